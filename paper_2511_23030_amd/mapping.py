"""One mapping iteration of the paper's optimisation loop (Sec. III-E):
select the keyframe's visible chunks, make them resident under the LRU
budget, compact their Gaussians, render RGB and depth, take the L1 loss,
back-propagate, and apply Adam to the pool.  Every step runs in libdcgs;
this class owns the device buffers and sequences the calls.
"""
from __future__ import annotations

import contextlib
import ctypes as C

import numpy as np
import torch

from . import dcgs as D

_nullctx = contextlib.nullcontext

DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4)


class MappingLoop:
    def __init__(self, ctx: D.Context, pool: D.Pool, sh_degree: int, chunk_size: float,
                 capacity: int, width: int, height: int, tile=(16, 16), bg=(0.0, 0.0, 0.0),
                 lr=DEFAULT_LR, ppt: int = 0, lambda_s: float = 0.0, lambda_depth: float = 0.0):
        self.ctx, self.pool = ctx, pool
        self.deg, self.s, self.tile, self.bg = sh_degree, float(chunk_size), tuple(tile), bg
        self.ppt = ppt
        self.R = 11 + 3 * (sh_degree + 1) ** 2
        dev = torch.device("cuda", ctx.device)
        self.cap = int(capacity)
        self.params = torch.empty(self.R, self.cap, dtype=torch.float32, device=dev)
        self.grad = torch.empty(self.R, self.cap, dtype=torch.float32, device=dev)
        self.src = torch.empty(self.cap, dtype=torch.int32, device=dev)
        self.rgb = torch.empty(3, height, width, dtype=torch.float32, device=dev)
        self.depth = torch.empty(height, width, dtype=torch.float32, device=dev)
        self.dl = torch.empty(3, height, width, dtype=torch.float32, device=dev)
        self.stats = torch.zeros(4, dtype=torch.float64, device=dev)
        # Eq. (3)'s SSIM weight and Eq. (2)'s depth weight (0: L1 only)
        self.lambda_s, self.lambda_depth = float(lambda_s), float(lambda_depth)
        self.dld = torch.empty(height, width, dtype=torch.float32, device=dev)
        self.state = D.RenderState(ctx)
        self.adam = D.AdamConfig.of(lr)
        self.iter = 0
        self.last = {}

    def _sel_buffers(self, n: int, side: bool):
        key = "_side_sel" if side else "_sel"
        buf = getattr(self, key, None)
        if buf is None or buf[0].numel() < n:
            dev = self.params.device
            m = max(n, 4096)
            buf = (torch.empty(m, dtype=torch.int64, device=dev),
                   torch.empty(m, dtype=torch.int16, device=dev),
                   torch.zeros(1, dtype=torch.int32, device=dev))
            setattr(self, key, buf)
        return buf

    def select_window(self, cams: list, stream: torch.cuda.Stream | None = None
                      ) -> tuple[np.ndarray, np.ndarray]:
        """Union of the chunks the views see (ascending ids) and each chunk's
        view mask (host copies).  Runs on `stream` (default: the current
        stream) and waits for that stream only."""
        addr, n = self.pool.device_ids()
        arr = (D.Camera * len(cams))(*[D.Camera.of(c) for c in cams])
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            # buffers of a side-stream selection come from that stream's
            # allocations: memory the compute stream released may still be
            # written by its queued kernels
            ids_t, mask_t, count_t = self._sel_buffers(n, stream is not None)
            self.ctx.check(D.lib().dcgs_select_chunks(
                self.ctx.h, C.cast(arr, C.c_void_p), len(cams), addr, n, self.s, D.ptr(ids_t),
                D.ptr(mask_t), D.ptr(count_t), D.stream_handle(stream)))
            k = int(count_t.item())
            return (ids_t[:k].cpu().numpy().view(np.uint64),
                    mask_t[:k].cpu().numpy().view(np.uint16))

    def _loss(self, rgb, target, depth, target_depth, dl, dld, stats=None):
        """The mapping loss of the rendered views (L1 only when both weights
        are 0); returns the depth gradient buffer or None."""
        H, W = rgb.shape[-2], rgb.shape[-1]
        st = self.stats if stats is None else stats
        if self.lambda_s == 0.0 and (self.lambda_depth == 0.0 or target_depth is None):
            self.ctx.loss_l1(rgb, target, dl, st, norm=3.0 * H * W)
            return None
        lam_d = self.lambda_depth if target_depth is not None else 0.0
        _, g, _ = self.ctx.loss_mapping(rgb, target, depth if lam_d else None,
                                        target_depth if lam_d else None, self.lambda_s, lam_d,
                                        dl_out=dl, dld_out=dld, stats=st)
        return g

    def schedule_window(self, keyframes: list, latest: int, n: int, grid: float = 200.0
                        ) -> np.ndarray:
        """Keyframe selection of a batching window (dcgs_keyframe_overlap):
        among the keyframes in the same `grid` cell as keyframe `latest`
        (the spatial candidate set), the n whose visible chunks are most
        resident in the pool (chunk overlap), ties to the more recent one."""
        res = self.ctx.keyframe_overlap(keyframes, latest, self.pool.device_ids(), self.s,
                                        self.pool.resident()[0], grid=grid, n_window=n)
        return res["window"]

    def select(self, cam: dict) -> np.ndarray:
        """Visible chunk ids of `cam` (host copy; one sync)."""
        return self.select_window([cam])[0]

    def prefetch_window(self, cams: list) -> tuple[np.ndarray, np.ndarray]:
        """Select the chunks of an upcoming window on a side stream (so the
        work already queued on the compute stream keeps running) and stage
        the missing ones on the pool's copy stream, evicting only chunks the
        frame just queued does not use.  Returns the selection, to be handed
        to that window's step so it is not computed twice."""
        if getattr(self, "_side_stream", None) is None:
            self._side_stream = torch.cuda.Stream(device=self.params.device)
        sel = self.select_window(cams, stream=self._side_stream)
        self.pool.prefetch(sel[0], now=self.iter - 1)
        return sel

    def prefetch_predicted(self, net, history: list, tau: float = 0.3) -> int:
        """Stage the chunks the prefetch network expects the next frames to
        need (from the last 8 cameras, history[0] the current one): its
        inference runs on a side stream, the copies on the pool's copy
        stream.  Returns the number of chunks asked for."""
        if getattr(self, "_side_stream", None) is None:
            self._side_stream = torch.cuda.Stream(device=self.params.device)
        if getattr(self, "_pool_ids", None) is None:
            self._pool_ids = self.pool.chunks()[0]
        ids = net.predict(history, self.s, tau, stream=self._side_stream)
        ids = ids[np.isin(ids, self._pool_ids)]
        self.pool.prefetch(ids, now=self.iter - 1)
        return int(ids.size)

    def _window_buffers(self, V: int):
        if getattr(self, "_wv", 0) != V:
            H, W = self.rgb.shape[1], self.rgb.shape[2]
            dev = self.rgb.device
            self.rgb_v = torch.empty(V, 3, H, W, dtype=torch.float32, device=dev)
            self.depth_v = torch.empty(V, H, W, dtype=torch.float32, device=dev)
            self.dl_v = torch.empty(V, 3, H, W, dtype=torch.float32, device=dev)
            self.dld_v = torch.empty(V, H, W, dtype=torch.float32, device=dev)
            self.gmask = torch.empty(self.cap, dtype=torch.int16, device=dev)
            self._wv = V

    def autotune(self, cams: list) -> tuple:
        """Pick the fastest raster shape for windows like `cams` (timed on
        this window's real Gaussians) and use it from now on."""
        V = len(cams)
        self._window_buffers(V)
        ids, masks = self.select_window(cams)
        self.pool.require(ids, now=self.iter)
        n = self.pool.compact(ids, self.params, self.src, masks=masks, out_gmask=self.gmask)
        shape, times = self.state.autotune(self.params, n, self.deg, list(cams), gmask=self.gmask)
        self.tile, self.ppt = shape[:2], shape[2]
        return shape, times

    def window_step(self, cams: list, targets: torch.Tensor, sel=None,
                    target_depths: torch.Tensor | None = None) -> dict:
        """One batched mapping iteration over a window of keyframes: one
        selection, one compaction of the union with per-Gaussian view masks,
        one forward and one backward launch sequence for all views, the loss
        summed over views, one Adam step.  `sel`: this window's selection
        if already made (prefetch_window)."""
        V = len(cams)
        self._window_buffers(V)
        ids, masks = self.select_window(cams) if sel is None else sel
        loaded, evicted = self.pool.require(ids, now=self.iter)
        n = self.pool.compact(ids, self.params, self.src, masks=masks, out_gmask=self.gmask)
        self.state.forward(self.params, n, self.deg, list(cams), self.bg, self.tile, self.rgb_v,
                           self.depth_v, ppt=self.ppt, gmask=self.gmask)
        dld = self._loss(self.rgb_v, targets, self.depth_v, target_depths, self.dl_v, self.dld_v)
        self.state.backward(self.params, n, self.dl_v, dld, self.grad, accumulate=False)
        self.pool.adam_step(self.src, self.grad, n, self.adam)
        self.iter += 1
        self.last = dict(n_active=n, n_chunks=int(ids.size), loaded=loaded, evicted=evicted,
                         views=V)
        return self.last

    def window_step_sequential(self, cams: list, targets: torch.Tensor, sel=None,
                               target_depths: torch.Tensor | None = None) -> dict:
        """The same update as window_step computed as one single-view forward
        and backward per view, accumulating gradients, then one Adam step
        (the per-view comparator of the batched path)."""
        V = len(cams)
        self._window_buffers(V)
        ids, masks = self.select_window(cams) if sel is None else sel
        loaded, evicted = self.pool.require(ids, now=self.iter)
        n = self.pool.compact(ids, self.params, self.src, masks=masks, out_gmask=self.gmask)
        H, W = self.rgb.shape[1], self.rgb.shape[2]
        stats = torch.zeros(4, dtype=torch.float64, device=self.rgb.device)
        for v in range(V):
            self.state.forward(self.params, n, self.deg, cams[v], self.bg, self.tile,
                               self.rgb_v[v], self.depth_v[v], ppt=self.ppt, gmask=self.gmask,
                               mask_shift=v)
            dld = self._loss(self.rgb_v[v], targets[v], self.depth_v[v],
                             None if target_depths is None else target_depths[v],
                             self.dl_v[v], self.dld_v[v])
            stats += self.stats
            self.state.backward(self.params, n, self.dl_v[v], dld, self.grad, accumulate=v > 0)
        self.stats.copy_(stats)
        self.pool.adam_step(self.src, self.grad, n, self.adam)
        self.iter += 1
        self.last = dict(n_active=n, n_chunks=int(ids.size), loaded=loaded, evicted=evicted,
                         views=V)
        return self.last

    def build_graph(self, V: int, pair_capacity: int):
        """(Re)build the graph-captured window for V views with room for
        `pair_capacity` (tile, Gaussian) pairs, using the current raster
        shape."""
        self._window_buffers(V)
        H, W = self.rgb.shape[1], self.rgb.shape[2]
        if getattr(self, "gtargets", None) is None or self.gtargets.shape[0] != V:
            self.gtargets = torch.empty(V, 3, H, W, dtype=torch.float32, device=self.rgb.device)
            self.gdtargets = torch.empty(V, H, W, dtype=torch.float32, device=self.rgb.device)
        if getattr(self, "win", None) is not None:
            self.win.close()
        ppt = self.ppt or {8: 1, 16: 2}.get(self.tile[0], 4)
        self.win = D.Window(self.ctx, self.pool, self.deg, W, H, V, self.tile, ppt, self.cap,
                            int(pair_capacity), self.bg, self.adam, self.params, self.grad,
                            self.src, self.gmask, self.rgb_v, self.depth_v, self.dl_v,
                            self.gtargets, self.stats, 3.0 * H * W, self.lambda_s,
                            self.lambda_depth, self.gdtargets, self.dld_v)
        self.win_pairs = int(pair_capacity)
        self._pending = []
        return self.win

    def _launch_graph(self, cams, targets, sel, target_depths=None) -> int:
        ids, masks = sel
        self.gtargets.copy_(targets)
        if self.lambda_depth > 0.0:
            self.gdtargets.copy_(target_depths)
        return self.win.launch(ids, masks, cams)

    def window_step_graph(self, cams: list, targets: torch.Tensor, sel=None,
                          target_depths: torch.Tensor | None = None) -> dict:
        """window_step through the graph-captured window (build_graph first),
        with the loss the loop was made with (L1, or the full loss with SSIM
        and, when lambda_depth > 0, the depth term: target_depths then
        required).  If a window overflowed its pair capacity (it and every
        later launch then changed nothing), the window is rebuilt with room
        for the pairs and the skipped windows run again, in order."""
        if self.lambda_depth > 0.0 and target_depths is None:
            raise ValueError("the graph's loss has a depth term: target_depths required")
        V = len(cams)
        ids, masks = self.select_window(cams) if sel is None else sel
        loaded, evicted = self.pool.require(ids, now=self.iter)
        try:
            n = self._launch_graph(cams, targets, (ids, masks), target_depths)
        except D.DcgsError as e:
            if e.status != 2:
                raise
            n = self._recover_graph(cams, targets, (ids, masks), target_depths)
        self._pending = (self._pending + [(cams, targets, (ids, masks), target_depths)])[-2:]
        self.iter += 1
        self.last = dict(n_active=n, n_chunks=int(ids.size), loaded=loaded, evicted=evicted,
                         views=V)
        return self.last

    def _redo(self, need: int, skipped: int, V: int):
        """Rebuild with room for `need` pairs and launch the `skipped` most
        recent windows again, in order."""
        redo = self._pending[len(self._pending) - skipped:] if skipped else []
        self.build_graph(V, max(int(need * 1.25) + 1024, 2 * self.win_pairs))
        for c, t, s_, d_ in redo:
            self.pool.require(s_[0], now=self.iter)
            self._launch_graph(c, t, s_, d_)
        self._pending = list(redo)

    def _recover_graph(self, cams, targets, sel, target_depths=None) -> int:
        need, skipped = self.win.sync()
        self._redo(need, skipped, len(cams))
        self.pool.require(sel[0], now=self.iter)
        return self._launch_graph(cams, targets, sel, target_depths)

    def sync_graph(self):
        """Wait for the graph launches; run again any that overflowed."""
        need, skipped = self.win.sync()
        while need:
            self._redo(need, skipped, self.win.n_views)
            need, skipped = self.win.sync()

    def step(self, cam: dict, target: torch.Tensor, ids: np.ndarray | None = None,
             target_depth: torch.Tensor | None = None) -> dict:
        """One plain mapping iteration for one keyframe; returns host stats."""
        if ids is None:
            ids = self.select(cam)
        loaded, evicted = self.pool.require(ids, now=self.iter)
        n = self.pool.compact(ids, self.params, self.src)
        self.state.forward(self.params, n, self.deg, cam, self.bg, self.tile, self.rgb, self.depth,
                           ppt=self.ppt)
        dld = self._loss(self.rgb, target, self.depth, target_depth, self.dl, self.dld)
        self.state.backward(self.params, n, self.dl, dld, self.grad, accumulate=False)
        self.pool.adam_step(self.src, self.grad, n, self.adam)
        self.iter += 1
        self.last = dict(n_active=n, n_chunks=int(ids.size), loaded=loaded, evicted=evicted)
        return self.last

    def loss_psnr(self, numel: int) -> tuple[float, float]:
        s = self.stats.cpu().numpy()
        mse = s[1] / numel
        return float(s[0] / numel), float(10.0 * np.log10(1.0 / max(mse, 1e-30)))
