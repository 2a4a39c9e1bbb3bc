"""One mapping iteration of the paper's optimisation loop (Sec. III-E):
select the keyframe's visible chunks, make them resident under the LRU
budget, compact their Gaussians, render RGB and depth, take the L1 loss,
back-propagate, and apply Adam to the pool.  Every step runs in libdcgs;
this class owns the device buffers and sequences the calls.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import dcgs as D

DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4)


class MappingLoop:
    def __init__(self, ctx: D.Context, pool: D.Pool, sh_degree: int, chunk_size: float,
                 capacity: int, width: int, height: int, tile=(16, 16), bg=(0.0, 0.0, 0.0),
                 lr=DEFAULT_LR):
        self.ctx, self.pool = ctx, pool
        self.deg, self.s, self.tile, self.bg = sh_degree, float(chunk_size), tuple(tile), bg
        self.R = 11 + 3 * (sh_degree + 1) ** 2
        dev = torch.device("cuda", ctx.device)
        self.cap = int(capacity)
        self.params = torch.empty(self.R, self.cap, dtype=torch.float32, device=dev)
        self.grad = torch.empty(self.R, self.cap, dtype=torch.float32, device=dev)
        self.src = torch.empty(self.cap, dtype=torch.int32, device=dev)
        self.rgb = torch.empty(3, height, width, dtype=torch.float32, device=dev)
        self.depth = torch.empty(height, width, dtype=torch.float32, device=dev)
        self.dl = torch.empty(3, height, width, dtype=torch.float32, device=dev)
        self.stats = torch.zeros(2, dtype=torch.float64, device=dev)
        self.sel_ids = torch.empty(4096, dtype=torch.int64, device=dev)
        self.sel_mask = torch.empty(4096, dtype=torch.int16, device=dev)
        self.sel_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.state = D.RenderState(ctx)
        self.adam = D.AdamConfig.of(lr)
        self.iter = 0
        self.last = {}

    def select(self, cam: dict) -> np.ndarray:
        """Visible chunk ids of `cam` (host copy; one sync)."""
        addr, n = self.pool.device_ids()
        if n > self.sel_ids.numel():
            dev = self.sel_ids.device
            self.sel_ids = torch.empty(n, dtype=torch.int64, device=dev)
            self.sel_mask = torch.empty(n, dtype=torch.int16, device=dev)
        camc = D.Camera.of(cam)
        self.ctx.check(D.lib().dcgs_select_chunks(
            self.ctx.h, C.byref(camc), 1, addr, n, self.s, D.ptr(self.sel_ids),
            D.ptr(self.sel_mask), D.ptr(self.sel_count), D.stream_handle()))
        k = int(self.sel_count.item())
        return self.sel_ids[:k].cpu().numpy().view(np.uint64)

    def step(self, cam: dict, target: torch.Tensor, ids: np.ndarray | None = None) -> dict:
        """One plain mapping iteration for one keyframe; returns host stats."""
        if ids is None:
            ids = self.select(cam)
        loaded, evicted = self.pool.require(ids, now=self.iter)
        n = self.pool.compact(ids, self.params, self.src)
        self.state.forward(self.params, n, self.deg, cam, self.bg, self.tile, self.rgb, self.depth)
        self.ctx.loss_l1(self.rgb, target, self.dl, self.stats)
        self.state.backward(self.params, n, self.dl, None, self.grad, accumulate=False)
        self.pool.adam_step(self.src, self.grad, n, self.adam)
        self.iter += 1
        self.last = dict(n_active=n, n_chunks=int(ids.size), loaded=loaded, evicted=evicted)
        return self.last

    def loss_psnr(self, numel: int) -> tuple[float, float]:
        s = self.stats.cpu().numpy()
        mse = s[1] / numel
        return float(s[0] / numel), float(10.0 * np.log10(1.0 / max(mse, 1e-30)))
