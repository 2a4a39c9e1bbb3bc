"""Learned chunk prefetch: binding of the prefetch calls of libdcgs and the
training / evaluation driver around them.

The network predicts, from the last 8 camera poses, which of the 64 x 64
chunk cells around the camera the exact frustum test (Sec. III-D) will
select in the next `horizon` frames; MappingLoop stages the predicted
chunks on the pool's copy stream while the current frame computes, and the
exact test of each frame still loads whatever was missed.  Every numeric
step (labels, features, forward, backward, loss, Adam, thresholding) runs in
libdcgs kernels; this module allocates tensors, draws the seeded batch
order, and sequences calls.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import dcgs as D

N_PARAMS = 81409
N_BF16 = 80896
N_CAND = 4096
IN_DIM = 59
HIDDEN = 256
HIST = 8


def _cams(cams: list):
    arr = (D.Camera * len(cams))(*[D.Camera.of(c) for c in cams])
    return arr, C.cast(arr, C.c_void_p)


def labels(ctx: D.Context, cams: list, chunk_size: float, horizon: int = 5,
           stream=None) -> torch.Tensor:
    """[T, 4096] uint8 exact labels of a trajectory (device)."""
    out = torch.empty(len(cams), N_CAND, dtype=torch.uint8, device="cuda")
    arr, p = _cams(cams)
    ctx.check(D.lib().dcgs_prefetch_labels(ctx.h, p, len(cams), horizon, chunk_size, D.ptr(out),
                                           D.stream_handle(stream)))
    return out


def features(ctx: D.Context, cams: list, frames, chunk_size: float, pos_unit: float = 1.0,
             lab: torch.Tensor | None = None, X: torch.Tensor | None = None,
             stream=None) -> tuple:
    """Input rows of the listed frames: X [F*4096, 59], cell ids [F*4096]
    (uint64 as int64), and labels y [F*4096] when `lab` is given."""
    frames = np.ascontiguousarray(frames, dtype=np.int32)
    F = frames.size
    if X is None or X.numel() < F * N_CAND * IN_DIM:
        X = torch.empty(F * N_CAND, IN_DIM, dtype=torch.float32, device="cuda")
    ids = torch.empty(F * N_CAND, dtype=torch.int64, device="cuda")
    y = torch.empty(F * N_CAND, dtype=torch.uint8, device="cuda") if lab is not None else None
    arr, p = _cams(cams)
    ctx.check(D.lib().dcgs_prefetch_features(ctx.h, p, len(cams), frames.ctypes.data, F,
                                             chunk_size, pos_unit, D.ptr(lab), D.ptr(X),
                                             D.ptr(ids), D.ptr(y), D.stream_handle(stream)))
    return X[:F * N_CAND], ids, y


class PrefetchNet:
    """The 59 -> 256 -> 256 -> 1 network: float32 master parameters, their
    bfloat16 copy, Adam moments and scratch, all on the device."""

    def __init__(self, ctx: D.Context, theta0: np.ndarray, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8):
        assert theta0.size == N_PARAMS
        self.ctx = ctx
        self.theta = torch.from_numpy(np.ascontiguousarray(theta0, np.float32)).cuda()
        self.wb = torch.empty(N_BF16, dtype=torch.int16, device="cuda")
        self.m = torch.zeros(N_PARAMS, dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.m)
        self.grad = torch.zeros_like(self.m)
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.lr, self.betas, self.eps = lr, betas, eps
        self.step_count = 0
        self._act_n = 0
        ctx.check(D.lib().dcgs_mlp_round(ctx.h, D.ptr(self.theta), D.ptr(self.wb),
                                         D.stream_handle(None)))

    def _acts(self, n: int):
        if n > self._act_n:
            self.act = torch.empty(4, n, HIDDEN, dtype=torch.float32, device="cuda")
            self.logit = torch.empty(n, dtype=torch.float32, device="cuda")
            self._act_n = n
        return self.act, self.logit

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        n = X.shape[0]
        act, logit = self._acts(n)
        self.ctx.check(D.lib().dcgs_mlp_forward(
            self.ctx.h, D.ptr(self.theta), D.ptr(self.wb), D.ptr(X), n, D.ptr(act[0]),
            D.ptr(act[1]), D.ptr(act[2]), D.ptr(act[3]), D.ptr(logit), D.stream_handle(stream)))
        return logit[:n]

    def backward(self, X: torch.Tensor, y: torch.Tensor, pos_weight: float, stream=None):
        n = X.shape[0]
        act, logit = self.act, self.logit
        self.ctx.check(D.lib().dcgs_mlp_backward(
            self.ctx.h, D.ptr(self.theta), D.ptr(self.wb), D.ptr(X), D.ptr(act[0]),
            D.ptr(act[1]), D.ptr(act[2]), D.ptr(act[3]), D.ptr(logit), D.ptr(y), n,
            float(pos_weight), D.ptr(self.grad), D.ptr(self.loss), D.stream_handle(stream)))
        return self.grad

    def adam(self, lr: float | None = None, stream=None):
        self.step_count += 1
        self.ctx.check(D.lib().dcgs_mlp_adam(
            self.ctx.h, D.ptr(self.theta), D.ptr(self.wb), D.ptr(self.m), D.ptr(self.v),
            D.ptr(self.grad), self.step_count, self.lr if lr is None else lr, self.betas[0],
            self.betas[1], self.eps, D.stream_handle(stream)))

    def train_step(self, X, y, pos_weight: float, lr: float | None = None, stream=None):
        self.forward(X, stream)
        self.backward(X, y, pos_weight, stream)
        self.adam(lr, stream)
        return self.loss

    def predict(self, history: list, chunk_size: float, tau: float = 0.5, pos_unit: float = 1.0,
                stream=None) -> np.ndarray:
        """EncodedIDs of the cells with P(visible in the next frames) >= tau,
        from the last 8 cameras (history[0] = current).  One sync of
        `stream`."""
        hist = list(history)[:HIST]
        hist += [hist[-1]] * (HIST - len(hist))
        arr, p = _cams(hist)
        thr = math.log(tau / (1.0 - tau))
        with torch.cuda.stream(stream) if stream is not None else _null():
            # output buffers from the stream the prediction runs on (memory
            # released on another stream may still be written by its queue)
            if not hasattr(self, "_pick") or self._pick_stream is not stream:
                self._pick = torch.empty(N_CAND, dtype=torch.int64, device="cuda")
                self._pick_n = torch.zeros(1, dtype=torch.int32, device="cuda")
                self._pick_logit = torch.empty(N_CAND, dtype=torch.float32, device="cuda")
                self._pick_stream = stream
            self.ctx.check(D.lib().dcgs_prefetch_predict(
                self.ctx.h, D.ptr(self.theta), D.ptr(self.wb), p, chunk_size, pos_unit, thr,
                D.ptr(self._pick), D.ptr(self._pick_n), D.ptr(self._pick_logit),
                D.stream_handle(stream)))
            k = int(self._pick_n.item())
            return self._pick[:k].cpu().numpy().view(np.uint64)

    def state(self) -> np.ndarray:
        return self.theta.cpu().numpy()


def _null():
    import contextlib
    return contextlib.nullcontext()


def train(ctx: D.Context, trajectories: list, chunk_size: float, steps: int = 1500,
          frames_per_batch: int = 16, horizon: int = 5, pos_weight: float = 4.0,
          lr: float = 1e-3, seed: int = 0, theta0: np.ndarray | None = None,
          log_every: int = 0) -> tuple:
    """Train on the exact labels of `trajectories` (lists of cameras).  Each
    step takes `frames_per_batch` frames of one trajectory (seeded choice),
    all 4096 candidates of each.  Returns the network and the loss of every
    step (host floats, read once at the end)."""
    import scenegen
    if theta0 is None:
        theta0 = scenegen.mlp_init(seed)
    net = PrefetchNet(ctx, theta0, lr=lr)
    labs = [labels(ctx, cams, chunk_size, horizon) for cams in trajectories]
    rng = np.random.default_rng(seed)
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda")
    X = None
    for it in range(steps):
        k = int(rng.integers(len(trajectories)))
        T = len(trajectories[k])
        frames = rng.integers(0, max(T - horizon, 1), frames_per_batch)
        X, _, y = features(ctx, trajectories[k], frames, chunk_size, lab=labs[k], X=X)
        lr_it = lr * (0.1 + 0.9 * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1))))
        losses[it:it + 1].copy_(net.train_step(X, y, pos_weight, lr=lr_it))
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(f"prefetch train step {it}: loss {losses[it].item():.5f}", flush=True)
    return net, losses.cpu().numpy()


def evaluate(ctx: D.Context, net: PrefetchNet, cams: list, chunk_size: float,
             tau: float = 0.5, every: int = 1, occupied: np.ndarray | None = None) -> dict:
    """Chunk misses along a trajectory, judged by the exact test: a cell the
    exact test selects at frame t+1 that it did not select at frame t is a
    miss unless the network's prediction at frame t staged it.  Reports the
    miss rate with the network and without it (every such cell missed), and
    the volume staged.  `occupied` (EncodedIDs) restricts the count to
    cells that hold Gaussians."""
    lab1 = labels(ctx, cams, chunk_size, horizon=1)         # visible at t+1
    T = len(cams)
    occ = None if occupied is None else set(np.asarray(occupied, np.uint64).tolist())
    need_next = []                                          # cells visible at t+1
    for f0 in range(0, T - 1, 256):
        fr = np.arange(f0, min(f0 + 256, T - 1), dtype=np.int32)
        _, ids, y = features(ctx, cams, fr, chunk_size, lab=lab1)
        ids = ids.view(-1, N_CAND).cpu().numpy().view(np.uint64)
        y = y.view(-1, N_CAND).cpu().numpy().astype(bool)
        for r in range(fr.size):
            cells = set(ids[r][y[r]].tolist())
            need_next.append(cells if occ is None else cells & occ)
    new = missed = needed = staged = 0
    frames = range(1, T - 1, every)
    for t in frames:
        hist = [cams[max(t - k, 0)] for k in range(HIST)]
        pred = set(net.predict(hist, chunk_size, tau).tolist())
        if occ is not None:
            pred &= occ
        enter = need_next[t] - need_next[t - 1]
        new += len(enter)
        missed += len(enter - pred)
        needed += len(need_next[t])
        staged += len(pred)
    nf = len(frames)
    return dict(frames=nf, needed=needed, entering=new, missed=missed,
                miss_rate=missed / max(needed, 1), miss_rate_without=new / max(needed, 1),
                entering_covered=1.0 - missed / max(new, 1), staged_per_frame=staged / max(nf, 1))
