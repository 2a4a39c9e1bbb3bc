"""ctypes binding of libdcgs (``include/dcgs.h``): argument marshalling only.

Every computation happens in the HIP library; this module converts torch
tensors to device pointers, cameras to ``dcgs_camera`` structs, and status
codes to exceptions.  Importing it does not load the library; the first use
does, and raises ``LibraryMissing`` if ``libdcgs.so`` was not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcgs.so")

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_CAPACITY", 3: "E_BUDGET", 4: "E_NOT_RESIDENT",
          5: "E_HIP", 6: "E_RANGE"}


class LibraryMissing(RuntimeError):
    pass


class DcgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("z_near", C.c_double),
                ("z_far", C.c_double)]

    @staticmethod
    def of(cam: dict) -> "Camera":
        c = Camera()
        c.R[:] = [float(x) for x in np.asarray(cam["R"], np.float64).reshape(9)]
        c.t[:] = [float(x) for x in np.asarray(cam["t"], np.float64).reshape(3)]
        c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
        c.width, c.height = cam["width"], cam["height"]
        c.z_near, c.z_far = cam["z_near"], cam["z_far"]
        return c


class AdamConfig(C.Structure):
    _fields_ = [("lr", C.c_float * 6), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]

    @staticmethod
    def of(lr, beta1=0.9, beta2=0.999, eps=1e-15) -> "AdamConfig":
        a = AdamConfig()
        a.lr[:] = [float(x) for x in lr]
        a.beta1, a.beta2, a.eps = beta1, beta2, eps
        return a


class WindowConfig(C.Structure):
    _fields_ = [("sh_degree", C.c_int), ("width", C.c_int), ("height", C.c_int),
                ("n_views", C.c_int), ("tile_w", C.c_int), ("tile_h", C.c_int),
                ("pixels_per_lane", C.c_int), ("capacity", C.c_int64),
                ("pair_capacity", C.c_int64), ("bg", C.c_float * 3), ("loss_norm", C.c_double),
                ("adam", AdamConfig), ("params", C.c_void_p), ("grad", C.c_void_p),
                ("src", C.c_void_p), ("gmask", C.c_void_p), ("rgb", C.c_void_p),
                ("depth", C.c_void_p), ("dl_drgb", C.c_void_p), ("targets", C.c_void_p),
                ("stats", C.c_void_p), ("lambda_s", C.c_double), ("lambda_depth", C.c_double),
                ("depth_targets", C.c_void_p), ("dl_ddepth", C.c_void_p)]


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
INT = C.c_int
DBL = C.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "dcgs_version": (C.c_char_p, []),
    "dcgs_create": (INT, [C.POINTER(P), INT]),
    "dcgs_destroy": (None, [P]),
    "dcgs_last_error": (C.c_char_p, [P]),
    "dcgs_chunk_ids": (INT, [P, P, I64, I64, DBL, P, P]),
    "dcgs_select_chunks": (INT, [P, P, INT, P, INT, DBL, P, P, P, P]),
    "dcgs_select_chunks_noalloc": (INT, [P, P, INT, P, INT, DBL, P, P, P, P]),
    "dcgs_keyframe_overlap": (INT, [P, P, INT, INT, DBL, P, INT, DBL, P, INT, P, P, P, P, INT,
                                    P, P, P]),
    "dcgs_pool_create": (INT, [P, INT, I64, C.POINTER(P)]),
    "dcgs_pool_destroy": (None, [P]),
    "dcgs_pool_ingest": (INT, [P, P, I64, DBL, P]),
    "dcgs_pool_chunks": (INT, [P, P, P, INT, C.POINTER(INT)]),
    "dcgs_pool_device_ids": (P, [P, C.POINTER(INT)]),
    "dcgs_pool_require": (INT, [P, P, INT, I64, C.POINTER(INT), C.POINTER(INT), P]),
    "dcgs_pool_read_chunk": (INT, [P, C.c_uint64, P, P, P, P]),
    "dcgs_pool_prefetch": (INT, [P, P, INT, I64, C.POINTER(INT), P]),
    "dcgs_pool_stats": (INT, [P, P, INT]),
    "dcgs_pool_resident": (INT, [P, P, INT, C.POINTER(INT), C.POINTER(I64)]),
    "dcgs_compact": (INT, [P, P, P, INT, P, I64, P, P, I64, C.POINTER(I64), P]),
    "dcgs_pool_loop_closure": (INT, [P, P, P, INT, P, INT, P, INT, P]),
    "dcgs_state_create": (INT, [P, C.POINTER(P)]),
    "dcgs_state_destroy": (None, [P]),
    "dcgs_render_fwd": (INT, [P, P, P, I64, I64, INT, P, INT, P, INT, P, INT, INT, INT, P, P, P,
                              P]),
    "dcgs_render_bwd": (INT, [P, P, P, I64, I64, P, P, P, I64, INT, P, P]),
    "dcgs_loss_l1": (INT, [P, P, P, I64, DBL, P, P, P]),
    "dcgs_adam_step": (INT, [P, P, P, I64, I64, P, P]),
    "dcgs_loss_mapping": (INT, [P, P, P, P, P, INT, INT, INT, DBL, DBL, P, P, P, P]),
    "dcgs_sample_pixels": (INT, [P, P, P, P, INT, INT, DBL, DBL, P, P, P, P]),
    "dcgs_autotune": (INT, [P, P, P, I64, I64, INT, P, P, INT, INT, P, P, P, P]),
    "dcgs_window_create": (INT, [P, P, P, C.POINTER(P)]),
    "dcgs_window_destroy": (None, [P]),
    "dcgs_window_launch": (INT, [P, P, P, INT, P, C.POINTER(I64), P]),
    "dcgs_window_sync": (INT, [P, C.POINTER(I64), C.POINTER(INT)]),
    "dcgs_window_pairs": (INT, [P, C.POINTER(I64)]),
    "dcgs_prefetch_labels": (INT, [P, P, INT, INT, DBL, P, P]),
    "dcgs_prefetch_features": (INT, [P, P, INT, P, INT, DBL, DBL, P, P, P, P, P]),
    "dcgs_mlp_forward": (INT, [P, P, P, P, I64, P, P, P, P, P, P]),
    "dcgs_mlp_backward": (INT, [P, P, P, P, P, P, P, P, P, P, I64, C.c_float, P, P, P]),
    "dcgs_mlp_adam": (INT, [P, P, P, P, P, P, I64, DBL, DBL, DBL, DBL, P]),
    "dcgs_mlp_round": (INT, [P, P, P, P]),
    "dcgs_prefetch_predict": (INT, [P, P, P, P, DBL, DBL, C.c_float, P, P, P, P]),
    "dcgs_profile_enable": (INT, [P, INT]),
    "dcgs_profile_read": (INT, [P, P, P, INT]),
    "dcgs_state_info": (INT, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32), C.POINTER(I32)]),
    "dcgs_pairs_fit": (INT, [I64, I64]),
    "dcgs_state_work": (INT, [P, C.POINTER(I64), C.POINTER(I64), P]),
    "dcgs_state_export": (INT, [P, P, P, P, P, P, P, P, P]),
}

_lib = None


def lib():
    """The loaded library (raises LibraryMissing when it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} not found; build it with "
                                 "`python -m paper_2511_23030_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ptr(t) -> int | None:
    """Device (or host) address of a torch tensor / numpy array, None for None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """A libdcgs context on one HIP device."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libdcgs needs a HIP device; none is visible")
        self.device = device
        torch.cuda.set_device(device)
        h = P()
        self._check(lib().dcgs_create(C.byref(h), device), None)
        self.h = h

    def _check(self, st: int, handle=None):
        if st != 0:
            msg = lib().dcgs_last_error(handle if handle is not None else getattr(self, "h", None))
            raise DcgsError(st, (msg or b"").decode())

    def check(self, st: int):
        self._check(st, self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().dcgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- chunks ----
    def chunk_ids(self, mean, chunk_size: float, stream=None):
        import torch
        n = mean.shape[1]
        out = torch.empty(n, dtype=torch.int64, device=mean.device)
        self.check(lib().dcgs_chunk_ids(self.h, ptr(mean), n, mean.stride(0), chunk_size,
                                        ptr(out), stream_handle(stream)))
        return out

    def select_chunks(self, cams: list, ids, chunk_size: float, stream=None):
        """ids: device int64 (uint64 bit patterns), ascending.  Returns
        (out_ids, out_mask, count) device tensors; count is a 1-element int32."""
        import torch
        n = ids.numel()
        arr = (Camera * len(cams))(*[Camera.of(c) for c in cams])
        out_ids = torch.empty(max(n, 1), dtype=torch.int64, device=ids.device)
        out_mask = torch.empty(max(n, 1), dtype=torch.int16, device=ids.device)
        count = torch.empty(1, dtype=torch.int32, device=ids.device)
        self.check(lib().dcgs_select_chunks(self.h, C.cast(arr, P), len(cams), ptr(ids), n,
                                            chunk_size, ptr(out_ids), ptr(out_mask), ptr(count),
                                            stream_handle(stream)))
        return out_ids, out_mask, count

    def keyframe_overlap(self, keyframes: list, latest: int, ids, chunk_size: float,
                         active_ids: np.ndarray, grid: float = 200.0, n_window: int = 0,
                         stream=None) -> dict:
        """Keyframe selection quantities (dcgs_keyframe_overlap) for host
        cameras `keyframes`: in_set (Eq. 8 membership of K(p_latest)),
        n_visible, n_overlap, overlap (Eq. 7) and, when n_window > 0, the
        window chosen from the candidate set.  ids: the device chunk grid
        (int64 tensor of uint64 bit patterns, or a pool's (address, count)
        from Pool.device_ids()); active_ids: host uint64."""
        m = len(keyframes)
        addr, n_ids = ids if isinstance(ids, tuple) else (ptr(ids), ids.numel())
        arr = (Camera * m)(*[Camera.of(c) for c in keyframes])
        act = np.ascontiguousarray(np.unique(np.asarray(active_ids, np.uint64)))
        out = dict(in_set=np.zeros(m, np.uint8), n_visible=np.zeros(m, np.int32),
                   n_overlap=np.zeros(m, np.int32), overlap=np.zeros(m, np.float64))
        win = np.zeros(max(n_window, 1), np.int32)
        nw = I32(0)
        self.check(lib().dcgs_keyframe_overlap(
            self.h, C.cast(arr, P), m, int(latest), float(grid), addr, n_ids,
            float(chunk_size), act.ctypes.data if act.size else None, act.size,
            out["in_set"].ctypes.data, out["n_visible"].ctypes.data,
            out["n_overlap"].ctypes.data, out["overlap"].ctypes.data, int(n_window),
            win.ctypes.data if n_window > 0 else None, C.byref(nw), stream_handle(stream)))
        out["window"] = win[:nw.value].copy() if n_window > 0 else None
        return out

    STAGES = ("select", "compact", "preprocess", "depth_sort", "scan_emit", "tile_sort",
              "ranges", "raster_fwd", "loss", "raster_bwd", "preprocess_bwd", "adam")

    def profile(self, enable: bool):
        self.check(lib().dcgs_profile_enable(self.h, int(enable)))

    def profile_read(self) -> dict:
        n = len(self.STAGES)
        ms = np.zeros(n, np.float64)
        calls = np.zeros(n, np.int64)
        self.check(lib().dcgs_profile_read(self.h, ms.ctypes.data, calls.ctypes.data, n))
        return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(self.STAGES)}

    def loss_l1(self, rgb, target, dl_out=None, stats=None, stream=None, norm=None):
        """L1 loss gradient sign(rgb - target) / norm (norm defaults to the
        element count of one image: 3HW for rgb [.., 3, H, W])."""
        import torch
        dl = torch.empty_like(rgb) if dl_out is None else dl_out
        st = torch.empty(2, dtype=torch.float64, device=rgb.device) if stats is None else stats
        if norm is None:
            norm = float(rgb.shape[-1] * rgb.shape[-2] * rgb.shape[-3]) if rgb.dim() >= 3 \
                else float(rgb.numel())
        self.check(lib().dcgs_loss_l1(self.h, ptr(rgb), ptr(target), rgb.numel(), float(norm),
                                      ptr(dl), ptr(st), stream_handle(stream)))
        return dl, st

    def loss_mapping(self, rgb, target, depth=None, depth_target=None, lambda_s=0.2,
                     lambda_depth=0.0, dl_out=None, dld_out=None, stats=None, stream=None):
        """Eqs. (2)-(4): rgb, target [V, 3, H, W] (or [3, H, W]); depth,
        depth_target [V, H, W].  Returns (dL/drgb, dL/ddepth or None,
        stats [4]); no host synchronisation (see loss_value)."""
        import torch
        V = rgb.shape[0] if rgb.dim() == 4 else 1
        H, W = rgb.shape[-2], rgb.shape[-1]
        dl = torch.empty_like(rgb) if dl_out is None else dl_out
        dld = None
        if depth is not None and lambda_depth != 0.0:
            dld = torch.empty_like(depth) if dld_out is None else dld_out
        st = torch.empty(4, dtype=torch.float64, device=rgb.device) if stats is None else stats
        self.check(lib().dcgs_loss_mapping(
            self.h, ptr(rgb), ptr(target), ptr(depth), ptr(depth_target), V, H, W,
            float(lambda_s), float(lambda_depth), ptr(dl), ptr(dld), ptr(st),
            stream_handle(stream)))
        return dl, dld, st

    def sample_pixels(self, image, render, u, beta=2.0, sigma=1.0, stream=None):
        """LoG sampling: (P_s map [H, W], raster indices of the sampled
        pixels) for image, render [3, H, W] and draws u [H, W]."""
        import torch
        H, W = image.shape[-2], image.shape[-1]
        ps = torch.empty(H, W, dtype=torch.float32, device=image.device)
        idx = torch.empty(H * W, dtype=torch.int32, device=image.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=image.device)
        self.check(lib().dcgs_sample_pixels(self.h, ptr(image), ptr(render), ptr(u), H, W,
                                            float(beta), float(sigma), ptr(ps), ptr(idx),
                                            ptr(cnt), stream_handle(stream)))
        return ps, idx[:int(cnt.item())]

    @staticmethod
    def loss_value(stats, n_views: int, H: int, W: int, lambda_s: float,
                   lambda_depth: float) -> float:
        """The loss of Eq. (2) summed over views from loss_mapping's stats."""
        s = stats.cpu().numpy()
        n = 3.0 * H * W
        return float((1 - lambda_s) * s[0] / n + lambda_s * (n_views - s[2] / n) +
                     lambda_depth * s[3] / (H * W))


class Pool:
    """Chunk store (pinned host) plus device residency pool with an LRU budget."""

    def __init__(self, ctx: Context, sh_degree: int, budget: int):
        h = P()
        ctx.check(lib().dcgs_pool_create(ctx.h, sh_degree, int(budget), C.byref(h)))
        self.ctx, self.h, self.sh_degree = ctx, h, sh_degree
        self.R = 11 + 3 * (sh_degree + 1) ** 2

    def close(self):
        if getattr(self, "h", None):
            lib().dcgs_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ingest(self, params: np.ndarray, chunk_size: float, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape[0] == self.R
        self.ctx.check(lib().dcgs_pool_ingest(self.h, p.ctypes.data, p.shape[1], chunk_size,
                                              stream_handle(stream)))

    def chunks(self):
        n = INT()
        lib().dcgs_pool_chunks(self.h, None, None, 0, C.byref(n))
        ids = np.zeros(n.value, np.uint64)
        counts = np.zeros(n.value, np.int64)
        self.ctx.check(lib().dcgs_pool_chunks(self.h, ids.ctypes.data, counts.ctypes.data,
                                              n.value, C.byref(n)))
        return ids, counts

    def device_ids(self):
        """(device address, count) of the ascending occupied chunk ids."""
        n = INT()
        addr = lib().dcgs_pool_device_ids(self.h, C.byref(n))
        return addr, n.value

    def require(self, ids: np.ndarray, now: int, stream=None):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        lo, ev = INT(), INT()
        self.ctx.check(lib().dcgs_pool_require(self.h, ids.ctypes.data, ids.size, now,
                                               C.byref(lo), C.byref(ev), stream_handle(stream)))
        return lo.value, ev.value

    def prefetch(self, ids: np.ndarray, now: int, stream=None) -> int:
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        k = INT()
        self.ctx.check(lib().dcgs_pool_prefetch(self.h, ids.ctypes.data, ids.size, now,
                                                C.byref(k), stream_handle(stream)))
        return k.value

    STAT_NAMES = ("loads", "evictions", "prefetched", "misses", "hits", "bytes_h2d", "bytes_d2h",
                  "resident")

    def stats(self) -> dict:
        out = np.zeros(8, np.int64)
        self.ctx.check(lib().dcgs_pool_stats(self.h, out.ctypes.data, 8))
        return dict(zip(self.STAT_NAMES, out.tolist()))

    def read_chunk(self, cid: int, count: int):
        p = np.zeros((self.R, count), np.float32)
        m = np.zeros_like(p)
        v = np.zeros_like(p)
        s = np.zeros(count, np.int32)
        self.ctx.check(lib().dcgs_pool_read_chunk(self.h, int(cid), p.ctypes.data, m.ctypes.data,
                                                  v.ctypes.data, s.ctypes.data))
        return p, m, v, s

    LOOP_STAT_NAMES = ("affected_chunks", "corrected", "moved", "chunks_rebuilt",
                       "chunks_written", "reset", "chunks_after")

    def loop_closure(self, keyframes: list, corrections, junctions: list = (), stream=None) -> dict:
        """Sec. III-G correction of the store.  corrections: [K][3][4] or
        [K][12] float64, rotation rows then translation (R | t)."""
        K = len(keyframes)
        corr = np.zeros((max(K, 1), 12), np.float64)
        if K:
            c = np.asarray(corrections, np.float64).reshape(K, -1)
            if c.shape[1] == 12 and np.asarray(corrections).ndim == 3:   # [K][3][4]
                c3 = np.asarray(corrections, np.float64)
                c = np.concatenate([c3[:, :, :3].reshape(K, 9), c3[:, :, 3]], 1)
            corr[:K] = c
        kf = (Camera * max(K, 1))(*[Camera.of(x) for x in keyframes])
        J = len(junctions)
        jc = (Camera * max(J, 1))(*[Camera.of(x) for x in junctions])
        out = np.zeros(7, np.int64)
        self.ctx.check(lib().dcgs_pool_loop_closure(self.h, C.cast(kf, P), corr.ctypes.data, K,
                                                    C.cast(jc, P), J, out.ctypes.data, 7,
                                                    stream_handle(stream)))
        return dict(zip(self.LOOP_STAT_NAMES, out.tolist()))

    def resident(self):
        n, g = INT(), I64()
        lib().dcgs_pool_resident(self.h, None, 0, C.byref(n), C.byref(g))
        ids = np.zeros(max(n.value, 1), np.uint64)
        self.ctx.check(lib().dcgs_pool_resident(self.h, ids.ctypes.data, ids.size, C.byref(n),
                                                C.byref(g)))
        return ids[:n.value], g.value

    def compact(self, ids: np.ndarray, out, out_src, masks: np.ndarray | None = None,
                out_gmask=None, stream=None) -> int:
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        mk = None if masks is None else np.ascontiguousarray(masks, dtype=np.uint16)
        n = I64()
        self.ctx.check(lib().dcgs_compact(self.h, ids.ctypes.data, None if mk is None else mk.ctypes.data,
                                          ids.size, ptr(out), out.stride(0), ptr(out_src),
                                          ptr(out_gmask), out.shape[1], C.byref(n),
                                          stream_handle(stream)))
        return n.value

    def adam_step(self, src, grad, n: int, cfg: AdamConfig, stream=None):
        self.ctx.check(lib().dcgs_adam_step(self.h, ptr(src), ptr(grad), n, grad.stride(0),
                                            C.byref(cfg), stream_handle(stream)))


class RenderState:
    """Forward state of one render (records, sorted pairs, ranges, per-pixel
    transmittance and last position) kept for its backward."""

    def __init__(self, ctx: Context):
        h = P()
        ctx.check(lib().dcgs_state_create(ctx.h, C.byref(h)))
        self.ctx, self.h = ctx, h

    def close(self):
        if getattr(self, "h", None):
            lib().dcgs_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, params, n: int, sh_degree: int, cam, bg, tile=(16, 16),
                rgb=None, depth=None, T=None, stream=None, ppt: int = 0, gmask=None,
                mask_shift: int = 0):
        """Render one camera (dict) or a window of cameras (list of dicts).
        Outputs are [3, H, W] / [H, W] for one camera and [V, 3, H, W] /
        [V, H, W] for a list.  gmask: device int16 [n] view bits or None."""
        import torch
        cams = cam if isinstance(cam, (list, tuple)) else [cam]
        V = len(cams)
        H, W = cams[0]["height"], cams[0]["width"]
        dev = params.device
        lead = (V,) if isinstance(cam, (list, tuple)) else ()
        rgb = torch.empty(*lead, 3, H, W, dtype=torch.float32, device=dev) if rgb is None else rgb
        depth = torch.empty(*lead, H, W, dtype=torch.float32, device=dev) if depth is None else depth
        bgv = (C.c_float * 3)(*[float(x) for x in bg])
        arr = (Camera * V)(*[Camera.of(c) for c in cams])
        self.ctx.check(lib().dcgs_render_fwd(self.ctx.h, self.h, ptr(params), n, params.stride(0),
                                             sh_degree, ptr(gmask), mask_shift, C.cast(arr, P),
                                             V, bgv,
                                             tile[0], tile[1], ppt, ptr(rgb), ptr(depth), ptr(T),
                                             stream_handle(stream)))
        self.n_views = V
        return rgb, depth

    def backward(self, params, n: int, dl_drgb, dl_ddepth=None, grad=None, accumulate=False,
                 grad2d=None, stream=None):
        import torch
        if grad is None:
            grad = torch.empty(params.shape[0], max(n, 1), dtype=torch.float32, device=params.device)
        self.ctx.check(lib().dcgs_render_bwd(self.ctx.h, self.h, ptr(params), n, params.stride(0),
                                             ptr(dl_drgb), ptr(dl_ddepth), ptr(grad),
                                             grad.stride(0), int(accumulate), ptr(grad2d),
                                             stream_handle(stream)))
        return grad

    def autotune(self, params, n: int, sh_degree: int, cams: list, gmask=None, force=False,
                 stream=None):
        """Fastest raster shape (tile_w, tile_h, pixels_per_lane) for this
        window, and the per-shape forward+backward times in ms (empty when
        the context's cache answered)."""
        shape = (C.c_int * 3)()
        times = np.zeros(16, np.float64)
        k = INT()
        arr = (Camera * len(cams))(*[Camera.of(c) for c in cams])
        times[:] = -1.0
        self.ctx.check(lib().dcgs_autotune(self.ctx.h, self.h, ptr(params), n, params.stride(0),
                                           sh_degree, ptr(gmask), C.cast(arr, P), len(cams),
                                           int(force), shape, times.ctypes.data, C.byref(k),
                                           stream_handle(stream)))
        return (shape[0], shape[1], shape[2]), [t for t in times[:k.value] if t >= 0]

    def work(self, stream=None) -> tuple:
        """(list positions walked, in-box evaluations) of the last forward."""
        a, b = I64(), I64()
        self.ctx.check(lib().dcgs_state_work(self.h, C.byref(a), C.byref(b),
                                             stream_handle(stream)))
        return a.value, b.value

    def info(self):
        n, p, tx, ty = I64(), I64(), I32(), I32()
        lib().dcgs_state_info(self.h, C.byref(n), C.byref(p), C.byref(tx), C.byref(ty))
        return dict(n=n.value, n_pairs=p.value, tiles_x=tx.value, tiles_y=ty.value)

    def export(self, device, H: int, W: int, stream=None) -> dict:
        """Copy the last forward's keys, values, ranges, counts, records, boxes
        and per-pixel last positions to torch tensors (records indexed
        v * n + i over the views of the last forward)."""
        import torch
        inf = self.info()
        V = getattr(self, "n_views", 1)
        P_, n, nt = inf["n_pairs"], inf["n"] * V, inf["tiles_x"] * inf["tiles_y"] * V
        out = dict(keys=torch.empty(max(P_, 1), dtype=torch.int64, device=device),
                   values=torch.empty(max(P_, 1), dtype=torch.int32, device=device),
                   ranges=torch.empty(nt, 2, dtype=torch.int32, device=device),
                   counts=torch.empty(max(n, 1), dtype=torch.int32, device=device),
                   records=torch.empty(10, max(n, 1), dtype=torch.float32, device=device),
                   box=torch.empty(4, max(n, 1), dtype=torch.int32, device=device),
                   last=torch.empty(V, H, W, dtype=torch.int32, device=device))
        self.ctx.check(lib().dcgs_state_export(self.h, ptr(out["keys"]), ptr(out["values"]),
                                               ptr(out["ranges"]), ptr(out["counts"]),
                                               ptr(out["records"]), ptr(out["box"]),
                                               ptr(out["last"]), stream_handle(stream)))
        out["keys"] = out["keys"][:P_]
        out["values"] = out["values"][:P_]
        out["counts"] = out["counts"][:n]
        out["records"] = out["records"][:, :n]
        out["box"] = out["box"][:, :n]
        if V == 1:
            out["last"] = out["last"][0]
        return out


class Window:
    """A graph-captured mapping window (dcgs_window_*): compaction, then one
    graph replay of forward, loss, backward and Adam for all views."""

    def __init__(self, ctx: "Context", pool: "Pool", sh_degree: int, width: int, height: int,
                 n_views: int, tile, ppt: int, capacity: int, pair_capacity: int, bg, adam,
                 params, grad, src, gmask, rgb, depth, dl, targets, stats, loss_norm: float,
                 lambda_s: float = 0.0, lambda_depth: float = 0.0, depth_targets=None,
                 dl_ddepth=None):
        self.ctx, self.pool = ctx, pool
        c = WindowConfig()
        c.sh_degree, c.width, c.height, c.n_views = sh_degree, width, height, n_views
        c.tile_w, c.tile_h, c.pixels_per_lane = int(tile[0]), int(tile[1]), int(ppt)
        c.capacity, c.pair_capacity = int(capacity), int(pair_capacity)
        c.bg[:] = [float(x) for x in bg]
        c.loss_norm = float(loss_norm)
        c.lambda_s, c.lambda_depth = float(lambda_s), float(lambda_depth)
        c.depth_targets, c.dl_ddepth = ptr(depth_targets), ptr(dl_ddepth)
        c.adam = adam
        for name, t in (("params", params), ("grad", grad), ("src", src), ("gmask", gmask),
                        ("rgb", rgb), ("depth", depth), ("dl_drgb", dl), ("targets", targets),
                        ("stats", stats)):
            setattr(c, name, ptr(t))
        self._keep = (params, grad, src, gmask, rgb, depth, dl, targets, stats, depth_targets,
                      dl_ddepth)
        self.cfg = c
        h = P()
        ctx.check(lib().dcgs_window_create(ctx.h, pool.h, C.byref(c), C.byref(h)))
        self.h = h
        self.n_views = n_views

    def launch(self, ids: np.ndarray, masks: np.ndarray, cams: list, stream=None) -> int:
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        masks = np.ascontiguousarray(masks, dtype=np.uint16)
        arr = (Camera * len(cams))(*[Camera.of(c) for c in cams])
        n = I64()
        self.ctx.check(lib().dcgs_window_launch(self.h, ids.ctypes.data, masks.ctypes.data,
                                                ids.size, C.cast(arr, P), C.byref(n),
                                                stream_handle(stream)))
        return n.value

    def sync(self) -> tuple:
        """Wait for the launches; (pairs needed, launches skipped) after an
        overflow, else (0, 0)."""
        need, skipped = I64(), INT()
        st = lib().dcgs_window_sync(self.h, C.byref(need), C.byref(skipped))
        if st == 2:
            return need.value, skipped.value
        self.ctx.check(st)
        return 0, 0

    def pairs(self) -> int:
        v = I64()
        self.ctx.check(lib().dcgs_window_pairs(self.h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "h", None):
            lib().dcgs_window_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
