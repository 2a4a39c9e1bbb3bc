"""The allocation-free selection entry point, called through the C ABI,
equals dcgs_select_chunks bit for bit on two calls in a row (the second on
a smaller grid and fewer views, so stale scratch from the first call would
show), and rejects a grid beyond its static scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenegen
from oracle import chunks as oc
from paper_2511_23030_amd import dcgs as D

pytestmark = pytest.mark.gpu

MAX_CHUNKS = 65536


def _call(ctx, fn, cams, ids_dev, s):
    n = ids_dev.numel()
    arr = (D.Camera * len(cams))(*[D.Camera.of(c) for c in cams])
    out_ids = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda")
    out_mask = torch.full((max(n, 1),), -1, dtype=torch.int16, device="cuda")
    count = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    st = fn(ctx.h, C.cast(arr, C.c_void_p), len(cams), D.ptr(ids_dev), n, s, D.ptr(out_ids),
            D.ptr(out_mask), D.ptr(count), D.stream_handle(None))
    torch.cuda.synchronize()
    k = int(count.item())
    return st, out_ids[:k].cpu().numpy(), out_mask[:k].cpu().numpy(), k


def _grid(side, z_layers, s, offset):
    ax = np.arange(side) + offset
    cx, cy, cz = np.meshgrid(ax, ax, np.arange(z_layers) - z_layers // 2, indexing="ij")
    return np.sort(oc.encode_id(np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)))


def test_noalloc_select_equals_select_on_two_calls(ctx):
    L = D.lib()
    s = 1.0
    cases = [
        # a large grid seen by 16 views, then a smaller one seen by 3: the
        # second call's masks must not pick up the first call's entries
        (_grid(40, 5, s, -20), scenegen.random_cameras(16, seed=71, extent=6.0)),
        (_grid(9, 3, s, -4), scenegen.random_cameras(3, seed=72, extent=3.0)),
    ]
    for ids, cams in cases:
        dev = torch.from_numpy(ids.view(np.int64)).cuda()
        st0, ids0, m0, k0 = _call(ctx, L.dcgs_select_chunks, cams, dev, s)
        st1, ids1, m1, k1 = _call(ctx, L.dcgs_select_chunks_noalloc, cams, dev, s)
        assert st0 == 0 and st1 == 0, (st0, st1, L.dcgs_last_error(ctx.h))
        print(f"grid {ids.size} chunks, {len(cams)} views: {k1} visible", flush=True)
        assert k1 == k0 and k1 > 0
        assert (ids1 == ids0).all() and (m1 == m0).all()
        if ids.size > 1000:
            continue  # the oracle's vertex enumeration takes a minute here
        # and both equal the oracle's exact visibility
        ref = oc.select_chunks(cams, ids, s)
        assert not ref["tie"].any()
        assert (ids1.view(np.uint64) == ref["union_ids"]).all()
        assert (m1.view(np.uint16) == ref["view_mask"]).all()


def test_noalloc_select_rejects_grids_beyond_its_scratch(ctx):
    L = D.lib()
    cams = scenegen.random_cameras(1, seed=73, extent=3.0)
    ids = torch.zeros(MAX_CHUNKS + 1, dtype=torch.int64, device="cuda")
    st, _, _, _ = _call(ctx, L.dcgs_select_chunks_noalloc, cams, ids, 1.0)
    assert st == 2  # DCGS_E_CAPACITY, nothing launched
    assert b"scratch" in L.dcgs_last_error(ctx.h)
