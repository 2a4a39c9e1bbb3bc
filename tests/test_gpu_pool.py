"""GPU parity of the residency pool (LRU plan), compaction and Adam."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import chunks as oc
from oracle import optim as oo
from paper_2511_23030_amd import dcgs as D

pytestmark = pytest.mark.gpu

LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4)
LR32 = [float(np.float32(x)) for x in LR]


@pytest.fixture(scope="module")
def room():
    sc = scenegen.room_scene(60_000, seed=10, sh_degree=3)
    s = 2.0
    cid = oc.encode_id(oc.chunk_coord(sc["params"][0:3].T, s))
    ids, counts = np.unique(cid, return_counts=True)
    return sc["params"], s, cid, ids, counts


def test_ingest_groups_by_chunk(ctx, room):
    params, s, cid, ids, counts = room
    pool = D.Pool(ctx, 3, budget=10**9)
    pool.ingest(params, s)
    got_ids, got_counts = pool.chunks()
    assert (got_ids == ids).all() and (got_counts == counts).all()
    for k in (0, len(ids) // 2, len(ids) - 1):
        p, m, v, st = pool.read_chunk(ids[k], counts[k])
        assert (p == params[:, cid == ids[k]]).all()       # input order kept
        assert (m == 0).all() and (v == 0).all() and (st == 0).all()
    pool.close()


def test_lru_matches_oracle_plan(ctx, room):
    params, s, cid, ids, counts = room
    cmap = {int(i): int(c) for i, c in zip(ids, counts)}
    budget = int(counts.sum() * 0.35)
    pool = D.Pool(ctx, 3, budget=budget)
    pool.ingest(params, s)
    rng = np.random.default_rng(7)
    resident = {}
    for it in range(40):
        k = int(rng.integers(1, 8))
        need = [int(x) for x in rng.choice(ids, k, replace=False)]
        try:
            plan = oc.residency_plan(need, resident, cmap, budget, now=it)
        except oc.BudgetError:
            with pytest.raises(D.DcgsError) as e:
                pool.require(np.array(need, np.uint64), now=it)
            assert e.value.status == 3
            continue
        loaded, evicted = pool.require(np.array(need, np.uint64), now=it)
        assert loaded == len(plan["load"]) and evicted == len(plan["evict"])
        resident = plan["resident"]
        got, g = pool.resident()
        assert set(int(x) for x in got) == set(resident)
        assert g == sum(cmap[c] for c in resident)
    pool.close()


def test_compact_adam_and_round_trip(ctx, room):
    params, s, cid, ids, counts = room
    cmap = {int(i): int(c) for i, c in zip(ids, counts)}
    pool = D.Pool(ctx, 3, budget=int(counts.sum() * 0.5))
    pool.ingest(params, s)
    act = [int(x) for x in ids[[1, 4, 9, 2]]]
    pool.require(np.array(act, np.uint64), now=0)
    R = params.shape[0]
    cap = sum(cmap[c] for c in act) + 100
    out = torch.empty(R, cap, device="cuda")
    src = torch.empty(cap, dtype=torch.int32, device="cuda")
    n = pool.compact(np.array(act, np.uint64), out, src)
    chunk_arrays = {c: (params[:, cid == c], np.arange(cmap[c])) for c in act}
    ref, _ = oc.compact(act, chunk_arrays)
    assert n == ref.shape[1]
    assert (out[:, :n].cpu().numpy() == ref).all()
    # two Adam steps on the compacted set, then an eviction and a reload.
    # Each step is checked on its own: the oracle (float64) starts from the
    # float32 state the device holds before the step and gets the same
    # float32 gradients; every stored value is within 2 ulp of the oracle's
    # result rounded to float32.
    rng = np.random.default_rng(3)
    cfg = D.AdamConfig.of(LR)
    order = sorted(act)

    def f32_ulp(x):
        return np.spacing(np.abs(np.asarray(x, np.float32))).astype(np.float64)

    for step in range(2):
        g = (rng.normal(0, 1e-4, (R, n)) * (rng.uniform(0, 1, (R, n)) > 0.2)).astype(np.float32)
        before = {c: pool.read_chunk(c, cmap[c]) for c in order}
        pool.adam_step(src, torch.from_numpy(g).cuda(), n, cfg)
        off = 0
        for c in order:
            k = cmap[c]
            p0, m0, v0, s0 = before[c]
            # the ABI carries the learning rates, beta1, beta2 and eps as
            # float32: give the oracle those values
            P, M, V, S = oo.adam_step(p0, m0, v0, s0, g[:, off:off + k], np.arange(k), LR32,
                                      beta1=float(np.float32(0.9)),
                                      beta2=float(np.float32(0.999)),
                                      eps=float(np.float32(1e-15)))
            off += k
            p, m, v, st = pool.read_chunk(c, k)
            assert (st == S).all()
            for got, ref, name in ((p, P, "params"), (m, M, "m"), (v, V, "v")):
                r32 = ref.astype(np.float32)
                err = np.abs(got.astype(np.float64) - r32.astype(np.float64))
                assert (err <= 2 * f32_ulp(r32)).all(), (name, step, (err / f32_ulp(r32)).max())
    after = {c: pool.read_chunk(c, cmap[c]) for c in order}
    others = [int(x) for x in ids if int(x) not in act][:6]
    pool.require(np.array(others, np.uint64), now=5)        # may evict some of `act`
    pool.require(np.array(act, np.uint64), now=6)           # back on the device
    for c in order:
        for a, b in zip(pool.read_chunk(c, cmap[c]), after[c]):
            assert np.array_equal(a, b)                     # the round trip is exact
    pool.close()


def test_budget_error_changes_nothing(ctx, room):
    params, s, cid, ids, counts = room
    pool = D.Pool(ctx, 3, budget=int(counts.max()) + 10)
    pool.ingest(params, s)
    pool.require(ids[:1], now=0)
    big = ids[np.argsort(counts)[-2:]]
    with pytest.raises(D.DcgsError) as e:
        pool.require(big, now=1)
    assert e.value.status == 3
    got, _ = pool.resident()
    assert list(got) == [ids[0]]
    pool.close()


def test_loss_l1(ctx):
    rgb = scenegen.upstream_grad(97, 61, seed=4, scale=0.5) + 0.5
    tgt = scenegen.target_image(97, 61, seed=5)
    rgb[0, 0, :5] = tgt[0, 0, :5]                    # exact ties: sign(0) = 0
    from oracle import splat as osp
    loss, g, _ = osp.l1_loss(rgb, tgt)
    dl, st = ctx.loss_l1(torch.from_numpy(rgb).cuda(), torch.from_numpy(tgt).cuda())
    dl = dl.cpu().numpy()
    assert np.abs(dl - g).max() <= 1e-7 * np.abs(g).max()
    assert (dl[0, 0, :5] == 0).all()
    st = st.cpu().numpy()
    assert abs(st[0] / rgb.size - loss) <= 1e-6 * loss
    mse = np.mean((np.clip(rgb, 0, 1) - tgt) ** 2)
    assert abs(st[1] / rgb.size - mse) <= 1e-6 * mse
