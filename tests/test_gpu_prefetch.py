"""The learned-prefetch kernels against the FP64 oracle: exact labels and
cell ids bit-exact, features, network forward, gradient and Adam within
tolerances derived from float32 arithmetic, thresholding exact; and a short
training run that lowers the chunk miss rate on a held-out trajectory."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import prefetch as op
from paper_2511_23030_amd import prefetch as P

pytestmark = pytest.mark.gpu

S = 50.0
U = 2.0 ** -24          # float32 unit roundoff


@pytest.fixture(scope="module")
def traj():
    path = scenegen.driving_path(101, length=800.0)
    return scenegen.driving_trajectory(path, 130, width=1241, height=376, focal=718.0,
                                       z_far=350.0)


def _on_boundary(cam, s=S):
    """Camera centre within rounding distance of a cell face: its base cell
    (Eq. 5) may round either way, so the frame is not compared."""
    c = op.centre(cam)
    f = (c + s / 2) / s
    return bool((np.abs(f - np.round(f)) < 1e-9).any())


def _frames(cams, want):
    out = [t for t in want if not _on_boundary(cams[t])]
    assert len(out) >= len(want) - 2
    return out


def test_labels_bit_exact(ctx, traj):
    lab = P.labels(ctx, traj, S, horizon=5).cpu().numpy()
    frames = _frames(traj, [0, 41, 97, 126, 129])
    print("case prefetch labels frames", frames, flush=True)
    n_pos = 0
    for t in frames:
        ref, tie = op.labels(traj, t, S, horizon=5)
        ok = ~tie
        assert tie.sum() <= 4
        assert (lab[t][ok] == ref[ok]).all(), t
        n_pos += int(ref.sum())
    assert n_pos > 20
    assert lab[129].sum() == 0           # no future frames


def test_features_and_ids(ctx, traj):
    lab = P.labels(ctx, traj, S, horizon=5)
    frames = _frames(traj, [0, 3, 9, 57, 129])
    X, ids, y = P.features(ctx, traj, frames, S, pos_unit=2.0, lab=lab)
    X = X.view(len(frames), 4096, 59).cpu().numpy()
    ids = ids.view(len(frames), 4096).cpu().numpy().view(np.uint64)
    y = y.view(len(frames), 4096).cpu().numpy()
    labh = lab.cpu().numpy()
    for r, t in enumerate(frames):
        Xr, idr = op.features(traj, t, S, pos_unit=2.0)
        assert (ids[r] == idr).all(), t
        # float64 values rounded once to float32 on both sides, up to the
        # order of a few float64 operations
        assert (np.abs(X[r] - Xr) <= 2 * U * np.maximum(np.abs(Xr), 1e-3)).all(), t
        assert (y[r] == labh[t]).all()


def _bound(w, f, X):
    """Elementwise error bounds of a float32 forward against the float64
    one: a length-K float32 dot product errs by at most K u sum|a_k b_k|
    (plus the bias rounding); GELU's float32 evaluation adds a few ulps and
    passes input errors through with slope at most 1.13."""
    Xa = torch.as_tensor(np.abs(X))
    e1 = 59 * U * (Xa @ w["W1"].abs().T) + U * w["b1"].abs()
    eh1 = 1.13 * e1 + 8 * U * f["h1"].abs() + 1e-30
    e2 = 256 * U * (f["h1"].abs() @ w["W2"].abs().T) + eh1 @ w["W2"].abs().T + U * w["b2"].abs()
    eh2 = 1.13 * e2 + 8 * U * f["h2"].abs() + 1e-30
    el = 256 * U * (f["h2"].abs() @ w["w3"].abs()) + eh2 @ w["w3"].abs() + U * abs(w["b3"][0])
    return dict(z1=e1, h1=eh1, z2=e2, h2=eh2, logit=el)


@pytest.mark.parametrize("n", [1, 64, 1037])
def test_mlp_forward(ctx, n):
    lay = op.layout()
    theta = scenegen.mlp_init(3, bias_sd=0.1)
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 59)).astype(np.float32)
    net = P.PrefetchNet(ctx, theta)
    logit = net.forward(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    w = op.unpack(theta, lay)
    f = op.mlp_forward(w, X.astype(np.float64))
    b = _bound(w, f, X.astype(np.float64))
    got = dict(z1=net.act[0, :n], h1=net.act[1, :n], z2=net.act[2, :n], h2=net.act[3, :n],
               logit=logit)
    for k in ("z1", "h1", "z2", "h2", "logit"):
        g = got[k].cpu().double()
        assert ((g - f[k].detach()).abs() <= 2 * b[k]).all(), k
    # the bfloat16 copy is the master rounded to nearest even
    wb = net.wb.cpu().numpy().view(np.uint16)
    o, m = lay["master"]["W2"]
    ob, _ = lay["bf16"]["W2"]
    ref = op.bf16_round(theta[o:o + m]).view(np.uint32) >> 16
    assert (wb[ob:ob + m] == ref).all()


def test_mlp_backward(ctx):
    lay = op.layout()
    theta = scenegen.mlp_init(4, bias_sd=0.1)
    n = 3001
    rng = np.random.default_rng(7)
    X = rng.normal(size=(n, 59)).astype(np.float32)
    y = (rng.uniform(size=n) < 0.1).astype(np.uint8)
    net = P.PrefetchNet(ctx, theta)
    Xt, yt = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    net.forward(Xt)
    g = net.backward(Xt, yt, 4.0).cpu().numpy().astype(np.float64)
    loss = net.loss.item()
    ref_loss, ref = op.mlp_grad(theta, X.astype(np.float64), y, 4.0, lay)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        o, m = lay["master"][name]
        scale = np.abs(ref[o:o + m]).max()
        err = np.abs(g[o:o + m] - ref[o:o + m]).max()
        assert err <= 1e-3 * scale, (name, err, scale)
    # deterministic: a second backward gives the same bits
    net.forward(Xt)
    g2 = net.backward(Xt, yt, 4.0).cpu().numpy()
    assert (g2 == g.astype(np.float32)).all()


def test_mlp_adam(ctx):
    theta = scenegen.mlp_init(5, bias_sd=0.1)
    net = P.PrefetchNet(ctx, theta, lr=3e-3)
    rng = np.random.default_rng(9)
    for step in (1, 2, 3):
        g = rng.normal(size=P.N_PARAMS).astype(np.float32) * 1e-2
        th0, m0, v0 = (t.cpu().numpy().copy() for t in (net.theta, net.m, net.v))
        net.grad.copy_(torch.from_numpy(g))
        net.adam()
        th_ref, m_ref, v_ref = op.adam(th0, m0, v0, g.astype(np.float64), step, 3e-3, 0.9, 0.999,
                                       1e-8)
        th, m, v = (t.cpu().numpy() for t in (net.theta, net.m, net.v))
        for a, r in ((th, th_ref), (m, m_ref), (v, v_ref)):
            # float64 arithmetic on both sides, one rounding to float32
            assert (np.abs(a - r) <= 1.01 * U * np.abs(r) * 2 + 1e-45).all()
        lay = op.layout()
        wb = net.wb.cpu().numpy().view(np.uint16)
        for name in ("W1", "W2", "w3"):
            o, m_ = lay["master"][name]
            ob, _ = lay["bf16"][name]
            assert (wb[ob:ob + m_] == (op.bf16_round(th[o:o + m_]).view(np.uint32) >> 16)).all()


def test_predict_thresholds_exactly(ctx, traj):
    theta = scenegen.mlp_init(6, bias_sd=0.5)
    net = P.PrefetchNet(ctx, theta)
    t = _frames(traj, [40])[0]
    hist = op.history(traj, t)
    ids = net.predict(hist, S, tau=0.5)
    logit = net._pick_logit.cpu().numpy()
    Xr, idr = op.features(traj, t, S)
    keep = logit >= 0.0
    assert (ids == idr[keep]).all()
    # the logits are those of the network on the oracle's features
    w = op.unpack(theta, op.layout())
    f = op.mlp_forward(w, Xr)
    b = _bound(w, f, Xr)
    assert (np.abs(logit - f["logit"].detach().numpy()) <= 2 * b["logit"].numpy() + 1e-5).all()
    assert 0 < keep.sum() < 4096


def test_training_lowers_misses_on_held_out_trajectory(ctx):
    trajs = []
    for seed in (100, 101, 102, 103):
        path = scenegen.driving_path(seed, length=1500.0)
        trajs.append(scenegen.driving_trajectory(path, None, width=1241, height=376,
                                                 focal=718.0, z_far=350.0))
    net, losses = P.train(ctx, trajs, S, steps=600, frames_per_batch=8, seed=1)
    print("case prefetch training loss", losses[:5].round(4), losses[-5:].round(4), flush=True)
    assert losses[-50:].mean() < 0.5 * losses[:10].mean()
    held = scenegen.driving_trajectory(scenegen.driving_path(120, length=800.0), None,
                                       width=1241, height=376, focal=718.0, z_far=350.0)
    ev = P.evaluate(ctx, net, held, S, tau=0.3, every=2)
    print("case prefetch held-out", ev, flush=True)
    assert ev["entering"] > 20
    assert ev["miss_rate"] < 0.5 * ev["miss_rate_without"]
