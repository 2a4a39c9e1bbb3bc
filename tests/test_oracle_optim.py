"""Pins of the Adam oracle."""
import numpy as np
import torch

import scenegen
from oracle import optim as oo

LR = [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4]


def test_first_step_closed_form():
    """From zero moments: m_hat = g, v_hat = g^2, so theta moves by
    -lr g / (|g| + eps)."""
    d = scenegen.adam_inputs(59, 200, seed=1, n_slots=300)
    m = np.zeros_like(d["m"])
    v = np.zeros_like(d["v"])
    step = np.zeros_like(d["step"])
    P, M, V, S = oo.adam_step(d["params"], m, v, step, d["grad"], d["src"], LR)
    lr = np.asarray(LR)[oo.group_of_rows(59)][:, None]
    g = d["grad"].astype(np.float64)
    exp = d["params"][:, d["src"]].astype(np.float64) - lr * g / (np.abs(g) + 1e-15)
    assert np.abs(P[:, d["src"]] - exp).max() < 1e-15
    untouched = np.setdiff1d(np.arange(300), d["src"])
    assert (P[:, untouched] == d["params"][:, untouched]).all()
    assert (S[d["src"]] == 1).all() and (S[untouched] == 0).all()


def test_matches_torch_adam():
    """Equal step counters reduce to torch.optim.Adam (float64)."""
    rng = np.random.default_rng(4)
    n, R = 50, 14
    p0 = rng.normal(size=(R, n))
    grads = [rng.normal(size=(R, n)) * 1e-3 for _ in range(4)]
    lr = np.asarray(LR)[oo.group_of_rows(R)]
    tp = [torch.nn.Parameter(torch.tensor(p0[r:r + 1].copy())) for r in range(R)]
    opt = torch.optim.Adam([{"params": [tp[r]], "lr": float(lr[r])} for r in range(R)], betas=(0.9, 0.999), eps=1e-15)
    P, M, V, S = p0, np.zeros((R, n)), np.zeros((R, n)), np.zeros(n, np.int64)
    src = np.arange(n)
    for g in grads:
        for r in range(R):
            tp[r].grad = torch.tensor(g[r:r + 1].copy())
        opt.step()
        P, M, V, S = oo.adam_step(P, M, V, S, g, src, LR)
    ref = np.concatenate([t.detach().numpy() for t in tp], 0)
    assert np.abs(P - ref).max() < 1e-14
