"""Oracle: the per-Gaussian Adam step of the mapping iteration.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper keeps per-Gaussian optimiser state and resets it at loop closure
(Sec. III-G, "Post-Correction Refinement") but does not name the optimiser.
Reading: Adam (Kingma and Ba) with beta1 = 0.9, beta2 = 0.999 and a small
epsilon, one step counter per Gaussian, every Gaussian of the active set
updated each step (zero gradients included), one learning rate per parameter
group.  Written out in float64:

    t += 1;  m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Pinned (tests/test_oracle_optim.py) by the closed-form first step from zero
moments, and by torch.optim.Adam (float64) where all counters are equal.
"""
from __future__ import annotations

import numpy as np


def group_of_rows(n_rows: int) -> np.ndarray:
    """Parameter group of each row of the parameter block: 0 means, 1 log-
    scales, 2 quaternions, 3 opacity logit, 4 SH degree 0, 5 higher SH."""
    grp = np.full(n_rows, 5, np.int64)
    grp[0:3], grp[3:6], grp[6:10], grp[10], grp[11:14] = 0, 1, 2, 3, 4
    return grp


def adam_step(params, m, v, step, grad, src, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """Update pool slots `src` (one per compacted Gaussian) with gradients
    `grad` [R, n].  Arrays are not modified; float64 results are returned as
    (params, m, v, step)."""
    P = np.asarray(params, np.float64).copy()
    M = np.asarray(m, np.float64).copy()
    V = np.asarray(v, np.float64).copy()
    S = np.asarray(step, np.int64).copy()
    g = np.asarray(grad, np.float64)
    src = np.asarray(src, np.int64)
    lr_row = np.asarray(lr, np.float64)[group_of_rows(P.shape[0])][:, None]
    t = S[src] + 1
    M[:, src] = beta1 * M[:, src] + (1 - beta1) * g
    V[:, src] = beta2 * V[:, src] + (1 - beta2) * g * g
    mhat = M[:, src] / (1 - beta1 ** t)
    vhat = V[:, src] / (1 - beta2 ** t)
    P[:, src] -= lr_row * mhat / (np.sqrt(vhat) + eps)
    S[src] = t
    return P, M, V, S
