"""The mapping loss of Eqs. (2)-(4) (L1 + SSIM + depth L1) against the FP64
oracle: loss value and gradients, ragged image sizes, the L1-only case
bit-identical to dcgs_loss_l1, identical images."""
import numpy as np
import pytest
import torch

from oracle import loss as ol

pytestmark = pytest.mark.gpu


def _inputs(V, H, W, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(size=(V, 3, H, W)).astype(np.float32)
    # a target correlated with x so SSIM is far from 0
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1).astype(np.float32)
    d = rng.uniform(1, 5, size=(V, H, W)).astype(np.float32)
    dt = (d + rng.choice([-1, 1], size=d.shape) * rng.uniform(0.01, 0.5, size=d.shape)
          ).astype(np.float32)
    return x, y, d, dt


@pytest.mark.parametrize("V,H,W", [(1, 16, 16), (2, 37, 53), (3, 96, 128)])
def test_loss_and_gradient_match_oracle(ctx, V, H, W):
    x, y, d, dt = _inputs(V, H, W, V * 100 + H)
    ls, ld = 0.2, 0.5
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    dtt, dtgt = torch.from_numpy(d).cuda(), torch.from_numpy(dt).cuda()
    dl, dld, st = ctx.loss_mapping(xt, yt, dtt, dtgt, lambda_s=ls, lambda_depth=ld)
    loss = ctx.loss_value(st, V, H, W, ls, ld)
    L, gx, gd = ol.mapping_loss_grad(x.astype(np.float64), y.astype(np.float64),
                                     d.astype(np.float64), dt.astype(np.float64), ls, ld)
    print(f"case loss V={V} {H}x{W}: {loss:.8f} vs {L:.8f}", flush=True)
    # float32 moments: m_xx - m_x^2 cancels to ~4u m_xx against C2 = 9e-4
    assert abs(loss - L) <= 1e-5 * abs(L)
    g = dl.cpu().numpy()
    assert np.abs(g - gx).max() <= 1e-3 * np.abs(gx).max()
    assert (np.sign(g) == np.sign(gx))[np.abs(gx) > 1e-2 * np.abs(gx).max()].all()
    assert np.array_equal(dld.cpu().numpy(), gd.astype(np.float32))
    ssim_ref = sum(ol.ssim_map(torch.tensor(x[v], dtype=torch.float64),
                               torch.tensor(y[v], dtype=torch.float64)).sum().item()
                   for v in range(V))
    assert abs(st[2].item() - ssim_ref) <= 1e-5 * abs(ssim_ref)


def test_l1_only_equals_l1_kernel_and_identical_images(ctx):
    x, y, _, _ = _inputs(2, 40, 33, 7)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    dl, _, st = ctx.loss_mapping(xt, yt, lambda_s=0.0)
    dl1, st1 = ctx.loss_l1(xt, yt, norm=3.0 * 40 * 33)
    assert torch.equal(dl, dl1)
    assert abs(st[0].item() - st1[0].item()) <= 1e-6 * st1[0].item()
    dl, _, st = ctx.loss_mapping(xt, xt.clone(), lambda_s=1.0)
    loss = ctx.loss_value(st, 2, 40, 33, 1.0, 0.0)
    assert abs(loss) < 1e-5
    assert abs(st[2].item() - 2 * 3 * 40 * 33) < 1e-3
