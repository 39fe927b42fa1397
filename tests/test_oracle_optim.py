"""Pins of the oracle's loss/adjoint and Adam against torch (autograd and
torch.optim.Adam in float64 on the CPU)."""
import numpy as np
import torch


def test_loss_adjoint_matches_autograd(orc):
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 2, size=(50, 3))
    tgt = rng.uniform(0, 2, size=(50, 3))
    tgt[3, 1] = img[3, 1]
    for kind in (0, 1):
        E, w = orc.loss_adjoint(img, tgt, kind)
        x = torch.tensor(img, dtype=torch.float64, requires_grad=True)
        t = torch.tensor(tgt, dtype=torch.float64)
        loss = torch.mean((x - t) ** 2) if kind == 0 else torch.mean(torch.abs(x - t))
        loss.backward()
        assert abs(E - loss.item()) < 1e-14
        assert np.allclose(w, x.grad.numpy(), atol=1e-16)


def test_projected_adam_matches_torch(orc):
    rng = np.random.default_rng(1)
    n = 40
    scale = np.where(np.arange(n) >= 30, 15.0, 1.0)
    lo = np.zeros(n)
    hi = np.ones(n)
    lo[5] = 1e-3
    tr = np.ones(n, np.uint8)
    tr[7] = 0
    theta0 = rng.uniform(0, 1, n)
    p = theta0 * scale
    m = np.zeros(n)
    v = np.zeros(n)
    th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([th], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 30):
        g_p = rng.normal(size=n) * 3
        orc.adam(p, g_p, m, v, step, 1e-2, scale=scale, lo=lo, hi=hi, trainable=tr)
        opt.zero_grad()
        gt = torch.tensor(g_p * scale)
        gt[7] = 0.0
        th.grad = gt
        keep = th.detach()[7].clone()
        opt.step()
        with torch.no_grad():
            th.copy_(torch.maximum(torch.minimum(th, torch.tensor(hi)), torch.tensor(lo)))
            th[7] = keep
        ref = th.detach().numpy() * scale
        mask = np.arange(n) != 7
        assert np.allclose(p[mask], ref[mask], rtol=1e-12, atol=1e-12)
        assert p[7] == theta0[7] * scale[7]
