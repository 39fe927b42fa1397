"""Pins of the learned-proposal parts of the oracle (C: network, mixture,
sampling, guided estimator; torch: network, loss and its gradient) against
what mathematics fixes: the vMF normalisation and its closed-form cosine
distribution, exact lobe-selection frequencies, a network whose weights make
its output a known function, a cross-entropy that reaches the target's
closed-form entropy, finite differences of the loss, and the closed-form
white-furnace radiance that a guided (one-sample MIS) estimator must still
reach on average."""
import math

import numpy as np
import pytest
import torch

from oracle import guide_ref
from paper_1903_07145_amd import scenes
import _guide


def _fib_sphere(n):
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    r = np.sqrt(1 - z * z)
    phi = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def _mix(mus, kappas, weights):
    m = np.zeros(40)
    for j in range(8):
        m[5 * j:5 * j + 3] = mus[j]
        m[5 * j + 3] = kappas[j]
        m[5 * j + 4] = weights[j]
    return m


def _random_mix(rng, kmax=50.0):
    mus = _guide.random_unit(rng, 8)
    kappas = np.exp(rng.uniform(np.log(0.02), np.log(kmax), 8))
    w = rng.uniform(0.1, 1, 8)
    return _mix(mus, kappas, w / w.sum())


def test_vmf_mixture_integrates_to_one(orc):
    # equal-area quadrature over the sphere (Fibonacci lattice)
    rng = np.random.default_rng(1)
    pts = torch.as_tensor(_fib_sphere(400_000))
    for kmax in (0.05, 5.0, 200.0):
        m = _random_mix(rng, kmax)
        mu = torch.as_tensor(m.reshape(8, 5)[:, :3])[None].expand(pts.shape[0], 8, 3)
        kap = torch.as_tensor(m.reshape(8, 5)[:, 3])[None].expand(pts.shape[0], 8)
        wt = torch.as_tensor(m.reshape(8, 5)[:, 4])[None].expand(pts.shape[0], 8)
        q = torch.exp(guide_ref.log_q(mu, kap, wt, pts)).numpy()
        assert abs(q.mean() * 4 * np.pi - 1.0) < 1e-4
        # the C oracle's density is the same function
        for i in range(0, pts.shape[0], 40000):
            assert orc.mixture_pdf(m, pts[i].numpy()) == pytest.approx(float(q[i]), rel=1e-12)


@pytest.mark.parametrize("kappa", [0.03, 1.0, 8.0, 300.0])
def test_vmf_sampling_cosine_distribution(orc, kappa):
    # P(mu.w <= t) = (e^{kappa (t-1)} - e^{-2 kappa}) / (1 - e^{-2 kappa}); azimuth uniform
    rng = np.random.default_rng(2)
    mu = _guide.random_unit(rng, 1)[0]
    m = _mix([mu] * 8, [kappa] * 8, [1.0] + [0.0] * 7)
    n = 4000
    u = rng.random((n, 3))
    c = np.empty(n)
    xs = np.empty((n, 3))
    for i in range(n):
        w = orc.mixture_sample(m, u[i, 0], u[i, 1], u[i, 2])
        assert abs(np.linalg.norm(w) - 1) < 1e-12
        c[i] = w @ mu
        xs[i] = w
    c.sort()
    F = (np.exp(kappa * (c - 1)) - np.exp(-2 * kappa)) / -np.expm1(-2 * kappa)
    ks = np.max(np.abs(F - (np.arange(n) + 0.5) / n))
    assert ks < 1.63 / math.sqrt(n) + 0.5 / n           # Kolmogorov-Smirnov, 1 %
    # mean cosine = coth(kappa) - 1/kappa (Langevin function)
    L = 1 / math.tanh(kappa) - 1 / kappa
    assert abs(c.mean() - L) < 5 * c.std() / math.sqrt(n) + 1e-12
    # the perpendicular part has zero mean (uniform azimuth)
    perp = xs - np.outer(xs @ mu, mu)
    assert np.linalg.norm(perp.mean(0)) < 5 * math.sqrt(max(1e-30, (perp ** 2).sum(1).mean()) / n)


def test_lobe_selection_frequencies(orc):
    axes = np.eye(3)
    mus = [axes[0], -axes[0], axes[1], -axes[1], axes[2], -axes[2], axes[0], axes[1]]
    weights = [0.1, 0.2, 0.3, 0.4, 0.0, 0.0, 0.0, 0.0]
    m = _mix(mus, [1e4] * 8, weights)
    n = 1000
    counts = np.zeros(4)
    for i in range(n):
        w = orc.mixture_sample(m, (i + 0.5) / n, 0.5, 0.25)
        j = int(np.argmax([w @ mus[k] for k in range(4)]))
        counts[j] += 1
    assert np.allclose(counts / n, weights[:4], atol=1.0 / n)


def test_network_layout_by_construction(orc):
    # W1 copies the 25 inputs into the first 25 units, W2..W4 are identities,
    # so for non-negative inputs the raw output is y = x A + b5 exactly.
    S = 3
    rng = np.random.default_rng(3)
    W1 = np.zeros((25, 64)); W1[np.arange(25), np.arange(25)] = 1
    I = np.eye(64)
    A = np.zeros((64, 40)); A[:25] = rng.uniform(-1, 1, (25, 40))
    b5 = rng.uniform(-1, 1, 40)
    emb = rng.uniform(0, 1, (S, 16))
    w = np.concatenate([W1.ravel(), np.zeros(64), I.ravel(), np.zeros(64), I.ravel(), np.zeros(64),
                        I.ravel(), np.zeros(64), A.ravel(), b5, emb.ravel()]).astype(np.float32)
    n = 5
    feat = rng.uniform(0, 1, (n, 9)).astype(np.float32).astype(np.float64)
    seg = np.array([0, 1, 2, 1, 0], np.int32)
    x = np.concatenate([feat, emb.astype(np.float32).astype(np.float64)[seg]], 1)
    y = x @ A.astype(np.float32).astype(np.float64)[:25] + b5.astype(np.float32)
    yt = guide_ref.network(w, feat, seg).numpy()
    assert np.allclose(yt, y, rtol=1e-12, atol=1e-12)
    # the C oracle's mixture equals the mixture of these raw outputs
    mix_c = orc.guide_eval(w, feat, seg)
    mix_t = guide_ref.mixture_flat(torch.as_tensor(y)).numpy()
    assert np.allclose(mix_c, mix_t, rtol=1e-12, atol=1e-14)
    # and the mixture is what its definition says for one lobe
    l = y[0, 5:10]
    assert np.allclose(mix_c[0, 5:8], l[:3] / np.linalg.norm(l[:3]), atol=1e-14)
    assert mix_c[0, 8] == pytest.approx(min(math.log1p(math.exp(l[3])) + 0.01, 1e4), rel=1e-13)
    lg = y[0, 4::5]
    assert mix_c[0, 9] == pytest.approx(math.exp(lg[1]) / np.exp(lg).sum(), rel=1e-13)


def test_c_and_torch_networks_agree(orc):
    S = 5
    w = _guide.random_weights(S, seed=4, out_gain=2.0)
    rng = np.random.default_rng(4)
    feat = rng.uniform(-1, 1, (200, 9))
    seg = rng.integers(0, S, 200).astype(np.int32)
    a = orc.guide_eval(w, feat.astype(np.float32).astype(np.float64), seg)
    b = guide_ref.mixture_flat(guide_ref.network(w, feat, seg)).numpy()
    assert np.allclose(a, b, rtol=1e-11, atol=1e-13)


def test_loss_gradient_matches_finite_differences():
    S = 4
    w = _guide.random_weights(S, seed=5, out_gain=1.5).astype(np.float64)
    rec = _guide.random_records(64, S, seed=5)
    L0, g = guide_ref.loss_grad(w, rec)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(guide_ref.N_NET, 24, replace=False),
                          guide_ref.N_NET + rng.choice(16 * S, 8, replace=False)])
    for i in idx:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (float(guide_ref.loss(torch.as_tensor(wp), rec)) - float(guide_ref.loss(torch.as_tensor(wm), rec))) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(g[i]))


def test_loss_reaches_target_entropy_and_is_larger_elsewhere():
    # records drawn from a vMF target with equal weights: the loss is the
    # cross-entropy, equal to the target's entropy when q is the target.
    kappa = 6.0
    mu = np.array([0.0, 0.6, 0.8])
    rng = np.random.default_rng(6)
    n = 20000
    # inverse-CDF sample of the target
    u = rng.random((n, 2))
    c = 1 + np.log(u[:, 0] + (1 - u[:, 0]) * np.exp(-2 * kappa)) / kappa
    t = np.cross(mu, [1.0, 0, 0]); t /= np.linalg.norm(t)
    b = np.cross(mu, t)
    s = np.sqrt(1 - c * c)
    d = np.outer(c, mu) + np.outer(s * np.cos(2 * np.pi * u[:, 1]), t) + np.outer(s * np.sin(2 * np.pi * u[:, 1]), b)
    mus = torch.as_tensor(np.tile(mu, (n, 8, 1)))
    wt = torch.as_tensor(np.tile([1.0] + [0.0] * 7, (n, 1)))
    ce = lambda k: float(-guide_ref.log_q(mus, torch.full((n, 8), k, dtype=torch.float64), wt,
                                          torch.as_tensor(d)).mean())
    H = -(math.log(kappa / (2 * math.pi * -math.expm1(-2 * kappa))) + kappa * (1 / math.tanh(kappa) - 1 / kappa - 1))
    assert abs(ce(kappa) - H) < 0.03
    assert ce(2.0) > H + 0.1 and ce(20.0) > H + 0.1


@pytest.mark.parametrize("mis", [0, 2])
def test_guided_furnace_unbiased(orc, mis):
    # closed cube, one Lambertian emitter segment: L = E sum_{k=0}^{D} rho^k
    # whatever the direction sampler, as long as its density is positive
    rho, E, D = 0.5, 1.0, 3
    s = scenes.furnace(rho, E)
    rho, E = float(s["params"][0]), float(s["params"][7])
    sc = orc.Scene(s["verts"], s["tris"], s["tri_seg"], s["num_segments"], s["emitter_seg"], s["normals"])
    lo, inv = _guide.box(s["verts"])
    w = _guide.random_weights(s["num_segments"], seed=7, out_gain=3.0, kappa_bias=2.0)
    r = sc.run(s["cams"], s["params"], spp=256, max_depth=D, mis=mis, want_path_L=True, want_hash=True,
               guide_w=w, guide_mix=0.5, bb_lo=lo, bb_inv=inv)
    x = r["path_L"][:, :, 0].ravel()
    L = E * sum(rho ** k for k in range(D + 1))
    se = x.std() / math.sqrt(x.size)
    assert se > 0                                       # the guide makes the estimator non-constant
    assert abs(x.mean() - L) < 5 * se
    g = sc.run(s["cams"], s["params"], spp=64, max_depth=D, mis=mis, w=np.tile([1.0, 0, 0], (64, 1)),
               want_grad=True, guide_w=w, guide_mix=0.5, bb_lo=lo, bb_inv=inv)["grad"]
    npix = 64
    dL_drho = E * sum(k * rho ** (k - 1) for k in range(1, D + 1))
    assert abs(g[0] / npix - dL_drho) < 0.1 * dL_drho


def test_mfma_backward_reference_bookkeeping():
    """The manual backward that rounds where the matrix-core path rounds
    (guide_ref.loss_grad_mfma) equals autograd exactly when no rounding is
    applied, and stays within bfloat16 accuracy of the straight-through
    gradient when it is."""
    S = 5
    w = _guide.random_weights(S, seed=3, out_gain=2.0)
    rec = _guide.random_records(700, S, seed=4)
    L0, g0 = guide_ref.loss_grad(w, rec, bf16=False)
    L1, g1 = guide_ref.loss_grad_mfma(w, rec, round_bf16=False)
    assert abs(L0 - L1) <= 1e-12 * abs(L0)
    assert np.allclose(g1, g0, rtol=1e-10, atol=1e-14 * np.abs(g0).max())
    L2, g2 = guide_ref.loss_grad(w, rec, bf16=True)
    L3, g3 = guide_ref.loss_grad_mfma(w, rec, round_bf16=True)
    assert abs(L2 - L3) <= 1e-12 * abs(L2)
    assert np.linalg.norm(g3 - g2) <= 2e-2 * np.linalg.norm(g2)

