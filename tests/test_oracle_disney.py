"""Pins of the oracle's Disney material model (the paper's material, Sec. 4.1;
Burley 2012): special cases that reduce to the separately pinned GGX lobe,
reciprocity, the complex-step derivatives of all 13 parameters against
central differences of the value, the sampler against its own pdf (pdf mass
and a chi-square test), energy of the metallic lobe, and central differences
of the whole estimator with frozen sampling on a Disney Cornell box.

The model itself is not energy-conserving: its diffuse term (Burley's
retro-reflection) sends up to 1.36 times the incident energy back for a
white, rough surface seen at grazing angles, so no energy bound is pinned for
it; the metallic lobe (GGX with Schlick's Fresnel) stays below 1."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1903_07145_amd import scenes

N = np.array([0.0, 0.0, 1.0])
X = np.array([1.0, 0.0, 0.0])


def _unit(rng, up=True):
    v = rng.normal(size=3)
    if up:
        v[2] = abs(v[2]) + 0.05
    return v / np.linalg.norm(v)


def _rand_params(rng):
    p = rng.uniform(0, 1, 13)
    p[7] = rng.uniform(0.15, 0.95)     # roughness away from the 1e-3 clamp of alpha
    p[8] = rng.uniform(0, 0.9)
    return p


def _hemisphere_grid(n_t=160, n_p=320):
    c = (np.arange(n_t) + 0.5) / n_t
    ph = (np.arange(n_p) + 0.5) / n_p * 2 * math.pi
    C, PH = np.meshgrid(c, ph, indexing="ij")
    S = np.sqrt(1 - C * C)
    return np.stack([S * np.cos(PH), S * np.sin(PH), C], -1).reshape(-1, 3), (1.0 / n_t) * (2 * math.pi / n_p)


def test_metallic_white_reduces_to_ggx(orc):
    """metallic 1, white base, no anisotropy, no clearcoat: F = 1 and the
    model is the GGX lobe with alpha = roughness^2 -- the oracle's Lambert +
    GGX material with kd = 0, ks = 1 (pinned in test_oracle_brdf)."""
    rng = np.random.default_rng(0)
    for _ in range(40):
        r = rng.uniform(0.1, 1.0)
        mp = np.array([1, 1, 1, rng.uniform(), 1.0, rng.uniform(), rng.uniform(), r, 0.0, rng.uniform(),
                       rng.uniform(), 0.0, rng.uniform()])
        wo, wi = _unit(rng), _unit(rng)
        f, _, _ = orc.disney_eval(mp, N, X, wo, wi)
        g, _, _, _ = orc.brdf_eval([0, 0, 0, 1, 1, 1, r * r], N, wo, wi)
        assert np.allclose(f, g, rtol=1e-12, atol=0), (f, g)


def test_reciprocity_and_below_surface(orc):
    rng = np.random.default_rng(1)
    for _ in range(60):
        mp = _rand_params(rng)
        t = rng.normal(size=3)
        a, b = _unit(rng), _unit(rng)
        fa, _, da = orc.disney_eval(mp, N, t, a, b)
        fb, _, db = orc.disney_eval(mp, N, t, b, a)
        assert np.allclose(fa, fb, rtol=1e-12)
        assert np.allclose(da, db, rtol=1e-10, atol=1e-13 * np.abs(da).max())
        below = b * np.array([1, 1, -1.0])
        f0, p0, d0 = orc.disney_eval(mp, N, t, a, below)
        assert not f0.any() and p0 == 0.0 and not d0.any()


def test_complex_step_derivatives_match_central_differences(orc):
    """All 13 derivatives of all 3 channels against central differences of
    the value (h = 1e-6), away from the alpha clamp."""
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(40):
        mp = _rand_params(rng)
        t = rng.normal(size=3)
        wo, wi = _unit(rng), _unit(rng)
        f, _, df = orc.disney_eval(mp, N, t, wo, wi)
        assert np.all(np.isfinite(df))
        for j in range(13):
            pp, pm = mp.copy(), mp.copy()
            pp[j] += h
            pm[j] -= h
            fd = (orc.disney_eval(pp, N, t, wo, wi)[0] - orc.disney_eval(pm, N, t, wo, wi)[0]) / (2 * h)
            scale = np.abs(df).max() + np.abs(f).max()
            assert np.allclose(df[j], fd, rtol=1e-5, atol=1e-7 * scale), (j, df[j], fd)


def test_parameters_act_where_the_model_says(orc):
    """Structural zeros of the derivatives: with metallic 1 the diffuse,
    subsurface and sheen parameters have no effect; with clearcoat 0 the
    clearcoat gloss has none; channel c of f does not depend on the other
    base-colour channels unless a tint (specular or sheen) is on."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        wo, wi = _unit(rng), _unit(rng)
        mp = _rand_params(rng)
        mp[4] = 1.0          # metallic
        mp[11] = 0.0         # clearcoat
        _, _, df = orc.disney_eval(mp, N, X, wo, wi)
        for j in (3, 9, 10, 12):   # subsurface, sheen, sheen tint, clearcoat gloss
            assert not df[j].any(), j
        mp = _rand_params(rng)
        mp[6] = 0.0          # specular tint
        mp[9] = 0.0          # sheen
        _, _, df = orc.disney_eval(mp, N, X, wo, wi)
        for c in range(3):
            for j in range(3):
                if j != c:
                    assert df[j][c] == 0.0, (j, c)


@pytest.mark.parametrize("case", ["diffuse", "metal", "coat", "mixed"])
def test_sampler_against_pdf(orc, case):
    """The pdf integrates (by quadrature over the hemisphere) to the fraction
    of sampled directions that land above the surface, and a histogram of the
    samples in (cos theta, phi) cells matches the pdf integrated over each
    cell (chi-square)."""
    mp = {"diffuse": [0.6, 0.5, 0.4, 0.3, 0.0, 0.2, 0.1, 0.8, 0.0, 0.5, 0.3, 0.0, 0.2],
          "metal": [0.8, 0.6, 0.5, 0.0, 1.0, 0.5, 0.0, 0.6, 0.7, 0.0, 0.0, 0.0, 0.0],
          "coat": [0.05, 0.05, 0.05, 0.0, 0.0, 0.0, 0.0, 0.7, 0.0, 0.0, 0.0, 1.0, 0.0],
          "mixed": [0.4, 0.6, 0.2, 0.5, 0.3, 0.7, 0.4, 0.55, 0.4, 0.6, 0.5, 0.6, 0.3]}[case]
    mp = np.array(mp, np.float64)
    wo = np.array([0.5, 0.1, 0.0])
    wo[2] = math.sqrt(1 - wo[0] ** 2 - wo[1] ** 2)
    dirs, dw = _hemisphere_grid(240, 240)
    ptot = sum(orc.disney_eval(mp, N, X, wo, wi)[1] for wi in dirs) * dw
    rng = np.random.default_rng(9)
    Ns = 40000
    nt, npb = 10, 12
    counts = np.zeros((nt, npb))
    ok = 0
    for u in rng.random((Ns, 3)):
        lobe, wi = orc.disney_sample(mp, N, X, wo, *u)
        if lobe < 0 or wi[2] <= 0:
            continue
        ok += 1
        it = min(nt - 1, int(wi[2] * nt))
        ip = int(((math.atan2(wi[1], wi[0]) + 2 * math.pi) % (2 * math.pi)) / (2 * math.pi) * npb) % npb
        counts[it, ip] += 1
    frac = ok / Ns
    assert abs(ptot - frac) < 4 * math.sqrt(frac * (1 - frac) / Ns) + 3e-3, (ptot, frac)
    sub = 8
    exp = np.zeros((nt, npb))
    for it in range(nt):
        for ip in range(npb):
            acc = 0.0
            for a in range(sub):
                for b in range(sub):
                    c = (it + (a + 0.5) / sub) / nt
                    ph = (ip + (b + 0.5) / sub) / npb * 2 * math.pi
                    s = math.sqrt(1 - c * c)
                    acc += orc.disney_eval(mp, N, X, wo, np.array([s * math.cos(ph), s * math.sin(ph), c]))[1]
            exp[it, ip] = acc / (sub * sub) * (1.0 / nt) * (2 * math.pi / npb) * Ns
    mask = exp > 20
    chi2 = np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask])
    assert stats.chi2.sf(chi2, mask.sum() - 1) > 1e-4, chi2


def test_metallic_energy_bounded(orc):
    """The metallic lobe (GGX with Schlick's Fresnel toward the base colour)
    reflects at most the incident energy, less for a darker base."""
    dirs, dw = _hemisphere_grid(120, 120)
    for r in (0.4, 0.7, 1.0):
        for th in (0.2, 1.0, 1.4):
            wo = np.array([math.sin(th), 0, math.cos(th)])
            e_white = sum(orc.disney_eval([1, 1, 1, 0, 1, 0, 0, r, 0, 0, 0, 0, 0], N, X, wo, wi)[0][0] * wi[2]
                          for wi in dirs) * dw
            e_grey = sum(orc.disney_eval([0.3, 0.3, 0.3, 0, 1, 0, 0, r, 0, 0, 0, 0, 0], N, X, wo, wi)[0][0] * wi[2]
                         for wi in dirs) * dw
            assert 0.0 < e_grey < e_white <= 1.0 + 2e-3, (r, th, e_grey, e_white)


def test_estimator_fd_disney_cornell(orc):
    """Central differences (h = 1e-3 and h/2, Richardson) of the whole
    estimator with frozen sampling against the product-rule gradient, on
    every Disney parameter of three segments and on the emitter."""
    s = scenes.disney(scenes.cornell(), seed=4)
    sc = orc.Scene(s["verts"], s["tris"], s["tri_seg"], s["num_segments"], s["emitter_seg"], s["normals"],
                   material=1)
    assert sc.P == 13 * 8 + 3
    rng = np.random.default_rng(5)
    pix = np.arange(0, 64 * 64, 41, dtype=np.int64)
    w = rng.normal(size=(pix.size, 3))
    opts = dict(spp=4, max_depth=3, mis=2, seed=5, stream_tag=2)
    p = s["params"].astype(np.float64)
    g = sc.run(s["cams"], p, pixel_list=pix, w=w, want_grad=True, **opts)["grad"]
    gmax = np.abs(g).max()

    def cd(i, h):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        Ip = sc.run(s["cams"], pp, sampling_params=p, pixel_list=pix, **opts)["image"]
        Im = sc.run(s["cams"], pm, sampling_params=p, pixel_list=pix, **opts)["image"]
        return np.sum(w * (Ip - Im)) / (2 * h)

    idx = [13 * seg + j for seg in (0, 2, 5) for j in range(13)] + [104, 105, 106]
    for i in idx:
        fd = (4 * cd(i, 5e-4) - cd(i, 1e-3)) / 3
        assert abs(fd - g[i]) <= 2e-5 * max(abs(g[i]), 1e-2 * gmax), (i, fd, g[i])
    assert np.count_nonzero(g[idx]) > 0.8 * len(idx)
