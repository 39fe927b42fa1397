"""Pins of the oracle's estimator and its derivatives against closed forms
(white furnace, Lambert's polygon irradiance), against central finite
differences of its own forward renders (the derivative code and the forward
code are separate), and against exact invariants (linearity in emission)."""
import math

import numpy as np
import pytest

from paper_1903_07145_amd import scenes


def _oscene(orc, s):
    return orc.Scene(s["verts"], s["tris"], s["tri_seg"], s["num_segments"], s["emitter_seg"],
                     s["normals"])


# --------------------------------------------------------------------------
# White furnace: closed cube, all faces one Lambertian emitter (rho, E).
# L = E sum_{k=0}^{D} rho^k ; dL/drho = E sum_{k=1}^{D} k rho^{k-1};
# dL/dE = sum_{k=0}^{D} rho^k.  BRDF-only sampling has zero variance.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("D", [1, 3, 6])
def test_furnace_brdf_only_exact(orc, D):
    rho, E = 0.6, 2.0
    s = scenes.furnace(rho, E)
    rho, E = float(s["params"][0]), float(s["params"][7])   # float32-rounded inputs
    sc = _oscene(orc, s)
    r = sc.run(s["cams"], s["params"], spp=4, max_depth=D, mis=0, want_path_L=True)
    L = E * sum(rho ** k for k in range(D + 1))
    assert np.allclose(r["path_L"], L, rtol=1e-12)
    # gradient of sum_j w_j I_j with w = 1 on channel 0 of every pixel
    npix = 64
    w = np.zeros((npix, 3))
    w[:, 0] = 1.0
    g = sc.run(s["cams"], s["params"], spp=4, max_depth=D, mis=0, w=w, want_grad=True)["grad"]
    dL_drho = E * sum(k * rho ** (k - 1) for k in range(1, D + 1))
    dL_dE = sum(rho ** k for k in range(D + 1))
    assert abs(g[0] - npix * dL_drho) < 1e-9 * npix * dL_drho
    assert abs(g[7] - npix * dL_dE) < 1e-9 * npix * dL_dE
    assert np.allclose(g[[1, 2, 8, 9]], 0.0, atol=1e-12)


@pytest.mark.parametrize("mis", [1, 2, 3])
def test_furnace_with_light_sampling_unbiased(orc, mis):
    rho, E, D = 0.5, 1.0, 3
    s = scenes.furnace(rho, E)
    rho, E = float(s["params"][0]), float(s["params"][7])
    sc = _oscene(orc, s)
    r = sc.run(s["cams"], s["params"], spp=256, max_depth=D, mis=mis, want_path_L=True)
    x = r["path_L"][:, :, 0].ravel()
    L = E * sum(rho ** k for k in range(D + 1))
    se = x.std() / math.sqrt(x.size)
    assert abs(x.mean() - L) < 5 * se + 1e-12


def _polygon_irradiance(x, n, poly):
    """Lambert's formula: E/L = 1/2 sum_i Theta_i (n . gamma_i)."""
    tot = 0.0
    m = len(poly)
    for i in range(m):
        a = poly[i] - x
        b = poly[(i + 1) % m] - x
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        th = math.acos(np.clip(np.dot(a, b), -1, 1))
        g = np.cross(a, b)
        g /= np.linalg.norm(g)
        tot += th * np.dot(n, g)
    return 0.5 * abs(tot)


@pytest.mark.parametrize("mis", [0, 1, 2])
def test_area_light_direct_lighting_closed_form(orc, mis):
    """Depth 1, pixel centres: E[L] = rho/pi * Le * (polygon form factor)."""
    rho, Le, hl, hgt = 0.6, 5.0, 0.5, 1.0
    s = scenes.area_light_plane(rho, Le, hl, hgt)
    sc = _oscene(orc, s)
    cams = s["cams"]
    W, H = cams["width"], cams["height"]
    r = sc.run(cams, s["params"], spp=2048, max_depth=1, mis=mis, jitter=0, want_path_L=True)
    poly = [np.array(p, np.float64) for p in
            [(-hl, hgt, -hl), (hl, hgt, -hl), (hl, hgt, hl), (-hl, hgt, hl)]]
    checked = 0
    for pix in range(W * H):
        y, xx = divmod(pix, W)
        o, d = orc.camera_ray(cams["cam_to_world"][0], cams["fov_y"][0], W, H, xx + 0.5, y + 0.5)
        tri, _ = sc.closest_hit(o, d)
        samples = r["path_L"][pix, :, 0]
        if tri < 0 or s["tri_seg"][tri] != 0:
            continue
        t = -o[1] / d[1]
        x = o + t * d
        Eirr = Le * _polygon_irradiance(x, np.array([0, 1.0, 0]), poly)
        expect = rho / math.pi * Eirr
        se = samples.std() / math.sqrt(samples.size)
        assert abs(samples.mean() - expect) < 5 * se + 1e-9, (pix, samples.mean(), expect, se)
        checked += 1
    assert checked > 20


# --------------------------------------------------------------------------
# Finite differences with frozen sampling parameters: sum_j w_j I_j(theta)
# is, per sample, a smooth function of theta, so central differences with
# h = 1e-3 match the analytic product-rule gradient to ~1e-6.
# --------------------------------------------------------------------------
def _fd_check(orc, s, params, pix, opts, idx, rng, rtol=2e-5):
    """Central differences (h = 1e-3 and h/2, Richardson-extrapolated so the
    roughness terms, which are not polynomial, are also O(h^4))."""
    sc = _oscene(orc, s)
    w = rng.normal(size=(pix.size, 3))
    base = sc.run(s["cams"], params, pixel_list=pix, w=w, want_grad=True, **opts)
    g = base["grad"]
    scale = np.max(np.abs(g)) + 1e-30

    def cd(i, h):
        pp = params.astype(np.float64).copy()
        pm = pp.copy()
        pp[i] += h
        pm[i] -= h
        Ip = sc.run(s["cams"], pp, sampling_params=params, pixel_list=pix, **opts)["image"]
        Im = sc.run(s["cams"], pm, sampling_params=params, pixel_list=pix, **opts)["image"]
        return np.sum(w * (Ip - Im)) / (2 * h)

    for i in idx:
        h = 1e-3
        fd = (4 * cd(i, h / 2) - cd(i, h)) / 3
        assert abs(fd - g[i]) <= rtol * max(abs(g[i]), 1e-2 * scale), (i, fd, g[i])
    return g


def test_fd_cornell_lambert(orc):
    s = scenes.cornell()
    rng = np.random.default_rng(0)
    pix = np.arange(0, 64 * 64, 37, dtype=np.int64)
    opts = dict(spp=4, max_depth=3, mis=2, seed=5, stream_tag=2)
    g = _fd_check(orc, s, s["params"], pix, opts, range(s["params"].size), rng)
    assert np.count_nonzero(g) >= 27


def test_fd_zero_albedo_and_emission(orc):
    """Derivatives stay exact at kd = 0 and e = 0 (the paper initialises there)."""
    s = scenes.cornell()
    p = s["params"].copy()
    p[0:3] = 0.0            # floor albedo
    p[7 * 2:7 * 2 + 3] = 0.0  # back wall albedo
    p[56:59] = [3.0, 0.0, 0.0]  # emitter: two zero channels
    rng = np.random.default_rng(1)
    pix = np.arange(0, 64 * 64, 29, dtype=np.int64)
    opts = dict(spp=4, max_depth=3, mis=2, seed=6, stream_tag=2)
    g = _fd_check(orc, s, p, pix, opts, [0, 1, 2, 14, 15, 16, 56, 57, 58], rng)
    # at kd_r = 0 (red light present) and at e_g = 0 the derivatives are live
    assert abs(g[0]) > 0 and abs(g[57]) > 0


@pytest.mark.parametrize("variant", ["ggx", "rr_profile", "power_mis"])
def test_fd_room_ggx(orc, variant):
    s = scenes.room()
    rng = np.random.default_rng(2)
    W, H = s["cams"]["width"], s["cams"]["height"]
    pix = np.array([(y * W + x) for y in range(100, 112, 3) for x in range(140, 180, 4)], np.int64)
    opts = dict(spp=4, max_depth=4, mis=2, seed=9, stream_tag=2)
    if variant == "rr_profile":
        opts.update(rr_depth=2, emission_profile=1)
    if variant == "power_mis":
        opts.update(mis=3)
    sc = _oscene(orc, s)
    w = rng.normal(size=(pix.size, 3))
    g = sc.run(s["cams"], s["params"], pixel_list=pix, w=w, want_grad=True, **opts)["grad"]
    nz = np.flatnonzero(np.abs(g) > 1e-3 * np.abs(g).max())
    idx = rng.choice(nz, size=min(24, nz.size), replace=False)
    # include some roughness and specular entries if touched
    extra = [i for i in nz if i < 7 * s["num_segments"] and i % 7 in (3, 6)][:6]
    _fd_check(orc, s, s["params"], pix, opts, sorted(set(idx) | set(extra)), rng)


def test_linearity_in_emission(orc):
    """L is linear in the emission: sum_k e_k dI/de_k = I, per sample."""
    s = scenes.room()
    sc = _oscene(orc, s)
    W = s["cams"]["width"]
    pix = np.arange(50 * W + 100, 50 * W + 164, dtype=np.int64)
    rng = np.random.default_rng(3)
    w = rng.normal(size=(pix.size, 3))
    r = sc.run(s["cams"], s["params"], pixel_list=pix, w=w, want_grad=True, spp=4,
               max_depth=4, mis=2, seed=3)
    S = s["num_segments"]
    e = s["params"][7 * S:].astype(np.float64)
    lhs = np.dot(e, r["grad"][7 * S:])
    rhs = np.sum(w * r["image"])
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs))


def test_pixel_list_matches_full_render(orc):
    s = scenes.cornell()
    sc = _oscene(orc, s)
    full = sc.run(s["cams"], s["params"], spp=2, max_depth=3)["image"]
    pix = np.array([5, 100, 2000, 4095], np.int64)
    part = sc.run(s["cams"], s["params"], spp=2, max_depth=3, pixel_list=pix)["image"]
    assert np.array_equal(full[pix], part)


def test_light_probabilities(orc):
    s = scenes.room()
    sc = _oscene(orc, s)
    pr = sc.light_probs(s["params"])
    assert pr.size == 8 and abs(pr.sum() - 1) < 1e-12
    p0 = s["params"].copy()
    S = s["num_segments"]
    p0[7 * S:] = 0.0
    pz = sc.light_probs(p0)     # all emission zero: area-proportional
    assert np.allclose(pz, pz[0])
    p1 = s["params"].copy()
    p1[7 * S:7 * S + 3] = 0.0   # one dark emitter keeps a small floor probability
    pr1 = sc.light_probs(p1)
    assert pr1[0] > 0 and pr1[0] < 1e-3


def test_conditioning_probes(orc):
    """The parity probes: most Lambertian paths in the Cornell box are well
    conditioned (radiance and gradient change by far less than 1e-4 under a
    1e-6 perturbation), while sharp GGX lobes in the room make path gradients
    more ill-conditioned than their radiance."""
    s = scenes.cornell()
    sc = _oscene(orc, s)
    pix = np.arange(0, 64 * 64, 61, dtype=np.int64)
    w = np.random.default_rng(3).normal(size=(pix.size, 3))
    r = sc.run(s["cams"], s["params"], pixel_list=pix, w=w, want_cond=True, spp=4, max_depth=3, mis=2, seed=9)
    assert r["gcond"].shape == r["cond"].shape
    fin = np.isfinite(r["cond"])
    assert fin.mean() > 0.95
    for c in (r["cond"][fin], r["gcond"][fin]):
        assert np.median(c) < 1e-4 and np.percentile(c, 95) < 1e-3
    s2 = scenes.room()
    sc2 = _oscene(orc, s2)
    W, H = s2["cams"]["width"], s2["cams"]["height"]
    pix2 = np.arange(0, 4 * W * H, 997, dtype=np.int64)
    w2 = np.random.default_rng(4).normal(size=(pix2.size, 3))
    r2 = sc2.run(s2["cams"], s2["params"], pixel_list=pix2, w=w2, want_cond=True, spp=4, max_depth=5, mis=2,
                 seed=9)
    both = np.isfinite(r2["cond"]) & np.isfinite(r2["gcond"])
    assert np.median(r2["gcond"][both]) < 1e-3
    assert (r2["gcond"][both] > r2["cond"][both]).mean() > 0.5


def test_conditioning_probe_flags_chaotic_paths(orc):
    """What the probe is for: a path whose radiance moves by more than 1e-2
    (with unchanged events) when the camera moves by 1e-5 m (about ten float32 ulps of its
    coordinates, along a direction the probe itself does not use) cannot be
    reproduced in float32, so the probe must rate it above the 1e-3 that
    admits a path to the tight comparison.  Apartment, the benchmark's
    sampling (8 spp, depth 7, RR from 3); cylinders with smooth normals make
    some paths chaotic."""
    import copy
    s = scenes.apartment()
    sc = _oscene(orc, s)
    V, W, H = s["cams"]["cam_to_world"].shape[0], s["cams"]["width"], s["cams"]["height"]
    pix = np.arange(0, V * W * H, 2003, dtype=np.int64)
    kw = dict(pixel_list=pix, seed=11, stream_tag=2, iteration=4, spp=8, max_depth=7, rr_depth=3, mis=2)
    p = scenes.init_theta(s, "uniform", seed=7)   # the benchmark's starting point
    base = sc.run(s["cams"], p, want_hash=True, want_path_L=True, want_cond=True, **kw)
    sens = np.zeros(base["cond"].shape, bool)
    for sign in (1.0, -1.0):
        cams = copy.deepcopy(s["cams"])
        shift = sign * 1e-5 * np.array([0.6, -0.48, 0.64]) / np.linalg.norm([0.6, -0.48, 0.64])
        c2w = cams["cam_to_world"].astype(np.float64)
        c2w[:, :3, 3] += shift
        cams["cam_to_world"] = c2w.astype(np.float32)
        r = sc.run(cams, p, want_hash=True, want_path_L=True, **kw)
        lm = np.abs(base["path_L"]).max(axis=2)
        ch = np.abs(r["path_L"] - base["path_L"]).max(axis=2) / np.maximum(lm, 1e-12)
        # continuous sensitivity: the same events, the radiance moved (an event
        # that flips under one particular shift is a near-tie, the margin's case)
        sens |= (r["hash"] == base["hash"]) & (ch > 1e-2)
    assert sens.sum() >= 5                           # the scene does have chaotic paths
    assert np.all(base["cond"][sens] > 1e-3), np.sort(base["cond"][sens])[:5]
    assert (base["cond"] <= 1e-3).mean() > 0.7      # and most paths are well conditioned
