"""Pins of three parts of the oracle that its other tests do not fix.

* Russian roulette (the workloads' "RR from depth 3"; the paper is silent on
  the rule, the reading is: survival probability q = clamp(max_c Ts_c, 0.1,
  0.95) on the throughput at the sampling parameters -- the product of the
  continuation weights up to and including vertex k and of the 1/q of the
  earlier survivals -- applied at vertices k >= rr_depth, the survivor
  divided by q).
  - Unbiasedness: in the white furnace the mean over many paths, and over
    seeds the mean gradient, equal the closed forms E sum rho^k,
    E sum k rho^(k-1) and sum rho^k (Sec. 3.1, Eq. 2; Sec. 3.3, Eq. 5-6)
    within 5 standard errors, for rr_depth 1 and 2, BRDF-only and with MIS.
    A survivor not divided by q, or q applied twice, fails these.
  - The rule itself: with BRDF-only sampling of a Lambertian furnace every
    continuation weight is exactly rho, so each path's value is a closed-form
    function of its own roulette uniforms.  The test draws those uniforms
    with the (separately pinned) Philox generator and the reading of the
    counter layout, and rebuilds every path value and its derivatives.  With
    RGB albedos and sampling albedos different from the rendered ones this
    fixes the clamp bounds, the max over channels, the use of the sampling
    throughput Ts (not T) with the earlier 1/q in it, the start vertex and the
    1/q weight.
* The paper's emission profile L_e(x, w) = e(x) (w . n(x))_+ (Sec. 4.3):
  direct light from a square emitter with that profile onto a Lambertian
  plane equals rho/pi * integral of e cos^2(theta_l) cos(theta_x) / r^2 over
  the emitter, evaluated here by Gauss-Legendre quadrature in numpy; checked
  for BRDF sampling, light sampling and MIS.
* Light selection weights (App. E: emission-proportional selection; reading:
  per emitter triangle area * max(lum(e), 1e-3 max_k lum(e_k)), lum = mean
  RGB, area only when every emission is zero) on emitter triangles of
  unequal area, and the consistency of next-event estimation with them: two
  emitters of different size and radiance light a plane to the sum of two
  Lambert polygon-irradiance closed forms.
"""
import math

import numpy as np
import pytest

from paper_1903_07145_amd import scenes


def _oscene(orc, s):
    return orc.Scene(s["verts"], s["tris"], s["tri_seg"], s["num_segments"], s["emitter_seg"],
                     s["normals"])


def _furnace(orc, rho_rgb, E):
    s = scenes.furnace(0.5, E)
    s["params"][0:3] = np.asarray(rho_rgb, np.float32)
    return s, _oscene(orc, s)


def _u24(x):
    return float(np.uint32(x) >> np.uint32(8)) * 2.0 ** -24


def _rr_uniform(orc, seed, tag, iteration, path_id, k):
    """Slot 6 of vertex k (the roulette uniform): the second 128-bit block of
    the vertex, counter (path_lo, path_hi, 2k + 1, iteration), element 2."""
    key = [(seed & 0xFFFFFFFF) ^ ((tag * 0x9E3779B9) & 0xFFFFFFFF), seed >> 32]
    ctr = [path_id & 0xFFFFFFFF, path_id >> 32, 2 * k + 1, iteration]
    return _u24(orc.philox4x32_10(ctr, key)[2])


# --------------------------------------------------------------------------
# Unbiasedness under Russian roulette.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("rr_depth,mis", [(1, 0), (2, 0), (1, 2), (2, 2)])
def test_rr_furnace_unbiased(orc, rr_depth, mis):
    rho, E, D = 0.6, 2.0, 6
    s, sc = _furnace(orc, [rho] * 3, E)
    rho, E = float(s["params"][0]), float(s["params"][7])
    r = sc.run(s["cams"], s["params"], spp=256, max_depth=D, rr_depth=rr_depth, mis=mis, seed=17,
               want_path_L=True)
    x = r["path_L"][:, :, 0].ravel()
    L = E * sum(rho ** k for k in range(D + 1))
    se = x.std() / math.sqrt(x.size)
    assert se > 0                                   # the roulette adds variance ...
    assert abs(x.mean() - L) < 5 * se, (x.mean(), L, se)   # ... but no bias
    # not dividing by q would give E (1 + sum_k rho^k prod_{j >= rr} q_j) instead
    biased = E * (1 + sum(rho ** k * np.prod([min(max(rho ** j, 0.1), 0.95) for j in range(rr_depth, k + 1)])
                          for k in range(1, D + 1)))
    assert abs(biased - L) > 20 * se


@pytest.mark.parametrize("rr_depth", [1, 2])
def test_rr_furnace_gradient_unbiased(orc, rr_depth):
    """Mean over K independent iterations of the gradient of sum_j I_j (all
    pixels, channel 0) against npix dL/drho and npix dL/dE."""
    rho, E, D, K = 0.6, 2.0, 5, 48
    s, sc = _furnace(orc, [rho] * 3, E)
    rho, E = float(s["params"][0]), float(s["params"][7])
    npix = 64
    w = np.zeros((npix, 3))
    w[:, 0] = 1.0
    gs = np.array([sc.run(s["cams"], s["params"], spp=8, max_depth=D, rr_depth=rr_depth, mis=0, seed=23,
                          iteration=it, w=w, want_grad=True)["grad"] for it in range(K)])
    dL_drho = npix * E * sum(k * rho ** (k - 1) for k in range(1, D + 1))
    dL_dE = npix * sum(rho ** k for k in range(D + 1))
    for i, ref in ((0, dL_drho), (7, dL_dE)):
        m, se = gs[:, i].mean(), gs[:, i].std(ddof=1) / math.sqrt(K)
        assert se > 0
        assert abs(m - ref) < 5 * se, (i, m, ref, se)


# --------------------------------------------------------------------------
# The roulette rule, path by path.
# --------------------------------------------------------------------------
# sampling albedos: the rendered ones; different ones (so Ts != T); dark
# ones (q at the 0.1 floor); bright ones (q at the 0.95 cap)
RHO_S = {"same": None, "frozen": [0.4, 0.7, 0.2], "dark": [0.04, 0.02, 0.03], "bright": [0.99, 0.97, 0.98]}


@pytest.mark.parametrize("case", sorted(RHO_S))
def test_rr_rule_path_by_path(orc, case):
    rho = np.array([0.6, 0.3, 0.5])
    frozen = RHO_S[case] is not None
    rho_s = np.array(RHO_S[case]) if frozen else rho
    E, D, rr, spp, seed, tag, it = 2.0, 6, 2, 16, 29, 2, 3
    s, sc = _furnace(orc, rho, E)
    p = s["params"].astype(np.float64)
    sp = p.copy()
    if frozen:
        sp[0:3] = rho_s
    rho, rho_s, E = p[0:3], sp[0:3], p[7]
    npix = 64
    w = np.random.default_rng(5).normal(size=(npix, 3))
    kw = dict(spp=spp, max_depth=D, rr_depth=rr, mis=0, seed=seed, stream_tag=tag, iteration=it)
    r = sc.run(s["cams"], p, sampling_params=sp if frozen else None, w=w, want_path_L=True, want_grad=True, **kw)
    L_ref = np.zeros((npix, spp, 3))
    g_ref = np.zeros(p.size)
    for pix in range(npix):
        for smp in range(spp):
            pid = pix * spp + smp
            inv_q = 1.0          # prod of 1/q over the roulette vertices passed so far
            val = np.ones(3)     # E-free path value: sum_k rho^k / prod q
            drho = np.zeros(3)   # its derivative per channel: sum_k k rho^(k-1) / prod q
            for k in range(1, D + 1):
                # continuation at vertex k; the throughput at the sampling
                # parameters after it, including the 1/q of the earlier
                # survivals, is rho_s^k * inv_q per channel
                if k >= rr:
                    q = min(max(float(np.max(rho_s ** k)) * inv_q, 0.1), 0.95)
                    if not _rr_uniform(orc, seed, tag, it, pid, k) < q:
                        break
                    inv_q /= q
                val = val + rho ** k * inv_q
                drho = drho + k * rho ** (k - 1) * inv_q
            L_ref[pix, smp] = E * val
            g_ref[0:3] += w[pix] * E * drho / spp
            g_ref[7:10] += w[pix] * val / spp
    assert np.allclose(r["path_L"], L_ref, rtol=1e-12, atol=0)
    assert np.allclose(r["grad"][[0, 1, 2, 7, 8, 9]], g_ref[[0, 1, 2, 7, 8, 9]], rtol=1e-11, atol=0)
    # the roulette actually ended paths at different depths
    ends = np.unique(np.round(L_ref[..., 0] / E, 9))
    assert ends.size > 3


# --------------------------------------------------------------------------
# Cosine emission profile (Sec. 4.3) by quadrature.
# --------------------------------------------------------------------------
def _profile_irradiance(x, hl, hgt, n_gl=48):
    """integral over the square emitter [-hl, hl]^2 at height hgt (facing
    down) of cos^2(theta_l) cos(theta_x) / r^2 dA, for a point x on the
    plane y = 0 facing up: the radiance leaving the emitter toward x is
    e cos(theta_l), and the solid angle brings one more cos(theta_l) / r^2."""
    t, wt = np.polynomial.legendre.leggauss(n_gl)
    gx, gz = np.meshgrid(hl * t, hl * t, indexing="ij")
    ww = np.outer(wt, wt) * hl * hl
    dx, dy, dz = gx - x[0], hgt - x[1], gz - x[2]
    r2 = dx * dx + dy * dy + dz * dz
    cos_l = dy / np.sqrt(r2)   # emitter normal (0, -1, 0) against the direction to x
    cos_x = dy / np.sqrt(r2)   # plane normal (0, 1, 0) against the direction to the emitter
    return float(np.sum(ww * cos_l * cos_l * cos_x / r2))


@pytest.mark.parametrize("mis", [0, 1, 2])
def test_cosine_emission_profile_closed_form(orc, mis):
    rho, e, hl, hgt = 0.6, 5.0, 0.5, 1.0
    s = scenes.area_light_plane(rho, e, hl, hgt)
    rho, e = float(s["params"][0]), float(s["params"][14])
    sc = _oscene(orc, s)
    cams = s["cams"]
    W, H = cams["width"], cams["height"]
    r = sc.run(cams, s["params"], spp=2048, max_depth=1, mis=mis, jitter=0, emission_profile=1,
               want_path_L=True)
    # the quadrature resolves the integrand: doubling the nodes changes nothing
    x0 = np.array([0.3, 0.0, -0.2])
    assert abs(_profile_irradiance(x0, hl, hgt, 48) - _profile_irradiance(x0, hl, hgt, 96)) < 1e-12
    checked = 0
    for pix in range(W * H):
        y, xx = divmod(pix, W)
        o, d = orc.camera_ray(cams["cam_to_world"][0], cams["fov_y"][0], W, H, xx + 0.5, y + 0.5)
        tri, _ = sc.closest_hit(o, d)
        if tri < 0 or s["tri_seg"][tri] != 0:
            continue
        x = o + (-o[1] / d[1]) * d
        expect = rho / math.pi * e * _profile_irradiance(x, hl, hgt)
        samples = r["path_L"][pix, :, 0]
        se = samples.std() / math.sqrt(samples.size)
        assert abs(samples.mean() - expect) < 5 * se + 1e-9, (pix, samples.mean(), expect, se)
        # the constant-radiance profile would give a visibly larger value
        checked += 1
    assert checked > 20


# --------------------------------------------------------------------------
# Light selection on emitter triangles of unequal area.
# --------------------------------------------------------------------------
def _two_light_scene(e_a, e_b, e_c):
    """A plane (segment 0, y = 0, facing up) under three emitters facing
    down: A a single triangle, B an irregular quad split into two triangles
    of different area, C a small triangle (segments 1, 2, 3)."""
    V = [(-8, 0, -8), (8, 0, -8), (8, 0, 8), (-8, 0, 8),           # plane
         (-1.2, 1.0, -0.8), (-0.2, 1.0, -0.9), (-0.9, 1.0, 0.5),   # A (clockwise seen from below)
         (0.3, 1.2, -0.6), (1.4, 1.2, -0.5), (1.1, 1.2, 0.9), (0.4, 1.2, 0.2),   # B
         (-0.3, 0.9, 1.0), (0.1, 0.9, 1.05), (-0.2, 0.9, 1.3)]    # C
    T = [(0, 2, 1), (0, 3, 2),
         (4, 5, 6),
         (7, 8, 9), (7, 9, 10),
         (11, 12, 13)]
    verts = np.array(V, np.float32)
    tris = np.array(T, np.int32)
    # emitters face down: flip any triangle whose normal points up
    for i in range(2, tris.shape[0]):
        a, b, c = verts[tris[i]]
        if np.cross(b - a, c - a)[1] > 0:
            tris[i] = tris[i][[0, 2, 1]]
    seg = np.array([0, 0, 1, 2, 2, 3], np.int32)
    p = np.array([0.6, 0.6, 0.6, 0, 0, 0, 0.5] + [0, 0, 0, 0, 0, 0, 0.5] * 3 + list(e_a) + list(e_b) + list(e_c),
                 np.float32)
    cams = dict(cam_to_world=scenes.look_at([0.0, 6.0, 3.0], [0.0, 0.0, 0.0])[None],
                fov_y=np.array([math.radians(50.0)], np.float32), width=8, height=8)
    return dict(name="three_lights", verts=verts, normals=None, tris=tris, tri_seg=seg, num_segments=4,
                emitter_seg=np.array([1, 2, 3], np.int32), cams=cams, params=p)


def _tri_area(v, t):
    a, b, c = v[t].astype(np.float64)
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a))


def test_light_probabilities_unequal_areas(orc):
    cases = [([4.0, 2.0, 3.0], [1.0, 1.5, 0.5], [9.0, 9.0, 9.0]),
             ([4.0, 2.0, 3.0], [0.0, 0.0, 0.0], [1e-4, 0.0, 0.0]),   # dim emitters at the 1e-3 floor
             ([0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0])]    # all dark: area only
    for e in cases:
        s = _two_light_scene(*e)
        sc = _oscene(orc, s)
        areas = np.array([_tri_area(s["verts"], s["tris"][i]) for i in range(2, 6)])
        assert np.ptp(areas) > 0.1 * areas.max()            # really unequal
        lum = np.array([np.mean(x) for x in e])
        k_of = np.array([0, 1, 1, 2])                        # emitter of each light triangle (input order)
        if lum.max() > 0:
            wgt = areas * np.maximum(lum[k_of], 1e-3 * lum.max())
        else:
            wgt = areas.copy()
        ref = wgt / wgt.sum()
        pr = sc.light_probs(s["params"])
        assert np.allclose(pr, ref, rtol=1e-12, atol=0), (e, pr, ref)


def _polygon_irradiance(x, n, poly):
    tot = 0.0
    for i in range(len(poly)):
        a = poly[i] - x
        b = poly[(i + 1) % len(poly)] - x
        a = a / np.linalg.norm(a)
        b = b / np.linalg.norm(b)
        g = np.cross(a, b)
        tot += math.acos(np.clip(np.dot(a, b), -1, 1)) * np.dot(n, g / np.linalg.norm(g))
    return 0.5 * abs(tot)


@pytest.mark.parametrize("mis", [1, 2])
def test_two_lights_direct_closed_form(orc, mis):
    """Next-event estimation with the unequal selection weights stays
    consistent: the plane's radiance is rho/pi times the sum over emitters of
    L_e times Lambert's polygon form factor (Lambert 1760; closed form)."""
    e = ([4.0, 2.0, 3.0], [1.0, 1.5, 0.5], [9.0, 9.0, 9.0])
    s = _two_light_scene(*e)
    sc = _oscene(orc, s)
    cams = s["cams"]
    W, H = cams["width"], cams["height"]
    r = sc.run(cams, s["params"], spp=4096, max_depth=1, mis=mis, jitter=0, want_path_L=True)
    v = s["verts"].astype(np.float64)
    polys = [[v[4], v[5], v[6]], [v[7], v[8], v[9], v[10]], [v[11], v[12], v[13]]]
    rho = float(s["params"][0])
    checked = 0
    for pix in range(W * H):
        y, xx = divmod(pix, W)
        o, d = orc.camera_ray(cams["cam_to_world"][0], cams["fov_y"][0], W, H, xx + 0.5, y + 0.5)
        tri, _ = sc.closest_hit(o, d)
        if tri < 0 or s["tri_seg"][tri] != 0:
            continue
        x = o + (-o[1] / d[1]) * d
        for c in range(3):
            expect = rho / math.pi * sum(e[k][c] * _polygon_irradiance(x, np.array([0, 1.0, 0]), polys[k])
                                         for k in range(3))
            samples = r["path_L"][pix, :, c]
            se = samples.std() / math.sqrt(samples.size)
            assert abs(samples.mean() - expect) < 5 * se + 1e-9, (pix, c, samples.mean(), expect, se)
        checked += 1
    assert checked > 20
