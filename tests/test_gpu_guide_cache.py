"""The cached proposal (ipt_guide_cache_build + guide_cached) on the GPU,
through the C ABI, against the oracle.

* Rows filled by the float32 network: images at 1e-4 and gradients at 1e-3
  against the oracle's guided estimator, which evaluates its float64 network
  at the query of the cell each vertex lies in (same cell rule), with the
  same near-tie and conditioning masks as the other parity tests; Cornell
  (flat, one-sided views) and the room (smooth normals, GGX, many cells per
  triangle on the walls).
* Rows filled by the bfloat16 MFMA network: the estimator keeps the mean of
  BRDF sampling.
* Host-side errors: no rows for the scene, bad cell area.
"""
import math

import numpy as np
import pytest
import torch

import _guide
from _gpu import check_mismatches, GRAD_ILL_COND, banner, both, comparable, dev, gpu_grad, gpu_render, mismatch_stats, oracle_opts
from paper_1903_07145_amd import ipt, scenes

pytestmark = pytest.mark.gpu

PIX_REL = 1e-4
GRAD_REL = 1e-3


def _guide_with(g, w):
    gd = ipt.Guide(g)
    gd.set_weights(w)
    return gd


def _kw(kw, gd, mix=0.5):
    return dict(kw, guide=gd, guide_mix=mix, guide_cached=1)


def _parity(sc, g, o, dc, gd, w, cell_area, kw, pix=None, mix=0.5):
    lo, inv = _guide.box(sc["verts"])
    ok = dict(guide_w=w, guide_mix=mix, bb_lo=lo, bb_inv=inv, guide_cell_area=cell_area)
    _, h_g = gpu_render(g, dc, sc["params"], _kw(kw, gd, mix), pixel_list=pix)
    r = o.run(sc["cams"], sc["params"], pixel_list=pix, want_hash=True, want_margin=True, want_cond=True,
              **oracle_opts(kw), **ok)
    b = check_mismatches(h_g, r, 3, label="cached proposal")
    n_mis, n_hard = b["mismatch"], b["hard"]
    keep = comparable(h_g, r)
    print("paths %d mismatching %d (hard %d), compared %.1f%%" % (h_g.size, n_mis, n_hard, 100 * keep.mean()))
    assert n_hard <= 1e-5 * 3 * h_g.size
    assert keep.mean() > 0.9
    img_g, _ = gpu_render(g, dc, sc["params"], _kw(kw, gd, mix), pixel_list=pix, mask=keep)
    ro = o.run(sc["cams"], sc["params"], pixel_list=pix, path_mask=keep.astype(np.uint8), **oracle_opts(kw), **ok)
    mean = np.abs(ro["image"]).mean()
    err = np.abs(img_g - ro["image"]) / np.maximum(np.abs(ro["image"]), 1e-4 * mean)
    print("pixel rel err p50 %.2e max %.2e" % (np.median(err), err.max()))
    assert err.max() <= PIX_REL
    npix = img_g.shape[0]
    wimg = np.random.default_rng(5).normal(size=(npix, 3))
    # paths whose gradient contribution is ill-conditioned are left out, as in
    # the unguided parity tests
    gcond = o.run(sc["cams"], sc["params"], pixel_list=pix, w=wimg, want_cond=True, **oracle_opts(kw), **ok)["gcond"]
    keep_g = keep & (gcond <= GRAD_ILL_COND)
    print("gradient compared on %.1f%% of paths" % (100 * keep_g.mean()))
    gg = gpu_grad(g, dc, sc["params"], wimg, _kw(kw, gd, mix), pixel_list=pix, mask=keep_g)
    go = o.run(sc["cams"], sc["params"], pixel_list=pix, w=wimg, path_mask=keep_g.astype(np.uint8), want_grad=True,
               **oracle_opts(kw), **ok)["grad"]
    rms = math.sqrt(np.mean(go ** 2))
    gerr = np.abs(gg - go) / np.maximum(np.abs(go), 1e-2 * rms)
    print("grad rel err max %.2e" % gerr.max())
    assert gerr.max() <= GRAD_REL


@pytest.mark.parametrize("mis", [0, 2])
def test_cached_guided_parity_cornell(mis):
    banner("cached proposal parity (float32 rows), cornell, mis=%d" % mis)
    sc = scenes.cornell()
    g, o = both(sc)
    dc = ipt.make_cameras(sc["cams"])
    w = _guide.random_weights(sc["num_segments"], seed=21, out_gain=3.0, kappa_bias=1.0)
    gd = _guide_with(g, w)
    cell_area = 2e-3   # walls: n = 16 (256 cells per triangle); box faces and the emitter fewer
    ncell = gd.cache_build(cell_area, mode=1)
    print("cells per side %d" % ncell)
    assert ncell > 36 * 4
    kw = dict(seed=41, stream_tag=1, iteration=2, spp=4, max_depth=3, mis=mis)
    _parity(sc, g, o, dc, gd, w, cell_area, kw)


def test_cached_guided_parity_room():
    banner("cached proposal parity (float32 rows), room: smooth normals, GGX")
    sc = scenes.room()
    g, o = both(sc)
    dc = ipt.make_cameras(sc["cams"])
    W, H = sc["cams"]["width"], sc["cams"]["height"]
    w = _guide.random_weights(sc["num_segments"], seed=22, out_gain=3.0, kappa_bias=1.0)
    gd = _guide_with(g, w)
    with pytest.raises(ipt.IPTError):
        gd.cache_build(1e-9)                        # more than 2^24 cells per side
    cell_area = 0.05
    ncell = gd.cache_build(cell_area, mode=1)
    print("cells per side %d for %d triangles" % (ncell, sc["tris"].shape[0]))
    assert ncell > sc["tris"].shape[0]
    pix = np.sort(np.random.default_rng(3).choice(4 * W * H, size=600, replace=False)).astype(np.int64)
    kw = dict(seed=43, stream_tag=1, iteration=1, spp=4, max_depth=3, mis=2)
    _parity(sc, g, o, dc, gd, w, cell_area, kw, pix=pix)


def _path_radiance(g, dc, params, kw, npix):
    L = torch.zeros(npix * kw["spp"] * 3, dtype=torch.float32, device="cuda")
    g.render(dc, dev(params), ipt.render_opts(debug_path_radiance=L, **kw))
    torch.cuda.synchronize()
    return L.cpu().numpy().astype(np.float64).reshape(-1, 3)


def test_cached_mfma_estimator_unbiased():
    banner("cached proposal (bf16 MFMA rows): same mean as BRDF sampling")
    sc = scenes.cornell()
    g = ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    gd = _guide_with(g, _guide.random_weights(sc["num_segments"], seed=23, out_gain=3.0, kappa_bias=1.5))
    gd.cache_build(2e-3, mode=0)
    # a second fill of the same scene reuses the table
    assert gd.cache_build(2e-3, mode=0) > 0
    for mis in (0, 2):
        kw = dict(seed=61, stream_tag=1, iteration=0, spp=64, max_depth=3, mis=mis)
        a = _path_radiance(g, dc, sc["params"], kw, 4096)
        b = _path_radiance(g, dc, sc["params"], dict(_kw(kw, gd), seed=62), 4096)
        se = np.sqrt(a.var(0) / a.shape[0] + b.var(0) / b.shape[0])
        print("mis %d mean brdf %s cached guide %s se %s" % (mis, a.mean(0), b.mean(0), se))
        assert np.all(np.abs(a.mean(0) - b.mean(0)) < 5 * se)


def test_cache_errors():
    banner("cached proposal: host-side errors")
    sc = scenes.cornell()
    g = ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    gd = _guide_with(g, _guide.random_weights(sc["num_segments"], seed=24))
    o = ipt.render_opts(spp=1, max_depth=2, guide=gd, guide_mix=0.5, guide_cached=1)
    with pytest.raises(ipt.IPTError):
        g.render(dc, dev(sc["params"]), o)          # no rows built yet
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(ipt.IPTError):
            gd.cache_build(bad)
    assert gd.cache_build(1e-9) == 36 * 64 * 64     # n capped at 64
    assert gd.cache_build(1e-2) > 0
    g.render(dc, dev(sc["params"]), o)
    torch.cuda.synchronize()
