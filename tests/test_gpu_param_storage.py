"""Parameters in global memory (ipt_build_opts.param_storage, automatic above
4096 parameters) through the C ABI: per-triangle materials (the paper's
coarse-to-fine refinement, App. E) make the parameter vector grow with the
triangle count, so the path kernels read it through the caches and the
adjoint adds float64 atomics into one accumulator instead of per-block LDS
copies and partials.

* Same scene, LDS vs forced global storage: the same events, images equal to
  float32 rounding (separately compiled kernels), gradients equal up to
  summation order (global storage
  sums float64 atomics into replicated accumulators, then the copies in a
  fixed order).
* Against the oracle at the usual bars: per-triangle Cornell (forced global),
  the textured Cornell ground truth (8256 parameters, global by size) and the
  per-triangle room (about 49k segments, 345k parameters) on pixel subsets.
  Parameters no compared path reaches must be zero on both sides; the rms
  that scales the gradient bar is taken over the parameters reached.
"""
import math

import numpy as np
import pytest
import torch

from _gpu import check_mismatches, GRAD_ILL_COND, banner, comparable, dev, gpu_grad, gpu_render, mismatch_stats, oracle_opts
from oracle import oracle
from paper_1903_07145_amd import ipt, scenes

pytestmark = pytest.mark.gpu

PIX_REL = 1e-4
GRAD_REL = 1e-3


def _oracle(sc):
    return oracle.Scene(sc["verts"], sc["tris"], sc["tri_seg"], sc["num_segments"], sc["emitter_seg"],
                        sc["normals"])


def _parity(sc, g, o, kw, pix=None, min_keep=0.9):
    dc = ipt.make_cameras(sc["cams"])
    p = sc["params"]
    _, h_g = gpu_render(g, dc, p, kw, pixel_list=pix)
    r = o.run(sc["cams"], p, pixel_list=pix, want_hash=True, want_margin=True, want_cond=True, **oracle_opts(kw))
    b = check_mismatches(h_g, r, 3, label="global params")
    n_mis, n_hard = b["mismatch"], b["hard"]
    keep = comparable(h_g, r)
    print("paths %d mismatching %d (hard %d), compared %.1f%%" % (h_g.size, n_mis, n_hard, 100 * keep.mean()))
    assert n_hard <= 1e-5 * 3 * h_g.size
    assert keep.mean() > min_keep
    img_g, _ = gpu_render(g, dc, p, kw, pixel_list=pix, mask=keep)
    ro = o.run(sc["cams"], p, pixel_list=pix, path_mask=keep.astype(np.uint8), **oracle_opts(kw))
    mean = np.abs(ro["image"]).mean()
    err = np.abs(img_g - ro["image"]) / np.maximum(np.abs(ro["image"]), 1e-4 * mean)
    print("pixel rel err max %.2e" % err.max())
    assert err.max() <= PIX_REL
    wimg = np.random.default_rng(4).normal(size=(img_g.shape[0], 3))
    gcond = o.run(sc["cams"], p, pixel_list=pix, w=wimg, want_cond=True, **oracle_opts(kw))["gcond"]
    keep_g = keep & (gcond <= GRAD_ILL_COND)
    gg = gpu_grad(g, dc, p, wimg, kw, pixel_list=pix, mask=keep_g)
    go = o.run(sc["cams"], p, pixel_list=pix, w=wimg, path_mask=keep_g.astype(np.uint8), want_grad=True,
               **oracle_opts(kw))["grad"]
    # with one material per triangle most parameters are reached by none of
    # the compared paths: those must be exactly zero on both sides, and the
    # scale of the relative bar (rms) is taken over the parameters reached,
    # not diluted by the structural zeros
    touched = go != 0
    assert np.all(gg[~touched] == 0.0)
    rms = math.sqrt(np.mean(go[touched] ** 2))
    gerr = np.abs(gg - go) / np.maximum(np.abs(go), 1e-2 * rms)
    worst = int(np.argmax(gerr))
    print("grad rel err max %.2e over %d parameters (%d reached; worst %d, entry %d of its block)" % (
        gerr.max(), go.size, int(touched.sum()), worst, worst % 7 if worst < 7 * sc["num_segments"] else -1))
    assert gerr.max() <= GRAD_REL
    return gg, go


def test_lds_and_global_storage_agree():
    banner("per-triangle Cornell: LDS vs global parameter storage")
    sc = scenes.per_triangle(scenes.cornell())
    ga = ipt.Scene.from_dict(sc)
    gb = ipt.Scene.from_dict(sc, param_storage=ipt.PARAMS_GLOBAL)
    assert ga.info()["params_global"] == 0 and gb.info()["params_global"] == 1
    dc = ipt.make_cameras(sc["cams"])
    kw = dict(seed=3, stream_tag=1, iteration=1, spp=8, max_depth=3, mis=2)
    ia, ha = gpu_render(ga, dc, sc["params"], kw)
    ib, hb = gpu_render(gb, dc, sc["params"], kw)
    assert np.array_equal(ha, hb)
    # two separately compiled kernels: the same arithmetic up to instruction
    # selection (contraction), so equal to float32 rounding, well inside the
    # 1e-4 oracle bar
    rel = np.abs(ia - ib) / np.maximum(np.abs(ia), 1e-4 * np.abs(ia).mean())
    print("image max rel diff %.2e" % rel.max())
    assert rel.max() <= 1e-5
    w = np.random.default_rng(1).normal(size=(64 * 64, 3))
    gk = dict(kw, stream_tag=2)
    a = gpu_grad(ga, dc, sc["params"], w, gk)
    b = gpu_grad(gb, dc, sc["params"], w, gk)
    rms = math.sqrt(np.mean(a ** 2))
    print("grad max diff %.2e (rms %.2e)" % (np.abs(a - b).max(), rms))
    assert np.abs(a - b).max() <= 1e-5 * rms


def test_global_storage_parity_cornell():
    banner("per-triangle Cornell, global storage, vs oracle")
    sc = scenes.per_triangle(scenes.cornell())
    g = ipt.Scene.from_dict(sc, param_storage=ipt.PARAMS_GLOBAL)
    _parity(sc, g, _oracle(sc), dict(seed=7, stream_tag=1, iteration=2, spp=4, max_depth=3, mis=2))


def test_global_storage_parity_textured():
    banner("textured Cornell ground truth: 1179 segments, 8256 parameters (global by size)")
    tc = scenes.textured_cornell()
    sc = scenes.per_triangle(tc, tri_params=tc["tri_params"])
    g = ipt.Scene.from_dict(sc)
    assert g.info()["params_global"] == 1
    pix = np.sort(np.random.default_rng(2).choice(128 * 128, size=1500, replace=False)).astype(np.int64)
    gg, go = _parity(sc, g, _oracle(sc), dict(seed=9, stream_tag=1, iteration=1, spp=8, max_depth=3, mis=2), pix=pix)
    assert (go != 0).sum() > 300


def test_global_storage_parity_room_per_triangle():
    banner("per-triangle room: ~49k segments, ~345k parameters")
    sc = scenes.per_triangle(scenes.room())
    g = ipt.Scene.from_dict(sc)
    assert g.info()["params_global"] == 1
    W, H = sc["cams"]["width"], sc["cams"]["height"]
    pix = np.sort(np.random.default_rng(3).choice(4 * W * H, size=400, replace=False)).astype(np.int64)
    _parity(sc, g, _oracle(sc), dict(seed=11, stream_tag=1, iteration=1, spp=4, max_depth=3, mis=2), pix=pix,
            min_keep=0.85)


def test_global_storage_with_cached_proposal():
    """The cached proposal on a scene whose parameters are in global memory
    (the kernels of proposal kind 3 with global storage): images and
    gradients against the oracle's guided estimator, and the guide's
    training records written by the gradient pass."""
    banner("per-triangle Cornell (global storage) with the cached proposal")
    import _guide
    sc = scenes.per_triangle(scenes.cornell())
    g = ipt.Scene.from_dict(sc, param_storage=ipt.PARAMS_GLOBAL)
    o = _oracle(sc)
    w = _guide.random_weights(sc["num_segments"], seed=31, out_gain=3.0, kappa_bias=1.0)
    gd = ipt.Guide(g, record_stride=1)
    gd.set_weights(w)
    cell_area = 2e-3
    gd.cache_build(cell_area, mode=1)
    lo, inv = _guide.box(sc["verts"])
    kw = dict(seed=17, stream_tag=1, iteration=3, spp=4, max_depth=3, mis=2, guide=gd, guide_mix=0.5, guide_cached=1)
    okw = dict(guide_w=w, guide_mix=0.5, bb_lo=lo, bb_inv=inv, guide_cell_area=cell_area)
    dc = ipt.make_cameras(sc["cams"])
    p = sc["params"]
    _, h_g = gpu_render(g, dc, p, kw)
    r = o.run(sc["cams"], p, want_hash=True, want_margin=True, want_cond=True, **oracle_opts(kw), **okw)
    b = check_mismatches(h_g, r, 3, label="global params")
    n_mis, n_hard = b["mismatch"], b["hard"]
    keep = comparable(h_g, r)
    print("paths %d mismatching %d (hard %d), compared %.1f%%" % (h_g.size, n_mis, n_hard, 100 * keep.mean()))
    assert n_hard <= 1e-5 * 3 * h_g.size and keep.mean() > 0.9
    img_g, _ = gpu_render(g, dc, p, kw, mask=keep)
    ro = o.run(sc["cams"], p, path_mask=keep.astype(np.uint8), **oracle_opts(kw), **okw)
    err = np.abs(img_g - ro["image"]) / np.maximum(np.abs(ro["image"]), 1e-4 * np.abs(ro["image"]).mean())
    print("pixel rel err max %.2e" % err.max())
    assert err.max() <= PIX_REL
    wimg = np.random.default_rng(6).normal(size=(64 * 64, 3))
    n0 = gd.records()
    gg = gpu_grad(g, dc, p, wimg, kw, mask=keep)
    go = o.run(sc["cams"], p, w=wimg, path_mask=keep.astype(np.uint8), want_grad=True, **oracle_opts(kw), **okw)["grad"]
    touched = go != 0
    rms = math.sqrt(np.mean(go[touched] ** 2))
    gerr = np.abs(gg - go) / np.maximum(np.abs(go), 1e-2 * rms)
    print("grad rel err max %.2e; training records written %d" % (gerr.max(), gd.records() - n0))
    assert gerr.max() <= GRAD_REL
    assert gd.records() - n0 > 1000
