"""The paper's own optimisation setting on the HIP path, against the FP64
oracle: every segment emissive (App. E: an unknown emission per object, most
of it zero, light selection proportional to the current emission), small
pixel batches with many paths per pixel, the L1 loss with its sign adjoint
(Sec. 3.2, Eq. 3; Sec. 3.3, Eq. 4) and the L1 emission regulariser
(Sec. 4.4, "Regularization")."""
import math

import numpy as np
import pytest
import torch

from _gpu import (check_mismatches, GRAD_ILL_COND, banner, both, comparable, dev, gpu_grad, gpu_render, image_parity,
                  mismatch_stats, oracle_opts)
from paper_1903_07145_amd import ipt, scenes

pytestmark = pytest.mark.gpu

PIX_REL = 1e-4
GRAD_REL = 1e-3


def _grad_err(gg, go):
    rms = math.sqrt(np.mean(go ** 2)) + 1e-30
    err = np.abs(gg - go) / np.maximum(np.abs(go), 1e-2 * rms)
    return err.max(), int(np.argmax(err))


def test_all_emissive_cornell_batch_parity():
    """8 pixels drawn from the image, 256 paths each: image and gradient
    parity with every one of the 36 triangles a light (light table in LDS)."""
    banner("all-emissive cornell, 8-pixel batch x 256 spp")
    sc = scenes.all_emissive(scenes.cornell())
    g, o = both(sc)
    dc = ipt.make_cameras(sc["cams"])
    assert g.info()["num_light_triangles"] == 36
    p = sc["params"].copy()
    p[7 * 8 + 3 * 2:7 * 8 + 3 * 2 + 3] = [0.3, 0.1, 0.0]   # a small emission on the back wall
    pix = np.sort(np.random.default_rng(0).choice(64 * 64, size=8, replace=False)).astype(np.int64)
    kw = dict(seed=5, stream_tag=2, iteration=3, spp=256, max_depth=3, mis=2)
    img_g, h_g = gpu_render(g, dc, p, kw, pixel_list=pix)
    r = o.run(sc["cams"], p, pixel_list=pix, want_hash=True, want_margin=True, **oracle_opts(kw))
    ok, mfrac, emax, _ = image_parity(img_g, r["image"], h_g, r["hash"])
    print("path mismatch %.2e, pixel rel err %.2e" % (mfrac, emax))
    assert emax <= PIX_REL
    mask = (h_g == r["hash"]).astype(np.uint8)
    w = np.random.default_rng(1).normal(size=(pix.size, 3))
    gg = gpu_grad(g, dc, p, w, kw, pixel_list=pix, mask=mask)
    go = o.run(sc["cams"], p, pixel_list=pix, w=w, path_mask=mask, want_grad=True, **oracle_opts(kw))["grad"]
    emax, arg = _grad_err(gg, go)
    print("grad rel err %.2e (param %d)" % (emax, arg))
    assert emax <= GRAD_REL
    # the back wall's emission derivative is live
    assert abs(gg[7 * 8 + 3 * 2]) > 0


def test_all_emissive_room_global_light_table():
    """Room with all 32 segments emissive: ~49k light triangles, so the light
    table and its CDF are read from global memory instead of LDS."""
    banner("all-emissive room: light table in global memory")
    sc = scenes.all_emissive(scenes.room())
    g, o = both(sc)
    assert g.info()["num_light_triangles"] > 1024
    dc = ipt.make_cameras(sc["cams"])
    W, H = sc["cams"]["width"], sc["cams"]["height"]
    p = sc["params"].copy()
    S = sc["num_segments"]
    p[7 * S + 3 * 3:7 * S + 3 * 3 + 3] = [0.5, 0.4, 0.2]   # a dim emission on a room surface
    rng = np.random.default_rng(2)
    pix = np.sort(rng.choice(4 * W * H, size=400, replace=False)).astype(np.int64)
    kw = dict(seed=8, stream_tag=2, iteration=1, spp=8, max_depth=3, mis=2)
    img_g, h_g = gpu_render(g, dc, p, kw, pixel_list=pix)
    r = o.run(sc["cams"], p, pixel_list=pix, want_hash=True, want_margin=True, want_cond=True, **oracle_opts(kw))
    # ~49k light triangles: the light pick compares u against a table of
    # float32 prefix sums whose neighbouring entries lie ~2e-5 of the total
    # apart, so about every path meets a pick near a boundary and a few
    # percent take the neighbouring light (near-ties, bounded here at 3%)
    b = check_mismatches(h_g, r, 3, label="paper setting", near_tie_bar=0.03)
    n_mis, n_hard = b["mismatch"], b["hard"]
    keep = comparable(h_g, r)
    print("paths %d mismatching %d (hard %d), compared %.1f%%" % (h_g.size, n_mis, n_hard, 100 * keep.mean()))
    assert n_hard <= 1e-5 * 3 * h_g.size
    # with ~49k light triangles most of them dim, a light choice often falls
    # within the 1e-5 near-tie margin of a CDF boundary (light probabilities
    # are ~1e-5), so fewer paths are compared than in the 8-light room
    assert keep.mean() > 0.6
    img_g, _ = gpu_render(g, dc, p, kw, pixel_list=pix, mask=keep)
    ro = o.run(sc["cams"], p, pixel_list=pix, path_mask=keep.astype(np.uint8), **oracle_opts(kw))
    mean = np.abs(ro["image"]).mean()
    err = np.abs(img_g - ro["image"]) / np.maximum(np.abs(ro["image"]), 1e-4 * mean)
    print("pixel rel err max %.2e" % err.max())
    assert err.max() <= PIX_REL
    w = rng.normal(size=(pix.size, 3))
    gcond = o.run(sc["cams"], p, pixel_list=pix, w=w, want_cond=True, **oracle_opts(kw))["gcond"]
    keep_g = keep & (gcond <= GRAD_ILL_COND)
    gg = gpu_grad(g, dc, p, w, kw, pixel_list=pix, mask=keep_g)
    go = o.run(sc["cams"], p, pixel_list=pix, w=w, path_mask=keep_g.astype(np.uint8), want_grad=True,
               **oracle_opts(kw))["grad"]
    emax, arg = _grad_err(gg, go)
    print("grad rel err %.2e (param %d), compared %.1f%%" % (emax, arg, 100 * keep_g.mean()))
    assert emax <= GRAD_REL


def test_l1_loss_batch_and_regulariser():
    """ipt_loss_grad with the L1 loss on a pixel batch, plus ipt_l1_reg, against
    the oracle's loss, sign adjoint and gradient on the same paths."""
    banner("L1 loss + L1 emission regulariser on an 8-pixel batch")
    from oracle import oracle as orc_mod
    sc = scenes.all_emissive(scenes.cornell())
    g, o = both(sc)
    dc = ipt.make_cameras(sc["cams"])
    pix = np.sort(np.random.default_rng(3).choice(64 * 64, size=8, replace=False)).astype(np.int64)
    target = o.run(sc["cams"], sc["params"], pixel_list=pix, spp=1024, max_depth=3, stream_tag=0, seed=1)["image"]
    p0 = np.zeros_like(sc["params"])
    p0[:56] = 0.3
    p0[56:] = 0.05 * sc["scale"][56:]
    co = dict(seed=9, stream_tag=1, iteration=2, spp=256, max_depth=3, mis=2)
    go_ = dict(co, stream_tag=2)
    _, h_b = gpu_render(g, dc, p0, go_, pixel_list=pix)
    rb = o.run(sc["cams"], p0, pixel_list=pix, want_hash=True, **oracle_opts(go_))
    mask = (h_b == rb["hash"]).astype(np.uint8)
    pl = dev(pix, torch.int64)
    imgA = torch.empty((pix.size, 3), dtype=torch.float32, device="cuda")
    loss, grad = g.loss_grad(dc, dev(p0), dev(target), ipt.render_opts(pixel_list=pl, **co),
                             ipt.render_opts(pixel_list=pl, path_mask=dev(mask.reshape(-1), torch.uint8), **go_),
                             1, image=imgA)
    # L1 on the emission entries
    lam = np.zeros_like(p0)
    lam[56:] = 1e-3
    ipt.l1_reg(dev(p0), grad, dev(lam), loss)
    torch.cuda.synchronize()
    img_gpu = imgA.cpu().numpy().astype(np.float64)
    E, w = orc_mod.loss_adjoint(img_gpu, target, 1)
    E_reg = E + float(np.sum(lam * np.abs(p0)))
    assert abs(loss.item() - E_reg) <= 1e-5 * E_reg
    go = o.run(sc["cams"], p0, pixel_list=pix, w=w, path_mask=mask, want_grad=True, **oracle_opts(go_))["grad"]
    go = go + lam * np.sign(p0)
    emax, arg = _grad_err(grad.cpu().numpy().astype(np.float64), go)
    print("loss %.6f (oracle %.6f), grad rel err %.2e (param %d)" % (loss.item(), E_reg, emax, arg))
    assert emax <= GRAD_REL
