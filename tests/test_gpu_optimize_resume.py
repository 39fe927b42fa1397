"""A split optimisation run (state saved after part of the iterations,
then resumed in a fresh call) reproduces the uninterrupted run on the BRDF
arm (to float32 rounding of the gradient's summation order): parameters,
Adam moments, the iteration count driving the cosine schedule and the Philox
streams all carry over.  With the learned proposal the run continues from
the saved weights and training records."""
import numpy as np
import pytest
import torch

from paper_1903_07145_amd import ipt, optimize, scenes

pytestmark = pytest.mark.gpu


def _setup():
    sc = scenes.cornell()
    g = ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    target = optimize.render_target(g, dc, torch.as_tensor(sc["params"], device="cuda"), 64, 3, -1)
    cov = optimize.coverage(g, sc)
    return sc, g, target, optimize.identifiable_masks(sc, cov), optimize.unrecoverable_mask(sc, cov)


def test_split_run_equals_uninterrupted(tmp_path):
    sc, g, target, masks, fixed = _setup()
    kw = dict(iters=40, seed=3, target=target, g=g, masks=masks, fixed=fixed, lr_schedule="cos", beta2=0.9)
    full = optimize.optimize(sc, **kw)
    p_full = optimize.optimize.last["params"].cpu().numpy()
    a = optimize.optimize(sc, stop_after=15, want_state=True, **kw)
    assert not a["done"] and a["iters"] == 15
    path = str(tmp_path / "st")
    optimize.save_state(path, a["state"])
    st = optimize.load_state(path)
    b = optimize.optimize(sc, state=st, want_state=True, **kw)
    assert b["done"] and b["iters"] == 40
    p_split = optimize.optimize.last["params"].cpu().numpy()
    assert np.allclose(p_full, p_split, rtol=1e-5, atol=1e-7)
    assert np.allclose(full["history"]["rmse_all"], b["history"]["rmse_all"], rtol=1e-5)
    assert np.allclose(full["history"]["loss"], b["history"]["loss"], rtol=1e-4)


def test_split_guided_run_resumes_guide():
    sc, g, target, masks, fixed = _setup()
    kw = dict(iters=30, seed=4, target=target, g=g, masks=masks, fixed=fixed, guide=True, warmup=5,
              guide_batch=1024, lr_schedule="cos", beta2=0.9)
    a = optimize.optimize(sc, stop_after=12, want_state=True, **kw)
    w = a["state"]["guide_w"]
    assert a["state"]["guide_rec"].shape[1] == 16 and len(a["state"]["guide_rec"]) > 0
    b = optimize.optimize(sc, state=a["state"], **kw)
    assert b["done"] and b["iters"] == 30
    # the resumed guide started from the saved weights and kept training
    w2 = optimize.optimize.last["guide"].get_weights()
    assert np.isfinite(w2).all() and not np.array_equal(w, w2)
    assert np.isfinite(b["final_rmse_all"])
