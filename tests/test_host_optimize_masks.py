"""Host logic of the optimisation driver, without a GPU: which parameters the
images determine (the RMSE subsets), which ones no view can recover (held at
their true values), and the per-group RMSE, for both material models.

A four-segment scene: segment 0 and 1 seen in 200 and 150 pixels, segment 2
an emitter seen in 500, segment 3 seen in 10 (below the 100-pixel floor);
segment 1's specular reflectance is below the roughness floor."""
import numpy as np
import pytest
import torch

from paper_1903_07145_amd import optimize

S = 4
COV = np.array([200, 150, 500, 10])


def _scene(material):
    nm = 13 if material == 1 else 7
    rng = np.random.default_rng(3)
    p = rng.uniform(0.2, 0.8, nm * S + 3).astype(np.float32)
    if nm == 7:
        p[7 * 1 + 3:7 * 1 + 6] = 0.01          # segment 1: specular below 0.05
    return dict(num_segments=S, emitter_seg=np.array([2], np.int32), params=p,
                trainable=np.ones(p.size, np.uint8), material=material), nm


def _idx(mask):
    return set(np.flatnonzero(mask).tolist())


@pytest.mark.parametrize("material", [0, 1])
def test_identifiable_and_unrecoverable_sets(material):
    sc, nm = _scene(material)
    assert optimize.params_per_segment(sc) == nm
    kd_e, all_id = optimize.identifiable_masks(sc, COV)
    fixed = optimize.unrecoverable_mask(sc, COV)
    E0 = nm * S                                  # the emitter's emission
    assert _idx(kd_e) == {0, 1, 2, nm, nm + 1, nm + 2, E0, E0 + 1, E0 + 2}
    if nm == 7:
        # diffuse and specular of the seen segments, roughness only where
        # the specular reflectance is large enough
        want = set(range(0, 7)) | set(range(7, 13)) | {E0, E0 + 1, E0 + 2}
    else:
        want = set(range(0, 2 * nm)) | {E0, E0 + 1, E0 + 2}
    assert _idx(all_id) == want
    # the emitting segment's reflectance and the barely seen segment are held
    assert _idx(fixed) == set(range(2 * nm, 4 * nm))
    assert not (fixed & all_id).any()
    # a barely seen emitter: its emission is held too
    cov2 = COV.copy()
    cov2[2] = 5
    assert _idx(optimize.unrecoverable_mask(sc, cov2)) == set(range(2 * nm, 4 * nm)) | {E0, E0 + 1, E0 + 2}
    # precision gate: a parameter the target cannot pin leaves both subsets
    sigma = np.zeros(sc["params"].size)
    sigma[1] = 1.0
    kd2, all2 = optimize.identifiable_masks(sc, COV, sigma=sigma)
    assert _idx(kd2) == _idx(kd_e) - {1} and _idx(all2) == _idx(all_id) - {1}
    # untrainable parameters are never in a subset
    sc3 = dict(sc, trainable=sc["trainable"].copy())
    sc3["trainable"][0] = 0
    kd3, all3 = optimize.identifiable_masks(sc3, COV)
    assert 0 not in _idx(kd3) and 0 not in _idx(all3)


@pytest.mark.parametrize("material", [0, 1])
def test_group_rmse(material):
    sc, nm = _scene(material)
    P = sc["params"].size
    p_true = torch.as_tensor(sc["params"])
    scale = torch.full((P,), 2.0)
    off = torch.zeros(P)
    idx = np.arange(P)
    if nm == 7:
        offs = dict(kd=0.1, ks=0.2, alpha=0.4, e=0.8)
        masks = dict(kd=(idx < 7 * S) & (idx % 7 < 3), ks=(idx < 7 * S) & (idx % 7 >= 3) & (idx % 7 < 6),
                     alpha=(idx < 7 * S) & (idx % 7 == 6), e=idx >= 7 * S)
    else:
        offs = dict(base=0.1, other=0.3, e=0.8)
        masks = dict(base=(idx < nm * S) & (idx % nm < 3), other=(idx < nm * S) & (idx % nm >= 3), e=idx >= nm * S)
    for k, m in masks.items():
        off[torch.as_tensor(m)] = offs[k]
    g = optimize.group_rmse(p_true + off, p_true, scale, torch.ones(P, dtype=torch.uint8), S, nm=nm)
    assert set(g) == set(offs)
    for k, v in offs.items():
        assert g[k] == pytest.approx(v / 2.0, rel=1e-6), k
    # the all-parameter RMSE is the root of the size-weighted group means
    total = optimize.param_rmse(p_true + off, p_true, scale, torch.ones(P, dtype=torch.uint8))
    want = np.sqrt(sum(masks[k].sum() * (offs[k] / 2.0) ** 2 for k in offs) / P)
    assert total == pytest.approx(want, rel=1e-6)
