"""Host-side scene tools (no GPU): the per-triangle re-parameterisation of the
coarse-to-fine refinement (App. A) and the textured Cornell box."""
import numpy as np

from paper_1903_07145_amd import scenes


def test_per_triangle_keeps_every_material_and_emission():
    sc = scenes.cornell()
    pt = scenes.per_triangle(sc)
    S, S2 = sc["num_segments"], pt["num_segments"]
    T = sc["tris"].shape[0]
    emit = set(int(x) for x in sc["emitter_seg"])
    n_emit_tris = sum(int(sc["tri_seg"][t]) in emit for t in range(T))
    assert S2 == (T - n_emit_tris) + len(emit)
    assert pt["params"].size == 7 * S2 + 3 * len(sc["emitter_seg"])
    for t in range(T):
        a = pt["params"][7 * pt["tri_seg"][t]:7 * pt["tri_seg"][t] + 7]
        b = sc["params"][7 * sc["tri_seg"][t]:7 * sc["tri_seg"][t] + 7]
        assert np.array_equal(a, b)
        assert pt["parent"][pt["tri_seg"][t]] == sc["tri_seg"][t]
    assert np.array_equal(pt["params"][7 * S2:], sc["params"][7 * S:])
    # emitter segments stay whole, one per emitter, in the same order
    for k, s in enumerate(sc["emitter_seg"]):
        tris = np.nonzero(sc["tri_seg"] == s)[0]
        assert len(set(pt["tri_seg"][tris].tolist())) == 1
        assert pt["parent"][pt["emitter_seg"][k]] == s


def test_per_triangle_subset_and_given_materials():
    sc = scenes.cornell()
    pick = np.array([0, 1, 5])
    tp = np.random.default_rng(0).uniform(0, 1, (sc["tris"].shape[0], 7)).astype(np.float32)
    pt = scenes.per_triangle(sc, tris=pick, tri_params=tp)
    segs = pt["tri_seg"]
    assert len(set(segs[pick].tolist())) == 3
    for t in pick:
        assert np.array_equal(pt["params"][7 * segs[t]:7 * segs[t] + 7], tp[t])
    rest = np.setdiff1d(np.arange(sc["tris"].shape[0]), pick)
    for t in rest:
        assert np.array_equal(pt["params"][7 * segs[t]:7 * segs[t] + 7],
                              sc["params"][7 * sc["tri_seg"][t]:7 * sc["tri_seg"][t] + 7])


def test_textured_cornell_object_means():
    tc = scenes.textured_cornell()
    for s in range(tc["num_segments"] - 1):
        m = tc["tri_seg"] == s
        assert np.allclose(tc["params"][7 * s:7 * s + 3], tc["tri_params"][m, :3].mean(axis=0), atol=1e-6)
    # textured walls vary, boxes and the ceiling are constant
    for s in (0, 2, 3, 4):
        assert tc["tri_params"][tc["tri_seg"] == s, :3].std(axis=0).min() > 0.02
    for s in (1, 5, 6):
        assert tc["tri_params"][tc["tri_seg"] == s, :3].std(axis=0).max() < 1e-6
