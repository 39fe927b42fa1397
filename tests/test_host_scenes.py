"""Host-side scene tools (no GPU): the per-triangle re-parameterisation of the
coarse-to-fine refinement (App. E) and the textured Cornell box."""
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


def test_cell_area_for_matches_surface_area():
    import torch  # noqa: F401  (optimize imports torch)
    from paper_1903_07145_amd import optimize
    sc = scenes.cornell()
    # unit room: floor, ceiling and three walls (5 m^2), two boxes and the emitter quad
    v = sc["verts"].astype(np.float64)
    t = sc["tris"].astype(np.int64)
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1).sum()
    boxes = 2 * (0.3 * 0.6 + 0.3 * 0.3 + 0.6 * 0.3) + 2 * (3 * 0.3 * 0.3)
    assert abs(area - (5.0 + boxes + 0.0625)) < 1e-5
    assert abs(optimize.cell_area_for(sc, 1000) - area / 1000) < 1e-6 * area


def test_texture_rmse_and_triangle_errors():
    import torch
    from paper_1903_07145_amd import optimize
    tc = scenes.textured_cornell()
    T = tc["tris"].shape[0]
    tri_kd = tc["tri_params"][:, :3].astype(np.float64)
    cnt = np.ones(T)
    # per-object parameters (object means): the RMSE is the texture's spread
    r = optimize.texture_rmse(tc, tc["params"], tri_kd, cnt)
    seg = tc["tri_seg"]
    kd = tc["params"][7 * seg[:, None] + np.arange(3)[None, :]]
    assert abs(r - np.sqrt(np.mean((kd - tri_kd) ** 2))) < 1e-9 and r > 0.05
    # the ground truth has none
    gt = scenes.per_triangle(tc, tri_params=tc["tri_params"])
    assert optimize.texture_rmse(gt, gt["params"], tri_kd, cnt) < 1e-6
    # triangle errors: mean over the pixels each triangle covers
    img = torch.zeros((6, 3))
    tgt = torch.tensor([[1.0, 1, 1], [2, 2, 2], [0, 0, 0], [3, 3, 3], [0, 0, 0], [0, 0, 0]])
    pix_tri = np.array([0, 0, 1, 2, -1, 1])
    err, c = optimize.triangle_errors(img, tgt, pix_tri, 4)
    assert np.allclose(c, [2, 2, 1, 0])
    assert np.allclose(err, [(1 + 4) / 2, 0.0, 9.0, 0.0])


def test_refined_scene_inherits_current_values():
    from paper_1903_07145_amd import optimize
    sc = scenes.cornell()
    T = sc["tris"].shape[0]
    vals = np.random.default_rng(3).uniform(0, 1, (T, 7)).astype(np.float32)
    # unrefined triangles of an object share its value
    for s in range(sc["num_segments"]):
        m = sc["tri_seg"] == s
        vals[m] = vals[np.nonzero(m)[0][0]]
    refined = np.array([0, 3, 12])
    vals[refined] = np.random.default_rng(4).uniform(0, 1, (3, 7))
    em = np.array([1.0, 2.0, 3.0], np.float32)
    ns = optimize._refined_scene(sc, refined, vals, em)
    for t in range(T):
        assert np.array_equal(ns["params"][7 * ns["tri_seg"][t]:7 * ns["tri_seg"][t] + 7], vals[t])
    assert np.array_equal(ns["params"][-3:], em)
    assert len(set(ns["tri_seg"][refined].tolist())) == 3


def test_paper_setting_masks():
    from paper_1903_07145_amd import optimize
    sc = scenes.all_emissive(scenes.cornell())
    S = sc["num_segments"]
    cov = np.full(S, 500)
    cov[6] = 50            # a box seen in too few pixels: held fixed
    fixed, head = optimize.paper_setting_masks(sc, cov)
    e0 = int(sc["true_emitters"][0])
    assert fixed[7 * 6:7 * 6 + 7].all() and fixed[7 * S + 18:7 * S + 21].all()
    assert fixed[7 * e0:7 * e0 + 7].all() and not fixed[7 * S + 3 * e0]
    assert head[0:3].all() and not head[3:7].any()          # albedo only (ks, roughness not trainable)
    assert head[7 * S:7 * S + 3].all()                       # every seen segment's emission
    sigma = np.zeros(sc["params"].size)
    sigma[1] = 1.0
    _, head2 = optimize.paper_setting_masks(sc, cov, sigma=sigma)
    assert not head2[1] and head2[0]


def test_subdivide_shares_midpoints_and_keeps_area():
    sc = scenes.cornell()
    T = sc["tris"].shape[0]
    pick = np.array([0, 1])          # the two triangles of the floor quad share an edge
    sd = scenes.subdivide(sc, pick)
    assert sd["tris"].shape[0] == T + 3 * pick.size
    # 3 midpoints each, the shared edge's once: 5 new vertices
    assert sd["verts"].shape[0] == sc["verts"].shape[0] + 5
    assert np.array_equal(np.bincount(sd["parent_tri"], minlength=T), np.where(np.isin(np.arange(T), pick), 4, 1))
    # children keep the parent's segment; every child lies in its parent's plane, areas add up
    v = sd["verts"].astype(np.float64)
    f = sd["tris"].astype(np.int64)
    area = 0.5 * np.linalg.norm(np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]), axis=1)
    v0 = sc["verts"].astype(np.float64)
    f0 = sc["tris"].astype(np.int64)
    area0 = 0.5 * np.linalg.norm(np.cross(v0[f0[:, 1]] - v0[f0[:, 0]], v0[f0[:, 2]] - v0[f0[:, 0]]), axis=1)
    for t in pick:
        ch = np.nonzero(sd["parent_tri"] == t)[0]
        assert np.all(sd["tri_seg"][ch] == sc["tri_seg"][t])
        assert np.allclose(area[ch], area0[t] / 4)
        n0 = np.cross(v0[f0[t, 1]] - v0[f0[t, 0]], v0[f0[t, 2]] - v0[f0[t, 0]])
        for c in ch:
            n = np.cross(v[f[c, 1]] - v[f[c, 0]], v[f[c, 2]] - v[f[c, 0]])
            assert np.dot(n, n0) > 0 and np.linalg.norm(np.cross(n, n0)) < 1e-9 * np.linalg.norm(n0) ** 2
    assert abs(area.sum() - area0.sum()) < 1e-9


def test_workload_recipes():
    """The synthetic workloads have the sizes the benchmarks are quoted on:
    apartment (about 500k triangles, 128 segments, 8 emitters, 16 views of
    640x480, 8 spp, depth 7, roulette from depth 3) and office floor (about
    2M triangles, 256 segments, 16 emitters, 30 views, 64 spp, depth 8); the
    parameter vector is 7 S + 3 E with the emission after the materials."""
    for make, tri, S, E, V, spp, D in ((scenes.apartment, 500000, 128, 8, 16, 8, 7),
                                       (scenes.office_floor, 2000000, 256, 16, 30, 64, 8)):
        sc = make()
        nt = sc["tris"].shape[0]
        assert abs(nt - tri) <= 0.01 * tri, nt
        assert sc["num_segments"] == S and len(sc["emitter_seg"]) == E
        assert np.asarray(sc["cams"]["cam_to_world"]).reshape(-1, 4, 4).shape[0] == V
        assert (sc["cams"]["width"], sc["cams"]["height"]) == (640, 480)
        r = sc["render"]
        assert (r["spp"], r["max_depth"], r["rr_depth"]) == (spp, D, 3)
        assert sc["params"].size == 7 * S + 3 * E
        assert sc["tri_seg"].min() >= 0 and sc["tri_seg"].max() < S
        assert np.isfinite(sc["verts"]).all() and sc["tris"].min() >= 0 and sc["tris"].max() < len(sc["verts"])
        for k in ("scale", "lo", "hi", "trainable"):
            assert sc[k].size == sc["params"].size, k
        # bounds are on the normalised parameters (value / scale)
        u = sc["params"] / sc["scale"]
        assert ((u >= sc["lo"] - 1e-6) & (u <= sc["hi"] + 1e-6)).all()


def test_disney_recipe():
    """The Disney variant: 13 parameters per segment, the base colour taken
    from the diffuse albedo, every material parameter in [0, 1] with its
    stated distribution's range, emission unchanged after the materials."""
    base = scenes.room()
    sc = scenes.disney(base, seed=6)
    S, E = sc["num_segments"], len(sc["emitter_seg"])
    assert sc["material"] == 1 and sc["params"].size == 13 * S + 3 * E
    d = sc["params"][:13 * S].reshape(S, 13)
    p7 = base["params"][:7 * S].reshape(S, 7)
    assert np.array_equal(d[:, 0:3], p7[:, 0:3])
    assert np.array_equal(sc["params"][13 * S:], base["params"][7 * S:])
    assert ((d >= 0) & (d <= 1)).all()
    assert ((d[:, 7] >= 0.25) & (d[:, 7] <= 0.9)).all()        # roughness
    assert (d[:, 8] <= 0.8).all() and (d[:, 12] <= 0.7).all()  # anisotropic, clearcoat gloss
    assert ((d[:, 4] == 0) | (d[:, 4] >= 0.2)).all()            # metallic: 0 or U(0.2, 1)
    assert (d[:, 4] == 0).any() and (d[:, 4] > 0).any() and (d[:, 11] == 0).any() and (d[:, 11] > 0).any()
    assert (sc["trainable"][:13 * S] == 1).all() and (sc["scale"][:13 * S] == 1).all()
