"""Host logic of the four-child BVH, without a GPU: the host builder (the same
split rule as the GPU builder), the greedy collapse into four-child nodes and
the quantization of the child boxes, built with g++ from the library's own
sources through a small C harness (tests/bvh_wide_harness.cpp).

Checked on random triangle soups, a soup of coincident centroids, the
Cornell box and the 50k-triangle room:
* the four-child tree covers every triangle exactly once, in leaves of at
  most two triangles, each node reached once, inner children stored
  contiguously;
* the greedy collapse fills a node to four children unless all its children
  are leaves;
* every child box contains every triangle of its subtree;
* every quantized child box (origin + q 2^e, decoded exactly) contains the
  float child box widened by 2^-20 of the node's largest extent; empty slots
  hold an inside-out box (q lo 255, q hi 0) and the reference ~0;
* the reported number of node levels is the tree's depth;
* the node visit's float32 slab test, emulated, admits every ancestor box of
  a hit (a build without the margin fails it)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1903_07145_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1903_07145_amd", "csrc")
NONE = 0x7FFFFFFF
LEAF_MAX = 2


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("bvhh") / "libbvhh.so")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                           os.path.join(HERE, "bvh_wide_harness.cpp"), os.path.join(CSRC, "bvh_host.cpp"),
                           os.path.join(CSRC, "bvh_wide.cpp"), "-o", out])
    lib = ctypes.CDLL(out)
    lib.harness_build.restype = ctypes.c_longlong
    return lib


def _build(lib, verts, tris, quantize):
    v = np.ascontiguousarray(verts, np.float32)
    t = np.ascontiguousarray(tris, np.int32)
    lv, bd = ctypes.c_int(), ctypes.c_int()
    n = lib.harness_build(v.ctypes.data_as(ctypes.c_void_p), t.ctypes.data_as(ctypes.c_void_p), t.shape[0],
                          quantize, ctypes.byref(lv), ctypes.byref(bd))
    assert n > 0
    nodes = np.zeros((n, 16 if quantize else 32), np.float32)
    order = np.zeros(t.shape[0], np.int32)
    lib.harness_copy(nodes.ctypes.data_as(ctypes.c_void_p), order.ctypes.data_as(ctypes.c_void_p))
    return nodes, order, lv.value


def _coincident(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.05, 0.4, size=(n, 1))
    b = rng.uniform(0.05, 0.4, size=(n, 1)) * rng.choice([-1.0, 1.0], size=(n, 1))
    z = np.zeros((n, 1))
    tri = np.stack([np.hstack([-a, -b, z]), np.hstack([a, -b, z]), np.hstack([z, b, z])], axis=1)
    v = np.concatenate([tri.reshape(-1, 3), scenes.random_soup(50, seed=seed)[0]]).astype(np.float32)
    return v, np.arange(v.shape[0], dtype=np.int32).reshape(-1, 3)


CASES = {
    "one triangle": lambda: scenes.random_soup(1, seed=1),
    "two triangles": lambda: scenes.random_soup(2, seed=2),
    "three triangles": lambda: scenes.random_soup(3, seed=3),
    "five triangles": lambda: scenes.random_soup(5, seed=4),
    "soup 1000": lambda: scenes.random_soup(1000, seed=5),
    "soup 20000": lambda: scenes.random_soup(20000, seed=6),
    "coincident centroids 2000": lambda: _coincident(2000, 7),
    "cornell": lambda: (lambda s: (s["verts"], s["tris"]))(scenes.scene_arrays(scenes.cornell())),
    "room (50k)": lambda: (lambda s: (s["verts"], s["tris"]))(scenes.scene_arrays(scenes.room())),
}


def _float_layout(nodes):
    lo = np.stack([nodes[:, 0:4], nodes[:, 8:12], nodes[:, 16:20]], axis=2)     # [node][slot][axis]
    hi = np.stack([nodes[:, 4:8], nodes[:, 12:16], nodes[:, 20:24]], axis=2)
    return lo.astype(np.float64), hi.astype(np.float64), nodes[:, 24:28].view(np.int32)


def _walk(refs):
    """Depth-first walk from the root: (node -> level, leaf refs, parent/slot
    of every inner child)."""
    level = {0: 0}
    leaves = []
    stack = [0]
    while stack:
        n = stack.pop()
        inner = [int(r) for r in refs[n] if r != NONE and r >= 0]
        assert inner == list(range(inner[0], inner[0] + len(inner))) if inner else True, "inner children contiguous"
        for r in refs[n]:
            r = int(r)
            if r == NONE:
                continue
            if r >= 0:
                assert r not in level, "node reached twice"
                level[r] = level[n] + 1
                stack.append(r)
            else:
                leaves.append(r)
    return level, leaves


@pytest.mark.parametrize("case", list(CASES))
def test_collapse_and_quantization(harness, case):
    verts, tris = CASES[case]()
    verts = np.asarray(verts, np.float32)
    tris = np.asarray(tris, np.int32)
    nt = tris.shape[0]
    fnodes, order, levels = _build(harness, verts, tris, 0)
    qnodes, order_q, levels_q = _build(harness, verts, tris, 1)
    assert np.array_equal(order, order_q) and levels == levels_q
    assert np.array_equal(np.sort(order), np.arange(nt))
    lo, hi, refs = _float_layout(fnodes)
    n = fnodes.shape[0]

    # tree shape: every node reached once, every leaf position covered once
    level, leaves = _walk(refs)
    assert len(level) == n
    assert max(level.values()) + 1 == levels
    covered = np.zeros(nt, np.int32)
    for r in leaves:
        code = ~r
        first, cnt = code >> 3, (code & 7) + 1
        assert cnt <= LEAF_MAX
        covered[first:first + cnt] += 1
    assert (covered == 1).all()

    # greedy collapse: fewer than four children only when all are leaves
    valid = refs != NONE
    nval = valid.sum(axis=1)
    has_inner = ((refs >= 0) & valid).any(axis=1)
    assert not (has_inner & (nval < 4)).any()

    # containment: every child box holds its subtree's triangles
    tri_lo = verts[tris].min(axis=1).astype(np.float64)
    tri_hi = verts[tris].max(axis=1).astype(np.float64)
    sub_lo = np.full((n, 4, 3), np.inf)
    sub_hi = np.full((n, 4, 3), -np.inf)
    for node in sorted(level, key=lambda k: -level[k]):   # children before parents
        for j in range(4):
            r = int(refs[node, j])
            if r == NONE:
                continue
            if r >= 0:
                sub_lo[node, j] = sub_lo[r].min(axis=0)
                sub_hi[node, j] = sub_hi[r].max(axis=0)
            else:
                code = ~r
                ids = order[(code >> 3):(code >> 3) + (code & 7) + 1]
                sub_lo[node, j] = tri_lo[ids].min(axis=0)
                sub_hi[node, j] = tri_hi[ids].max(axis=0)
    assert (lo[valid] <= sub_lo[valid]).all() and (hi[valid] >= sub_hi[valid]).all()

    # quantized boxes: decoded planes enclose the float boxes widened by delta
    org = qnodes[:, 0:3].astype(np.float64)
    ew = qnodes[:, 3].view(np.uint32)
    ex = np.stack([((ew >> (8 * a)) & 0xFF).astype(np.int64) - 127 for a in range(3)], axis=1)
    assert (ex >= -126).all() and (ex <= 127).all()
    qrows = qnodes[:, 4:10].view(np.uint32)                  # xl xh yl yh zl zh
    qb = np.stack([(qrows >> (8 * j)) & 0xFF for j in range(4)], axis=2).astype(np.float64)  # [node][row][slot]
    cell = np.ldexp(1.0, ex)                                 # [node][axis]
    dlo = org[:, None, :] + np.stack([qb[:, 0], qb[:, 2], qb[:, 4]], axis=2) * cell[:, None, :]
    dhi = org[:, None, :] + np.stack([qb[:, 1], qb[:, 3], qb[:, 5]], axis=2) * cell[:, None, :]
    mn = np.where(valid[:, :, None], lo, np.inf).min(axis=1)
    mx = np.where(valid[:, :, None], hi, -np.inf).max(axis=1)
    ext = np.max(np.where(mx >= mn, mx - mn, 0.0), axis=1)
    delta = np.ldexp(np.maximum(ext, 1e-30), -20)[:, None, None]
    assert (dlo[valid] <= (lo - delta)[valid]).all() and (dhi[valid] >= (hi + delta)[valid]).all()
    # origin at or below the lowest plane minus the margin
    assert (org <= mn - delta[:, :, 0] + 0.0).all()
    # empty slots: inside out on every axis, reference ~0
    qrefs = qnodes[:, 12:16].view(np.int32)
    for row, want in zip(range(6), (255, 0, 255, 0, 255, 0)):
        assert (qb[:, row][~valid] == want).all()
    assert (qrefs[~valid] == -1).all() and np.array_equal(qrefs[valid], refs[valid])


def _f32(x):
    return np.float32(x)


@pytest.mark.parametrize("case,nrays", [("soup 20000", 1500), ("room (50k)", 1500)])
def test_quantized_boxes_admit_every_hit_in_float32(harness, case, nrays):
    """The node visit's float32 slab test, emulated on the CPU (planes as
    q 2^-24 times 1/d scaled by 2^(e+24), plus (origin - o)/d; one rounding
    per plane; the relative slack 1.0000005), admits every ancestor box of a
    triangle for a ray that reaches that triangle, with the ray's far limit
    at that hit (the tightest the traversal uses): from origins anywhere in
    and around the scene and from points on other triangles (continuation
    rays, with the scene's tmin).  This is what makes the quantized tree
    conservative; 1/d is perturbed by up to 2 ulp, more than the hardware
    reciprocal's error."""
    verts, tris = CASES[case]()
    verts = np.asarray(verts, np.float32)
    tris = np.asarray(tris, np.int32)
    qnodes, order, _ = _build(harness, verts, tris, 1)
    fnodes, _, _ = _build(harness, verts, tris, 0)
    _, _, refs = _float_layout(fnodes)
    # parent links: (node, slot) of every inner node and of every leaf position
    parent = {}
    leaf_of = {}
    for n in range(refs.shape[0]):
        for j in range(4):
            r = int(refs[n, j])
            if r == NONE:
                continue
            if r >= 0:
                parent[r] = (n, j)
            else:
                code = ~r
                for pos in range(code >> 3, (code >> 3) + (code & 7) + 1):
                    leaf_of[pos] = (n, j)
    pos_of_tri = np.empty(tris.shape[0], np.int64)
    pos_of_tri[order] = np.arange(tris.shape[0])
    org = qnodes[:, 0:3]
    ew = qnodes[:, 3].view(np.uint32)
    qrows = qnodes[:, 4:10].view(np.uint32)
    lo_s, hi_s = verts.min(axis=0).astype(np.float64), verts.max(axis=0).astype(np.float64)
    diag = float(np.linalg.norm(hi_s - lo_s))
    tmin = _f32(1e-6 * diag)
    rng = np.random.default_rng(17)

    def admits(n, j, o, inv, tmx):
        ns, fs = [], []
        for a in range(3):
            e = int((ew[n] >> (8 * a)) & 0xFF) - 127
            A = np.ldexp(np.float64(inv[a]), e)                   # exact: 1/d times 2^e
            B = _f32(_f32(org[n, a] - o[a]) * inv[a])
            ql = float((qrows[n, 2 * a] >> (8 * j)) & 0xFF)
            qh = float((qrows[n, 2 * a + 1] >> (8 * j)) & 0xFF)
            tl, th = _f32(ql * A + np.float64(B)), _f32(qh * A + np.float64(B))
            near, far = (th, tl) if inv[a] < 0 else (tl, th)
            ns.append(near)
            fs.append(far)
        tn = max(max(ns[0], ns[1]), max(ns[2], tmin))
        tf = min(min(fs[0], fs[1]), min(fs[2], tmx))
        return tn <= _f32(tf * _f32(1.0000005))

    bad = 0
    for i in range(nrays):
        t_id = int(rng.integers(tris.shape[0]))
        b = rng.dirichlet([1.0, 1.0, 1.0])
        P = (b[:, None] * verts[tris[t_id]].astype(np.float64)).sum(axis=0)
        if i % 2 == 0:   # an origin in or around the scene
            O = rng.uniform(lo_s - 0.1 * (hi_s - lo_s), hi_s + 0.1 * (hi_s - lo_s))
        else:            # a continuation ray from another triangle's surface
            s_id = int(rng.integers(tris.shape[0]))
            b2 = rng.dirichlet([1.0, 1.0, 1.0])
            O = (b2[:, None] * verts[tris[s_id]].astype(np.float64)).sum(axis=0)
        d = P - O
        dist = float(np.linalg.norm(d))
        if dist < 1e-3 * diag:
            continue
        d = (d / dist).astype(np.float32)
        o = O.astype(np.float32)
        inv = np.empty(3, np.float32)
        for a in range(3):
            da = d[a] if abs(d[a]) > 1e-20 else np.float32(np.copysign(1e-20, d[a]))
            x = _f32(np.float32(1.0) / da)
            inv[a] = np.nextafter(np.nextafter(x, np.float32(np.inf if rng.random() < 0.5 else -np.inf)),
                                  np.float32(np.inf if rng.random() < 0.5 else -np.inf)) if rng.random() < 0.7 else x
        # the far limit the traversal uses once this hit is the best: t + tmin
        tmx = _f32(_f32(dist) + tmin)
        n, j = leaf_of[int(pos_of_tri[t_id])]
        while True:
            if not admits(n, j, o, inv, tmx):
                bad += 1
                break
            if n == 0:
                break
            n, j = parent[n]
    assert bad == 0, bad
