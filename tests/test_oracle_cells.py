"""Pins of the oracle's cell rule for the cached proposal (oracle/ipt_oracle.c,
cell_subdiv / cell_query), checked against geometry computed here from
scratch: the subdivision is the smallest n whose cells are no larger than the
requested area (closed form, away from float32 ties), the cells of a triangle
partition it into n^2 congruent sub-triangles whose centroids are the
queries (brute force point-in-triangle tests in barycentric space), and the
query normal is the interpolated vertex normal at the centroid, negated on
the back side."""
import numpy as np
import pytest

from oracle import oracle


def _scene(verts, tris, normals=None):
    n = len(tris)
    return oracle.Scene(np.asarray(verts, np.float32), np.asarray(tris, np.int32), np.zeros(n, np.int32), 1,
                        np.zeros(0, np.int32), None if normals is None else np.asarray(normals, np.float32))


def _bary(p0, e1, e2, x):
    A = np.stack([e1, e2], 1)
    uv, *_ = np.linalg.lstsq(A, x - p0, rcond=None)
    return uv


def test_subdivision_is_smallest_n_with_small_enough_cells():
    rng = np.random.default_rng(0)
    checked = 0
    for k in range(200):
        v = rng.normal(size=(3, 3)).astype(np.float32)
        o = _scene(v, [[0, 1, 2]])
        area = 0.5 * np.linalg.norm(np.cross(v[1].astype(np.float64) - v[0], v[2].astype(np.float64) - v[0]))
        ca = float(np.float32(area / rng.uniform(1.0, 3000.0)))
        n, _, _ = o.cell_query(0, 0.1, 0.1, 0, ca)
        exact = max(1, int(np.ceil(np.sqrt(area / ca))))
        # skip cases within float32 rounding of a boundary n^2 = area / ca
        r = np.sqrt(area / ca)
        if abs(r - round(r)) < 1e-4:
            continue
        assert n == min(exact, 64), (k, n, exact)
        checked += 1
    assert checked > 150
    # a cell area larger than the triangle: one cell
    o = _scene([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]])
    assert o.cell_query(0, 0.3, 0.3, 0, 10.0)[0] == 1
    # tiny cells: capped at 64
    assert o.cell_query(0, 0.3, 0.3, 0, 1e-9)[0] == 64


@pytest.mark.parametrize("n_want", [1, 2, 5])
def test_cells_partition_the_triangle(n_want):
    v = np.array([[0.2, -0.1, 0.3], [1.7, 0.2, 0.1], [0.5, 1.3, -0.4]], np.float32)
    o = _scene(v, [[0, 1, 2]])
    p0, e1, e2 = v[0].astype(np.float64), (v[1] - v[0]).astype(np.float64), (v[2] - v[0]).astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(e1, e2))
    ca = float(np.float32(area / (n_want * n_want - 0.5)))   # smallest n with n^2 >= n_want^2 - 0.5
    rng = np.random.default_rng(n_want)
    uv = rng.uniform(0, 1, (6000, 2))
    uv = np.where(uv.sum(1, keepdims=True) > 1, 1 - uv[:, ::-1], uv)
    groups = {}
    for u, w in uv:
        n, xq, _ = o.cell_query(0, u, w, 0, ca)
        assert n == n_want
        c = _bary(p0, e1, e2, xq)
        key = tuple(np.round(c * 3 * n).astype(int))
        groups.setdefault(key, []).append((u, w, c))
    assert len(groups) == n_want * n_want
    for key, pts in groups.items():
        c = pts[0][2]
        # the cell's corners from its centroid: lower cells (1/3, 1/3) above a
        # grid corner, upper cells (2/3, 2/3)
        base = np.floor(c * n_want)
        frac = c * n_want - base
        if np.allclose(frac, 1 / 3, atol=1e-9):
            corners = (base + np.array([[0, 0], [1, 0], [0, 1]])) / n_want
        else:
            assert np.allclose(frac, 2 / 3, atol=1e-9)
            corners = (base + np.array([[1, 1], [0, 1], [1, 0]])) / n_want
        assert np.allclose(corners.mean(0), c, atol=1e-12)
        a, b, d = corners
        M = np.stack([b - a, d - a], 1)
        for u, w, _ in pts:
            s, t = np.linalg.solve(M, np.array([u, w]) - a)
            assert s >= -1e-9 and t >= -1e-9 and s + t <= 1 + 1e-9
    # equal areas: the samples spread evenly over the cells
    counts = np.array([len(p) for p in groups.values()])
    expect = uv.shape[0] / n_want ** 2
    assert np.all(np.abs(counts - expect) < 6 * np.sqrt(expect))


def test_query_normal_and_side():
    v = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0]], np.float32)
    # flat: the geometric normal, negated on the back side
    o = _scene(v, [[0, 1, 2]])
    _, _, nf = o.cell_query(0, 0.2, 0.2, 0, 0.5)
    _, _, nb = o.cell_query(0, 0.2, 0.2, 1, 0.5)
    assert np.allclose(nf, [0, 0, 1]) and np.allclose(nb, [0, 0, -1])
    # vertex normals: the normalised barycentric interpolation at the centroid
    nv = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1]], np.float64)
    nv /= np.linalg.norm(nv, axis=1, keepdims=True)
    o = _scene(v, [[0, 1, 2]], nv)
    n, xq, nq = o.cell_query(0, 0.05, 0.05, 0, 0.5)   # area 2: n = 2, cell (0, 0) lower
    assert n == 2
    c = np.array([1 / 6, 1 / 6])
    assert np.allclose(xq, [2 * c[0], 2 * c[1], 0])
    want = (1 - c.sum()) * nv[0] + c[0] * nv[1] + c[1] * nv[2]
    assert np.allclose(nq, want / np.linalg.norm(want))
    assert np.allclose(o.cell_query(0, 0.05, 0.05, 1, 0.5)[2], -want / np.linalg.norm(want))
