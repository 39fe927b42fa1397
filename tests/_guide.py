"""Seeded inputs for the learned-proposal tests (no method arithmetic).

Parameter blocks in the library's layout (see oracle/guide_ref.py), synthetic
training records, and the float32 scene box the library uses for the
position features.
"""
import numpy as np

N_NET = 16744
N_EMB = 16


def random_weights(num_segments, seed=0, out_gain=1.0, kappa_bias=0.0):
    """He-normal hidden layers; output layer scaled by out_gain (larger = peakier lobes)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out, gain in [(25, 64, 1.0), (64, 64, 1.0), (64, 64, 1.0), (64, 64, 1.0), (64, 40, out_gain)]:
        parts.append(rng.normal(0.0, gain * np.sqrt(2.0 / fan_in), fan_in * fan_out))
        b = rng.normal(0.0, 0.05, fan_out)
        if fan_out == 40:
            b[3::5] += kappa_bias
        parts.append(b)
    parts.append(rng.normal(0.0, 0.3, num_segments * N_EMB))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == N_NET + N_EMB * num_segments
    return w


def box(verts):
    """(lo, inv) in float32 as the library computes them from the vertices."""
    v = np.asarray(verts, np.float32)
    lo = v.min(axis=0)
    hi = v.max(axis=0)
    inv = (np.float32(1.0) / np.maximum(hi - lo, np.float32(1e-6))).astype(np.float32)
    return lo.astype(np.float64), inv.astype(np.float64)


def random_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_records(n, num_segments, seed=0, target=None):
    """Records [n, 16] (float32, ring layout) with random features; the
    direction is drawn from `target(rng, n)` (unit vectors) if given, else
    uniformly, and the weight is U(0.1, 2)."""
    rng = np.random.default_rng(seed)
    r = np.zeros((n, 16), np.float32)
    r[:, 0:3] = rng.uniform(-1, 1, (n, 3))
    r[:, 3] = np.arange(n, dtype=np.int32).__mod__(num_segments).astype(np.int32).view(np.float32)
    r[:, 4:7] = random_unit(rng, n)
    r[:, 7] = rng.uniform(0.1, 2.0, n)
    r[:, 8:11] = random_unit(rng, n)
    r[:, 11] = np.full(n, -1, np.int32).view(np.float32)
    r[:, 12:15] = target(rng, n) if target is not None else random_unit(rng, n)
    r[:, 15] = np.ones(n, np.int32).view(np.float32)
    return r
