"""The C-ABI library loads, exports every symbol include/ipt.h declares, and
rejects bad arguments on the host before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_07145_amd", "libipt.so")


@pytest.fixture(scope="module")
def ipt():
    if not os.path.exists(LIB):
        from paper_1903_07145_amd import build
        build.build()
    from paper_1903_07145_amd import ipt as m
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "ipt.h")).read()
    return sorted(set(re.findall(r"\b(ipt_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(ipt):
    names = _declared()
    assert "ipt_render" in names and "ipt_loss_grad" in names
    L = ipt.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(ipt.EXPORTS) >= set(names)


def test_scene_build_validation(ipt):
    L = ipt.lib()
    v = np.zeros((3, 3), np.float32)
    v[1, 0] = 1
    v[2, 1] = 1
    t = np.array([[0, 1, 3]], np.int32)     # vertex 3 out of range
    s = np.zeros(1, np.int32)
    e = np.zeros(0, np.int32)
    h = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    st = L.ipt_scene_build(p(v), 3, None, p(t), p(s), 1, 1, p(e), 0, None, ctypes.byref(h))
    assert st == 2 and b"out of range" in L.ipt_last_error()
    t = np.array([[0, 1, 2]], np.int32)
    s = np.array([4], np.int32)             # segment out of range
    st = L.ipt_scene_build(p(v), 3, None, p(t), p(s), 1, 1, p(e), 0, None, ctypes.byref(h))
    assert st == 2
    v2 = v.copy()
    v2[0, 0] = np.nan
    s = np.zeros(1, np.int32)
    st = L.ipt_scene_build(p(v2), 3, None, p(t), p(s), 1, 1, p(e), 0, None, ctypes.byref(h))
    assert st == 2 and b"finite" in L.ipt_last_error()
    v2[0, 0] = -2e12                        # beyond the coordinate range
    st = L.ipt_scene_build(p(v2), 3, None, p(t), p(s), 1, 1, p(e), 0, None, ctypes.byref(h))
    assert st == 2 and b"beyond 1e12" in L.ipt_last_error()
    e2 = np.array([0, 0], np.int32)         # duplicate emitter
    st = L.ipt_scene_build(p(v), 3, None, p(t), p(s), 1, 1, p(e2), 2, None, ctypes.byref(h))
    assert st == 2
    st = L.ipt_scene_build(None, 3, None, p(t), p(s), 1, 1, p(e), 0, None, ctypes.byref(h))
    assert st == 1
    vz = np.zeros((3, 3), np.float32)       # zero-area emitter triangle
    st = L.ipt_scene_build(p(vz), 3, None, p(t), p(s), 1, 1, p(np.array([0], np.int32)), 1, None,
                           ctypes.byref(h))
    assert st == 2 and b"zero area" in L.ipt_last_error()


def test_sgd_step_validation(ipt):
    L = ipt.lib()
    a = ipt.AdamOpts(1e-2, 0.9, 0.999, 1e-8)
    assert L.ipt_sgd_step(None, None, None, None, 4, 1, ctypes.byref(a), None, None, None, None, None) == 1
    bad = ipt.AdamOpts(-1.0, 0.9, 0.999, 1e-8)
    x = ctypes.c_void_p(16)
    assert L.ipt_sgd_step(x, x, x, x, 4, 1, ctypes.byref(bad), None, None, None, None, None) == 1
    assert L.ipt_sgd_step(x, x, x, x, 4, 0, ctypes.byref(a), None, None, None, None, None) == 1
