"""The ctypes structures of the Python binding against the C structures of
include/ipt.h: a small C program built with gcc prints every structure's size
and each field's offset, and those must equal what ctypes computes. A field
missing on either side, a wrong type or a reordering fails here instead of
silently shifting the fields the library reads."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1903_07145_amd import ipt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    ("ipt_cameras", ipt.Cameras),
    ("ipt_render_opts", ipt.RenderOpts),
    ("ipt_adam_opts", ipt.AdamOpts),
    ("ipt_scene_info_t", ipt.SceneInfo),
    ("ipt_build_opts", ipt.BuildOpts),
    ("ipt_kernel_profile", ipt.KernelProfile),
    ("ipt_guide_opts", ipt.GuideOpts),
]


def _c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ipt.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append('    printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for field, _ in cls._fields_:
            lines.append('    printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, field, cname, field))
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    layout = {}
    for line in out:
        if line:
            a, b, v = line.split()
            layout[(a, b)] = int(v)
    return layout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_ctypes_structures_match_the_header(tmp_path):
    layout = _c_layout(tmp_path)
    for cname, cls in PAIRS:
        assert layout[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert layout[(cname, field)] == getattr(cls, field).offset, (cname, field)
