"""The C ABI library loads and exports every function declared in include/*.h (no GPU calls)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_14053_amd", "libdirectl.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(dl_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dl_create", "dl_scene_create", "dl_display_create", "dl_render", "dl_render_standard",
              "dl_display_view_map", "dl_project", "dl_interleave", "dl_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdirectl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdirectl.so not built")
def test_default_opts_and_error_string_without_gpu():
    from paper_2407_14053_amd import api
    o = api.default_opts()
    assert abs(o.z_near - 0.2) < 1e-7 and o.q_cut == 9.0 and abs(o.alpha_min - 1 / 255) < 1e-9
    assert abs(o.alpha_max - 0.99) < 1e-7 and abs(o.t_min - 1e-4) < 1e-10 and abs(o.dilation - 0.3) < 1e-7
    assert o.sh_degree == 3
    lib = api.load()
    assert lib.dl_create(-1, ctypes.byref(ctypes.c_void_p())) != 0
    assert len(lib.dl_last_error()) > 0
