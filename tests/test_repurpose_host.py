"""Host logic of subpixel repurposing (Alg. 2, run on the host when a display is created): a harness compiled
against the library's walk gives, for the view map of the oracle, the same source pixel for every subpixel as the
oracle's repurpose_map, bit for bit, on panels with positive and negative slants, offsets, N below and above L_x
and P_w from 1 to 4 (no GPU involved)."""
import os
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import repurpose as orep
from oracle.viewmap import view_map

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PANELS = [
    # w, h, N, tan(alpha), L_x, K_offset, P_w
    (48, 40, 8, F(1, 3), F(53, 10), F(0), 2),
    (64, 48, 45, F(1, 6), F(37, 5), F(0), 1),
    (64, 48, 45, F(1, 6), F(37, 5), F(3, 2), 4),
    (60, 40, 60, F(1197, 10000), F(53344, 10000), F(12547, 10000), 2),
    (40, 60, 48, F(-1, 27), F(16, 3), F(0), 2),
    (40, 30, 3, F(1, 3), F(53, 10), F(0), 3),
]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("rep") / "repurpose_harness")
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "repurpose_harness.cpp"),
           "-x", "hip", os.path.join(ROOT, "paper_2407_14053_amd", "csrc", "repurpose.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


@pytest.mark.parametrize("w,h,N,t,L,K,pw", PANELS)
def test_host_walk_equals_oracle(harness, tmp_path, w, h, N, t, L, K, pw):
    V = view_map(w, h, N, t, L, K).astype(np.uint8)
    vfile, ofile = str(tmp_path / "V.u8"), str(tmp_path / "src.i32")
    V.tofile(vfile)
    args = [harness, str(w), str(h), str(N), str(t.numerator), str(t.denominator), str(L.numerator),
            str(L.denominator), str(K.numerator), str(K.denominator), str(pw), vfile, ofile]
    r = subprocess.run(args, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    got = np.fromfile(ofile, dtype=np.int32).reshape(h, w, 3).astype(np.int64)
    sx, sy = orep.repurpose_map(w, h, N, t, L, K, pw)
    assert np.array_equal(got, sx * w + sy), int((got != sx * w + sy).sum())
