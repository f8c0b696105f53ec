"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the library's BVH builder and
Alg. 2 walk through their host harnesses, and the oracle's C++ (compositing with near-tie groups, the adjoint,
the projection, the compiled walk) through a small driver.  Any invalid access, leak or undefined operation
aborts the program and fails the test."""
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
# the sanitizers apply to the host pass only (-Xarch_host before each -fsanitize=); no device code is involved
SAN_HIP = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _hip_harness(tmp_path_factory, name, harness, src):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp(name) / name)
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"] + SAN_HIP + ["-I", os.path.join(ROOT, "include"), os.path.join(HERE, harness),
                                            "-x", "hip", os.path.join(ROOT, "paper_2407_14053_amd", "csrc", src),
                                            "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


@pytest.fixture(scope="module")
def bvh_asan(tmp_path_factory):
    return _hip_harness(tmp_path_factory, "bvh_asan", "bvh_harness.cpp", "bvh.hip")


@pytest.fixture(scope="module")
def walk_asan(tmp_path_factory):
    return _hip_harness(tmp_path_factory, "walk_asan", "repurpose_harness.cpp", "repurpose.hip")


@pytest.mark.parametrize("n,kind", [(1, 0), (5, 0), (9, 2), (3000, 1), (200, 2)])
def test_bvh_builder_sanitized(bvh_asan, n, kind):
    r = subprocess.run([bvh_asan, str(n), str(kind)], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.startswith("ok")


@pytest.mark.parametrize("w,h,N,t,L,K,pw", [(48, 40, 8, F(1, 3), F(53, 10), F(0), 2),
                                            (40, 60, 48, F(-1, 27), F(16, 3), F(7, 3), 3)])
def test_alg2_walk_sanitized(walk_asan, tmp_path, w, h, N, t, L, K, pw):
    V = view_map(w, h, N, t, L, K).astype(np.uint8)
    vfile, ofile = str(tmp_path / "V.u8"), str(tmp_path / "src.i32")
    V.tofile(vfile)
    args = [walk_asan, str(w), str(h), str(N), str(t.numerator), str(t.denominator), str(L.numerator),
            str(L.denominator), str(K.numerator), str(K.denominator), str(pw), vfile, ofile]
    r = subprocess.run(args, capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    got = np.fromfile(ofile, dtype=np.int32).reshape(h, w, 3).astype(np.int64)
    sx, sy = orep.repurpose_map(w, h, N, t, L, K, pw)
    assert np.array_equal(got, sx * w + sy)


def test_oracle_sanitized(tmp_path):
    out = str(tmp_path / "oracle_san")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_san_driver.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([out], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.startswith("ok")
