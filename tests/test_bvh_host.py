"""Host logic of the ray-order BVH (Eq. (21), built on the host): a harness compiled against the library's own
builder checks, on uniform, clustered and coincident synthetic Gaussians and on the smallest cases, that child
references are in range, every Gaussian of the BVH sits in exactly one leaf (those with opacity >= alpha_min),
boxes nest, each Gaussian's q <= q_lim ellipsoid lies inside its leaf box, and a push-all-children walk stays within
the reported stack bound."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("bvh") / "bvh_harness")
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "bvh_harness.cpp"),
           "-x", "hip", os.path.join(ROOT, "paper_2407_14053_amd", "csrc", "bvh.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


@pytest.mark.parametrize("n,kind", [(1, 0), (2, 0), (5, 0), (9, 2), (3000, 0), (3000, 1), (200, 2), (60000, 1)])
def test_bvh_invariants(harness, n, kind):
    r = subprocess.run([harness, str(n), str(kind)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
