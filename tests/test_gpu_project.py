"""Per-view EWA projection and SH colour on the GPU path against the FP64 oracle (C ABI)."""
import numpy as np
import pytest

from oracle import render as orender
from paper_2407_14053_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_14053_amd import api
    c = api.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", ["tiny", "uhd45_sub"])
def test_projected_records_match_oracle(ctx, case):
    from paper_2407_14053_amd import api
    log("project", case)
    if case == "tiny":
        d = synth.make_named_display("tiny")
        sc = synth.make_scene("tiny")
    else:
        d = synth.make_named_display("uhd45")
        sc = synth.make_scene("uhd45").subset(slice(0, 20000))
    c2w = synth.pose_sweep(9)[2]
    S = api.Scene(ctx, sc.arrays())
    D = api.Display(ctx, d)
    rec, depth = api.project(ctx, S, D, c2w)
    rec = rec.cpu().numpy().astype(np.float64)
    depth = depth.cpu().numpy()
    R, t, eye = orender.cameras_for(d, c2w)
    opts = orender.Opts()
    f, cx, cy = orender.intrinsics(d)
    amin = opts.alpha_min
    for v in sorted({0, d.n_views // 2, d.n_views - 1}):
        o = orender.project(sc, R[v], t[v], eye[v], f, cx, cy, opts)
        vis = np.isfinite(depth[v])
        assert not np.any(rec[v][~vis])  # a culled Gaussian's record is all zeros
        # visible on the GPU only in front of the near plane and with opacity able to reach alpha_min
        assert np.all(o[vis, 9] > opts.z_near)
        # every Gaussian whose cutoff ellipse certainly reaches a pixel centre must be visible
        qlim = np.minimum(opts.q_cut, 2 * np.log(np.maximum(o[:, 5], 1e-30) / amin))
        ex = np.sqrt(np.maximum(qlim, 0) * o[:, 10])
        ey = np.sqrt(np.maximum(qlim, 0) * o[:, 12])
        sure = (o[:, 9] > opts.z_near * 1.001) & (o[:, 5] > amin * 1.001) & \
               (o[:, 0] + 0.99 * ex > 0.5 + 1) & (o[:, 0] - 0.99 * ex < d.width - 1.5) & \
               (o[:, 1] + 0.99 * ey > 1.5) & (o[:, 1] - 0.99 * ey < d.height - 1.5)
        assert np.all(vis[sure])
        g, r = rec[v][vis], o[vis]
        assert np.allclose(depth[v][vis], r[:, 9], rtol=1e-13)
        assert np.allclose(g[:, 0], r[:, 0], rtol=2e-7, atol=2e-4)
        assert np.allclose(g[:, 1], r[:, 1], rtol=2e-7, atol=2e-4)
        # the GPU record holds the conic scaled by log2(e)/2 (a, c) and log2(e) (b)
        ks = np.log2(np.e) / 2
        conic = g[:, 2:5] / np.array([ks, 2 * ks, ks])
        scale = np.sqrt(np.abs(r[:, 2] * r[:, 4]))
        for k in (0, 1, 2):
            assert np.all(np.abs(conic[:, k] - r[:, 2 + k]) <= 1e-6 * scale + 1e-12)
        assert np.allclose(g[:, 8], r[:, 5], rtol=1e-7)
        assert np.allclose(g[:, 9:12], r[:, 6:9], atol=5e-6)
    S.close()
    D.close()
