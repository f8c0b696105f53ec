"""dl_project_noalloc, the entry point that allocates nothing (its scratch is a fixed device array), against
dl_project through the C ABI: the same records and depths bit for bit on two calls in a row, the second on a
smaller input, and the size limit refused before any launch."""
import numpy as np
import pytest

from paper_2407_14053_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _check_case(ctx, dname, sname, c2w):
    import torch
    from paper_2407_14053_amd import api
    d = synth.make_named_display(dname)
    sc = synth.make_scene(sname)
    S = api.Scene(ctx, sc.arrays())
    D = api.Display(ctx, d)
    ref_rec, ref_depth = api.project(ctx, S, D, c2w)
    # outputs pre-filled with values the projection never writes, so that a record left unwritten shows
    out = torch.full((d.n_views, sc.n, 12), float("nan"), dtype=torch.float32, device="cuda")
    depth = torch.full((d.n_views, sc.n), -7.0, dtype=torch.float64, device="cuda")
    api.project_noalloc(ctx, S, D, c2w, out, depth)
    log("  no-alloc projection %s: %d views x %d Gaussians" % (dname, d.n_views, sc.n))
    assert torch.equal(out, ref_rec)
    nan = torch.isnan(ref_depth)
    assert torch.equal(torch.isnan(depth), nan)
    assert torch.equal(depth[~nan], ref_depth[~nan])
    assert int((~nan).sum()) > 0
    S.close()
    D.close()


def test_project_noalloc_equals_project_on_two_calls():
    from paper_2407_14053_amd import api
    ctx = api.Context(0)
    # two calls in a row on the device's one scratch array, the second smaller (8 x 2000, then 4 x 200 pairs)
    _check_case(ctx, "tiny", "tiny", synth.pose_sweep(8)[2])
    _check_case(ctx, "fd64", "fd64", synth.pose_sweep(9)[1])
    ctx.close()


def test_project_noalloc_refuses_inputs_beyond_its_scratch():
    import torch
    from paper_2407_14053_amd import api
    ctx = api.Context(0)
    d = synth.make_named_display("uhd45")          # 45 views
    sc = synth.scene_uniform(200_000, 2.0, 9)      # 9M (view, Gaussian) keys: 72 MB > 64 MiB of scratch
    S = api.Scene(ctx, sc.arrays())
    D = api.Display(ctx, d)
    out = torch.zeros((d.n_views, sc.n, 12), dtype=torch.float32, device="cuda")
    depth = torch.zeros((d.n_views, sc.n), dtype=torch.float64, device="cuda")
    with pytest.raises(api.DLError) as ei:
        api.project_noalloc(ctx, S, D, synth.pose_front(), out, depth)
    assert ei.value.code == api.DL_ERANGE
    assert "scratch" in str(ei.value)
    assert float(out.abs().sum()) == 0.0          # nothing was launched
    S.close()
    D.close()
    ctx.close()
