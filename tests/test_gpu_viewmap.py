"""View map (Eq. (1)-(3)) and rig on the GPU path, bit-exact against the oracle (C ABI)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import rig as orig
from oracle import viewmap as oviewmap
from paper_2407_14053_amd import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2407_14053_amd import api
    c = api.Context(0)
    yield c
    c.close()


EXTRA = {
    "offset_pos": dict(width=301, height=77, n_views=7, tan_slant=Fraction(2, 7), pitch=Fraction(23, 5),
                       offset=Fraction(13, 4)),
    "neg_slant_offset": dict(width=129, height=65, n_views=5, tan_slant=Fraction(-3, 8), pitch=Fraction(9, 2),
                             offset=Fraction(-5, 3)),
    "one_view": dict(width=64, height=48, n_views=1, tan_slant=Fraction(1, 3), pitch=Fraction(53, 10)),
    "max_views": dict(width=333, height=101, n_views=255, tan_slant=Fraction(1, 7), pitch=Fraction(255, 1)),
    "one_pixel": dict(width=1, height=1, n_views=3, tan_slant=Fraction(1, 3), pitch=Fraction(5, 1)),
}


def _display(name):
    if name.startswith("table1_"):
        # the display table's panels; the 65-inch one needs the view map's per-product reduction (Q (3W + H) is
        # above 2^62 there)
        return synth.table1_display(name[len("table1_"):])
    if name in EXTRA:
        return synth.make_display(name=name, **EXTRA[name])
    return synth.make_named_display(name)


@pytest.mark.parametrize("name", ["tiny", "uhd45", "8k60", "fhd16", "fhd45", "fd64", "fig2b"] + list(EXTRA) +
                         ["table1_7.9in", "table1_15.6in", "table1_65in"])
def test_view_map_bit_exact(ctx, name):
    from paper_2407_14053_amd import api
    log("view map", name)
    d = _display(name)
    D = api.Display(ctx, d)
    got = D.view_map().cpu().numpy()
    ref = oviewmap.view_map(d.width, d.height, d.n_views, d.tan_slant, d.pitch, d.offset)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref.astype(np.uint8))
    rv, rx, ry, index = oviewmap.subpixel_rays(ref)
    assert D.num_rays() == len(rv)
    D.close()


@pytest.mark.parametrize("name", ["tiny", "uhd45", "fd64", "one_view"])
def test_cameras_match_oracle_rig(ctx, name):
    from paper_2407_14053_amd import api
    d = _display(name)
    D = api.Display(ctx, d)
    for c2w in [synth.pose_front(3.0), synth.pose_orbit(120)[17], synth.look_at_c2w((0.3, 1.0, 2.5))]:
        cams = D.cameras(c2w)
        R, t, eye = orig.cameras(c2w, float(np.linalg.norm(c2w[:3, 3])), d.baseline, d.n_views)
        assert np.allclose(cams[:, :9].reshape(-1, 3, 3), R, atol=1e-14)
        assert np.allclose(cams[:, 9:12], t, atol=1e-13)
        assert np.allclose(cams[:, 12:15], eye, atol=1e-14)
    D.close()


def test_invalid_descriptors_rejected(ctx):
    from paper_2407_14053_amd import api
    bad = [
        dict(width=0, height=10, n_views=3, tan_slant=Fraction(1, 3), pitch=Fraction(5)),
        dict(width=10, height=10, n_views=0, tan_slant=Fraction(1, 3), pitch=Fraction(5)),
        dict(width=10, height=10, n_views=256, tan_slant=Fraction(1, 3), pitch=Fraction(5)),
        dict(width=10, height=10, n_views=3, tan_slant=Fraction(1, 3), pitch=Fraction(0)),
        dict(width=10, height=10, n_views=3, tan_slant=Fraction(1, 3), pitch=Fraction(-5)),
    ]
    for kw in bad:
        with pytest.raises(api.DLError) as e:
            api.Display(ctx, synth.make_display(**kw))
        assert e.value.code == api.DL_EINVAL
    d = synth.make_display(10, 10, 3, Fraction(1, 3), Fraction(5))
    desc = api.make_desc(d)
    desc.pitch.den = 0
    import ctypes
    h = ctypes.c_void_p()
    assert api.load().dl_display_create(ctx.h, ctypes.byref(desc), None, ctypes.byref(h)) == api.DL_EINVAL
    # exact arithmetic that cannot fit 64-bit integers
    huge = synth.make_display(10, 10, 3, Fraction(1, 2 ** 40 + 1), Fraction(2 ** 30 + 7, 3))
    with pytest.raises(api.DLError) as e:
        api.Display(ctx, huge)
    assert e.value.code == api.DL_ERANGE
