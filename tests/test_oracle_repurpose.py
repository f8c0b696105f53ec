"""Oracle subpixel repurposing (Sec. "Subpixel Repurposing", Eq. (11)-(14)) pinned by what the paper fixes for any
reading of its heuristic: every subpixel keeps its view and channel (Eq. (11)-(13)), a ray's channel fills at most
one subpixel, a repurposed subpixel takes a pixel rendered earlier in the same area and inside the search window of
Eq. (14) (rows below, columns to the left), the ray count lies in [wh, 3wh] and never exceeds that of the identity
map, and with an empty search window the map is the identity (Alg. 1).  The reading itself is pinned by the one
table the paper prints for it: the rendered pixel ratio beta against P_w on the panels of its display table
(values within 0.2 of the printed ones, and falling as P_w grows, as printed), computed by the compiled walk, which
the tests also check against the pure-Python one."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import repurpose as R
from oracle.viewmap import view_map

PANELS = [
    # w, h, N, tan(alpha), L_x, K_offset, P_w
    (48, 40, 8, F(1, 3), F(53, 10), F(0), 2),
    (64, 48, 16, F(1, 6), F(37, 5), F(0), 2),
    (64, 48, 45, F(1, 6), F(37, 5), F(0), 1),
    (64, 48, 45, F(1, 6), F(37, 5), F(3, 2), 4),
    (60, 40, 60, F(1197, 10000), F(53344, 10000), F(12547, 10000), 2),   # a 15.6-inch-like panel (Tab. 1)
    (40, 60, 48, F(-1, 27), F(16, 3), F(0), 2),                          # negative slant
]


def _views(V):
    return np.stack([V[:, k::3] for k in range(3)], axis=2).astype(np.int64)


def _area(w, h, t, L, K, pw):
    # the area of subpixel (x, 3y + k) is that of its pixel
    return np.repeat(R.pixel_areas(w, h, t, L, K, pw), 3, axis=1)


@pytest.mark.parametrize("w,h,N,t,L,K,pw", PANELS)
def test_repurposing_invariants(w, h, N, t, L, K, pw):
    V = view_map(w, h, N, t, L, K).astype(np.int64)
    A = _area(w, h, t, L, K, pw)
    sx, sy = R.repurpose_map(w, h, N, t, L, K, pw)
    v = _views(V)
    xs, ys = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    # the source pixel shows the subpixel's view on one of its subpixels, and that subpixel is its own source
    # (the pixel was rendered for it), in the same area
    for x in range(h):
        for y in range(w):
            for k in range(3):
                x2, y2, vv = sx[x, y, k], sy[x, y, k], v[x, y, k]
                own = [j for j in range(3) if V[x2, 3 * y2 + j] == vv and sx[x2, y2, j] == x2 and sy[x2, y2, j] == y2]
                assert own, (x, y, k)
                assert any(A[x2, 3 * y2 + j] == A[x, 3 * y + k] for j in own), (x, y, k)
    # a ray's channel fills at most one subpixel
    keys = np.stack([v.ravel(), sx.ravel(), sy.ravel(), np.broadcast_to(np.arange(3), v.shape).ravel()], axis=1)
    assert len(np.unique(keys, axis=0)) == keys.shape[0]
    # repurposed subpixels: rows at least 2 below the source (fewer only where Eq. (14) clamps the window to
    # the last row), columns at or left of it
    rep = (sx != xs[..., None]) | (sy != ys[..., None])
    dx = xs[..., None] - sx
    dy = sy - ys[..., None]
    near_bottom = np.broadcast_to(xs[..., None] >= h - 2, dx.shape)
    assert ((dx >= 2) | (near_bottom & (dx >= 0)))[rep].all() and (dy[rep] >= 0).all()
    # ray count between wh and 3wh, at most the identity map's
    n = len(R.rays_of(V, sx, sy))
    ident = len(np.unique(np.stack([v.ravel(), np.repeat(np.arange(w * h), 3)], axis=1), axis=0))
    assert w * h <= n <= ident <= 3 * w * h


def test_empty_search_window_is_the_identity_map():
    # 5 N / (2 L_x) < 2: no row lies in the window of Eq. (14) (except where min(x + 2, h - 1) clamps it onto
    # the last row), so every subpixel above the last two rows shows its own pixel (Alg. 1)
    w, h, N, t, L = 40, 30, 3, F(1, 3), F(53, 10)
    assert 5 * N / (2 * L) < 2
    sx, sy = R.repurpose_map(w, h, N, t, L, 0, 2)
    xs, ys = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    same = (sx == xs[..., None]) & (sy == ys[..., None])
    assert same[: h - 2].all()


def test_repurposing_reduces_rays_on_dense_panels():
    # N / L_x large: views repeat down the lens direction and idle channels find takers
    w, h, N, t, L = 64, 48, 45, F(1, 6), F(37, 5)
    V = view_map(w, h, N, t, L, 0).astype(np.int64)
    sx, sy = R.repurpose_map(w, h, N, t, L, 0, 2)
    beta = len(R.rays_of(V, sx, sy)) / (w * h)
    assert beta < 1.5


@pytest.mark.parametrize("w,h,N,t,L,K,pw", PANELS)
def test_compiled_walk_equals_python_walk(w, h, N, t, L, K, pw):
    sx, sy = R.repurpose_map(w, h, N, t, L, K, pw)
    V, src = R.repurpose_map_full(w, h, N, t, L, K, pw)
    assert np.array_equal(V.astype(np.int64), view_map(w, h, N, t, L, K).astype(np.int64))
    assert np.array_equal(src.astype(np.int64), sx * w + sy)


# Table 6 of the paper: beta for P_w = 1, 2, 3, 4 on the 7.9-, 15.6- and 65-inch panels of the display table
# (Table 1: w, h, L_x, tilt angle in degrees, K_offset, N_v).  The tilt is converted to tan(alpha) rounded to a
# denominator of 10^6 and the four-decimal pitch and offset are taken as exact decimals.
TABLE6 = {
    "7.9in": ((1536, 2048, "6.2221", 10.8232, "4.2077", 48), (1.4764, 1.4467, 1.3044, 1.0790)),
    "15.6in": ((3840, 2160, "5.3344", 6.8526, "1.2547", 60), (1.3701, 1.3694, 1.2868, 1.1109)),
    "65in": ((7680, 4320, "9.3597", 8.6517, "23.6677", 96), (1.5613, 1.3708, 1.2440, 1.2222)),
}
BETA_TOL = 0.2


def _table_panel(name):
    (w, h, L, deg, K, N), printed = TABLE6[name]
    t = F(round(math.tan(math.radians(deg)) * 10 ** 6), 10 ** 6)
    return w, h, N, t, F(L), F(K), printed


@pytest.mark.parametrize("name", ["7.9in", "15.6in"])
def test_beta_against_table6(name):
    w, h, N, t, L, K, printed = _table_panel(name)
    got = [R.beta(w, h, N, t, L, K, pw) for pw in (1, 2, 3, 4)]
    print(name, "beta", ["%.4f" % b for b in got], "printed", printed)
    for b, p in zip(got, printed):
        assert abs(b - p) <= BETA_TOL, (name, got, printed)
    # the printed trend: fewer rays as the areas grow
    assert all(got[i + 1] <= got[i] for i in range(3)), got
    assert got[3] < got[0]


def test_beta_against_table6_65in_at_pw2():
    # the 65-inch panel (99.5M subpixels) at the P_w the paper selects; the other P_w of this panel are in the
    # design notes' table
    w, h, N, t, L, K, printed = _table_panel("65in")
    b = R.beta(w, h, N, t, L, K, 2)
    print("65in beta(P_w = 2) %.4f printed %.4f" % (b, printed[1]))
    assert abs(b - printed[1]) <= BETA_TOL
