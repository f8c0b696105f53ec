"""Oracle (test infrastructure only): subpixel repurposing, Alg. 2 of the paper (Sec. "Subpixel Repurposing").

Nothing in the product imports this module; only tests use it.

What is computed: the encoded image index matrix M_i, which gives every subpixel (x, y, k) of the panel the
ray it shows: (v, x', y', k) with v = V(x, 3y + k) (the view and the channel are kept, Eq. (11)-(13)), i.e.
channel k of view v's pixel (x', y').  Without repurposing (x', y') = (x, y) (Alg. 1).  With it, a pixel of view
v that was rendered for one of its channels lends its other two channels to nearby subpixels of the same view
along the lens direction, so fewer distinct rays (v, x', y') need rendering.

The paper leaves the heuristic underdetermined; the readings taken here (each one a line of the design notes):
* Areas (SplitArea): the panel is cut into slanted strips of P_w grating units.  A subpixel's grating unit is
  floor(d_offset / L_x) with d_offset of Eq. (1), so its area is floor(d_offset / (P_w L_x)) (floored, also for
  negative d_offset).  Areas are processed in increasing index, the subpixels of an area in row-major order
  (row x, column y, channel k).
* The buffer B_rgb holds one pixel per (view, channel); it starts empty in every area.  Sampling a new
  subpixel (Eq. (11)) stores its pixel for the two other channels of that view (Eq. (12)), replacing what they
  held; repurposing (Eq. (13)) takes the pixel held for (v, k) and empties that slot.
* Search range (Eq. (14), whose parentheses are unbalanced): rows from min(x + 2, h - 1) to
  min(x + floor(5 N_v / (2 L_x)), h - 1), columns from max(y - floor(N_v / (3 L_x)), 0) to y.  The bounds are
  real-valued in the paper; integer rows and columns inside them are the ones searched.
* SearchTheSameViewpoint: among the subpixels in that range that belong to the same area, have view v and
  are not yet assigned, one whose channel has a pixel waiting in B_rgb is taken if there is one, else any;
  ties go to the first in row-major order (row, column, channel).  None: the chain ends and the view's buffer
  slots are emptied (ClearSubpixelBuffer).
"""
from __future__ import annotations

from fractions import Fraction
from math import floor

import numpy as np

from oracle.viewmap import view_map


def _area_map(width: int, height: int, tan_slant, pitch, offset, pw: int) -> np.ndarray:
    """A[x, s] = floor(d_offset / (P_w L_x)) for s = 3y + k, with d_offset of Eq. (1) (exact)."""
    ts, L, K = Fraction(tan_slant), Fraction(pitch), Fraction(offset)
    a, b = ts.numerator, ts.denominator
    p, q = L.numerator, L.denominator
    r, c = K.numerator, K.denominator
    s = np.arange(3 * width, dtype=object)
    A = np.empty((height, 3 * width), dtype=np.int64)
    for x in range(height):
        for j in range(3 * width):
            d = Fraction(int(s[j])) + 3 * x * Fraction(a, b) - Fraction(r, c)   # Eq. (1)
            A[x, j] = floor(d / (pw * L))
    return A


def repurpose_map(width: int, height: int, n_views: int, tan_slant, pitch, offset=0, pw: int = 2):
    """Alg. 2.  Returns (src_x, src_y) of shape [h, w, 3]: subpixel (x, y, k) shows channel k of view
    V(x, 3y + k) at pixel (src_x, src_y).  Pure Python loops: small panels only."""
    V = view_map(width, height, n_views, tan_slant, pitch, offset).astype(np.int64)
    A = _area_map(width, height, tan_slant, pitch, offset, pw)
    L = Fraction(pitch)
    drow = floor(Fraction(5 * n_views) / (2 * L))      # 2 N/L + N/(2L)
    dcol = floor(Fraction(n_views) / (3 * L))          # N/(3L)
    h, w = height, width
    src_x = np.full((h, w, 3), -1, dtype=np.int64)
    src_y = np.full((h, w, 3), -1, dtype=np.int64)
    # subpixels of every area in row-major order
    order = sorted(((int(A[x, 3 * y + k]), x, y, k) for x in range(h) for y in range(w) for k in range(3)))
    cur_area = None
    B = {}
    for area, x0, y0, k0 in order:
        if area != cur_area:
            cur_area = area
            B = {}                                        # CreateSubpixelBuffer: empty per area
        v = int(V[x0, 3 * y0 + k0])
        x, y, k = x0, y0, k0
        while src_x[x, y, k] < 0 and A[x, 3 * y + k] == area:
            if (v, k) in B:                               # Eq. (13): repurpose the waiting pixel
                src_x[x, y, k], src_y[x, y, k] = B.pop((v, k))
            else:                                         # Eq. (11)-(12): sample anew, lend the others
                src_x[x, y, k], src_y[x, y, k] = x, y
                B[(v, (k + 1) % 3)] = (x, y)
                B[(v, (k + 2) % 3)] = (x, y)
            # Eq. (14)
            x_lo, x_hi = min(x + 2, h - 1), min(x + drow, h - 1)
            y_lo, y_hi = max(y - dcol, 0), y
            first = preferred = None
            for xx in range(x_lo, x_hi + 1):
                for yy in range(y_lo, y_hi + 1):
                    for kk in range(3):
                        if V[xx, 3 * yy + kk] != v or src_x[xx, yy, kk] >= 0 or A[xx, 3 * yy + kk] != area:
                            continue
                        if first is None:
                            first = (xx, yy, kk)
                        if preferred is None and (v, kk) in B:
                            preferred = (xx, yy, kk)
                if preferred is not None:
                    break
            nxt = preferred if preferred is not None else first
            if nxt is None:
                break
            x, y, k = nxt
        for kk in range(3):                               # ClearSubpixelBuffer(v)
            B.pop((v, kk), None)
    assert (src_x >= 0).all()
    return src_x, src_y


def rays_of(V: np.ndarray, src_x: np.ndarray, src_y: np.ndarray) -> np.ndarray:
    """U_rays: the distinct (v, x', y') over all subpixels, sorted."""
    h, w, _ = src_x.shape
    v = np.stack([V[:, k::3] for k in range(3)], axis=2).astype(np.int64)
    keys = np.stack([v.ravel(), src_x.ravel(), src_y.ravel()], axis=1)
    return np.unique(keys, axis=0)


def encoded_from_rays(V: np.ndarray, src_x: np.ndarray, src_y: np.ndarray, ray_rgb) -> np.ndarray:
    """M_e[x, y, k] = channel k of the ray (V(x, 3y + k), src_x, src_y); ray_rgb(v, x', y') -> rgb."""
    h, w, _ = src_x.shape
    out = np.empty((h, w, 3))
    for x in range(h):
        for y in range(w):
            for k in range(3):
                out[x, y, k] = ray_rgb(int(V[x, 3 * y + k]), int(src_x[x, y, k]), int(src_y[x, y, k]))[k]
    return out
