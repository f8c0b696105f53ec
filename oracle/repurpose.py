"""Oracle (test infrastructure only): subpixel repurposing (paper Sec. "Subpixel Repurposing", Eq. (11)-(14)).

Nothing in the product imports this module; only tests use it.

What is computed: the encoded image index matrix M_i, which gives every subpixel (x, y, k) of the panel the
ray it shows: (v, x', y', k) with v = V(x, 3y + k) (the view and the channel are kept, Eq. (11)-(13)), i.e.
channel k of view v's pixel (x', y').  Without repurposing (x', y') = (x, y) (Alg. 1).  With it, a pixel of view
v that was rendered for one of its channels lends its other two channels to nearby subpixels of the same view
along the lens direction, so fewer distinct rays (v, x', y') need rendering.

The paper leaves the heuristic underdetermined.  The reading taken here (each point a line of the design notes)
was chosen among the variants the text allows as the one whose rays per pixel come closest to the paper's table
of beta against P_w on the three panels of its display table, with the same trend:

* Areas: a pixel lies in the slanted strip of P_w grating units that holds its left edge, i.e. its area is
  floor(d_offset(x, y, 0) / (P_w L_x)) with d_offset of Eq. (1); its three subpixels share it.  Areas are taken in
  increasing order, the subpixels of an area in row-major order (row x, column y, channel k).
* Every subpixel still unassigned when its turn comes starts a chain of its view v, holding nothing.  A chain
  assigns its current subpixel: a pixel it holds for that channel is shown there and released (Eq. (13)); if it
  holds none, the subpixel shows its own pixel, which is then held for the view's two other channels in place of
  whatever was held for them (Eq. (11)-(12)).
* The next subpixel of the chain comes from the window of Eq. (14) (whose parentheses are unbalanced): rows
  min(x + 2, h - 1) .. min(x + floor(5 N_v / (2 L_x)), h - 1), columns max(y - floor(N_v / (3 L_x)), 0) .. y.  It
  is a subpixel of view v not yet assigned, one whose channel has a held pixel if there is one, the first in
  row-major order (row, column, channel) either way.  The search itself ignores the areas; the chain goes on only
  if that subpixel lies in the chain's area, and otherwise (or if there is none) ends, dropping what it holds.

This module is pure Python for small panels; ``srwalk.cpp`` is the same reading compiled for full-size panels (the
tests check that the two agree).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from math import floor

import numpy as np

from oracle.viewmap import view_map

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srwalk.cpp")
_LIB = os.path.join(_HERE, "libdlo_sr.so")


def pixel_areas(width: int, height: int, tan_slant, pitch, offset, pw: int) -> np.ndarray:
    """A[x, y] = floor(d_offset(x, y, 0) / (P_w L_x)), with d_offset of Eq. (1) (exact)."""
    ts, L, K = Fraction(tan_slant), Fraction(pitch), Fraction(offset)
    A = np.empty((height, width), dtype=np.int64)
    for x in range(height):
        for y in range(width):
            d = 3 * y + 3 * x * ts - K                                     # Eq. (1) at k = 0
            A[x, y] = floor(d / (pw * L))
    return A


def repurpose_map(width: int, height: int, n_views: int, tan_slant, pitch, offset=0, pw: int = 2):
    """Returns (src_x, src_y) of shape [h, w, 3]: subpixel (x, y, k) shows channel k of view V(x, 3y + k) at
    pixel (src_x, src_y).  Pure Python loops: small panels only."""
    V = view_map(width, height, n_views, tan_slant, pitch, offset).astype(np.int64)
    A = pixel_areas(width, height, tan_slant, pitch, offset, pw)
    L = Fraction(pitch)
    rows_below = floor(Fraction(5 * n_views) / (2 * L))      # Eq. (14): 2 N/L + N/(2L)
    cols_left = floor(Fraction(n_views) / (3 * L))           # Eq. (14): N/(3L)
    h, w = height, width
    src_x = np.full((h, w, 3), -1, dtype=np.int64)
    src_y = np.full((h, w, 3), -1, dtype=np.int64)

    def next_in_window(x, y, v, holding):
        first = None
        for xx in range(min(x + 2, h - 1), min(x + rows_below, h - 1) + 1):
            for yy in range(max(y - cols_left, 0), y + 1):
                for kk in range(3):
                    if V[xx, 3 * yy + kk] != v or src_x[xx, yy, kk] >= 0:
                        continue
                    if kk in holding:
                        return xx, yy, kk
                    if first is None:
                        first = (xx, yy, kk)
        return first

    pixels = sorted((int(A[x, y]), x, y) for x in range(h) for y in range(w))
    for area, x0, y0 in pixels:
        for k0 in range(3):
            if src_x[x0, y0, k0] >= 0:
                continue
            v = int(V[x0, 3 * y0 + k0])
            holding = {}                        # channel -> pixel of view v lent to it
            x, y, k = x0, y0, k0
            while True:
                if k in holding:                # show a lent pixel (Eq. (13))
                    src_x[x, y, k], src_y[x, y, k] = holding.pop(k)
                else:                           # show the own pixel and lend it (Eq. (11)-(12))
                    src_x[x, y, k], src_y[x, y, k] = x, y
                    for other in ((k + 1) % 3, (k + 2) % 3):
                        holding[other] = (x, y)
                nxt = next_in_window(x, y, v, holding)
                if nxt is None or A[nxt[0], nxt[1]] != area:
                    break
                x, y, k = nxt
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


# ---- the compiled walk (full-size panels) ----

def build(force: bool = False) -> str:
    """Compile srwalk.cpp (g++ -O3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _clib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        _lib.dlo_repurpose.argtypes = [ctypes.c_int] * 3 + [i64] * 6 + [ctypes.c_int, P, P]
        _lib.dlo_repurpose.restype = ctypes.c_int
        _lib.dlo_count_rays.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.dlo_count_rays.restype = i64
    return _lib


def repurpose_map_full(width: int, height: int, n_views: int, tan_slant, pitch, offset=0, pw: int = 2):
    """The same map by the compiled walk: returns (V[h, 3w] uint8, src[h, w, 3] int32 = x' w + y')."""
    ts, L, K = Fraction(tan_slant), Fraction(pitch), Fraction(offset)
    V = np.empty((height, 3 * width), dtype=np.uint8)
    src = np.empty((height, width, 3), dtype=np.int32)
    rc = _clib().dlo_repurpose(width, height, n_views, ts.numerator, ts.denominator, L.numerator, L.denominator,
                               K.numerator, K.denominator, pw, V.ctypes.data, src.ctypes.data)
    if rc != 0:
        raise ValueError("panel parameters out of range for the compiled walk")
    return V, src


def beta(width: int, height: int, n_views: int, tan_slant, pitch, offset=0, pw: int = 2) -> float:
    """Rendered pixel ratio: distinct rays / (w h) (Sec. "Subpixel Repurposing"; 3 for the identity map when the
    three subpixels of every pixel belong to three views)."""
    V, src = repurpose_map_full(width, height, n_views, tan_slant, pitch, offset, pw)
    n = _clib().dlo_count_rays(width, height, V.ctypes.data, src.ctypes.data)
    if n < 0:
        raise AssertionError("a source pixel does not show its subpixel's view")
    return n / (width * height)
