"""Oracle (test infrastructure only): lenticular view map, Eq. (1)-(3), and interlacing, Alg. 1.

Nothing in the product imports this module; only tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.

Definitions followed (paper Sec. 3.1, "Interlacing and Display"):

* Eq. (1): d_offset = 3*y + 3*x*tan(alpha) + k - K_offset, for the subpixel in row x, pixel column y,
  colour channel k, measured in subpixel widths (a subpixel is 1 wide and 3 tall).
* Eq. (2): x_offset = d_offset mod L_x, which the text confines to [0, L_x) (a floored modulo, so that
  negative d_offset from negative slants or offsets still lands in that interval).
* Eq. (3): v = floor(N_v * x_offset / L_x).  The formula is 0-based; the prose calls the first slot
  "viewpoint 1".  We follow the formula: v in [0, N_v).

The parameters tan(alpha), L_x and K_offset are exact rationals, and the arithmetic is exact: evaluated in
binary floating point, Eq. (2)-(3) misassign subpixels that sit exactly on a lens boundary, which rational
panels hit systematically.

Alg. 1: M_e[x, y, k] = M_m[V[x, 3y + k], x, y, k] with the views already at panel resolution (the Resize
step is the identity here).
"""
from __future__ import annotations

from fractions import Fraction
from math import floor

import numpy as np


def view_of_subpixel(x: int, y: int, k: int, n_views: int, tan_slant: Fraction, pitch: Fraction,
                     offset: Fraction) -> int:
    """Eq. (1)-(3) evaluated literally with Python Fractions (the plain definition)."""
    d_offset = 3 * y + 3 * x * Fraction(tan_slant) + k - Fraction(offset)     # Eq. (1)
    L = Fraction(pitch)
    x_offset = d_offset - L * floor(d_offset / L)                              # Eq. (2), in [0, L)
    assert 0 <= x_offset < L
    return floor(n_views * x_offset / L)                                        # Eq. (3)


def view_map_fraction(width: int, height: int, n_views: int, tan_slant, pitch, offset=0) -> np.ndarray:
    """V[h, 3w] by the literal Fraction definition (slow: tiny panels and samples only)."""
    V = np.empty((height, 3 * width), dtype=np.int64)
    for x in range(height):
        for s in range(3 * width):
            V[x, s] = view_of_subpixel(x, s // 3, s % 3, n_views, tan_slant, pitch, offset)
    return V


def view_map(width: int, height: int, n_views: int, tan_slant, pitch, offset=0) -> np.ndarray:
    """V[h, 3w] (uint8 when N_v <= 256) by exact integer arithmetic.

    With tan(alpha) = a/b, L_x = p/q, K = r/s, multiply Eq. (1) by the common denominator b*s:
    D = (3y + k)*b*s + 3x*a*s - r*b.  Then d_offset / L_x = D*q / (b*s*p), so with Q = b*s*p the
    fractional part of d_offset / L_x is ((D*q) mod Q) / Q and Eq. (3) is v = (N * ((D*q) mod Q)) // Q.
    Python integers are unbounded, so rows are evaluated with object-free int64 only when safe.
    """
    ts, L, K = Fraction(tan_slant), Fraction(pitch), Fraction(offset)
    a, b = ts.numerator, ts.denominator
    p, q = L.numerator, L.denominator
    r, s = K.numerator, K.denominator
    Q = b * s * p
    # bound |D*q| and N*Q to stay inside int64
    maxD = (3 * width) * b * s + 3 * height * abs(a) * s + abs(r) * b
    if maxD * q >= 2 ** 62 or n_views * Q >= 2 ** 62:
        raise OverflowError("view map parameters exceed exact int64 evaluation")
    sub = np.arange(3 * width, dtype=np.int64)          # s = 3y + k
    rows = np.arange(height, dtype=np.int64)
    D = sub[None, :] * (b * s) + rows[:, None] * (3 * a * s) - r * b
    rho = np.mod(D * q, Q)                               # numpy mod is floored for a positive modulus
    V = (n_views * rho) // Q
    return V.astype(np.uint8 if n_views <= 256 else np.int64)


def resize_bilinear(img: np.ndarray, out_h: int, out_w: int) -> np.ndarray:
    """Alg. 1's Resize (the paper names no filter; this build reads it as bilinear): img[h, w, c] ->
    [out_h, out_w, c] in FP64 with half-pixel centres: output row i samples input row (i + 1/2) h / out_h - 1/2,
    clamped at 0, between its floor and the next row (the last row repeats); columns alike."""
    h, w = img.shape[:2]

    def axis(n_out, n_in):
        src = np.maximum((np.arange(n_out) + 0.5) * (n_in / n_out) - 0.5, 0.0)
        i0 = np.minimum(np.floor(src).astype(np.int64), n_in - 1)
        i1 = np.minimum(i0 + 1, n_in - 1)
        return i0, i1, src - i0

    r0, r1, ly = axis(out_h, h)
    c0, c1, lx = axis(out_w, w)
    a = img[r0][:, c0].astype(np.float64)
    b = img[r0][:, c1].astype(np.float64)
    c = img[r1][:, c0].astype(np.float64)
    d = img[r1][:, c1].astype(np.float64)
    ly = ly[:, None, None]
    lx = lx[None, :, None]
    return (1 - ly) * ((1 - lx) * a + lx * b) + ly * ((1 - lx) * c + lx * d)


def interleave(views: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Alg. 1: views[N, h, w, 3] and V[h, 3w] -> encoded image M_e[h, w, 3]."""
    n, h, w, _ = views.shape
    out = np.empty((h, w, 3), dtype=views.dtype)
    for k in range(3):
        vk = V[:, k::3].astype(np.int64)                 # view of subpixel (x, 3y + k)
        xs, ys = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        out[:, :, k] = views[vk, xs, ys, k]
    return out


def subpixel_rays(V: np.ndarray):
    """The ray of each subpixel (x, y, k): (v, x, y) with v = V[x, 3y + k] (paper Sec. 5: a subpixel is the
    ray from the camera of view v through pixel (x, y) of that view; channel k is kept).

    Returns (ray_v, ray_x, ray_y) of all distinct rays and ``index[h, w, 3]`` mapping each subpixel to its
    ray.  Two subpixels of one pixel share a ray only when they fall into the same view."""
    h, w3 = V.shape
    w = w3 // 3
    Vi = V.astype(np.int64).reshape(h, w, 3)
    xs = np.broadcast_to(np.arange(h)[:, None, None], (h, w, 3))
    ys = np.broadcast_to(np.arange(w)[None, :, None], (h, w, 3))
    code = (Vi * h + xs) * w + ys
    uniq, inv = np.unique(code.ravel(), return_inverse=True)
    ray_y = uniq % w
    ray_x = (uniq // w) % h
    ray_v = uniq // (w * h)
    return ray_v, ray_x, ray_y, inv.reshape(h, w, 3)
