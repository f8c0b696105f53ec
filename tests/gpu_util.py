"""Shared helpers of the GPU parity tests (inputs from the seeded generators, expected values from the
oracle only)."""
import sys

import numpy as np

from oracle import render as orender
from oracle import viewmap as oviewmap

TOL = 2e-4   # max |err| per colour channel on [0, 1]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sample_subpixels(h, w, n, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, h, n)
    ys = rng.integers(0, w, n)
    ks = rng.integers(0, 3, n)
    # corners and edges
    extra = [(0, 0), (0, w - 1), (h - 1, 0), (h - 1, w - 1), (h // 2, 0), (0, w // 2), (h - 1, w // 2),
             (h // 2, w - 1)]
    ex = np.array([e[0] for e in extra for _ in range(3)])
    ey = np.array([e[1] for e in extra for _ in range(3)])
    ek = np.array([k for _ in extra for k in range(3)])
    return np.r_[xs, ex], np.r_[ys, ey], np.r_[ks, ek]


def check_subpixels(scene, display, c2w, img, xs, ys, ks, opts=None, V=None, label="", src=None):
    """GPU image values at subpixels (xs, ys, ks) against the oracle's admissible outcomes of their rays: the
    ray of view V(x, 3y + k) through pixel (x, y), or through the pixel src = (src_x, src_y)[x, y, k] of a
    repurposed panel.  Returns (max error over rays within budget, number of over-budget rays, number of
    fragile rays)."""
    if V is None:
        V = orender.view_map_of(display)
    vs = V[xs, 3 * ys + ks].astype(np.int64)
    px, py = (xs, ys) if src is None else (src[0][xs, ys, ks], src[1][xs, ys, ks])
    code = (vs * display.height + px) * display.width + py
    uniq, inv = np.unique(code, return_inverse=True)
    rv = uniq // (display.width * display.height)
    rx = (uniq // display.width) % display.height
    ry = uniq % display.width
    res = orender.render_rays(scene, display, c2w, rv, rx, ry, opts)
    got = np.asarray(img)[xs, ys, ks].astype(np.float64)
    err = res.admissible_err_sub(got, inv, ks)
    over = res.info[inv, 0] > 0
    ok = ~over
    worst = float(err[ok].max()) if ok.any() else 0.0
    if worst > TOL:
        i = int(np.argmax(np.where(ok, err, -1)))
        log("%s worst subpixel (x=%d, y=%d, k=%d) view %d: gpu %.7f oracle %.7f nvar %d info %s" % (
            label, xs[i], ys[i], ks[i], vs[i], got[i], res.prim[inv[i], ks[i]], res.nvar[inv[i]],
            res.info[inv[i]]))
    return worst, int(over.sum()), int((res.info[inv, 1] > 0).sum())


def full_oracle_image(scene, display, c2w, opts=None):
    img, res, index = orender.render_directl(scene, display, c2w, opts)
    return img, res, index


def admissible_image_err(res, index, gpu_img):
    h, w, _ = index.shape
    ch = np.broadcast_to(np.arange(3)[None, None, :], index.shape)
    err = res.admissible_err_sub(np.asarray(gpu_img).reshape(-1), index.reshape(-1), ch.reshape(-1))
    over = res.info[index.reshape(-1), 0] > 0
    return err, over
