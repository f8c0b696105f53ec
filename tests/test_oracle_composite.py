"""Pins of the oracle's per-ray compositing (Eq. (5)-(6), (10)) and the DirectL = "N views + Alg. 1"
invariant, CPU only."""
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import render, viewmap
from paper_2407_14053_amd import synth

C0 = 1.0 / (2.0 * np.sqrt(np.pi))


def _scene(means, log_sigma, logits, rgb):
    n = len(means)
    sh = np.zeros((n, 16, 3), np.float32)
    sh[:, 0, :] = (np.asarray(rgb, np.float64) - 0.5) / C0
    return synth.Scene(np.asarray(means, np.float32), np.full((n, 3), log_sigma, np.float32),
                       np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), np.asarray(logits, np.float32), sh)


def _one_view_display(w=15, h=15, focal=60.0):
    return synth.Display(w, h, 1, Fraction(1, 3), Fraction(53, 10), Fraction(0), 0.0, focal)


def _logit(o):
    return float(np.log(o / (1 - o)))


def _ray(sc, d, x, y, opts=None):
    res = render.render_rays(sc, d, synth.pose_front(3.0), [0], [x], [y], opts)
    return res


def _rec(sc, d):
    from oracle import rig
    R, t, e = rig.cameras(synth.pose_front(3.0), 3.0, 0.0, 1)
    return render.project(sc, R[0], t[0], e[0], d.focal_px, d.width / 2, d.height / 2)


def test_single_gaussian_closed_form():
    d = _one_view_display(16, 16)
    o = 0.8
    sc = _scene([[0, 0, 0]], np.log(0.05), [_logit(o)], [[0.9, 0.2, 0.4]])
    rec = _rec(sc, d)
    s2 = rec[0, 10]
    rgb = sc.sh[0, 0].astype(np.float64) * C0 + 0.5
    for (x, y) in [(8, 8), (7, 8), (9, 10), (8, 5)]:
        r2 = (y + 0.5 - 8.0) ** 2 + (x + 0.5 - 8.0) ** 2
        alpha = min(float(np.float32(0.99)), float(np.float32(o)) * np.exp(-r2 / (2 * s2)))
        q = r2 / s2
        exp_c = alpha * rgb if (q <= 9 and alpha >= float(np.float32(1 / 255))) else 0 * rgb
        assert np.allclose(_ray(sc, d, x, y).prim[0], exp_c, atol=1e-12), (x, y)


def test_two_gaussians_front_to_back_and_swap():
    d = _one_view_display()
    o1, o2 = 0.6, 0.7
    c1, c2 = [0.9, 0.1, 0.2], [0.1, 0.8, 0.3]
    a1, a2 = float(np.float32(o1)), float(np.float32(o2))
    sc = _scene([[0, 0, 0.5], [0, 0, -0.5]], np.log(0.05), [_logit(o1), _logit(o2)], [c1, c2])
    cc1 = sc.sh[0, 0].astype(np.float64) * C0 + 0.5
    cc2 = sc.sh[1, 0].astype(np.float64) * C0 + 0.5
    got = _ray(sc, d, 7, 7).prim[0]          # pixel centre = principal point: q = 0, alpha = o
    assert np.allclose(got, a1 * cc1 + (1 - a1) * a2 * cc2, atol=1e-12)
    sc.means[:, 2] *= -1                     # swap depths
    got = _ray(sc, d, 7, 7).prim[0]
    assert np.allclose(got, a2 * cc2 + (1 - a2) * a1 * cc1, atol=1e-12)


def test_stack_terminates_before_transmittance_drops_below_t_min():
    """k identical Gaussians on the axis with alpha = 1/2: blending the j-th leaves T = 2^-j; the walk
    stops before the first j with 2^-j < 1e-4, i.e. after 13 blends: C = c (1 - 2^-13)."""
    d = _one_view_display()
    k = 20
    means = [[0, 0, 0.4 - 0.04 * i] for i in range(k)]
    sc = _scene(means, np.log(0.05), [0.0] * k, [[0.7, 0.3, 0.5]] * k)
    res = _ray(sc, d, 7, 7)
    c = sc.sh[0, 0].astype(np.float64) * C0 + 0.5
    assert res.info[0, 2] == 13
    assert np.allclose(res.prim[0], c * (1 - 0.5 ** 13), atol=1e-12)


def test_alpha_and_ellipse_thresholds_exclude():
    d = _one_view_display()
    # opacity just below / above 1/255 at q = 0
    for o, blended in [(0.0039, False), (0.0040, True)]:
        sc = _scene([[0, 0, 0]], np.log(0.05), [_logit(o)], [[0.9, 0.9, 0.9]])
        res = _ray(sc, d, 7, 7)
        assert (res.info[0, 2] == 1) == blended
    # pixel at q = 8.5 (in) and q = 9.5 (out) of a wide Gaussian: place the mean off the pixel centre
    sc = _scene([[0, 0, 0]], np.log(0.1), [_logit(0.99)], [[0.9, 0.9, 0.9]])
    s2 = _rec(sc, d)[0, 10]
    f = d.focal_px
    for q, blended in [(8.5, True), (9.5, False)]:
        off_px = np.sqrt(q * s2)                 # along the image x axis
        sc.means[0, 0] = np.float32(-off_px * 3.0 / f)   # world x maps to +image x
        s2b = _rec(sc, d)[0, 10]
        u = _rec(sc, d)[0, 0]
        qq = (7.5 - u) ** 2 / s2b
        res = _ray(sc, d, 7, 7)
        assert (res.info[0, 2] == 1) == (qq <= 9.0) == blended
        assert abs(qq - q) < 0.3


def test_near_plane_culls():
    d = _one_view_display()
    sc = _scene([[0, 0, 2.9], [0, 0, 2.7]], np.log(0.01), [_logit(0.9)] * 2, [[0.5, 0.5, 0.5]] * 2)
    res = _ray(sc, d, 7, 7)
    assert res.info[0, 2] == 1   # z = 0.1 culled, z = 0.3 blended


def test_fragile_threshold_yields_both_outcomes():
    """A Gaussian whose q at the pixel lies within the band around q_cut is explored both blended and not."""
    d = _one_view_display()
    sc = _scene([[0, 0, 0]], np.log(0.1), [_logit(0.99)], [[0.9, 0.9, 0.9]])
    f = d.focal_px
    s2 = _rec(sc, d)[0, 10]
    sc.means[0, 0] = np.float32(-np.sqrt(9.0 * s2) * 3.0 / f)
    rec = _rec(sc, d)
    q = (7.5 - rec[0, 0]) ** 2 / rec[0, 10]
    opts = render.Opts(band_q=abs(q - 9.0) / 9.0 * 2 + 1e-9)
    res = _ray(sc, d, 7, 7, opts)
    outs = res.var[0, :res.nvar[0]]
    assert res.nvar[0] >= 2
    assert np.any(np.all(outs == 0, axis=1)) and np.any(np.all(outs > 0, axis=1))


def test_brute_force_small_panel_with_scipy_gaussian_density():
    """Each subpixel recomposited in Python: alpha from scipy's 2D normal density of the projected Gaussian
    (o * 2 pi sqrt(det S') * pdf), per-pixel rule, depth sort, front-to-back blend with early stop."""
    d = synth.Display(24, 16, 6, Fraction(1, 3), Fraction(53, 10), Fraction(0), 0.3, 30.0)
    sc = synth.scene_uniform(40, 1.0, 21)
    sc.log_scales += 1.2
    c2w = synth.pose_front(3.0)
    img, res, index = render.render_directl(sc, d, c2w)
    V = render.view_map_of(d)
    R, t, e = render.cameras_for(d, c2w)
    recs = [render.project(sc, R[v], t[v], e[v], d.focal_px, d.width / 2, d.height / 2) for v in range(6)]
    opts = render.Opts()
    for x in range(d.height):
        for y in range(d.width):
            for k in range(3):
                v = int(V[x, 3 * y + k])
                rec = recs[v]
                cand = []
                for i in range(sc.n):
                    if rec[i, 9] <= opts.z_near:
                        continue
                    S = np.array([[rec[i, 10], rec[i, 11]], [rec[i, 11], rec[i, 12]]])
                    p = np.array([y + 0.5, x + 0.5])
                    g = multivariate_normal(mean=rec[i, :2], cov=S).pdf(p) * 2 * np.pi * np.sqrt(np.linalg.det(S))
                    diff = p - rec[i, :2]
                    q = diff @ np.linalg.solve(S, diff)
                    a = min(opts.alpha_max, rec[i, 5] * g)
                    if q <= opts.q_cut and a >= opts.alpha_min:
                        cand.append((rec[i, 9], i, a, rec[i, 6 + k]))
                cand.sort()
                T, C = 1.0, 0.0
                for _, _, a, c in cand:
                    if T * (1 - a) < opts.t_min:
                        break
                    C += a * T * c
                    T *= 1 - a
                assert abs(img[x, y, k] - C) < 1e-10, (x, y, k)


@pytest.mark.parametrize("name", ["tiny", "fd64"])
def test_directl_equals_views_then_interleave(name):
    """The paper's invariant (Table 3 "Required Only" = HR, RMSE 0): rendering only each subpixel's ray
    gives exactly Alg. 1 applied to the N full views."""
    d = synth.make_named_display(name)
    sc = synth.make_scene("tiny" if name == "tiny" else "fd64")
    c2w = synth.pose_sweep(7)[2]
    img, res, index = render.render_directl(sc, d, c2w)
    views = render.render_views(sc, d, c2w)
    enc = viewmap.interleave(views, render.view_map_of(d))
    assert np.array_equal(img, enc)
    assert res.info[:, 0].sum() == 0


def _alpha_at(rec, i, px, py):
    dx, dy = px - rec[i, 0], py - rec[i, 1]
    q = rec[i, 2] * dx * dx + 2 * rec[i, 3] * dx * dy + rec[i, 4] * dy * dy
    return min(float(np.float32(0.99)), rec[i, 5] * np.exp(-0.5 * q))


def test_near_tie_group_admits_every_order():
    """Three Gaussians whose depths differ by less than the depth band (2^-30 relative) form one near-tie group:
    the order among them is not defined at the renderer's depth precision, so the composite of each of the 3!
    orders is among the admissible outcomes, and the exact FP64 order gives the primary one."""
    from itertools import permutations
    d = _one_view_display()
    mz = [0.0, 2e-9, 4e-9]            # camera depths 3, 3 - 2e-9, 3 - 4e-9: adjacent gaps below 2^-30 * 3
    sc = _scene([[0, 0, z] for z in mz], np.log(0.2), [_logit(0.5), _logit(0.6), _logit(0.7)],
                [[0.9, 0.1, 0.1], [0.1, 0.9, 0.1], [0.1, 0.1, 0.9]])
    rec = _rec(sc, d)
    assert len(set(rec[:, 9])) == 3
    res = _ray(sc, d, 7, 7)
    assert res.info[0, 0] == 0 and res.info[0, 3] == 1
    outs = res.var[0, :res.nvar[0]]
    a = [_alpha_at(rec, i, 7.5, 7.5) for i in range(3)]
    comps = []
    for perm in permutations(range(3)):
        T, C = 1.0, np.zeros(3)
        for i in perm:
            C += a[i] * T * rec[i, 6:9]
            T *= 1 - a[i]
        comps.append(C)
        assert np.abs(outs - C[None, :]).max(axis=1).min() < 1e-12, perm
    exact = comps[list(permutations(range(3))).index(tuple(np.argsort(rec[:, 9], kind="stable")))]
    assert np.allclose(res.prim[0], exact, atol=1e-12)
    # the six orders give six different colours, so the check above is not vacuous
    assert min(np.abs(comps[i] - comps[j]).max() for i in range(6) for j in range(i)) > 1e-3


def test_near_tie_behind_terminated_walk_is_not_explored():
    """A near-tie pair behind three opaque Gaussians that end the walk (T would fall below t_min) cannot change
    the composite, so it is neither explored nor counted; in front of them it is."""
    d = _one_view_display()
    rgb = [[0.9, 0.1, 0.1], [0.1, 0.9, 0.1], [0.5, 0.5, 0.5], [0.3, 0.2, 0.1], [0.2, 0.3, 0.4]]
    for stack_z, explored in [(0.5, False), (-0.5, True)]:
        # the pair at camera depths 3 and 3 - 2e-9, the stack at 2.5-2.7 (in front) or 3.3-3.5 (behind)
        mz = [stack_z, stack_z * 0.8, stack_z * 0.6, 0.0, 2e-9]
        sc = _scene([[0, 0, z] for z in mz], np.log(0.3), [_logit(0.98)] * 3 + [_logit(0.5)] * 2, rgb)
        res = _ray(sc, d, 7, 7)
        assert res.info[0, 0] == 0
        assert res.info[0, 3] == (1 if explored else 0), stack_z
        assert (res.nvar[0] >= 2) == explored
