"""Oracle ray-order 3DGS (Alg. 3, Eq. (22)-(23)) pinned by what mathematics and the paper fix: the peak t_j
minimises the quadratic form along the ray (checked by a numerical minimiser), alpha_j is the maximum of
o_j G along the ray (checked by dense sampling), the covariance matches scipy's rotation of the quaternion, the
heap keeps exactly the c_h nearest hits (checked against a full sort), and blends of hand-placed Gaussians have
closed forms."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.transform import Rotation

from oracle import rayorder as RO
from oracle import render as orender
from paper_2407_14053_amd import synth


def _scene(means, log_scales, quats, logits, sh):
    return synth.Scene(np.asarray(means, np.float32), np.asarray(log_scales, np.float32),
                       np.asarray(quats, np.float32), np.asarray(logits, np.float32).reshape(-1, 1),
                       np.asarray(sh, np.float32).reshape(-1, 16, 3))


def _random_scene(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    return _scene(rng.uniform(-spread, spread, (n, 3)), rng.uniform(-3.0, -1.0, (n, 3)), rng.normal(size=(n, 4)),
                  rng.uniform(-1.0, 4.0, n), rng.normal(0, 0.3, (n, 16, 3)))


def test_covariance_matches_scipy_rotation():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(20, 4))
    s = np.exp(rng.uniform(-3, 0, (20, 3)))
    sc = _scene(np.zeros((20, 3)), np.log(s), q, np.zeros(20), np.zeros((20, 16, 3)))
    _, inv, _, _ = RO.gaussians(sc)
    for i in range(20):
        Rs = Rotation.from_quat(np.roll(np.asarray(q[i], np.float32).astype(np.float64), -1)).as_matrix()
        ss = np.exp(np.log(s[i]).astype(np.float32).astype(np.float64))
        Sigma = Rs @ np.diag(ss ** 2) @ Rs.T
        assert np.allclose(np.linalg.inv(inv[i]), Sigma, rtol=1e-9, atol=1e-12)


def test_peak_minimises_the_quadratic_form_along_the_ray():
    sc = _random_scene(30, 2)
    mu, inv, op, _ = RO.gaussians(sc)
    rng = np.random.default_rng(3)
    for _ in range(5):
        o = rng.uniform(-3, 3, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t, q = RO.peak(mu, inv, o, d)
        for j in range(30):
            Sig = np.linalg.inv(inv[j])
            f = lambda s: float((o + s * d - mu[j]) @ np.linalg.solve(Sig, o + s * d - mu[j]))
            lo = float((mu[j] - o) @ d) - 20.0
            res = minimize_scalar(f, bounds=(lo, lo + 40.0), method="bounded", options={"xatol": 1e-12})
            assert abs(res.x - t[j]) < 1e-6 * max(1.0, abs(t[j]))
            assert abs(res.fun - q[j]) < 1e-9 * max(1.0, q[j])


def test_alpha_is_the_maximum_response_along_the_ray():
    sc = _random_scene(10, 4, spread=0.3)
    mu, inv, op, _ = RO.gaussians(sc)
    o = np.array([0.05, -0.02, -2.0])
    d = np.array([0.01, 0.02, 1.0])
    d /= np.linalg.norm(d)
    t, q = RO.peak(mu, inv, o, d)
    s = np.linspace(0.0, 4.0, 400001)
    for j in range(10):
        x = o[None, :] + s[:, None] * d[None, :] - mu[j]
        G = np.exp(-0.5 * np.einsum("ni,ij,nj->n", x, inv[j], x))
        assert abs(op[j] * G.max() - op[j] * np.exp(-0.5 * q[j])) < 1e-8


def test_isotropic_closed_form():
    # sigma = 0.1 everywhere, mean off the ray by 0.15 perpendicular: t = (mu - o) . d, q = 0.15^2 / 0.01
    sc = _scene([[0.15, 0.0, 1.0]], [[np.log(0.1)] * 3], [[1, 0, 0, 0]], [0.0], np.zeros((1, 16, 3)))
    mu, inv, op, _ = RO.gaussians(sc)
    t, q = RO.peak(mu, inv, np.zeros(3), np.array([0.0, 0.0, 1.0]))
    s64 = np.exp(float(np.float32(np.log(0.1))))   # exp in FP64 of the FP32 log-scale
    assert abs(t[0] - float(np.float32(1.0))) < 1e-12
    assert abs(q[0] - float(np.float32(0.15)) ** 2 / s64 ** 2) < 1e-12


def test_direction_length_does_not_change_peak_point_or_alpha():
    sc = _random_scene(20, 5)
    mu, inv, op, _ = RO.gaussians(sc)
    o = np.array([0.3, 0.1, -2.5])
    d = np.array([0.1, -0.2, 1.0])
    t1, q1 = RO.peak(mu, inv, o, d)
    t2, q2 = RO.peak(mu, inv, o, 2.5 * d)
    assert np.allclose(t1, 2.5 * t2, rtol=1e-12) and np.allclose(q1, q2, rtol=1e-10, atol=1e-12)


def _dc_sh(rgb):
    sh = np.zeros((len(rgb), 16, 3))
    sh[:, 0, :] = (np.asarray(rgb) - 0.5) / 0.28209479177387814
    return sh


def test_two_gaussians_on_the_axis_closed_form_and_capacity_one():
    # two small isotropic Gaussians centred on the ray at z = 1 and z = 2, DC colours; alpha = sigmoid(logit)
    logits = np.array([0.3, 1.2], np.float32)
    sc = _scene([[0, 0, 2.0], [0, 0, 1.0]], [[np.log(0.05)] * 3] * 2, [[1, 0, 0, 0]] * 2, logits,
                _dc_sh([[0.9, 0.1, 0.2], [0.2, 0.7, 0.4]]))
    o, d = np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]])
    a = 1.0 / (1.0 + np.exp(-logits.astype(np.float64)))
    _, _, _, sh = RO.gaussians(sc)
    col = sh[:, 0, :] * 0.28209479177387814 + 0.5
    out = RO.trace(sc, o, d, heap_cap=8)
    exp = a[1] * col[1] + (1 - a[1]) * a[0] * col[0]                # nearer one (index 1) first
    assert np.allclose(out.rgb[0], exp, atol=1e-12) and out.hits[0] == 2 and out.blended[0] == 2
    out1 = RO.trace(sc, o, d, heap_cap=1)                            # c_h = 1 keeps only the nearest
    assert np.allclose(out1.rgb[0], a[1] * col[1], atol=1e-12) and out1.blended[0] == 1


def test_transmittance_stop_closed_form():
    # five Gaussians of alpha 0.9 centred on the ray: T = 0.1 after the first, 0.01 after the second, and the
    # third would take it to 0.001 < t_min = 0.005: the walk stops there
    opts = orender.Opts(t_min=orender.f32(0.005))
    lg = np.float32(np.log(9.0))
    sc = _scene([[0, 0, 1.0 + 0.5 * i] for i in range(5)], [[np.log(0.05)] * 3] * 5, [[1, 0, 0, 0]] * 5,
                [lg] * 5, _dc_sh([[0.5 + 0.1 * i, 0.3, 0.2] for i in range(5)]))
    out = RO.trace(sc, np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), heap_cap=16, opts=opts)
    a = 1.0 / (1.0 + np.exp(-float(lg)))
    _, _, _, sh = RO.gaussians(sc)
    c = sh[:, 0, 0] * 0.28209479177387814 + 0.5
    exp = a * c[0] + (1 - a) * a * c[1]
    assert out.hits[0] == 5 and out.blended[0] == 2 and abs(out.rgb[0, 0] - exp) < 1e-12


@pytest.mark.parametrize("cap", [1, 3, 7, 16, 64])
def test_heap_keeps_the_nearest_hits(cap):
    """The heap's result equals blending the c_h smallest t of all hits, sorted (full sort, no heap)."""
    sc = synth.make_scene("tiny")
    d = synth.make_named_display("tiny")
    c2w = synth.pose_sweep(8)[1]
    rng = np.random.default_rng(cap)
    rv, rx, ry = rng.integers(0, d.n_views, 60), rng.integers(0, d.height, 60), rng.integers(0, d.width, 60)
    opts = orender.Opts()
    out = RO.render_rays(sc, d, c2w, rv, rx, ry, cap, opts)
    mu, inv, op, sh = RO.gaussians(sc)
    o, dirs = RO.ray_dirs(d, orender.cameras_for(d, c2w), rv, rx, ry)
    Y = orender.sh_basis(dirs, 3)
    for r in range(60):
        t, q = RO.peak(mu, inv, o[r], dirs[r])
        a = op * np.exp(-0.5 * q)
        hit = np.nonzero((t >= opts.z_near) & (q <= opts.q_cut) & (a >= opts.alpha_min))[0]
        order = hit[np.lexsort((hit, t[hit]))][:cap]
        T, C = 1.0, np.zeros(3)
        for j in order:
            al = min(opts.alpha_max, a[j])
            if T * (1 - al) < opts.t_min:
                break
            C += T * al * np.maximum(Y[r] @ sh[j] + 0.5, 0)
            T *= 1 - al
        assert np.allclose(out.rgb[r], C, atol=1e-12), r
    assert out.hits.max() > cap or cap == 64
