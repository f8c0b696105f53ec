"""Pins of the oracle's projection (Eq. (8)-(9)), opacity and SH colour, CPU only."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import expit, sph_harm_y

from oracle import render, rig
from paper_2407_14053_amd import synth


def _camera(eye=(0.3, -0.2, 3.0)):
    c2w = synth.look_at_c2w(eye)
    R, t, e = rig.cameras(c2w, float(np.linalg.norm(eye)), 0.0, 1)
    return R[0], t[0], e[0]


def _real_sh_scipy(dirs, degree=3):
    """Real SH without the Condon-Shortley phase, from scipy's complex harmonics (which include it)."""
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    out = np.zeros((len(dirs), 16))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            if m == 0:
                val = sph_harm_y(l, 0, theta, phi).real
            elif m > 0:
                val = np.sqrt(2) * (-1) ** m * sph_harm_y(l, m, theta, phi).real
            else:
                val = np.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, theta, phi).imag
            out[:, l * l + l + m] = val
    return out


def test_sh_basis_matches_scipy_real_harmonics():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = np.r_[d, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0]]]
    assert np.allclose(render.sh_basis(d), _real_sh_scipy(d), atol=1e-13)


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi integrates products of degree <= 6 exactly
    zs, wz = np.polynomial.legendre.leggauss(10)
    phis = np.arange(16) * 2 * np.pi / 16
    Z, P = np.meshgrid(zs, phis, indexing="ij")
    W = (wz[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).ravel()
    s = np.sqrt(1 - Z ** 2)
    dirs = np.stack([(s * np.cos(P)).ravel(), (s * np.sin(P)).ravel(), Z.ravel()], axis=1)
    Y = render.sh_basis(dirs)
    gram = (Y * W[:, None]).T @ Y
    assert np.allclose(gram, np.eye(16), atol=1e-12)


def test_quaternion_rotation_and_covariance_against_numeric_jacobian():
    """Sigma' must equal J_num R Sigma R^T J_num^T + h I with J_num the central-difference Jacobian of the
    perspective map world point -> (f X / Z + cx, f Y / Z + cy), Sigma from scipy's rotation."""
    rng = np.random.default_rng(11)
    G = 64
    sc = synth.scene_uniform(G, 1.0, 5)
    R, t, eye = _camera()
    f, cx, cy = 400.0, 160.0, 90.0
    opts = render.Opts()
    rec = render.project(sc, R, t, eye, f, cx, cy, opts)

    def proj(p):
        X = R @ p + t
        return np.array([f * X[0] / X[2] + cx, f * X[1] / X[2] + cy])

    for i in range(G):
        mu = sc.means[i].astype(np.float64)
        q = sc.quats[i].astype(np.float64)
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = Rq @ np.diag(np.exp(2 * sc.log_scales[i].astype(np.float64))) @ Rq.T
        h = 1e-5
        Jn = np.stack([(proj(mu + h * e) - proj(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        cov = Jn @ Sig @ Jn.T + opts.dilation * np.eye(2)
        got = np.array([[rec[i, 10], rec[i, 11]], [rec[i, 11], rec[i, 12]]])
        assert np.allclose(got, cov, rtol=1e-7, atol=1e-9)
        assert np.allclose(rec[i, :2], proj(mu), rtol=1e-13, atol=1e-10)
        conic = np.array([[rec[i, 2], rec[i, 3]], [rec[i, 3], rec[i, 4]]])
        assert np.allclose(conic @ got, np.eye(2), atol=1e-10)
        assert np.isclose(rec[i, 9], (R @ mu + t)[2], rtol=1e-14)
        assert np.isclose(rec[i, 5], expit(float(sc.opacity_logits[i])), rtol=1e-14)


def test_isotropic_on_axis_closed_form():
    """An isotropic Gaussian of std s on the optical axis at depth z projects to the principal point with
    Sigma' = ((f s / z)^2 + h) I."""
    s = 0.07
    sc = synth.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), np.log(s), np.float32),
                     np.array([[1, 0, 0, 0]], np.float32), np.zeros(1, np.float32), np.zeros((1, 16, 3), np.float32))
    R, t, eye = _camera((0.0, 0.0, 2.5))
    f = 300.0
    rec = render.project(sc, R, t, eye, f, 50.0, 40.0)
    sig2 = (f * float(np.float32(s)) / 2.5) ** 2 + float(np.float32(0.3))
    assert np.allclose(rec[0, :2], [50.0, 40.0], atol=1e-12)
    assert np.allclose(rec[0, 10:13], [sig2, 0.0, sig2], rtol=1e-6)


def test_colour_from_sh_in_camera_to_mean_direction():
    sc = synth.scene_uniform(200, 1.0, 9)
    R, t, eye = _camera()
    rec = render.project(sc, R, t, eye, 300.0, 50.0, 40.0)
    d = sc.means.astype(np.float64) - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = _real_sh_scipy(d)
    raw = np.einsum("gl,glc->gc", Y, sc.sh.astype(np.float64)) + 0.5
    assert np.allclose(rec[:, 13:16], raw, atol=1e-12)
    assert np.allclose(rec[:, 6:9], np.maximum(raw, 0.0), atol=1e-12)
    # DC only: rgb = dc / (2 sqrt(pi)) + 1/2
    sc.sh[:, 1:, :] = 0
    rec = render.project(sc, R, t, eye, 300.0, 50.0, 40.0)
    assert np.allclose(rec[:, 13:16], sc.sh[:, 0, :].astype(np.float64) / (2 * np.sqrt(np.pi)) + 0.5, atol=1e-14)
