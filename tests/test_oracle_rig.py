"""Pins of the oracle's camera rig (Sec. 3.1 multiview rendering, Eq. (17)), CPU only."""
import numpy as np
import pytest

from oracle import rig
from paper_2407_14053_amd import synth


@pytest.mark.parametrize("n", [1, 2, 4, 8, 45, 60])
def test_rig_geometry(n):
    c2w = synth.look_at_c2w((0.4, -0.3, 3.1))
    conv = float(np.linalg.norm(c2w[:3, 3]))
    R, t, eye = rig.cameras(c2w, conv, 0.6, n)
    target = c2w[:3, 3] + conv * c2w[:3, 2]
    for v in range(n):
        # orthonormal, right-handed (right x down = forward)
        assert np.allclose(R[v] @ R[v].T, np.eye(3), atol=1e-14)
        assert np.isclose(np.linalg.det(R[v]), 1.0, atol=1e-14)
        assert np.allclose(np.cross(R[v][0], R[v][1]), R[v][2], atol=1e-14)
        # the optical axis passes through the convergence point
        p = R[v] @ target + t[v]
        assert abs(p[0]) < 1e-12 and abs(p[1]) < 1e-12 and p[2] > 0
        # t = -R eye
        assert np.allclose(R[v] @ eye[v] + t[v], 0, atol=1e-12)
        # cameras lie on the centre camera's horizontal (right) axis
        off = eye[v] - c2w[:3, 3]
        assert np.allclose(off, np.dot(off, c2w[:3, 0]) * c2w[:3, 0], atol=1e-14)
    if n > 1:
        # the outermost cameras are one baseline apart, view 0 on the left, spacing even
        assert np.isclose(np.linalg.norm(eye[-1] - eye[0]), 0.6, atol=1e-14)
        assert np.dot(eye[-1] - eye[0], c2w[:3, 0]) > 0
        gaps = np.linalg.norm(np.diff(eye, axis=0), axis=1)
        assert np.allclose(gaps, 0.6 / (n - 1), atol=1e-14)
    if n % 2 == 1:
        c = n // 2
        assert np.allclose(R[c], c2w[:3, :3].T, atol=1e-14)
        assert np.allclose(eye[c], c2w[:3, 3], atol=1e-14)
