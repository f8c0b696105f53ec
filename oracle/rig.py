"""Oracle (test infrastructure only): the multi-view camera rig in FP64.

Paper Sec. 3.1 ("Multiview Rendering"): N_v cameras evenly spaced, all aimed at the centre of the light
field, focal planes converging there; Eq. (17): each view's extrinsic is a rig transform applied to the
extrinsic L_0 of the light-field centre.

Reading of the unstated details:
* the centre camera's camera-to-world matrix (OpenCV axes: x right, y down, z forward) is the pose;
* camera v sits on the centre camera's right axis at s_v = baseline * (v / (N - 1) - 1/2) (view 0 is the
  leftmost, "baseline" is the distance between the outermost cameras; s_0 = 0 when N = 1);
* every camera is aimed (toe-in) at the convergence point eye_0 + converge_dist * forward_0, with the
  centre camera's down axis as the reference "down";
* intrinsics: square pixels, focal f in pixels, principal point (W/2, H/2); pixel (row x, column y) has its
  centre at image coordinates (y + 1/2, x + 1/2).
"""
from __future__ import annotations

import numpy as np


def _unit(v):
    return v / np.linalg.norm(v)


def cameras(c2w, converge_dist: float, baseline: float, n_views: int):
    """Returns (R[N,3,3], t[N,3], eye[N,3]): world-to-camera rotation rows (right, down, forward),
    translation t = -R eye, and camera centres."""
    c2w = np.asarray(c2w, dtype=np.float64)
    right0, down0, fwd0, eye0 = c2w[:3, 0], c2w[:3, 1], c2w[:3, 2], c2w[:3, 3]
    target = eye0 + converge_dist * fwd0
    R = np.empty((n_views, 3, 3))
    t = np.empty((n_views, 3))
    eyes = np.empty((n_views, 3))
    for v in range(n_views):
        s = baseline * (v / (n_views - 1) - 0.5) if n_views > 1 else 0.0
        eye = eye0 + s * right0
        fwd = _unit(target - eye)
        right = _unit(np.cross(down0, fwd))
        down = np.cross(fwd, right)
        R[v] = np.stack([right, down, fwd])
        t[v] = -R[v] @ eye
        eyes[v] = eye
    return R, t, eyes
