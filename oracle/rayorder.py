"""Oracle (test infrastructure only): ray-order 3DGS, Alg. 3 of the paper (Sec. "Ray-Order 3DGS"), in FP64.

Nothing in the product imports this module; only tests use it.

For a ray with origin o and unit direction d, and a Gaussian j with mean mu, covariance
Sigma = R S S^T R^T (R from the normalised quaternion (w, x, y, z), S = diag(exp(log-scale)), Eq. (8)) and
opacity o_j = sigmoid(logit):
* t_j = (mu - o)^T Sigma^-1 d / (d^T Sigma^-1 d), where the Gaussian's response along the ray peaks (Eq. (22));
* alpha_j = o_j G(o + t_j d), G(x) = exp(-q/2) with q = (x - mu)^T Sigma^-1 (x - mu) (Eq. (23) with Eq. (7));
* its colour: real SH of degree <= 3 evaluated in the ray direction d, plus 0.5, clamped below at 0.
Every intersecting Gaussian is offered to a max-heap of capacity c_h keyed by t (a full heap replaces its
root when the new t is smaller); the heap's contents are sorted by t and alpha-blended front to back.

Readings of what the paper leaves open (each one a line of the design notes):
* "intersects": the Gaussian passes the rasterizer's per-pixel rule at its peak on the ray: t_j >= z_near (d of
  unit length), q_j <= q_cut and o_j exp(-q_j / 2) >= alpha_min.  The BVH only accelerates finding that set
  (every such peak lies inside the Gaussian's q <= min(q_cut, 2 ln(o_j / alpha_min)) ellipsoid, hence inside
  its leaf box), so brute force over all Gaussians in index order is the same set.
* equal t: the heap orders (t, Gaussian index) lexicographically.
* blending: alpha = min(alpha_max, alpha_j); the walk stops before a Gaussian whose blend would take the
  transmittance below t_min; the background is added with the final transmittance (the rasterizer's rules).
* origin and direction: the view's camera centre and the direction through the pixel centre (row x, column y
  at image point (y + 1/2, x + 1/2)) of that view's pinhole camera.

Decisions that FP32 arithmetic can take differently from FP64 (q at q_cut, alpha at alpha_min, t at z_near,
near-equal t among the blended Gaussians or at the heap's capacity, the transmittance at t_min) mark the ray
"fragile" when they can change the result: a threshold decision only for a Gaussian nearer than where the walk
ended.  Tests compare only rays without such a decision.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass

import numpy as np

from . import render as orender

# relative bands of the fragile decisions (FP32 error of the GPU's peak, quadratic form and blend, with margin)
BAND_Q = 1e-4
BAND_T = 1e-5
BAND_STOP = 1e-3


def rotation(quats: np.ndarray) -> np.ndarray:
    """R[n, 3, 3] of unit quaternions (w, x, y, z) (normalised here)."""
    q = np.asarray(quats, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((len(q), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def gaussians(scene):
    """(mu[n, 3], Sigma^-1[n, 3, 3], opacity[n], sh[n, 16, 3]) in FP64 from the scene's FP32 parameters."""
    mu = np.asarray(scene.means, dtype=np.float32).astype(np.float64)
    s = np.exp(np.asarray(scene.log_scales, dtype=np.float32).astype(np.float64))
    R = rotation(np.asarray(scene.quats, dtype=np.float32).astype(np.float64))
    inv = np.einsum("nij,nj,nkj->nik", R, 1.0 / (s * s), R)          # R S^-2 R^T
    lg = np.asarray(scene.opacity_logits, dtype=np.float32).astype(np.float64).reshape(-1)
    op = 1.0 / (1.0 + np.exp(-lg))
    sh = np.asarray(scene.sh, dtype=np.float32).astype(np.float64).reshape(-1, 16, 3)
    return mu, inv, op, sh


def peak(mu, inv, o, d):
    """Eq. (22)-(23) for every Gaussian and one ray: (t[n], q[n]) with q the quadratic form at the peak."""
    diff = mu - o                                    # mu - o
    Ad = inv @ d                                     # Sigma^-1 d  [n, 3]
    den = Ad @ d                                     # d^T Sigma^-1 d
    t = np.einsum("ni,ni->n", diff, Ad) / den        # Eq. (22)
    r = o + t[:, None] * d - mu                      # o + t d - mu
    q = np.einsum("ni,nij,nj->n", r, inv, r)
    return t, q


@dataclass
class RayOut:
    rgb: np.ndarray       # [n, 3]
    hits: np.ndarray      # [n] intersecting Gaussians
    blended: np.ndarray   # [n] Gaussians blended (after the heap and the transmittance stop)
    fragile: np.ndarray   # [n] bool


def ray_dirs(display, cams, ray_v, ray_x, ray_y):
    """Origins and unit directions of rays (view v, pixel row x, column y)."""
    R, _, eye = cams
    f, cx, cy = orender.intrinsics(display)
    v = np.asarray(ray_v, dtype=np.int64)
    cam = np.stack([(np.asarray(ray_y) + 0.5 - cx) / f, (np.asarray(ray_x) + 0.5 - cy) / f,
                    np.ones(len(v))], axis=1)
    d = np.einsum("nji,nj->ni", R[v], cam)           # R^T (camera -> world)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return eye[v], d


def trace(scene, origins, dirs, heap_cap: int, opts: orender.Opts = None) -> RayOut:
    """Alg. 3 for each ray (origins[n, 3], unit dirs[n, 3])."""
    opts = opts or orender.Opts()
    mu, inv, op, sh = gaussians(scene)
    n = len(origins)
    rgb = np.zeros((n, 3))
    hits = np.zeros(n, dtype=np.int64)
    blended = np.zeros(n, dtype=np.int64)
    fragile = np.zeros(n, dtype=bool)
    Y = orender.sh_basis(np.asarray(dirs, dtype=np.float64), opts.sh_degree)     # [n, 16]
    a_min, q_cut = opts.alpha_min, opts.q_cut
    for r in range(n):
        o, d = np.asarray(origins[r], np.float64), np.asarray(dirs[r], np.float64)
        t, q = peak(mu, inv, o, d)
        a = op * np.exp(-0.5 * q)
        front = t >= opts.z_near
        hit = front & (q <= q_cut) & (a >= a_min)                                 # IntersectsBVH
        heap = []                                                                 # max-heap of (t, j) via negation
        for j in np.nonzero(hit)[0]:
            key = (float(t[j]), int(j))
            if len(heap) == heap_cap:
                if key < (-heap[0][0], -heap[0][1]):                              # t < Getmax(h)
                    heapq.heapreplace(heap, (-key[0], -key[1]))                   # Popmax + AddToHeap
            else:
                heapq.heappush(heap, (-key[0], -key[1]))
        kept = sorted((-a_, -b_) for a_, b_ in heap)                              # Sort(h)
        hits[r] = int(hit.sum())
        T = 1.0
        C = np.zeros(3)
        fr = False
        t_end = np.inf            # hits beyond this distance cannot change the result
        for i, (tj, j) in enumerate(kept):                                        # AlphaBlending
            alpha = min(opts.alpha_max, float(a[j]))
            nt = T * (1.0 - alpha)
            if abs(nt - opts.t_min) <= BAND_STOP * opts.t_min:
                fr = True
            if nt < opts.t_min:
                t_end = tj
                break
            col = np.maximum(Y[r] @ sh[j] + 0.5, 0.0)                             # CalculateFromSHS(d, g)
            C += T * alpha * col
            T = nt
            blended[r] += 1
        else:
            if len(kept) == heap_cap:                                             # the capacity ended the walk
                t_end = kept[-1][0]
                if hits[r] > heap_cap:
                    rest = np.sort(t[hit])
                    if rest[heap_cap] - rest[heap_cap - 1] <= BAND_T * abs(rest[heap_cap]):
                        fr = True
        rgb[r] = C + T * np.asarray([orender.f32(b) for b in opts.bg])
        # threshold decisions FP32 could take the other way, on Gaussians that would change the blended prefix
        near = t <= t_end * (1 + BAND_T)
        fr = fr or bool(np.any(near & front & (np.abs(q - q_cut) <= BAND_Q * q_cut) & (a >= a_min * (1 - BAND_Q)))
                        or np.any(near & front & (np.abs(a / a_min - 1) <= BAND_Q) & (q <= q_cut * (1 + BAND_Q)))
                        or np.any(near & (np.abs(t - opts.z_near) <= BAND_T * opts.z_near) & (q <= q_cut)
                                  & (a >= a_min)))
        ts = np.array([k[0] for k in kept[:blended[r] + 1]])
        if len(ts) > 1 and np.any(np.diff(ts) <= BAND_T * np.abs(ts[1:])):
            fr = True
        fragile[r] = fr
    return RayOut(rgb, hits, blended, fragile)


def render_rays(scene, display, c2w, ray_v, ray_x, ray_y, heap_cap: int, opts: orender.Opts = None,
                converge_dist=None) -> RayOut:
    """Alg. 3 for the rays (view, pixel row, pixel column) of the display's rig at pose c2w."""
    cams = orender.cameras_for(display, c2w, converge_dist)
    o, d = ray_dirs(display, cams, ray_v, ray_x, ray_y)
    return trace(scene, o, d, heap_cap, opts)
