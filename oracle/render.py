"""Oracle (test infrastructure only): Python side of the FP64 CPU renderer in ``dlo.cpp``.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import this module; the
product path never does.

``Opts`` holds the rasterizer constants (z_near, q_cut, alpha_min, alpha_max, t_min, dilation, background)
as the same float32 values the GPU uses, widened exactly to FP64, plus the fragile-decision bands.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

from . import rig, viewmap

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dlo.cpp")
_LIB = os.path.join(_HERE, "libdlo.so")


def build(force: bool = False) -> str:
    """Compile the oracle (g++ -O2 -fopenmp, IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _COpts(ctypes.Structure):
    _fields_ = [("focal", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("z_near", ctypes.c_double), ("q_cut", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double), ("dilation", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("band_q", ctypes.c_double), ("band_a", ctypes.c_double),
                ("band_z", ctypes.c_double), ("band_znear", ctypes.c_double), ("eps_alpha", ctypes.c_double),
                ("eps_mul", ctypes.c_double), ("budget", ctypes.c_int32), ("sh_degree", ctypes.c_int32)]


_lib = None
MAX_VAR = 32   # admissible outcomes per ray (kMaxVar in dlo.cpp)


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.dlo_project.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, P]
        _lib.dlo_render_rays.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int32, P, P, P, P,
                                         ctypes.c_int64, P, P, P, P, P, P, P]
        _lib.dlo_backward_rays.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int32, P, P, P, P,
                                           ctypes.c_int64, P, P, P, P, P, P, P, P, P]
        _lib.dlo_sh_basis.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P]
        _lib.dlo_num_threads.restype = ctypes.c_int
    return _lib


def f32(x) -> float:
    return float(np.float32(x))


@dataclass
class Opts:
    """Rasterizer constants; defaults are the 3DGS conventions this build adopts (as float32 values)."""
    z_near: float = f32(0.2)
    q_cut: float = f32(9.0)
    alpha_min: float = f32(1.0 / 255.0)
    alpha_max: float = f32(0.99)
    t_min: float = f32(1e-4)
    dilation: float = f32(0.3)
    bg: tuple = (0.0, 0.0, 0.0)
    sh_degree: int = 3
    # fragile-decision bands (relative), derived from the FP32 error of the GPU's blend
    band_q: float = 2e-4
    band_a: float = 2e-4
    band_z: float = 2.0 ** -30
    band_znear: float = 1e-9
    eps_alpha: float = 3e-5
    eps_mul: float = 1e-6
    budget: int = 4

    def c(self, focal, cx, cy) -> _COpts:
        o = _COpts()
        o.focal, o.cx, o.cy = focal, cx, cy
        for k in ("z_near", "q_cut", "alpha_min", "alpha_max", "t_min", "dilation", "band_q", "band_a",
                  "band_z", "band_znear", "eps_alpha", "eps_mul"):
            setattr(o, k, float(getattr(self, k)))
        o.bg = (ctypes.c_double * 3)(*[f32(b) for b in self.bg])
        o.budget = int(self.budget)
        o.sh_degree = int(self.sh_degree)
        return o


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _scene_arrays(scene):
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in scene.arrays()]
    return arrs


def cameras_for(display, c2w, converge_dist=None):
    if converge_dist is None:
        converge_dist = float(np.linalg.norm(np.asarray(c2w)[:3, 3]))
    return rig.cameras(c2w, converge_dist, display.baseline, display.n_views)


def intrinsics(display):
    return display.focal_px, display.width / 2.0, display.height / 2.0


def project(scene, R, t, eye, focal, cx, cy, opts: Opts = None) -> np.ndarray:
    """Projected FP64 records [G, 16] of one view (see ``dlo_project``)."""
    opts = opts or Opts()
    m, ls, q, lg, sh = _scene_arrays(scene)
    out = np.empty((scene.n, 16), dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    eye = np.ascontiguousarray(eye, dtype=np.float64)
    co = opts.c(focal, cx, cy)
    lib().dlo_project(scene.n, _ptr(m), _ptr(ls), _ptr(q), _ptr(lg), _ptr(sh), _ptr(R), _ptr(t), _ptr(eye),
                      ctypes.byref(co), _ptr(out))
    return out


@dataclass
class RayResult:
    prim: np.ndarray      # [n, 3] FP64 truth
    nvar: np.ndarray      # [n]
    var: np.ndarray       # [n, MAX_VAR, 3] admissible outcomes
    info: np.ndarray      # [n, 4]: over-budget flag, fragile decisions, Gaussians blended, near-tie groups

    def admissible_err(self, gpu: np.ndarray) -> np.ndarray:
        """Per ray: min over admissible outcomes of max_c |gpu[r, c] - outcome[c]|."""
        gpu = np.asarray(gpu, dtype=np.float64)
        d = np.abs(self.var - gpu[:, None, :]).max(axis=2)
        d = np.where(np.arange(MAX_VAR)[None, :] < self.nvar[:, None], d, np.inf)
        return np.minimum(d.min(axis=1), np.abs(self.prim - gpu).max(axis=1))

    def admissible_err_sub(self, gpu_vals, ray_idx, ch) -> np.ndarray:
        """Per subpixel: gpu_vals[n] is channel ch[n] of ray ray_idx[n]; min over admissible outcomes of
        |gpu - outcome|."""
        gpu_vals = np.asarray(gpu_vals, dtype=np.float64)
        ray_idx = np.asarray(ray_idx)
        ch = np.asarray(ch)
        v = self.var[ray_idx[:, None], np.arange(MAX_VAR)[None, :], ch[:, None]]
        d = np.abs(v - gpu_vals[:, None])
        d = np.where(np.arange(MAX_VAR)[None, :] < self.nvar[ray_idx][:, None], d, np.inf)
        return np.minimum(d.min(axis=1), np.abs(self.prim[ray_idx, ch] - gpu_vals))


def render_rays(scene, display, c2w, ray_v, ray_x, ray_y, opts: Opts = None, converge_dist=None,
                cams=None) -> RayResult:
    opts = opts or Opts()
    m, ls, q, lg, sh = _scene_arrays(scene)
    R, t, eye = cams if cams is not None else cameras_for(display, c2w, converge_dist)
    R = np.ascontiguousarray(R, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    eye = np.ascontiguousarray(eye, dtype=np.float64)
    rv = np.ascontiguousarray(ray_v, dtype=np.int32)
    rx = np.ascontiguousarray(ray_x, dtype=np.int32)
    ry = np.ascontiguousarray(ray_y, dtype=np.int32)
    n = len(rv)
    prim = np.zeros((n, 3))
    nvar = np.zeros(n, dtype=np.int32)
    var = np.zeros((n, MAX_VAR, 3))
    info = np.zeros((n, 4), dtype=np.int32)
    co = opts.c(*intrinsics(display))
    lib().dlo_render_rays(scene.n, _ptr(m), _ptr(ls), _ptr(q), _ptr(lg), _ptr(sh), display.n_views, _ptr(R),
                          _ptr(t), _ptr(eye), ctypes.byref(co), n, _ptr(rv), _ptr(rx), _ptr(ry), _ptr(prim),
                          _ptr(nvar), _ptr(var), _ptr(info))
    return RayResult(prim, nvar, var, info)


def render_views(scene, display, c2w, opts: Opts = None, converge_dist=None, views=None) -> np.ndarray:
    """The standard paradigm's multi-view images M_m[N, h, w, 3] (all pixels of every view)."""
    N, H, W = display.n_views, display.height, display.width
    vs = range(N) if views is None else views
    rv, rx, ry = [], [], []
    for v in vs:
        xs, ys = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rv.append(np.full(H * W, v))
        rx.append(xs.ravel())
        ry.append(ys.ravel())
    res = render_rays(scene, display, c2w, np.concatenate(rv), np.concatenate(rx), np.concatenate(ry), opts,
                      converge_dist)
    out = np.zeros((N, H, W, 3))
    out[list(vs)] = res.prim.reshape(len(list(vs)), H, W, 3)
    return out


def view_map_of(display) -> np.ndarray:
    return viewmap.view_map(display.width, display.height, display.n_views, display.tan_slant, display.pitch,
                            display.offset)


def render_directl(scene, display, c2w, opts: Opts = None, converge_dist=None):
    """The light-field image by rendering only each subpixel's own ray.  Returns (M_e[h, w, 3] from the
    FP64 truth, RayResult, subpixel->ray index[h, w, 3])."""
    V = view_map_of(display)
    rv, rx, ry, index = viewmap.subpixel_rays(V)
    res = render_rays(scene, display, c2w, rv, rx, ry, opts, converge_dist)
    ch = np.broadcast_to(np.arange(3)[None, None, :], index.shape)
    img = res.prim[index, ch]
    return img, res, index


def backward_rays(scene, display, c2w, ray_v, ray_x, ray_y, grad_rgb, opts: Opts = None, converge_dist=None):
    """FP64 adjoint: gradients of sum_r grad_rgb[r] . C(r) w.r.t. (means, log_scales, quats, logits, sh)."""
    opts = opts or Opts()
    m, ls, q, lg, sh = _scene_arrays(scene)
    R, t, eye = cameras_for(display, c2w, converge_dist)
    R, t, eye = (np.ascontiguousarray(a, dtype=np.float64) for a in (R, t, eye))
    rv = np.ascontiguousarray(ray_v, dtype=np.int32)
    rx = np.ascontiguousarray(ray_x, dtype=np.int32)
    ry = np.ascontiguousarray(ray_y, dtype=np.int32)
    g = np.ascontiguousarray(grad_rgb, dtype=np.float64)
    G = scene.n
    gm = np.zeros((G, 3)); gl = np.zeros((G, 3)); gq = np.zeros((G, 4)); go = np.zeros(G)
    gs = np.zeros((G, 16, 3))
    co = opts.c(*intrinsics(display))
    lib().dlo_backward_rays(G, _ptr(m), _ptr(ls), _ptr(q), _ptr(lg), _ptr(sh), display.n_views, _ptr(R), _ptr(t),
                            _ptr(eye), ctypes.byref(co), len(rv), _ptr(rv), _ptr(rx), _ptr(ry), _ptr(g), _ptr(gm),
                            _ptr(gl), _ptr(gq), _ptr(go), _ptr(gs))
    return gm, gl, gq, go, gs


def sh_basis(dirs: np.ndarray, degree: int = 3) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    Y = np.zeros((len(dirs), 16))
    lib().dlo_sh_basis(len(dirs), degree, _ptr(dirs), _ptr(Y))
    return Y
