"""Thin Python binding of the C ABI in ``include/directl.h`` (argument marshalling only).

Every step of the render runs in the gfx950 kernels of ``libdirectl.so``; PyTorch provides device memory
(tensors) and streams.  There is no CPU fallback: if the library is missing or no GPU is present, calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdirectl.so")

DL_OK, DL_EINVAL, DL_ERANGE, DL_ENOMEM, DL_EHIP, DL_ECAP, DL_ELATER = 0, -1, -2, -3, -4, -5, -6


class DLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("directl error %d: %s" % (code, msg))
        self.code = code


class dl_rational(ctypes.Structure):
    _fields_ = [("num", ctypes.c_int64), ("den", ctypes.c_int64)]


class dl_display_desc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("n_views", ctypes.c_int32),
                ("repurpose_pw", ctypes.c_int32), ("tan_slant", dl_rational), ("pitch", dl_rational),
                ("offset", dl_rational), ("baseline", ctypes.c_double), ("focal_px", ctypes.c_double)]


class dl_pose(ctypes.Structure):
    _fields_ = [("c2w", ctypes.c_double * 16), ("converge_dist", ctypes.c_double)]


class dl_render_opts(ctypes.Structure):
    _fields_ = [("z_near", ctypes.c_float), ("q_cut", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("sh_degree", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32)]


NSTAGES = 10
STAGES = ["upload", "project", "depth_sort", "bin_count", "scan", "bin_emit", "tile_sort", "bounds", "blend",
          "interleave"]


class dl_frame_stats(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double * NSTAGES), ("stage_launches", ctypes.c_int32 * NSTAGES),
                ("keys", ctypes.c_int64), ("visible", ctypes.c_int64), ("evaluations", ctypes.c_int64),
                ("blends", ctypes.c_int64), ("rays", ctypes.c_int64), ("batches", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("rays_per_lane", ctypes.c_int32),
                ("chunks", ctypes.c_int32), ("chunk_ms", (ctypes.c_double * NSTAGES) * 8), ("lanes", ctypes.c_int32)]


class dl_bvh_stats(ctypes.Structure):
    _fields_ = [("n_gaussians", ctypes.c_int64), ("n_prims", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("depth", ctypes.c_int32), ("stack_bound", ctypes.c_int32),
                ("sah_cost", ctypes.c_double), ("build_ms", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "dl_default_opts": (None, [ctypes.POINTER(dl_render_opts)]),
    "dl_last_error": (ctypes.c_char_p, []),
    "dl_create": (_I, [_I, ctypes.POINTER(_P)]),
    "dl_destroy": (None, [_P]),
    "dl_scene_create": (_I, [_P, ctypes.c_int64, _P, _P, _P, _P, _P, _I, _P, ctypes.POINTER(_P)]),
    "dl_scene_update": (_I, [_P, _P, _P, _P, _P, _P, _I, _P]),
    "dl_scene_size": (ctypes.c_int64, [_P]),
    "dl_scene_free": (None, [_P]),
    "dl_display_create": (_I, [_P, ctypes.POINTER(dl_display_desc), _P, ctypes.POINTER(_P)]),
    "dl_display_free": (None, [_P]),
    "dl_display_view_map": (_I, [_P, _P, _P]),
    "dl_display_num_rays": (ctypes.c_int64, [_P]),
    "dl_display_source_map": (_I, [_P, _P, _P]),
    "dl_cameras": (_I, [_P, ctypes.POINTER(dl_pose), _P]),
    "dl_project": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), _P, _P, _P]),
    "dl_project_noalloc": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), _P, _P, _P]),
    "dl_plan_batch_prepare": (_I, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), _P]),
    "dl_plan_render_batch": (_I, [_P, ctypes.POINTER(dl_pose), ctypes.c_int32, _P]),
    "dl_render": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), _P, _P]),
    "dl_render_standard": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), _P, _P,
                                _P]),
    "dl_render_multiview": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), ctypes.c_int32,
                                 ctypes.c_int32, _P, _P, _P]),
    "dl_interleave": (_I, [_P, _P, _P, _P]),
    "dl_render_backward": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), _P, _P, _P, _P,
                                _P, _P, _P, _P]),
    "dl_set_profiling": (_I, [_P, _I]),
    "dl_set_key_capacity": (_I, [_P, ctypes.c_int64]),
    "dl_key_capacity": (ctypes.c_int64, [_P]),
    "dl_frame_stats_get": (_I, [_P, ctypes.POINTER(dl_frame_stats)]),
    "dl_probe_issue_rates": (_I, [_I, ctypes.POINTER(ctypes.c_double), _I]),
    "dl_plan_create": (_I, [_P, _P, _P, ctypes.POINTER(dl_render_opts), ctypes.POINTER(dl_pose), ctypes.c_int64,
                            _P, _P, ctypes.POINTER(_P)]),
    "dl_plan_render": (_I, [_P, ctypes.POINTER(dl_pose), _P]),
    "dl_plan_check": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "dl_plan_first_chunk_only": (_I, [_P]),
    "dl_plan_use_all_chunks": (_I, [_P, _P]),
    "dl_plan_bytes": (ctypes.c_int64, [_P]),
    "dl_plan_estimate_bytes": (ctypes.c_int64, [_P, _P, ctypes.POINTER(dl_render_opts), ctypes.c_int64]),
    "dl_plan_free": (None, [_P]),
    "dl_bvh_build": (_I, [_P, _P, ctypes.POINTER(dl_render_opts), _P, ctypes.POINTER(_P)]),
    "dl_bvh_get_stats": (_I, [_P, ctypes.POINTER(dl_bvh_stats)]),
    "dl_bvh_free": (None, [_P]),
    "dl_render_rayorder": (_I, [_P, _P, _P, ctypes.POINTER(dl_pose), ctypes.POINTER(dl_render_opts), ctypes.c_int32,
                                _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libdirectl.so (built by ``paper_2407_14053_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libdirectl.so is not built (%s); run python -m paper_2407_14053_amd.build" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != DL_OK:
        raise DLError(rc, load().dl_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP path needs a GPU; none is visible")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


_DEFAULT_OPTS = None


def _opts(opts):
    """opts, or the library's defaults (made once; the library only reads them)."""
    global _DEFAULT_OPTS
    if opts is not None:
        return opts
    if _DEFAULT_OPTS is None:
        _DEFAULT_OPTS = default_opts()
    return _DEFAULT_OPTS


def default_opts(**over) -> dl_render_opts:
    o = dl_render_opts()
    load().dl_default_opts(ctypes.byref(o))
    for k, v in over.items():
        if k == "bg":
            o.bg = (ctypes.c_float * 3)(*v)
        else:
            setattr(o, k, v)
    return o


def make_pose(c2w, converge_dist=None) -> dl_pose:
    """The C pose of a camera-to-world matrix (converge_dist defaults to the camera's distance from the origin);
    a dl_pose is returned as it is, so that callers can build poses once."""
    if isinstance(c2w, dl_pose):
        return c2w
    c2w = np.asarray(c2w, dtype=np.float64).reshape(4, 4)
    p = dl_pose()
    p.c2w = (ctypes.c_double * 16)(*c2w.ravel().tolist())
    p.converge_dist = float(np.linalg.norm(c2w[:3, 3])) if converge_dist is None else float(converge_dist)
    return p


def _rat(x) -> dl_rational:
    f = Fraction(x)
    return dl_rational(f.numerator, f.denominator)


def make_desc(display) -> dl_display_desc:
    d = dl_display_desc()
    d.width, d.height, d.n_views = display.width, display.height, display.n_views
    d.tan_slant, d.pitch, d.offset = _rat(display.tan_slant), _rat(display.pitch), _rat(display.offset)
    d.baseline, d.focal_px = float(display.baseline), float(display.focal_px)
    d.repurpose_pw = int(getattr(display, "repurpose_pw", 0))
    return d


def probe_issue_rates(device: int = 0) -> dict:
    """Vector-ALU issue rates measured on the device (dl_probe_issue_rates)."""
    _torch()
    out = (ctypes.c_double * 16)()
    _check(load().dl_probe_issue_rates(int(device), out, 16))
    return {"fma_lane_ops_per_s": out[0], "exp_lane_ops_per_s": out[1], "fma4_exp1_steps_per_s": out[2],
            "blend_pairs_1ch_per_s": out[3], "blend_pairs_3ch_per_s": out[4], "engine_clock_hz": out[5],
            "compute_units": int(out[6]), "add_lane_ops_per_s": out[7], "fmac_lane_ops_per_s": out[8],
            "negmul_lane_ops_per_s": out[9], "fma3v_lane_ops_per_s": out[10],
            "cndmask_sgpr_lane_ops_per_s": out[11], "cmp_sgpr_add_steps_per_s": out[12],
            "fmac3r_lane_ops_per_s": out[13], "fma_sgpr_lane_ops_per_s": out[14],
            "exp1_fma4_steps_per_s": out[15]}


class Context:
    def __init__(self, device: int = 0):
        torch = _torch()
        torch.cuda.set_device(device)
        self.device = device
        h = ctypes.c_void_p()
        _check(load().dl_create(device, ctypes.byref(h)))
        self.h = h

    def set_key_capacity(self, keys: int):
        _check(load().dl_set_key_capacity(self.h, int(keys)))

    def key_capacity(self) -> int:
        return int(load().dl_key_capacity(self.h))

    def set_profiling(self, level):
        """0/False off, 1 blend timing, 2 every stage, 3/True every stage and the blend's work counters."""
        level = 3 if level is True else int(level)
        _check(load().dl_set_profiling(self.h, level))

    def frame_stats(self) -> dict:
        return self.stats_dict(self.frame_stats_raw())

    def frame_stats_raw(self) -> "dl_frame_stats":
        """The last frame's statistics as the C struct (cheap to take inside a timed loop; see stats_dict)."""
        st = dl_frame_stats()
        _check(load().dl_frame_stats_get(self.h, ctypes.byref(st)))
        return st

    @staticmethod
    def stats_dict(st) -> dict:
        d = {k: getattr(st, k) for k in ("keys", "visible", "evaluations", "blends", "rays", "batches", "tile_w",
                                         "tile_h", "rays_per_lane", "lanes")}
        d["stage_ms"] = {STAGES[i]: st.stage_ms[i] for i in range(NSTAGES)}
        d["stage_launches"] = {STAGES[i]: st.stage_launches[i] for i in range(NSTAGES)}
        d["chunk_ms"] = [{STAGES[i]: st.chunk_ms[c][i] for i in range(NSTAGES) if st.chunk_ms[c][i] > 0}
                         for c in range(st.chunks)]
        return d

    def close(self):
        if self.h:
            load().dl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """Library-owned SoA copy of a Gaussian scene.  ``arrays`` = (means[G,3], log_scales[G,3], quats[G,4],
    opacity_logits[G], sh[G,16,3]) as float32 torch CUDA tensors or numpy arrays."""

    def __init__(self, ctx: Context, arrays, stream=None):
        self.ctx = ctx
        arrs, on_dev = self._prep(arrays)
        self.n = int(arrs[0].shape[0])
        h = ctypes.c_void_p()
        _check(load().dl_scene_create(ctx.h, self.n, *[self._p(a, on_dev) for a in arrs], int(on_dev),
                                      _stream(stream), ctypes.byref(h)))
        self.h = h

    @staticmethod
    def _prep(arrays):
        torch = _torch()
        if isinstance(arrays[0], torch.Tensor):
            arrs = [a.detach().to(torch.float32).contiguous() for a in arrays]
            return arrs, arrs[0].is_cuda
        return [np.ascontiguousarray(a, dtype=np.float32) for a in arrays], False

    @staticmethod
    def _p(a, on_dev):
        return _ptr(a) if on_dev else a.ctypes.data_as(ctypes.c_void_p)

    def update(self, arrays, stream=None):
        arrs, on_dev = self._prep(arrays)
        assert int(arrs[0].shape[0]) == self.n
        _check(load().dl_scene_update(self.h, *[self._p(a, on_dev) for a in arrs], int(on_dev), _stream(stream)))
        self._keep = arrs   # keep the sources alive until the stream has consumed them

    def close(self):
        if self.h:
            load().dl_scene_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Display:
    def __init__(self, ctx: Context, display, stream=None):
        self.ctx = ctx
        self.info = display
        self.desc = make_desc(display)
        h = ctypes.c_void_p()
        _check(load().dl_display_create(ctx.h, ctypes.byref(self.desc), _stream(stream), ctypes.byref(h)))
        self.h = h

    @property
    def shape(self):
        return self.desc.height, self.desc.width

    @property
    def n_views(self):
        return self.desc.n_views

    def num_rays(self) -> int:
        return int(load().dl_display_num_rays(self.h))

    def view_map(self, stream=None):
        torch = _torch()
        out = torch.empty((self.desc.height, 3 * self.desc.width), dtype=torch.uint8, device="cuda")
        _check(load().dl_display_view_map(self.h, _ptr(out), _stream(stream)))
        return out

    def source_map(self, stream=None):
        """[H][W][3] int32: the pixel x' W + y' whose channel k subpixel (x, y, k) shows (Alg. 2's M_i)."""
        torch = _torch()
        out = torch.empty((self.desc.height, self.desc.width, 3), dtype=torch.int32, device="cuda")
        _check(load().dl_display_source_map(self.h, _ptr(out), _stream(stream)))
        return out

    def cameras(self, c2w, converge_dist=None) -> np.ndarray:
        out = np.zeros((self.desc.n_views, 16), dtype=np.float64)
        pose = make_pose(c2w, converge_dist)
        _check(load().dl_cameras(self.h, ctypes.byref(pose), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self.h:
            load().dl_display_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def project(ctx, scene, display, c2w, converge_dist=None, opts=None, stream=None):
    """(records[N, G, 12] float32, depth[N, G] float64 with NaN where culled)."""
    torch = _torch()
    N, G = display.n_views, scene.n
    rec = torch.empty((N, G, 12), dtype=torch.float32, device="cuda")
    depth = torch.empty((N, G), dtype=torch.float64, device="cuda")
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_project(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), _ptr(rec), _ptr(depth),
                             _stream(stream)))
    return rec, depth


def project_noalloc(ctx, scene, display, c2w, out, depth, converge_dist=None, opts=None, stream=None):
    """dl_project_noalloc into caller-owned out[N, G, 12] float32 and depth[N, G] float64 (the library allocates
    nothing; its scratch is a fixed device array)."""
    torch = _torch()
    N, G = display.n_views, scene.n
    if tuple(out.shape) != (N, G, 12) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape (%d, %d, 12)" % (N, G))
    if tuple(depth.shape) != (N, G) or depth.dtype != torch.float64 or not depth.is_contiguous():
        raise ValueError("depth must be a contiguous float64 tensor of shape (%d, %d)" % (N, G))
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_project_noalloc(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), _ptr(out),
                                     _ptr(depth), _stream(stream)))
    return out, depth


def render(ctx, scene, display, c2w, converge_dist=None, opts=None, out=None, stream=None):
    """DirectL: the encoded image [H, W, 3] float32."""
    torch = _torch()
    H, W = display.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_render(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), _ptr(out),
                            _stream(stream)))
    return out


def render_standard(ctx, scene, display, c2w, converge_dist=None, opts=None, out=None, views=None,
                    keep_views=False, stream=None):
    """Standard paradigm: N full views then Alg. 1.  Returns (encoded image, views or None)."""
    torch = _torch()
    H, W = display.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    if views is None and keep_views:
        views = torch.empty((display.n_views, H, W, 3), dtype=torch.float32, device="cuda")
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_render_standard(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), _ptr(out),
                                     _ptr(views) if views is not None else None, _stream(stream)))
    return out, views


def render_multiview(ctx, scene, display, c2w, view_w, view_h, converge_dist=None, opts=None, out=None, views=None,
                     keep_views=False, stream=None):
    """The multi-view baselines: N views at view_w x view_h, bilinear Resize to the panel, Alg. 1.  Returns
    (encoded image, views [N, view_h, view_w, 3] or None)."""
    torch = _torch()
    H, W = display.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    if views is None and keep_views:
        views = torch.empty((display.n_views, view_h, view_w, 3), dtype=torch.float32, device="cuda")
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_render_multiview(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), int(view_w),
                                      int(view_h), _ptr(out), _ptr(views) if views is not None else None,
                                      _stream(stream)))
    return out, views


class BVH:
    """The scene's 8-wide SAH BVH for ray-order rendering (built on the host from the scene's current
    parameters; q_cut and alpha_min of ``opts`` are baked into its boxes)."""

    def __init__(self, ctx: Context, scene: Scene, opts=None, stream=None):
        self.ctx = ctx
        h = ctypes.c_void_p()
        o = _opts(opts)
        _check(load().dl_bvh_build(ctx.h, scene.h, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.h = h

    def stats(self) -> dict:
        st = dl_bvh_stats()
        _check(load().dl_bvh_get_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if self.h:
            load().dl_bvh_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render_rayorder(ctx, bvh, display, c2w, heap_cap=128, converge_dist=None, opts=None, out=None, stream=None):
    """Ray-order 3DGS (Alg. 3) of the display's rays with heap capacity c_h = heap_cap: the encoded image."""
    torch = _torch()
    H, W = display.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_render_rayorder(ctx.h, bvh.h, display.h, ctypes.byref(pose), ctypes.byref(o), int(heap_cap),
                                     _ptr(out), _stream(stream)))
    return out


def render_backward(ctx, scene, display, c2w, out, grad_out, converge_dist=None, opts=None, stream=None):
    """Gradients (means[G,3], log_scales[G,3], quats[G,4], opacity_logits[G], sh[G,16,3]) of a loss whose
    gradient with respect to the DirectL image `out` is `grad_out`."""
    torch = _torch()
    G = scene.n
    dev = dict(dtype=torch.float32, device="cuda")
    g = (torch.empty((G, 3), **dev), torch.empty((G, 3), **dev), torch.empty((G, 4), **dev), torch.empty((G,), **dev),
         torch.empty((G, 16, 3), **dev))
    out = out.contiguous()
    grad_out = grad_out.to(torch.float32).contiguous()
    pose = make_pose(c2w, converge_dist)
    o = _opts(opts)
    _check(load().dl_render_backward(ctx.h, scene.h, display.h, ctypes.byref(pose), ctypes.byref(o), _ptr(out),
                                     _ptr(grad_out), *[_ptr(x) for x in g], _stream(stream)))
    return g


def interleave(display, views, out=None, stream=None):
    torch = _torch()
    H, W = display.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    _check(load().dl_interleave(display.h, _ptr(views), _ptr(out), _stream(stream)))
    return out


def plan_estimate_bytes(scene, display, opts=None, key_capacity: int = 0) -> int:
    """Device bytes a plan would hold (plus its output image) at the given tile-key capacity."""
    o = _opts(opts)
    n = int(load().dl_plan_estimate_bytes(scene.h, display.h, ctypes.byref(o), int(key_capacity)))
    if n < 0:
        raise DLError(DL_EINVAL, "cannot estimate a plan for these arguments")
    h, w = display.shape
    return n + 12 * h * w


class Plan:
    """A DirectL frame of one (scene, display, options) with fixed buffers, replayed as a HIP graph.

    `out` is the image every launch writes.  `launch` is asynchronous on `stream` (not the null stream);
    `check` is valid once that launch has completed and raises nothing: it returns (ok, keys_needed)."""

    def __init__(self, ctx: Context, scene: Scene, display: Display, probe_c2w, converge_dist=None, opts=None,
                 min_key_capacity: int = 0, stream=None):
        torch = _torch()
        H, W = display.shape
        self.ctx, self.scene, self.display = ctx, scene, display  # kept alive while the plan lives
        self.out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        self.opts = opts or default_opts()
        self.converge_dist = converge_dist
        pose = make_pose(probe_c2w, converge_dist)
        h = ctypes.c_void_p()
        _check(load().dl_plan_create(ctx.h, scene.h, display.h, ctypes.byref(self.opts), ctypes.byref(pose),
                                     int(min_key_capacity), _ptr(self.out), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.batch_max = 1
        self.needs_all_chunks = False
        self.bytes = int(load().dl_plan_bytes(self.h)) + self.out.numel() * 4

    def launch(self, c2w, stream=None, converge_dist=None):
        cd = self.converge_dist if converge_dist is None else converge_dist
        pose = make_pose(c2w, cd)
        _check(load().dl_plan_render(self.h, ctypes.byref(pose), _stream(stream)))
        return self.out

    def prepare_batch(self, max_frames: int, stream=None):
        """Capture graphs of 1..max_frames frames in a row (batched launches); allocates their output images
        outs[max_frames, H, W, 3] (counted in `bytes`)."""
        torch = _torch()
        H, W = self.display.shape
        self.outs = torch.empty((max_frames, H, W, 3), dtype=torch.float32, device="cuda")
        ptrs = (ctypes.c_void_p * max_frames)(*[self.outs[k].data_ptr() for k in range(max_frames)])
        _check(load().dl_plan_batch_prepare(self.h, int(max_frames), ptrs, _stream(stream)))
        self.batch_max = int(max_frames)
        self.bytes += self.outs.numel() * 4

    def launch_batch(self, c2ws, stream=None, converge_dist=None):
        """One launch rendering len(c2ws) frames in a row; returns outs[:n] (frame k is pose k)."""
        cd = self.converge_dist if converge_dist is None else converge_dist
        n = len(c2ws)
        poses = (dl_pose * n)(*[make_pose(c, cd) for c in c2ws])
        _check(load().dl_plan_render_batch(self.h, poses, int(n), _stream(stream)))
        return self.outs[:n]

    def check(self):
        """(ok, keys_needed) once the plan's launches have completed.  ok is False when a frame overflowed the
        key capacity, or when a frame of a first-chunk plan needed a later depth chunk: then `needs_all_chunks`
        is True, and use_all_chunks() makes the plan render such frames (launch them again)."""
        need = ctypes.c_int64(0)
        rc = load().dl_plan_check(self.h, ctypes.byref(need))
        if rc not in (DL_OK, DL_ECAP, DL_ELATER):
            _check(rc)
        self.needs_all_chunks = rc == DL_ELATER
        return rc == DL_OK, int(need.value)

    @property
    def first_chunk_only(self) -> bool:
        """The plan's graphs hold the first depth chunk only (its probe frame finished in it)."""
        return load().dl_plan_first_chunk_only(self.h) == 1

    def use_all_chunks(self, stream=None):
        """Recapture the plan's graphs with every depth chunk (waits for the plan's last launch)."""
        _check(load().dl_plan_use_all_chunks(self.h, _stream(stream)))
        self.needs_all_chunks = False

    def close(self):
        if getattr(self, "h", None):
            load().dl_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
