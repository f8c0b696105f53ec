"""Seeded synthetic inputs: Gaussian scenes, lenticular display descriptors, centre-camera poses.

This module only *draws inputs*. It contains none of the rendering arithmetic (no view map, no camera
rig, no projection, no compositing), so that the HIP path and the CPU oracle can both be fed from it
without sharing any of the method's code.

Scenes follow the distributions used for the light-field workloads (3D Gaussian splatting scenes as in
the paper's Sec. 3.3, synthetic stand-ins for its trained Blender / Mip-NeRF360 scenes):

* means uniform in a cube (or a clustered layout of blobs plus a background shell),
* log-scales ~ U(-4, -2) per axis,
* rotations: normalised N(0, I4) quaternions (uniform on SO(3)), stored (w, x, y, z),
* opacity logits ~ N(0, 1),
* spherical-harmonic colour of degree 3, DC ~ N(0, 0.5), higher bands ~ N(0, 0.05) (standard deviations),

all float32, user layout ``means[G,3]``, ``log_scales[G,3]``, ``quats[G,4]``, ``opacity_logits[G]``,
``sh[G,16,3]`` (coefficient-major, channel-minor, DC first).

Draw order from one numpy PCG64 stream: means, log-scales, quaternions, opacity logits, SH DC, SH rest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

__all__ = [
    "Scene", "Display", "scene_uniform", "scene_clustered", "make_scene", "make_display",
    "look_at_c2w", "pose_sweep", "pose_orbit", "DISPLAYS", "SCENES",
]


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)

    def subset(self, idx) -> "Scene":
        return Scene(*(a[idx] for a in self.arrays()))


@dataclass
class Display:
    """Lenticular panel descriptor: W x H pixels (3 subpixels each), N views, rational slant/pitch/offset.

    ``tan_slant``, ``pitch`` and ``offset`` are exact rationals (Eq. (1)-(3) parameters tan(alpha), L_x,
    K_offset, the latter two in subpixel widths).  ``baseline`` is the distance between the outermost
    cameras, ``focal_px`` the focal length in pixels (square pixels)."""
    width: int
    height: int
    n_views: int
    tan_slant: Fraction
    pitch: Fraction
    offset: Fraction = Fraction(0)
    baseline: float = 0.3
    focal_px: float = 0.0
    name: str = ""
    extra: dict = field(default_factory=dict)
    repurpose_pw: int = 0  # 0: identity map (Alg. 1); P_w >= 1: subpixel repurposing (Alg. 2)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _attributes(rng: np.random.Generator, n: int):
    log_scales = rng.uniform(-4.0, -2.0, size=(n, 3)).astype(np.float32)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    quats = q.astype(np.float32)
    opacity_logits = rng.standard_normal(n).astype(np.float32)
    sh = np.empty((n, 16, 3), dtype=np.float32)
    sh[:, 0, :] = rng.normal(0.0, 0.5, size=(n, 3))
    sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, 15, 3))
    return log_scales, quats, opacity_logits, sh


def scene_uniform(n: int, half_extent: float, seed: int) -> Scene:
    """Means uniform in [-half_extent, half_extent]^3."""
    rng = _rng(seed)
    means = rng.uniform(-half_extent, half_extent, size=(n, 3)).astype(np.float32)
    return Scene(means, *_attributes(rng, n))


def scene_clustered(n: int, seed: int, n_blobs: int = 64, blob_sigma: float = 0.3,
                    centre_extent: float = 2.0, shell_frac: float = 0.2, shell_radius: float = 4.0) -> Scene:
    """80% of the Gaussians in ``n_blobs`` isotropic blobs (centres uniform in the cube of half-width
    ``centre_extent``, offsets N(0, blob_sigma^2)), the rest uniform on a sphere of ``shell_radius``."""
    rng = _rng(seed)
    n_shell = int(round(n * shell_frac))
    n_blob = n - n_shell
    centres = rng.uniform(-centre_extent, centre_extent, size=(n_blobs, 3))
    which = rng.integers(0, n_blobs, size=n_blob)
    blob_pts = centres[which] + rng.normal(0.0, blob_sigma, size=(n_blob, 3))
    d = rng.standard_normal((n_shell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    shell_pts = d * shell_radius
    means = np.concatenate([blob_pts, shell_pts], axis=0)
    perm = rng.permutation(n)
    means = means[perm].astype(np.float32)
    return Scene(means, *_attributes(rng, n))


def focal_from_fov_y(height: int, fov_y_deg: float) -> float:
    """Focal length in pixels for a vertical field of view (input description of the camera)."""
    return (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)


def make_display(width, height, n_views, tan_slant, pitch, offset=0, baseline=0.3, fov_y_deg=40.0,
                 name="", repurpose_pw=0) -> Display:
    return Display(width, height, n_views, Fraction(tan_slant), Fraction(pitch), Fraction(offset),
                   float(baseline), focal_from_fov_y(height, fov_y_deg), name, repurpose_pw=int(repurpose_pw))


# Display descriptors of the workloads (rational forms of the stated slants and pitches).
DISPLAYS = {
    # 256x144, N=8, slant atan(1/3), pitch 5.3, baseline 0.3
    "tiny": dict(width=256, height=144, n_views=8, tan_slant=Fraction(1, 3), pitch=Fraction(53, 10),
                 baseline=0.3),
    # 3840x2160, N=45, slant atan(1/6), pitch 7.4, baseline 0.6
    "uhd45": dict(width=3840, height=2160, n_views=45, tan_slant=Fraction(1, 6), pitch=Fraction(37, 5),
                  baseline=0.6),
    # 7680x4320, N=60, slant atan(1/5), pitch 9.1, baseline 0.6
    "8k60": dict(width=7680, height=4320, n_views=60, tan_slant=Fraction(1, 5), pitch=Fraction(91, 10),
                 baseline=0.6),
    # 1920x1080, N=16, pitch 4.6 (slant unstated: atan(1/3))
    "fhd16": dict(width=1920, height=1080, n_views=16, tan_slant=Fraction(1, 3), pitch=Fraction(23, 5),
                  baseline=0.6),
    # 1920x1080, N=45, pitch 4.6 (slant unstated: atan(1/3))
    "fhd45": dict(width=1920, height=1080, n_views=45, tan_slant=Fraction(1, 3), pitch=Fraction(23, 5),
                  baseline=0.6),
    # gradient-check instance: 64x64, N=4, pitch 5.3, baseline 0.3
    "fd64": dict(width=64, height=64, n_views=4, tan_slant=Fraction(1, 3), pitch=Fraction(53, 10),
                 baseline=0.3),
    # the 7.9-inch panel layout of Fig. 2(b): alpha = atan(-1/27), L_x = 5 1/3, K = 0, N = 48
    "fig2b": dict(width=1536, height=2048, n_views=48, tan_slant=Fraction(-1, 27), pitch=Fraction(16, 3),
                  baseline=0.6),
}


# The three panels of the paper's display table (Table 1): (w, h, L_x, tilt angle in degrees, K_offset, N_v).
# Tilt angles become tan(alpha) rounded to a denominator of 10^6; four-decimal pitches and offsets are exact
# decimals.
TABLE1_PANELS = {
    "7.9in": (1536, 2048, "6.2221", 10.8232, "4.2077", 48),
    "15.6in": (3840, 2160, "5.3344", 6.8526, "1.2547", 60),
    "65in": (7680, 4320, "9.3597", 8.6517, "23.6677", 96),
}


def table1_display(name: str, repurpose_pw: int = 0, baseline: float = 0.6) -> Display:
    import math
    w, h, pitch, deg, off, n = TABLE1_PANELS[name]
    tan = Fraction(round(math.tan(math.radians(deg)) * 10 ** 6), 10 ** 6)
    return make_display(w, h, n, tan, Fraction(pitch), Fraction(off), baseline=baseline, name=name,
                        repurpose_pw=repurpose_pw)


def make_named_display(name: str, **over) -> Display:
    kw = dict(DISPLAYS[name])
    kw.update(over)
    return make_display(name=name, **kw)


SCENES = {
    "tiny": lambda: scene_uniform(2000, 1.0, 1001),
    "uhd45": lambda: scene_uniform(300_000, 2.0, 1002),
    "8k60": lambda: scene_clustered(3_000_000, 1003),
    "fd64": lambda: scene_uniform(200, 1.0, 1005),
    "train500k": lambda: scene_uniform(500_000, 2.0, 1005),
}


def make_scene(name: str) -> Scene:
    return SCENES[name]()


def serving_scene(n: int, seed: int) -> Scene:
    return scene_uniform(n, 2.0, seed)


# ----------------------------------------------------------------------------------------------------
# Centre-camera poses (inputs).  Camera-to-world matrices in OpenCV axes: columns are the camera's
# right (+x), down (+y) and forward (+z) directions and its position.
# ----------------------------------------------------------------------------------------------------
def look_at_c2w(eye, target=(0.0, 0.0, 0.0), world_up=(0.0, 1.0, 0.0)) -> np.ndarray:
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(world_up, dtype=np.float64)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    c2w = np.eye(4)
    c2w[:3, 0] = right
    c2w[:3, 1] = down
    c2w[:3, 2] = fwd
    c2w[:3, 3] = eye
    return c2w


def pose_sweep(n_frames: int, distance: float = 3.0, max_deg: float = 10.0) -> list:
    """Azimuth sweep of +-max_deg around the +z axis view of the origin."""
    out = []
    for t in range(n_frames):
        a = math.radians(max_deg) * math.sin(2.0 * math.pi * t / max(n_frames, 1))
        out.append(look_at_c2w((distance * math.sin(a), 0.0, distance * math.cos(a))))
    return out


def pose_orbit(n_frames: int, distance: float = 3.0) -> list:
    """Full orbit, eye_t = d (sin th, 0, cos th), th = 2 pi t / n, looking at the origin."""
    return [look_at_c2w((distance * math.sin(2 * math.pi * t / n_frames), 0.0,
                         distance * math.cos(2 * math.pi * t / n_frames))) for t in range(n_frames)]


def pose_front(distance: float = 3.0) -> np.ndarray:
    return look_at_c2w((0.0, 0.0, distance))
