"""Pin of the oracle's FP64 adjoint against central finite differences of the FP64 forward, CPU only.

Instance: 200 Gaussians, 64x64 panel, N = 4 views (fewer views than the lens pitch, so some rays serve two
subpixels), loss L = sum w * M_e with fixed random weights, plus a non-zero background to exercise the
final-transmittance term.  Threshold decisions (q_cut, alpha_min, t_min) make L piecewise smooth; a
parameter whose +-eps interval crosses one is detected by two step sizes disagreeing and is skipped (and
counted)."""
import numpy as np

from oracle import render, viewmap
from paper_2407_14053_amd import synth


def _setup():
    d = synth.make_named_display("fd64")
    sc = synth.make_scene("fd64")
    sc.log_scales += 0.8          # splats of a few pixels so that most Gaussians touch several rays
    c2w = synth.pose_sweep(9)[1]
    opts = render.Opts(bg=(0.1, 0.2, 0.3))
    V = render.view_map_of(d)
    rv, rx, ry, index = viewmap.subpixel_rays(V)
    w = np.random.default_rng(5).uniform(-1, 1, size=(d.height, d.width, 3))
    grad = np.zeros((len(rv), 3))
    for k in range(3):
        np.add.at(grad[:, k], index[:, :, k].ravel(), w[:, :, k].ravel())
    return d, sc, c2w, opts, (rv, rx, ry, index), w, grad


def _loss(sc, d, c2w, opts, rays, w):
    rv, rx, ry, index = rays
    res = render.render_rays(sc, d, c2w, rv, rx, ry, opts)
    ch = np.broadcast_to(np.arange(3)[None, None, :], index.shape)
    return float((res.prim[index, ch] * w).sum())


def test_adjoint_matches_central_differences():
    d, sc, c2w, opts, rays, w, grad = _setup()
    rv, rx, ry, _ = rays
    gm, gl, gq, go, gs = render.backward_rays(sc, d, c2w, rv, rx, ry, grad, opts)
    mag = np.abs(gm).sum(1) + np.abs(gl).sum(1) + np.abs(go)
    rng = np.random.default_rng(1)
    pick = rng.choice(np.nonzero(mag > 1e-3)[0], 14, replace=False)
    fields = [("means", 3, gm), ("log_scales", 3, gl), ("quats", 4, gq), ("opacity_logits", 1, go),
              ("sh", 48, gs.reshape(-1, 48))]
    checked = skipped = 0
    worst = 0.0
    for i in pick:
        for name, width, g in fields:
            comps = range(width) if name != "sh" else rng.choice(48, 6, replace=False)
            for c in comps:
                arr = getattr(sc, name)
                flat = arr.reshape(arr.shape[0], -1)
                base = flat[i, c].copy()
                fds = []
                for eps in (1e-4, 5e-5):
                    flat[i, c] = np.float32(base + eps)
                    hi = float(flat[i, c])
                    Lp = _loss(sc, d, c2w, opts, rays, w)
                    flat[i, c] = np.float32(base - eps)
                    lo = float(flat[i, c])
                    Lm = _loss(sc, d, c2w, opts, rays, w)
                    flat[i, c] = base
                    fds.append((Lp - Lm) / (hi - lo))
                adj = float(g.reshape(g.shape[0], -1)[i, c])
                scale = max(1e-3, abs(fds[0]))
                if abs(fds[0] - fds[1]) > 1e-5 * scale + 1e-9:
                    skipped += 1            # a threshold decision lies within +-eps
                    continue
                err = abs(adj - fds[0]) / scale
                worst = max(worst, err)
                assert err < 1e-4, (name, i, c, adj, fds)
                checked += 1
    assert checked > 180
    assert skipped <= 0.2 * (checked + skipped)
    assert worst < 1e-4
