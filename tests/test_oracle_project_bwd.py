"""Pins of the oracle's projection derivative: central finite differences
of the oracle's projection (itself pinned against closed forms and scipy)
for every input -- 3D means, log-scales, quaternions (unnormalized, through
the normalization), opacity, RGB and degree-3 SH coefficients -- under a
random linear loss of all projection outputs (means2D, conic (a, b, c),
opacity, rgb, depth).  Cases: an axis camera and a rotated orbit camera,
Gaussians on and off the optical axis, including ones whose x/z lies beyond
the Jacobian clamp (derivative through the clamp is 0), and SH colours with
one channel clamped at 0."""
import math

import numpy as np
import pytest

from workloads.scenes import Camera, _orbit_camera


def _cams():
    axis = Camera(width=96, height=64, fx=90.0, fy=80.0, cx=48.0, cy=32.0, R=np.eye(3), t=np.zeros(3))
    orbit = _orbit_camera(96, 64, az=0.7, el=0.3)
    return [axis, orbit]


def _gaussians(rng, P, sh_degree, cam):
    # centres in front of the camera, some beyond the 1.3 half-FOV clamp in x
    R, t = np.asarray(cam.R), np.asarray(cam.t)
    zc = rng.uniform(2.5, 5.0, P)
    xz = rng.uniform(-0.5, 0.5, P) * cam.width / cam.fx
    xz[0] = 1.6 * (0.5 * cam.width / cam.fx)  # beyond the clamp
    yz = rng.uniform(-0.4, 0.4, P) * cam.height / cam.fy
    pc = np.stack([xz * zc, yz * zc, zc], 1)
    mu = (pc - t) @ R  # world = R^T (p - t)
    ls = rng.normal(-2.0, 0.5, (P, 3))
    q = rng.standard_normal((P, 4)) * rng.uniform(0.5, 2.0, (P, 1))  # unnormalized
    op = rng.uniform(0.1, 0.9, P)
    if sh_degree < 0:
        col = rng.uniform(0.0, 1.0, (P, 3))
    else:
        K = (sh_degree + 1) ** 2
        col = rng.normal(0.0, 0.3, (P, K, 3))
        col[:, 0, :] = rng.uniform(0.5, 1.5, (P, 3))
        col[1, 0, 2] = -3.0  # that channel clamps at 0
    return [np.asarray(a, np.float32) for a in (mu, ls, q, op, col)]


def _loss(out, w):
    return float(np.sum(out["means2D"] * w[0]) + np.sum(out["conic_opacity"] * w[1]) +
                 np.sum(out["rgb"] * w[2]) + np.sum(out["depth"] * w[3]))


@pytest.mark.parametrize("sh_degree", [-1, 3])
@pytest.mark.parametrize("ci", [0, 1])
def test_project_bwd_matches_finite_differences(orc, sh_degree, ci):
    cam = _cams()[ci]
    rng = np.random.default_rng(40 + ci + 3 * sh_degree)
    P = 5
    inputs = _gaussians(rng, P, sh_degree, cam)
    base = orc.project(cam, *inputs, sh_degree)
    assert (base["radius"] > 0).all()
    w = [rng.standard_normal((P, 2)), rng.standard_normal((P, 4)), rng.standard_normal((P, 3)),
         rng.standard_normal(P)]
    an = orc.project_bwd(cam, *inputs, sh_degree, w[0], w[1], w[2], w[3])
    names = ["means3D", "log_scales", "quats", "opacity", "colors"]
    for k, name in enumerate(names):
        x = inputs[k]
        fd = np.zeros(x.shape)
        flat = x.reshape(-1)
        for i in range(flat.size):
            h = 1e-3 * max(abs(float(flat[i])), 0.1)
            xp, xm = flat.copy(), flat.copy()
            xp[i] = np.float32(flat[i] + h)
            xm[i] = np.float32(flat[i] - h)
            args_p = list(inputs)
            args_m = list(inputs)
            args_p[k] = xp.reshape(x.shape)
            args_m[k] = xm.reshape(x.shape)
            lp = _loss(orc.project(cam, *args_p, sh_degree), w)
            lm = _loss(orc.project(cam, *args_m, sh_degree), w)
            fd.reshape(-1)[i] = (lp - lm) / (float(xp[i]) - float(xm[i]))
        a = an[name]
        scale = max(float(np.sqrt(np.mean(a * a))), 1e-12)
        err = np.abs(a - fd) / np.maximum(np.abs(fd), scale)
        assert err.max() < 2e-4, (name, float(err.max()), np.unravel_index(np.argmax(err), err.shape))


def test_project_bwd_culled_is_zero(orc):
    cam = _cams()[0]
    mu = np.array([[0.0, 0.0, 0.1]], np.float32)  # behind the near plane
    ls = np.full((1, 3), -2.0, np.float32)
    q = np.array([[1.0, 0, 0, 0]], np.float32)
    op = np.array([0.5], np.float32)
    col = np.array([[0.2, 0.3, 0.4]], np.float32)
    g = orc.project_bwd(cam, mu, ls, q, op, col, -1, np.ones((1, 2)), np.ones((1, 4)), np.ones((1, 3)), np.ones(1))
    for v in g.values():
        assert not np.any(v)
