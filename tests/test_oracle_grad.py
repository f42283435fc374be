"""Pins of the oracle's backward (the exact derivative of the forward blend,
Eq. (4), with every skip / stop decision held fixed):

* central finite differences, in FP64, of the oracle's own forward for every
  per-Gaussian input (means2D, conic, opacity, colour, depth) and a loss that
  weights colour, alpha and depth;
* the single-Gaussian closed form d out / d opacity = G (rgb - bg).
"""
import math

import numpy as np
import pytest

from workloads import scenes


def _setup(orc, seed, n=24):
    s = scenes.scene_tiny(n=n, seed=seed, log_scale_mu=-1.6)
    cam = s.cameras[0]
    pr = orc.project_scene(s)
    b = orc.bin_sort_ranges(cam.width, cam.height, pr["means2D"], pr["radius"], pr["depth"])
    rng = np.random.default_rng(seed)
    g = dict(dL_dcolor=rng.standard_normal((3, cam.height, cam.width)),
             dL_dalpha=rng.standard_normal((cam.height, cam.width)),
             dL_ddepth=rng.standard_normal((cam.height, cam.width)))
    return s, cam, pr, b, g


def _loss(orc, cam, b, m2, co, rgb, depth, g, bg):
    f = orc.render_fwd(cam.width, cam.height, b["ranges"], b["point_list"], m2, co, rgb, depth, bg=bg)
    L = (g["dL_dcolor"] * f["color"]).sum() + (g["dL_dalpha"] * f["alpha"]).sum() + \
        (g["dL_ddepth"] * f["depth"]).sum()
    return L, (f["n_contrib"], f["n_examined"])


@pytest.mark.parametrize("seed", [21, 22])
def test_backward_matches_central_differences(orc, seed):
    s, cam, pr, b, g = _setup(orc, seed)
    bg = np.array([0.1, 0.3, 0.2])
    base = dict(m2=pr["means2D"].copy(), co=pr["conic_opacity"].copy(), rgb=pr["rgb"].copy(),
                depth=pr["depth"].copy())
    bw = orc.render_bwd(cam.width, cam.height, b["ranges"], b["point_list"], base["m2"], base["co"], base["rgb"],
                        base["depth"], g["dL_dcolor"], g["dL_dalpha"], g["dL_ddepth"], bg=bg)
    params = []  # (array key, index, analytic)
    for i in range(s.P):
        if pr["radius"][i] == 0:
            continue
        params += [("m2", (i, 0), bw["means2D"][i, 0]), ("m2", (i, 1), bw["means2D"][i, 1])]
        params += [("co", (i, k), bw["conic"][i, k]) for k in range(3)]
        params += [("co", (i, 3), bw["opacity"][i])]
        params += [("rgb", (i, k), bw["rgb"][i, k]) for k in range(3)]
        params += [("depth", (i,), bw["depth"][i])]
    checked = skipped = 0
    scale = max(1e-12, float(np.sqrt(np.mean([p[2] ** 2 for p in params]))))
    for key, idx, ana in params:
        fds = []
        fps = []
        for h in (1e-6, 5e-7):
            vals = []
            for sgn in (1, -1):
                arrs = {k: v.copy() for k, v in base.items()}
                arrs[key][idx] += sgn * h
                L, fp = _loss(orc, cam, b, arrs["m2"], arrs["co"], arrs["rgb"], arrs["depth"], g, bg)
                vals.append(L)
                fps.append(fp)
            fds.append((vals[0] - vals[1]) / (2 * h))
        stable = all(np.array_equal(fps[0][0], f[0]) and np.array_equal(fps[0][1], f[1]) for f in fps)
        if not stable or abs(fds[0] - fds[1]) > 1e-5 * (abs(fds[0]) + scale):
            skipped += 1
            continue
        checked += 1
        assert abs(fds[0] - ana) <= 2e-6 * (abs(ana) + scale), (key, idx, fds[0], ana)
    assert checked > 0.95 * len(params), (checked, skipped)


def test_single_gaussian_opacity_gradient_closed_form(orc):
    W, H = 32, 32
    inv = np.linalg.inv(np.array([[6.0, 1.0], [1.0, 4.0]]))
    mu = np.array([[15.2, 16.7]])
    o, rgb, bg = 0.6, np.array([[0.8, 0.3, 0.5]]), np.array([0.1, 0.2, 0.7])
    co = np.array([[inv[0, 0], inv[0, 1], inv[1, 1], o]])
    b = orc.bin_sort_ranges(W, H, mu, np.array([20], np.int32), np.array([1.0]))
    for (px, py, c) in [(15, 16, 0), (17, 15, 1), (13, 18, 2)]:
        gC = np.zeros((3, H, W))
        gC[c, py, px] = 1.0
        bw = orc.render_bwd(W, H, b["ranges"], b["point_list"], mu, co, rgb, np.array([1.0]), gC, bg=bg)
        d = np.array([px, py]) - mu[0]
        G = math.exp(-0.5 * d @ inv @ d)
        assert o * G < 0.99 and o * G > 1 / 255
        assert bw["opacity"][0] == pytest.approx(G * (rgb[0, c] - bg[c]), rel=1e-12)
        assert bw["rgb"][0, c] == pytest.approx(o * G, rel=1e-12)
