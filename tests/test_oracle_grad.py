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


# ---------------------------------------------------------------- mag pins
# The oracle's backward also returns, per gradient element, m = the sum over
# pixels of the absolute value of that pixel's term.  The parity rule uses m
# as a floor of the gradient tolerance, so it is pinned here on its own.  A
# Gaussian sits at most once in a pixel's list, so each pixel adds exactly
# one term to each element, and m is the sum over pixels of |the gradient the
# pixel alone produces|.

_KEYS = ("means2D", "conic", "opacity", "rgb", "depth")


def _small(orc, seed, W=20, H=18):
    s = scenes.scene_tiny(n=16, seed=seed, width=W, height=H, log_scale_mu=-1.4)
    cam = s.cameras[0]
    pr = orc.project_scene(s)
    b = orc.bin_sort_ranges(W, H, pr["means2D"], pr["radius"], pr["depth"])
    return cam, pr, b


def _bwd(orc, cam, pr, b, gC, gA=None, gD=None, bg=(0.2, 0.5, 0.1)):
    return orc.render_bwd(cam.width, cam.height, b["ranges"], b["point_list"], pr["means2D"], pr["conic_opacity"],
                          pr["rgb"], pr["depth"], gC, gA, gD, bg=bg)


@pytest.mark.parametrize("seed", [31, 32])
def test_mag_is_sum_of_per_pixel_absolute_terms(orc, seed):
    """Brute force: one backward per pixel with the upstream gradient of that
    pixel alone; m must equal the sum of the absolute per-pixel gradients."""
    cam, pr, b = _small(orc, seed)
    W, H = cam.width, cam.height
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, H, W))
    gA = rng.standard_normal((H, W))
    gD = rng.standard_normal((H, W))
    full = _bwd(orc, cam, pr, b, gC, gA, gD)
    acc = {k: np.zeros_like(full[k]) for k in _KEYS}
    summed = {k: np.zeros_like(full[k]) for k in _KEYS}
    for py in range(H):
        for px in range(W):
            one = [np.zeros_like(gC), np.zeros_like(gA), np.zeros_like(gD)]
            one[0][:, py, px] = gC[:, py, px]
            one[1][py, px] = gA[py, px]
            one[2][py, px] = gD[py, px]
            o = _bwd(orc, cam, pr, b, *one)
            for k in _KEYS:
                acc[k] += np.abs(o[k])
                summed[k] += o[k]
    for k in _KEYS:
        scale = float(np.abs(acc[k]).max()) + 1e-300
        np.testing.assert_allclose(full["mag"][k], acc[k], rtol=1e-12, atol=1e-13 * scale, err_msg=k)
        np.testing.assert_allclose(full[k], summed[k], rtol=1e-10, atol=1e-12 * scale, err_msg=k)
    assert any(float(np.abs(full[k]).max()) > 0 for k in _KEYS)


def test_mag_bounds_the_gradient(orc):
    """Triangle inequality m >= |y| element by element, with strict excess
    somewhere (terms of both signs cancel for the mean and conic gradients)."""
    cam, pr, b = _small(orc, 33, W=48, H=40)
    rng = np.random.default_rng(33)
    o = _bwd(orc, cam, pr, b, rng.standard_normal((3, 40, 48)), rng.standard_normal((40, 48)),
             rng.standard_normal((40, 48)))
    for k in _KEYS:
        assert np.all(o["mag"][k] >= np.abs(o[k]) * (1 - 1e-12)), k
    assert np.any(o["mag"]["means2D"] > 1.01 * np.abs(o["means2D"]))


def test_mag_equals_gradient_when_every_term_is_positive(orc):
    """With positive upstream colour and depth gradients every per-pixel term
    of d/drgb (w g_C) and d/ddepth (w g_D) is non-negative: m == y."""
    cam, pr, b = _small(orc, 34)
    W, H = cam.width, cam.height
    rng = np.random.default_rng(34)
    o = _bwd(orc, cam, pr, b, rng.uniform(0.1, 1.0, (3, H, W)), None, rng.uniform(0.1, 1.0, (H, W)))
    assert float(o["rgb"].max()) > 0 and float(o["depth"].max()) > 0
    np.testing.assert_allclose(o["mag"]["rgb"], o["rgb"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(o["mag"]["depth"], o["depth"], rtol=1e-13, atol=0)


def test_mag_single_gaussian_single_pixel(orc):
    """One Gaussian seen by one pixel: one term per element, so m == |y|."""
    W = H = 1
    inv = np.linalg.inv(np.array([[3.0, 0.7], [0.7, 2.0]]))
    mu = np.array([[0.4, -0.3]])
    co = np.array([[inv[0, 0], inv[0, 1], inv[1, 1], 0.7]])
    rgb, depth = np.array([[0.3, 0.9, 0.6]]), np.array([2.5])
    b = orc.bin_sort_ranges(W, H, mu, np.array([3], np.int32), depth)
    assert b["n_pairs"] == 1
    o = orc.render_bwd(W, H, b["ranges"], b["point_list"], mu, co, rgb, depth, np.array([[[0.8]], [[-1.3]], [[0.4]]]),
                       np.array([[0.6]]), np.array([[-0.9]]), bg=(0.2, 0.1, 0.4))
    for k in _KEYS:
        assert np.any(o[k] != 0), k
        np.testing.assert_allclose(o["mag"][k], np.abs(o[k]), rtol=1e-15, atol=0, err_msg=k)
