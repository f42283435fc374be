"""Pins of the oracle's binning, sort and forward blend (Eq. (4) with the skip /
stop rules of the paper's detailed naive per-pixel loop):

* tile membership and per-tile order against a geometric brute force and
  numpy's lexsort;
* a single Gaussian against the closed form alpha rgb + (1 - alpha) bg, with
  the density evaluated from numpy's matrix inverse of the 2D covariance;
* an all-transparent scene equals the background;
* the identical-alpha stack (golden fixture, derived by hand);
* brute-force per-pixel evaluation over a global depth sort;
* invariance to the input order of Gaussians; alpha + final_T = 1.
"""
import json
import math
import os

import numpy as np
import pytest

from workloads import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
A_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))
A_MAX = float(np.float32(0.99))


def _tiny(orc, n=24, seed=5, **kw):
    s = scenes.scene_tiny(n=n, seed=seed, **kw)
    cam = s.cameras[0]
    pr = orc.project_scene(s)
    b = orc.bin_sort_ranges(cam.width, cam.height, pr["means2D"], pr["radius"], pr["depth"])
    return s, cam, pr, b


def _brute_membership(u, v, r, tx, ty, tile=16):
    return r > 0 and (u - r < tile * (tx + 1)) and (u + r >= tile * tx) and \
        (v - r < tile * (ty + 1)) and (v + r >= tile * ty)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bin_sort_ranges_brute_force(orc, seed):
    s, cam, pr, b = _tiny(orc, n=40, seed=seed)
    TX = (cam.width + 15) // 16
    TY = (cam.height + 15) // 16
    order = sorted(range(s.P), key=lambda g: (pr["depth"][g], g))
    total = 0
    for ty in range(TY):
        for tx in range(TX):
            want = [g for g in order if _brute_membership(pr["means2D"][g, 0], pr["means2D"][g, 1],
                                                          pr["radius"][g], tx, ty)]
            t = ty * TX + tx
            st, en = b["ranges"][t]
            got = list(b["point_list"][st:en]) if en > st else []
            assert got == want, (tx, ty)
            total += len(want)
    assert total == b["n_pairs"]


def test_sort_matches_lexsort(orc):
    rng = np.random.default_rng(3)
    M, P = 5000, 300
    tid = rng.integers(0, 37, M).astype(np.int32)
    gid = rng.integers(0, P, M).astype(np.int32)
    depth = rng.uniform(1, 2, P)
    depth[::7] = depth[0]  # ties broken by Gaussian id
    t2, g2 = orc.sort_pairs(tid, gid, depth)
    order = np.lexsort((gid, depth[gid], tid))
    np.testing.assert_array_equal(t2, tid[order])
    np.testing.assert_array_equal(g2, gid[order])


def _frame_2d(orc, width, height, means2D, conic_opacity, rgb, depth, radius):
    b = orc.bin_sort_ranges(width, height, means2D, np.asarray(radius, np.int32), depth)
    return b


def test_single_gaussian_closed_form(orc):
    W, H = 40, 36
    S2 = np.array([[9.0, 2.5], [2.5, 5.0]])
    inv = np.linalg.inv(S2)
    mu = np.array([20.3, 17.6])
    o, rgb, bg = 0.8, np.array([0.9, 0.4, 0.1]), np.array([0.05, 0.1, 0.2])
    co = np.array([[inv[0, 0], inv[0, 1], inv[1, 1], o]])
    b = _frame_2d(orc, W, H, mu[None], co, rgb[None], np.array([2.0]), [40])
    f = orc.render_fwd(W, H, b["ranges"], b["point_list"], mu[None], co, rgb[None], np.array([2.0]), bg=bg)
    for py in range(H):
        for px in range(W):
            d = np.array([px, py]) - mu
            G = math.exp(-0.5 * d @ inv @ d)
            a = min(A_MAX, o * G)
            want = bg if a < A_MIN else a * rgb + (1 - a) * bg
            np.testing.assert_allclose(f["color"][:, py, px], want, atol=1e-13)
            assert f["n_contrib"][py, px] == (0 if a < A_MIN else 1)


def test_all_transparent_is_background(orc):
    s = scenes.scene_tiny(n=30, seed=9)
    s.opacity[:] = 0.0
    cam = s.cameras[0]
    pr = orc.project_scene(s)
    b = orc.bin_sort_ranges(cam.width, cam.height, pr["means2D"], pr["radius"], pr["depth"])
    bg = np.array([0.3, 0.6, 0.9])
    f = orc.render_fwd(cam.width, cam.height, b["ranges"], b["point_list"], pr["means2D"], pr["conic_opacity"],
                       pr["rgb"], pr["depth"], bg=bg)
    assert b["n_pairs"] > 0
    np.testing.assert_array_equal(f["color"], np.broadcast_to(bg[:, None, None], f["color"].shape))
    assert np.all(f["alpha"] == 0) and np.all(f["depth"] == 0) and np.all(f["final_T"] == 1)
    assert np.all(f["n_contrib"] == 0)


def test_identical_alpha_stack_golden(orc):
    with open(os.path.join(GOLDEN, "alpha_stack.json")) as fh:
        gold = json.load(fh)
    K = gold["stack_size"]
    W, H = 16, 16
    px, py = gold["pixel"]
    means = np.tile(np.array([[px, py]], np.float64), (K, 1))
    co = np.tile(np.array([[1.0, 0.0, 1.0, gold["alpha"]]]), (K, 1))
    rgb = np.tile(np.array([gold["rgb"]]), (K, 1))
    depth = np.arange(1, K + 1, dtype=np.float64)
    b = _frame_2d(orc, W, H, means, co, rgb, depth, [4] * K)
    f = orc.render_fwd(W, H, b["ranges"], b["point_list"], means, co, rgb, depth)
    assert f["n_contrib"][py, px] == gold["n_contrib"]
    assert f["n_examined"][py, px] == gold["n_examined"]
    assert f["n_blended"][py, px] == gold["n_contrib"]  # identical entries: every one before the stop blends
    assert f["final_T"][py, px] == pytest.approx(gold["final_T"], rel=1e-15)
    np.testing.assert_allclose(f["color"][:, py, px], gold["color"], rtol=1e-14)
    assert f["alpha"][py, px] == pytest.approx(gold["out_alpha"], rel=1e-14)
    assert f["depth"][py, px] == pytest.approx(gold["out_depth"], rel=1e-14)


def _brute_pixel(pr, order, px, py, tx, ty, bg):
    T, C, D, n, ex, nb = 1.0, np.zeros(3), 0.0, 0, 0, 0
    k = -1
    for g in order:
        if not _brute_membership(pr["means2D"][g, 0], pr["means2D"][g, 1], pr["radius"][g], tx, ty):
            continue
        k += 1
        ex += 1
        dx, dy = px - pr["means2D"][g, 0], py - pr["means2D"][g, 1]
        a, b_, c, o = pr["conic_opacity"][g]
        q = np.array([[a, b_], [b_, c]])
        d = np.array([dx, dy])
        power = -0.5 * d @ q @ d
        if power > 0:
            continue
        alpha = min(A_MAX, o * math.exp(power))
        if alpha < A_MIN:
            continue
        Tn = T * (1 - alpha)
        if Tn < T_MIN:
            break
        C += pr["rgb"][g] * alpha * T
        D += pr["depth"][g] * alpha * T
        T = Tn
        n = k + 1
        nb += 1
    return C + T * bg, D, T, n, ex, nb


@pytest.mark.parametrize("seed,n", [(4, 30), (6, 60)])
def test_render_brute_force(orc, seed, n):
    s, cam, pr, b = _tiny(orc, n=n, seed=seed, log_scale_mu=-1.5)
    bg = np.array([0.2, 0.1, 0.4])
    f = orc.render_fwd(cam.width, cam.height, b["ranges"], b["point_list"], pr["means2D"], pr["conic_opacity"],
                       pr["rgb"], pr["depth"], bg=bg)
    order = sorted(range(s.P), key=lambda g: (pr["depth"][g], g))
    for py in range(cam.height):
        for px in range(cam.width):
            C, D, T, nc, ex, nb = _brute_pixel(pr, order, px, py, px // 16, py // 16, bg)
            np.testing.assert_allclose(f["color"][:, py, px], C, rtol=1e-12, atol=1e-14)
            assert f["depth"][py, px] == pytest.approx(D, rel=1e-12, abs=1e-14)
            assert f["final_T"][py, px] == pytest.approx(T, rel=1e-12)
            assert f["n_contrib"][py, px] == nc
            assert f["n_examined"][py, px] == ex
            assert f["n_blended"][py, px] == nb
    assert np.abs(f["alpha"] + f["final_T"] - 1).max() < 1e-13
    assert f["blends"] == int(f["n_examined"].sum())
    assert f["contributors"] == int(f["n_blended"].sum())
    # some pixels skip entries inside their walked range: both counts are exercised
    assert np.any(f["n_blended"] < f["n_contrib"]) and np.all(f["n_blended"] <= f["n_contrib"])


def test_permutation_invariance(orc):
    s = scenes.scene_tiny(n=50, seed=8, log_scale_mu=-1.5)
    cam = s.cameras[0]

    def render(sc):
        pr = orc.project_scene(sc)
        b = orc.bin_sort_ranges(cam.width, cam.height, pr["means2D"], pr["radius"], pr["depth"])
        return orc.render_fwd(cam.width, cam.height, b["ranges"], b["point_list"], pr["means2D"],
                              pr["conic_opacity"], pr["rgb"], pr["depth"])

    f0 = render(s)
    perm = np.random.default_rng(0).permutation(s.P)
    s.means3D, s.log_scales, s.quats = s.means3D[perm], s.log_scales[perm], s.quats[perm]
    s.opacity, s.colors = s.opacity[perm], s.colors[perm]
    f1 = render(s)
    for k in ("color", "alpha", "depth", "final_T", "n_contrib"):
        np.testing.assert_array_equal(f0[k], f1[k])
