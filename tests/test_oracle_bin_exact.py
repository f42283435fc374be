"""Pins of the oracle's exact ellipse-tile binning (orc_bin_exact):

* the rectangle minimum of the quadratic form against a dense brute force
  and, for axis-aligned forms, the closed form a dx^2 + c dy^2 with dx, dy the
  distances from the origin to the rectangle's x and y ranges;
* the q bound against 2 ln(255 o) (alpha = o exp(-q/2) reaches 1/255 there);
* the exact pairs are the square rule's pairs with some removed, order kept;
* safety by brute force: no removed pair has a pixel centre in its tile where
  the Gaussian's alpha reaches 1/255;
* the forward and backward of Eq. (4) from the exact lists equal those from
  the square-rule lists (the removed entries are skipped at every pixel).
"""
import math

import numpy as np
import pytest

from workloads import scenes

A_MIN = float(np.float32(1.0) / np.float32(255.0))


def _rand_form(rng):
    a, c = np.exp(rng.uniform(-6, 2, 2))
    b = rng.uniform(-0.999, 0.999) * math.sqrt(a * c)
    return a, b, c


def test_rect_min_q_brute_force():
    import oracle
    rng = np.random.default_rng(0)
    for _ in range(300):
        a, b, c = _rand_form(rng)
        lx, ly = rng.uniform(-40, 30, 2)
        hx, hy = lx + rng.uniform(0, 25), ly + rng.uniform(0, 25)
        got = oracle.rect_min_q(a, b, c, lx, hx, ly, hy)
        xs, ys = np.linspace(lx, hx, 301), np.linspace(ly, hy, 301)
        X, Y = np.meshgrid(xs, ys)
        q = a * X * X + 2 * b * X * Y + c * Y * Y
        grid = float(q.min())
        # the exact minimum lies below every sample and within one grid step
        # (times the largest gradient on the rectangle) of the best one
        gx = np.abs(2 * a * X + 2 * b * Y).max()
        gy = np.abs(2 * b * X + 2 * c * Y).max()
        step = gx * (hx - lx) / 300 + gy * (hy - ly) / 300
        assert got <= grid * (1 + 1e-12) + 1e-12, (a, b, c, lx, hx, ly, hy, got, grid)
        assert grid - got <= step + 1e-9, (got, grid, step)


def test_rect_min_q_axis_aligned_closed_form():
    import oracle
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, c = np.exp(rng.uniform(-4, 2, 2))
        lx, ly = rng.uniform(-30, 30, 2)
        hx, hy = lx + rng.uniform(0, 20), ly + rng.uniform(0, 20)
        dx = 0.0 if lx <= 0 <= hx else min(abs(lx), abs(hx))
        dy = 0.0 if ly <= 0 <= hy else min(abs(ly), abs(hy))
        want = a * dx * dx + c * dy * dy
        assert math.isclose(oracle.rect_min_q(a, 0.0, c, lx, hx, ly, hy), want, rel_tol=1e-13, abs_tol=1e-300)


def test_q_limit():
    import oracle
    for o in (A_MIN, 0.01, 0.3, 0.99, 1.0):
        tau = 2 * math.log(o / A_MIN)
        lim = oracle.bin_q_limit(o)
        assert lim >= tau and lim - tau <= (abs(tau) + 1) / 1000
        # at q = tau the Gaussian's alpha is exactly the skip threshold
        assert math.isclose(o * math.exp(-tau / 2), A_MIN, rel_tol=1e-12)
    assert oracle.bin_q_limit(A_MIN * 0.5) < 0.0  # never blends: no tile


def _lists(orc, s, exact):
    cam = s.cameras[0]
    pr = orc.project_scene(s)
    co = pr["conic_opacity"] if exact else None
    return pr, orc.bin_sort_ranges(cam.width, cam.height, pr["means2D"], pr["radius"], pr["depth"],
                                   conic_opacity=co)


@pytest.mark.parametrize("seed,n", [(5, 24), (7, 120), (9, 300)])
def test_exact_pairs_are_a_filtered_square_rule(seed, n):
    import oracle
    s = scenes.scene_tiny(n=n, seed=seed, width=96, height=80)
    cam = s.cameras[0]
    pr, std = _lists(oracle, s, False)
    _, ex = _lists(oracle, s, True)
    assert ex["n_pairs"] <= std["n_pairs"]
    TX = (cam.width + 15) // 16
    for t in range(std["ranges"].shape[0]):
        a = std["point_list"][std["ranges"][t, 0]:std["ranges"][t, 1]]
        b = ex["point_list"][ex["ranges"][t, 0]:ex["ranges"][t, 1]]
        keep = np.isin(a, b)
        np.testing.assert_array_equal(a[keep], b)  # a subsequence, same order
        tx, ty = t % TX, t // TX
        for g in a[~keep]:  # removed: no pixel centre of the tile can blend g
            ca, cb, cc, o = pr["conic_opacity"][g]
            u, v = pr["means2D"][g]
            px = np.arange(tx * 16, min(tx * 16 + 16, cam.width), dtype=np.float64) - u
            py = np.arange(ty * 16, min(ty * 16 + 16, cam.height), dtype=np.float64) - v
            X, Y = np.meshgrid(px, py)
            power = -0.5 * (ca * X * X + cc * Y * Y) - cb * X * Y
            assert np.all(np.minimum(0.99, o * np.exp(power)) < A_MIN), (t, g)


def test_exact_lists_render_the_same():
    import oracle
    s = scenes.scene_tiny(n=300, seed=9, width=96, height=80)
    cam = s.cameras[0]
    pr, std = _lists(oracle, s, False)
    _, ex = _lists(oracle, s, True)
    assert ex["n_pairs"] < std["n_pairs"]
    args = (pr["means2D"], pr["conic_opacity"], pr["rgb"], pr["depth"])
    f_std = oracle.render_fwd(cam.width, cam.height, std["ranges"], std["point_list"], *args)
    f_ex = oracle.render_fwd(cam.width, cam.height, ex["ranges"], ex["point_list"], *args)
    for k in ("color", "alpha", "depth", "final_T"):
        np.testing.assert_array_equal(f_ex[k], f_std[k])
    # fewer entries examined per pixel (the removed ones were examined and skipped)
    assert np.all(f_ex["n_examined"] <= f_std["n_examined"]) and f_ex["blends"] < f_std["blends"]
    gC = np.random.default_rng(2).standard_normal((3, cam.height, cam.width))
    b_std = oracle.render_bwd(cam.width, cam.height, std["ranges"], std["point_list"], *args, gC)
    b_ex = oracle.render_bwd(cam.width, cam.height, ex["ranges"], ex["point_list"], *args, gC)
    for k in ("means2D", "conic", "opacity", "rgb", "depth"):
        # the same per-pixel terms, accumulated in another order
        np.testing.assert_allclose(b_ex[k], b_std[k], rtol=1e-11, atol=1e-12 * float(np.abs(b_std[k]).max()))
