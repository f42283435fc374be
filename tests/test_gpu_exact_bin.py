"""GPU parity of exact ellipse-tile binning (bgs_tile_lists_exact).

* Lists: the oracle's fp64 exact rule on the GPU's own fp32 splats.  The
  GPU evaluates the rule on a slightly larger ellipse, so it must hold every
  pair the oracle keeps, may hold extra pairs only where the rule's minimum of
  q over the tile comes within the fp32 padding of the bound, and each of its
  lists is a subsequence of the square rule's list (same order).
* Renders: forward images from exact lists equal those from the square rule's
  lists bit for bit for the pixel-wise kernels (the removed entries are
  skipped at every pixel); gradients agree to the accumulation order.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import to_np
from workloads import scenes

pytestmark = pytest.mark.gpu

# "tall": 300 Gaussians about 50 tile rows high on a 48 x 1600 image, so that a
# chunk's row intervals (64 Gaussians) overflow the emit's 1024-row buffer and
# are taken in several windows
CASES = ["tiny-300", "0", "sh3-tiny", "tall"]
PX_SLACK = 1.0 / 64.0


def _scene(name):
    if name == "sh3-tiny":
        return scenes.scene_tiny(n=200, seed=11, width=80, height=56, sh_degree=3)
    if name == "tall":
        return scenes.scene_tiny(n=300, seed=9, width=48, height=1600, log_scale_mu=2.4)
    return scenes.make(name)


@pytest.fixture(scope="module")
def rasts():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True), Rasterizer("cuda", binning="ellipse", poison_outputs=True)


def _near_boundary(W, H, tile_id, g, m2, co):
    """The pair's tile meets the ellipse enlarged by the GPU's fp32 padding."""
    TX = (W + 15) // 16
    tx, ty = tile_id % TX, tile_id // TX
    a, b, c, o = (float(v) for v in co[g])
    u, v = (float(x) for x in m2[g])
    lim = oracle.bin_q_limit(o)
    det = a * c - b * b
    px = PX_SLACK + math.sqrt(max(lim, 0.0) * c / det) / 1024 + 1e-3
    py = PX_SLACK + math.sqrt(max(lim, 0.0) * a / det) / 1024 + 1e-3
    q = oracle.rect_min_q(a, b, c, tx * 16 - px - u, tx * 16 + 15 + px - u, ty * 16 - py - v, ty * 16 + 15 + py - v)
    return q <= lim * (1 + 1 / 512) + 1 / 512


def _check_lists(W, H, prep_sq, prep_ex, window=None):
    m2, co = to_np(prep_ex.means2D).astype(np.float64), to_np(prep_ex.conic_opacity).astype(np.float64)
    ob = oracle.bin_sort_ranges(W, H, m2, to_np(prep_ex.radius), to_np(prep_ex.depth), window=window,
                                conic_opacity=co)
    rg_ex, pl_ex = to_np(prep_ex.ranges), to_np(prep_ex.point_list)
    rg_sq, pl_sq = to_np(prep_sq.ranges), to_np(prep_sq.point_list)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    tiles = range(TX * TY) if window is None else [ty * TX + tx for ty in range(window[1], window[3])
                                                   for tx in range(window[0], window[2])]
    extra = kept = 0
    for t in tiles:
        gpu = pl_ex[rg_ex[t, 0]:rg_ex[t, 1]]
        sq = pl_sq[rg_sq[t, 0]:rg_sq[t, 1]]
        orc = ob["point_list"][ob["ranges"][t, 0]:ob["ranges"][t, 1]]
        inside = np.isin(sq, gpu)
        np.testing.assert_array_equal(sq[inside], gpu)  # a subsequence of the square rule's list
        missing = orc[~np.isin(orc, gpu)]
        assert missing.size == 0, f"tile {t}: the GPU dropped pairs the rule keeps: {missing[:8]}"
        for g in gpu[~np.isin(gpu, orc)]:
            assert _near_boundary(W, H, t, int(g), m2, co), f"tile {t} Gaussian {g}: extra pair off the boundary"
            extra += 1
        kept += gpu.size
    return kept, extra


@pytest.mark.parametrize("name", CASES)
def test_exact_lists_vs_oracle(rasts, name):
    sq, ex = rasts
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[exact-bin] lists case={name} P={s.P}", flush=True)
    p_sq = sq.prepare_scene(s)
    p_ex = ex.prepare_scene(s)
    torch.cuda.synchronize()
    assert p_ex.n_pairs <= p_sq.n_pairs
    kept, extra = _check_lists(cam.width, cam.height, p_sq, p_ex)
    assert kept == p_ex.n_pairs
    assert extra <= max(4, kept // 50)  # the padding adds only a sliver of pairs


@pytest.mark.parametrize("name", CASES)
def test_exact_lists_render_the_same(rasts, name):
    from paper_2412_17378_amd import make_cfg
    sq, ex = rasts
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[exact-bin] render case={name}", flush=True)
    p_sq = sq.prepare_scene(s)
    p_ex = ex.prepare_scene(s)
    gC = torch.from_numpy(np.random.default_rng(4).standard_normal((3, cam.height, cam.width)).astype(np.float32))
    gC = gC.cuda()
    for v, sub, o in (("static", 16, "raster"), ("pixel", 8, "cost"), ("pixel", 16, "cost")):
        cfg = make_cfg(v, sub, o, tuple(s.bg))
        f_sq = sq.render_fwd(p_sq, cfg)
        f_ex = ex.render_fwd(p_ex, cfg)
        torch.cuda.synchronize()
        for k in ("color", "alpha", "depth", "final_T"):
            assert torch.equal(f_sq[k], f_ex[k]), (v, sub, k)
        assert bool(torch.all(f_ex["n_contrib"] <= f_sq["n_contrib"]))
        g_sq = sq.render_bwd(p_sq, cfg, f_sq, gC)
        g_ex = ex.render_bwd(p_ex, cfg, f_ex, gC)
        torch.cuda.synchronize()
        for k in g_sq:
            a, b = g_sq[k], g_ex[k]
            scale = float(a.abs().max()) + 1e-30
            assert float((a - b).abs().max()) <= 1e-4 * scale, (v, sub, k)


def test_exact_lists_full_size():
    """1920x1080, 500k Gaussians: lists in windows against the oracle, the
    whole forward image equal to the square rule's, and the pair count."""
    from paper_2412_17378_amd import Rasterizer, make_cfg
    s = scenes.make("1")
    cam = s.cameras[0]
    print(f"[exact-bin] full size P={s.P}", flush=True)
    sq = Rasterizer("cuda", reuse_pairs=False, poison_outputs=True)
    ex = Rasterizer("cuda", reuse_pairs=False, binning="ellipse", poison_outputs=True)
    p_sq = sq.prepare_scene(s)
    p_ex = ex.prepare_scene(s)
    torch.cuda.synchronize()
    print(f"[exact-bin] M square {p_sq.n_pairs} exact {p_ex.n_pairs}", flush=True)
    assert p_ex.n_pairs < 0.7 * p_sq.n_pairs
    rg = to_np(p_sq.ranges)
    heavy = int(np.argmax(rg[:, 1] - rg[:, 0]))
    TX = (cam.width + 15) // 16
    for tw in ([heavy % TX, heavy // TX, heavy % TX + 2, heavy // TX + 2], [10, 10, 14, 13], [60, 30, 63, 33]):
        _check_lists(cam.width, cam.height, p_sq, p_ex, window=tw)
    cfg = make_cfg("static", 16, "raster", tuple(s.bg))
    f_sq = sq.render_fwd(p_sq, cfg)
    f_ex = ex.render_fwd(p_ex, cfg)
    torch.cuda.synchronize()
    for k in ("color", "alpha", "depth", "final_T"):
        assert torch.equal(f_sq[k], f_ex[k]), k
