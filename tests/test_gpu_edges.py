"""Edge cases of the method on the GPU path, each against the oracle or a
closed form: empty and fully culled scenes, a 1x1 image, every Gaussian in one
tile (lists longer than several staging batches and chunks), equal depths
(order by id), the identical-alpha stack (golden fixture), zero opacity --
forward images and, for every backward variant, gradients (colour, alpha and
depth upstream) against the oracle's derivative."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from parity import MARGIN, compare_forward, compare_grads, oracle_bwd_from_gpu, oracle_render_from_gpu, to_np
from workloads import scenes

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
# (variant, sub-tile, order[, "split" / "pool": split walks / the persistent task pool])
VARIANTS = [("static", 16, "raster"), ("pixel", 8, "raster"), ("pixel", 8, "cost"), ("pixel", 16, "cost"),
            ("pixel", 16, "cost", "pool"), ("pixel", 32, "cost"), ("pixel", 32, "cost", "pool"),
            ("static_wave", 16, "raster"), ("gauss", 8, "cost"), ("hybrid", 8, "cost")]
BWD_VARIANTS = [v for v in VARIANTS if v[0] in ("static", "pixel", "static_wave")] + [("pixel", 16, "cost", "split")]


def _cfg(v, bg=(0.0, 0.0, 0.0)):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    flags = (B.FLAG_SPLIT_WALKS if "split" in v[3:] else 0) | (B.FLAG_PERSISTENT if "pool" in v[3:] else 0)
    return make_cfg(*v[:3], bg, flags=flags)


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _render_all(rast, prep, bg=(0.0, 0.0, 0.0)):
    outs = {}
    for v in VARIANTS:
        outs[v] = rast.render_fwd(prep, _cfg(v, bg))
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("method", ["fused", "sort"])
def test_empty_scene(rast, method):
    s = scenes.scene_tiny(n=1, seed=1)
    for k in ("means3D", "log_scales", "quats", "opacity", "colors"):
        setattr(s, k, getattr(s, k)[:0])
    print(f"[edge] empty method={method}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    assert prep.n_pairs == 0
    bg = (0.2, 0.4, 0.6)
    for key, out in _render_all(rast, prep, bg).items():
        assert torch.all(out["final_T"] == 1.0), key
        assert torch.all(out["n_contrib"] == 0), key
        for c in range(3):
            assert torch.allclose(out["color"][c], torch.full_like(out["color"][c], bg[c])), key


@pytest.mark.parametrize("method", ["fused", "sort"])
def test_all_culled(rast, method):
    s = scenes.scene_tiny(n=50, seed=2)
    s.means3D[:, 2] = -1.0  # behind the camera
    print(f"[edge] culled method={method}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    assert prep.n_pairs == 0
    assert int(prep.radius.abs().sum()) == 0
    for key, out in _render_all(rast, prep).items():
        assert torch.all(out["final_T"] == 1.0), key


@pytest.mark.parametrize("method", ["fused", "sort"])
def test_one_pixel_image(rast, method):
    s = scenes.scene_tiny(n=30, seed=4, width=1, height=1)
    s.means3D[:, :2] *= 0.01
    print(f"[edge] 1x1 method={method}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    assert prep.n_pairs > 0
    orc = oracle_render_from_gpu(prep)
    for key, out in _render_all(rast, prep).items():
        compare_forward(out, orc, name=f"1x1/{key}")


@pytest.mark.parametrize("method", ["fused", "sort"])
def test_one_tile_holds_everything(rast, method):
    # 3000 small Gaussians all inside pixel tile (1,1) of a 64x48 image
    rng = np.random.default_rng(5)
    s = scenes.scene_tiny(n=3000, seed=6, width=64, height=48, log_scale_mu=-5.5)
    z = rng.uniform(3, 5, s.P)
    # pixel centre (24, 24) -> camera ray x/z = (24.5 - 32)/64
    s.means3D[:, 0] = ((24.5 - 32.0) / 64.0 + rng.uniform(-0.05, 0.05, s.P)) * z
    s.means3D[:, 1] = ((24.5 - 24.0) / 64.0 + rng.uniform(-0.05, 0.05, s.P)) * z
    s.means3D[:, 2] = z
    s.log_scales[:] = -6.0
    s.opacity[:] = 0.05
    print(f"[edge] one-tile method={method}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    torch.cuda.synchronize()
    rg = to_np(prep.ranges)
    lens = rg[:, 1] - rg[:, 0]
    assert lens.max() >= 2000, lens.max()
    ob = oracle.bin_sort_ranges(64, 48, to_np(prep.means2D), to_np(prep.radius), to_np(prep.depth))
    np.testing.assert_array_equal(to_np(prep.point_list), ob["point_list"])
    np.testing.assert_array_equal(rg, ob["ranges"])
    orc = oracle_render_from_gpu(prep)
    for key, out in _render_all(rast, prep).items():
        compare_forward(out, orc, name=f"one-tile/{key}")


@pytest.mark.parametrize("method", ["fused", "sort"])
def test_equal_depths_keep_id_order(rast, method):
    s = scenes.scene_tiny(n=200, seed=7, log_scale_mu=-2.5)
    s.means3D[:, 2] = 4.0  # every depth equal
    print(f"[edge] equal-depth method={method}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    torch.cuda.synchronize()
    ob = oracle.bin_sort_ranges(s.cameras[0].width, s.cameras[0].height, to_np(prep.means2D), to_np(prep.radius),
                                to_np(prep.depth))
    np.testing.assert_array_equal(to_np(prep.point_list), ob["point_list"])
    rg = to_np(prep.ranges)
    pl = to_np(prep.point_list)
    for t in range(rg.shape[0]):
        seg = pl[rg[t, 0]:rg[t, 1]]
        assert np.all(np.diff(seg) > 0)


def _prep_2d(rast, W, H, means2D, conic_opacity, rgb, depth, radius):
    from paper_2412_17378_amd import bgs as B
    from paper_2412_17378_amd.pipeline import Prepared
    dev = torch.device("cuda")
    pr = dict(means2D=torch.tensor(means2D, dtype=torch.float32, device=dev).contiguous(),
              conic_opacity=torch.tensor(conic_opacity, dtype=torch.float32, device=dev).contiguous(),
              rgb=torch.tensor(rgb, dtype=torch.float32, device=dev).contiguous(),
              depth=torch.tensor(depth, dtype=torch.float32, device=dev).contiguous(),
              radius=torch.tensor(radius, dtype=torch.int32, device=dev).contiguous())
    pr["tiles_touched"] = torch.ones(len(depth), dtype=torch.int32, device=dev)  # nonzero: visible
    return rast.bin_sort_ranges(W, H, pr, "fused")


def test_identical_alpha_stack_golden(rast):
    with open(os.path.join(GOLDEN, "alpha_stack.json")) as fh:
        gold = json.load(fh)
    K = gold["stack_size"]
    px, py = gold["pixel"]
    prep = _prep_2d(rast, 16, 16, [[px, py]] * K, [[1.0, 0.0, 1.0, gold["alpha"]]] * K, [gold["rgb"]] * K,
                    list(range(1, K + 1)), [4] * K)
    for key, out in _render_all(rast, prep).items():
        assert int(out["n_contrib"][py, px]) == gold["n_contrib"], key
        assert float(out["final_T"][py, px]) == pytest.approx(gold["final_T"], rel=1e-6), key
        np.testing.assert_allclose(to_np(out["color"][:, py, px]), gold["color"], rtol=1e-6)
        assert float(out["depth"][py, px]) == pytest.approx(gold["out_depth"], rel=1e-6)


def test_zero_opacity_is_background(rast):
    s = scenes.scene_tiny(n=100, seed=9)
    s.opacity[:] = 0.0
    prep = rast.prepare_scene(s)
    assert prep.n_pairs > 0
    bg = (0.3, 0.6, 0.9)
    for key, out in _render_all(rast, prep, bg).items():
        assert torch.all(out["n_contrib"] == 0), key
        assert torch.all(out["final_T"] == 1.0), key


def _check_backward(rast, prep, name, bg=(0.0, 0.0, 0.0), seed=11):
    """Every backward variant against the oracle's derivative on the GPU's own
    splats and lists, with colour, alpha and depth upstream gradients (zero at
    the oracle's near-threshold pixels on both sides)."""
    from paper_2412_17378_amd import make_cfg
    H, W = prep.height, prep.width
    orc = oracle_render_from_gpu(prep, bg=bg)
    flagged = orc["margin"] < MARGIN
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, H, W)).astype(np.float32)
    gA = rng.standard_normal((H, W)).astype(np.float32)
    gD = rng.standard_normal((H, W)).astype(np.float32)
    gC[:, flagged] = 0.0
    gA[flagged] = 0.0
    gD[flagged] = 0.0
    ob = oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg)
    dev = torch.device("cuda")
    for v in BWD_VARIANTS:
        print(f"[edge-bwd] case={name} cfg={v}", flush=True)
        cfg = _cfg(v, bg)
        fwd = rast.render_fwd(prep, cfg)
        grads = rast.render_bwd(prep, cfg, fwd, torch.from_numpy(gC).to(dev), torch.from_numpy(gA).to(dev),
                                torch.from_numpy(gD).to(dev))
        torch.cuda.synchronize()
        compare_grads(grads, ob, name=f"{name}/{v}")
    return ob


def test_backward_one_pixel_image(rast):
    s = scenes.scene_tiny(n=30, seed=4, width=1, height=1)
    s.means3D[:, :2] *= 0.01
    prep = rast.prepare_scene(s)
    ob = _check_backward(rast, prep, "1x1", bg=(0.2, 0.4, 0.6))
    assert float(np.abs(ob["rgb"]).max()) > 0


def test_backward_one_tile_holds_everything(rast):
    rng = np.random.default_rng(5)
    s = scenes.scene_tiny(n=3000, seed=6, width=64, height=48, log_scale_mu=-5.5)
    z = rng.uniform(3, 5, s.P)
    s.means3D[:, 0] = ((24.5 - 32.0) / 64.0 + rng.uniform(-0.05, 0.05, s.P)) * z
    s.means3D[:, 1] = ((24.5 - 24.0) / 64.0 + rng.uniform(-0.05, 0.05, s.P)) * z
    s.means3D[:, 2] = z
    s.log_scales[:] = -6.0
    s.opacity[:] = 0.05
    prep = rast.prepare_scene(s)
    torch.cuda.synchronize()
    assert int((prep.ranges[:, 1] - prep.ranges[:, 0]).max()) >= 2000
    _check_backward(rast, prep, "one-tile", bg=(0.1, 0.1, 0.1))


def test_backward_equal_depths(rast):
    s = scenes.scene_tiny(n=200, seed=7, log_scale_mu=-2.5)
    s.means3D[:, 2] = 4.0
    prep = rast.prepare_scene(s)
    _check_backward(rast, prep, "equal-depth")


def test_backward_identical_alpha_stack(rast):
    with open(os.path.join(GOLDEN, "alpha_stack.json")) as fh:
        gold = json.load(fh)
    K = gold["stack_size"]
    px, py = gold["pixel"]
    prep = _prep_2d(rast, 16, 16, [[px, py]] * K, [[1.0, 0.0, 1.0, gold["alpha"]]] * K, [gold["rgb"]] * K,
                    list(range(1, K + 1)), [4] * K)
    _check_backward(rast, prep, "alpha-stack", bg=(0.2, 0.3, 0.4))


def test_backward_zero_opacity(rast):
    from paper_2412_17378_amd import make_cfg
    s = scenes.scene_tiny(n=100, seed=9)
    s.opacity[:] = 0.0
    prep = rast.prepare_scene(s)
    H, W = prep.height, prep.width
    gC = torch.randn(3, H, W, device="cuda")
    for v in BWD_VARIANTS:
        cfg = _cfg(v, (0.3, 0.6, 0.9))
        fwd = rast.render_fwd(prep, cfg)
        grads = rast.render_bwd(prep, cfg, fwd, gC)
        torch.cuda.synchronize()
        for k, t in grads.items():
            assert torch.all(t == 0), (v, k)
