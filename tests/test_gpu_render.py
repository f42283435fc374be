"""GPU parity of render_fwd / render_bwd against the FP64 oracle, through the
C ABI, for every kernel variant and queue order.

The oracle is fed the GPU path's own fp32 splats and per-tile lists (so this
isolates the render stage).  Images: 1e-4 relative (s = 1e-2) on unflagged
pixels, n_contrib exact.  Gradients: 1e-4 relative (s = RMS of the tensor)
with the upstream gradient zeroed at flagged pixels on both sides.  The
static and balanced forward kernels evaluate each pixel in the same order and
must agree bit for bit.
"""
import numpy as np
import pytest
import torch

from parity import (MARGIN, compare_forward, compare_grads, oracle_bwd_from_gpu, oracle_render_from_gpu, to_np)
from workloads import scenes

pytestmark = pytest.mark.gpu

# (variant, sub-tile, queue order[, "pool": the persistent task pool])
VARIANTS = [("static", 16, "raster"), ("pixel", 8, "raster"), ("pixel", 8, "cost"), ("pixel", 16, "cost"),
            ("pixel", 16, "raster"), ("pixel", 32, "cost"), ("static_wave", 16, "raster"), ("gauss", 8, "cost"),
            ("hybrid", 8, "cost"), ("pixel", 16, "cost", "pool"), ("pixel", 32, "cost", "pool")]


def _cfg(v, bg=(0.0, 0.0, 0.0)):
    """(variant, sub-tile, order[, "pool": the persistent task pool])"""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    return make_cfg(*v[:3], bg, flags=B.FLAG_PERSISTENT if "pool" in v[3:] else 0)


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _scene(name):
    if name == "ragged":  # image size not a multiple of 16 in either direction
        return scenes.scene_tiny(n=400, seed=3, width=83, height=45, log_scale_mu=-2.5)
    if name == "sh3":
        return scenes.scene_tiny(n=300, seed=11, width=80, height=56, sh_degree=3)
    return scenes.make(name)


@pytest.mark.parametrize("name", ["tiny-60", "ragged", "0", "sh3"])
@pytest.mark.parametrize("v", VARIANTS)
def test_forward_parity(rast, name, v):
    s = _scene(name)
    bg = (0.1, 0.2, 0.3)
    print(f"[fwd] case={name} cfg={v}", flush=True)
    prep = rast.prepare_scene(s)
    out = rast.render_fwd(prep, _cfg(v, bg))
    torch.cuda.synchronize()
    orc = oracle_render_from_gpu(prep, bg=bg)
    compare_forward(out, orc, name=f"{name}/{v}")


@pytest.mark.parametrize("name", ["tiny-60", "ragged", "0"])
def test_static_and_balanced_bit_identical(rast, name):
    from paper_2412_17378_amd import make_cfg
    s = _scene(name)
    print(f"[fwd-bitwise] case={name}", flush=True)
    prep = rast.prepare_scene(s)
    a = rast.render_fwd(prep, make_cfg("static"))
    for v in (("pixel", 8, "cost"), ("pixel", 16, "cost"), ("pixel", 16, "raster"), ("pixel", 32, "cost"),
              ("static_wave", 16, "raster"), ("pixel", 16, "cost", "pool"), ("pixel", 32, "cost", "pool")):
        b = rast.render_fwd(prep, _cfg(v))
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), (k, v)


@pytest.mark.parametrize("name", ["tiny-60", "ragged", "0", "sh3"])
@pytest.mark.parametrize("v", [v for v in VARIANTS if v[0] in ("static", "pixel", "static_wave")])
def test_backward_parity(rast, name, v):
    s = _scene(name)
    bg = (0.3, 0.1, 0.2)
    print(f"[bwd] case={name} cfg={v}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = _cfg(v, bg)
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    orc_f = oracle_render_from_gpu(prep, bg=bg)
    flagged = orc_f["margin"] < MARGIN
    cam = s.cameras[0]
    rng = np.random.default_rng(99)
    gC = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    gA = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gD = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    for g in (gC, gA[None], gD[None]):
        g[:, flagged] = 0.0
    dev = torch.device("cuda")
    grads = rast.render_bwd(prep, cfg, fwd, torch.from_numpy(gC).to(dev), torch.from_numpy(gA).to(dev),
                            torch.from_numpy(gD).to(dev))
    torch.cuda.synchronize()
    orc = oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg)
    compare_grads(grads, orc, name=f"{name}/{v}")


@pytest.mark.parametrize("name", ["tiny-60", "ragged", "0", "sh3"])
def test_examined_count(rast, name):
    """The forward's optional work count equals the oracle's examined count."""
    s = _scene(name)
    print(f"[examined] case={name}", flush=True)
    prep = rast.prepare_scene(s)
    n = to_np(rast.count_examined(prep))
    orc = oracle_render_from_gpu(prep)
    ok = orc["margin"] >= MARGIN
    np.testing.assert_array_equal(n[ok], orc["n_examined"][ok])


def test_autograd_function(rast):
    """RenderFn gives the same gradients as calling render_bwd directly."""
    from paper_2412_17378_amd import make_cfg, render
    s = scenes.make("0")
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 8, "cost")
    m2 = prep.means2D.clone().requires_grad_(True)
    co = prep.conic_opacity.clone().requires_grad_(True)
    rgb = prep.rgb.clone().requires_grad_(True)
    dep = prep.depth.clone().requires_grad_(True)
    color, alpha, depth = render(m2, co, rgb, dep, prep, cfg, rast)
    g = torch.randn_like(color)
    (color * g).sum().backward()
    fwd = rast.render_fwd(prep, cfg)
    ref = rast.render_bwd(prep, cfg, fwd, g.contiguous())
    torch.cuda.synchronize()
    for t, r in ((m2.grad, ref["means2D"]), (co.grad, ref["conic_opacity"]), (rgb.grad, ref["rgb"])):
        scale = float(r.abs().max()) + 1e-30
        assert float((t - r).abs().max()) <= 1e-4 * scale  # float atomics: order varies


@pytest.mark.parametrize("name", ["0", "sh3"])
def test_backward_split_walks_parity(rast, name):
    """Split backward walks (lower part front to back, upper part back to
    front) against the oracle, with colour, alpha and depth upstream."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    bg = (0.3, 0.1, 0.2)
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost", bg, flags=B.FLAG_SPLIT_WALKS)
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    orc_f = oracle_render_from_gpu(prep, bg=bg)
    flagged = orc_f["margin"] < MARGIN
    cam = s.cameras[0]
    rng = np.random.default_rng(21)
    gC = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    gA = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gD = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gC[:, flagged] = 0.0
    gA[flagged] = 0.0
    gD[flagged] = 0.0
    print(f"[bwd-split] case={name} deepest walk {int(fwd['n_contrib'].max())}", flush=True)
    grads = rast.render_bwd(prep, cfg, fwd, torch.from_numpy(gC).cuda(), torch.from_numpy(gA).cuda(),
                            torch.from_numpy(gD).cuda())
    torch.cuda.synchronize()
    ob = oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg)
    compare_grads(grads, ob, name=f"{name} split")
