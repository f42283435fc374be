"""Packed gradient records (FLAG_PACKED_GRADS, bgs_project_bwd_packed).

* Every backward variant writing [P][16] records against the FP64 oracle, at
  the bar of the four-array backward (compare_grads), with the record floats
  10-15 left untouched (still zero).
* bgs_project_bwd_packed against bgs_project_bwd on the same values unpacked
  into four arrays: the same arithmetic, so equal bit for bit.
* The FrameStep with records (its default) against the step with four arrays
  on the same frame: equal up to the order of the float atomics.
"""
import numpy as np
import pytest
import torch

from parity import MARGIN, compare_grads, oracle_bwd_from_gpu, oracle_render_from_gpu, to_np
from workloads import scenes

pytestmark = pytest.mark.gpu

# (variant, sub-tile, queue order, split walks)
BWD = [("static", 16, "raster", False), ("static_wave", 16, "raster", False), ("pixel", 8, "cost", False),
       ("pixel", 16, "cost", False), ("pixel", 16, "cost", True), ("pixel", 16, "raster", False),
       ("pixel", 32, "cost", False)]


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _scene(name):
    if name == "ragged":
        return scenes.scene_tiny(n=400, seed=3, width=83, height=45, log_scale_mu=-2.5)
    return scenes.make(name)


def _upstream(s, fwd, prep, bg, seed):
    orc_f = oracle_render_from_gpu(prep, bg=bg)
    flagged = orc_f["margin"] < MARGIN
    cam = s.cameras[0]
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    gA = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gD = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gC[:, flagged] = 0.0
    gA[flagged] = 0.0
    gD[flagged] = 0.0
    return gC, gA, gD


@pytest.mark.parametrize("name", ["tiny-60", "ragged", "0"])
@pytest.mark.parametrize("variant,sub,order,split", BWD)
def test_packed_backward_parity(rast, name, variant, sub, order, split):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    bg = (0.3, 0.1, 0.2)
    print(f"[bwd-packed] case={name} variant={variant}/{sub} order={order} split={split}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg(variant, sub, order, bg, flags=B.FLAG_PACKED_GRADS | (B.FLAG_SPLIT_WALKS if split else 0))
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    gC, gA, gD = _upstream(s, fwd, prep, bg, 31)
    dev = torch.device("cuda")
    grads = rast.render_bwd(prep, cfg, fwd, torch.from_numpy(gC).to(dev), torch.from_numpy(gA).to(dev),
                            torch.from_numpy(gD).to(dev))
    torch.cuda.synchronize()
    assert tuple(grads["records"].shape) == (prep.P, B.GRAD_RECORD)
    assert not bool(grads["records"][:, 10:].any()), "unused record floats were written"
    ob = oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg)
    compare_grads(grads, ob, name=f"{name} packed {variant}/{sub}/{order}")


@pytest.mark.parametrize("name", ["tiny-60", "0"])
def test_packed_deterministic_backward(rast, name):
    """The deterministic backward into records: oracle parity, and the same
    records bit for bit on a second run."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    bg = (0.3, 0.1, 0.2)
    print(f"[bwd-det-packed] case={name}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost", bg, flags=B.FLAG_PACKED_GRADS)
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    gC, gA, gD = _upstream(s, fwd, prep, bg, 32)
    dev = torch.device("cuda")
    up = [torch.from_numpy(a).to(dev) for a in (gC, gA, gD)]
    a = rast.render_bwd_det(prep, cfg, fwd, *up)
    b = rast.render_bwd_det(prep, cfg, fwd, *up)
    torch.cuda.synchronize()
    assert torch.equal(a["records"], b["records"])
    compare_grads(a, oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg), name=f"{name} packed det")


@pytest.mark.parametrize("name", ["0", "sh3"])
def test_project_bwd_packed_bit_identical(name):
    from paper_2412_17378_amd import Rasterizer
    from paper_2412_17378_amd import bgs as B
    s = scenes.scene_tiny(n=300, seed=11, width=80, height=56, sh_degree=3) if name == "sh3" else scenes.make(name)
    cam = s.cameras[0]
    P = s.P
    print(f"[proj-bwd-packed] case={name} P={P}", flush=True)
    rast = Rasterizer("cuda")
    dev = torch.device("cuda")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rng = np.random.default_rng(7)
    rec = torch.from_numpy(rng.standard_normal((P, B.GRAD_RECORD)).astype(np.float32)).to(dev)
    rec[:, 0:3] *= 1e-2
    v = B.record_views(rec)
    a = rast.project_bwd(cam, s.means3D, s.log_scales, s.quats, s.colors, s.sh_degree, v["means2D"],
                         v["conic_opacity"], v["rgb"], v["depth"])
    m3, ls, qu, co = T(s.means3D), T(s.log_scales), T(s.quats), T(s.colors)
    b = dict(means3D=torch.empty(P, 3, device=dev), log_scales=torch.empty(P, 3, device=dev),
             quats=torch.empty(P, 4, device=dev), opacity=torch.empty(P, device=dev), colors=torch.empty_like(co))
    B.bgs_project_bwd_packed(cam, m3, ls, qu, co, s.sh_degree, rec, b)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_step_records_match_arrays():
    """FrameStep with gradient records against the step with four arrays."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd.pipeline import FrameStep
    s = scenes.make("0")
    cam = s.cameras[0]
    dev = torch.device("cuda")
    params = {k: torch.from_numpy(getattr(s, k)).to(dev).contiguous()
              for k in ("means3D", "log_scales", "quats", "opacity", "colors")}
    up = torch.from_numpy(np.random.default_rng(3).standard_normal((3, cam.height, cam.width))
                          .astype(np.float32)).to(dev)
    for fwd_v, bwd_v in [(("static", 16, "raster"), ("pixel", 16, "cost")),
                         (("static_wave", 16, "raster"), ("static_wave", 16, "raster"))]:
        print(f"[step-packed] fwd={fwd_v} bwd={bwd_v}", flush=True)
        fc, bc = make_cfg(*fwd_v, tuple(s.bg)), make_cfg(*bwd_v, tuple(s.bg))
        a = FrameStep(cam, params, s.sh_degree, up, fc, bc, poison_outputs=True, packed_grads=True)
        b = FrameStep(cam, params, s.sh_degree, up, fc, bc, poison_outputs=True, packed_grads=False)
        a.run()
        b.run()
        torch.cuda.synchronize()
        for k in a.fwd:
            assert torch.equal(a.fwd[k], b.fwd[k]), k
        for k in b.grads:
            x, y = to_np(a.grads[k]).astype(np.float64), to_np(b.grads[k]).astype(np.float64)
            scale = max(float(np.abs(y).max()), 1e-30)
            assert float(np.abs(x - y).max()) <= 1e-5 * scale, k
        assert not bool(a.grad_records[:, 10:].any())


def test_autotune_on_records(rast):
    """bgs_autotune with FLAG_PACKED_GRADS times the backward candidates on
    gradient records and returns a backward configuration carrying the flag."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene("0")
    print("[autotune-packed] case=0", flush=True)
    prep = rast.prepare_scene(s)
    H, W, P, dev = prep.height, prep.width, prep.P, torch.device("cuda")
    out = dict(color=torch.empty(3, H, W, device=dev), alpha=torch.empty(H, W, device=dev),
               depth=torch.empty(H, W, device=dev), final_T=torch.empty(H, W, device=dev),
               n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
    f = prep.frame()
    base = make_cfg("pixel", 16, "cost", tuple(s.bg), flags=B.FLAG_PACKED_GRADS)
    ws = torch.empty(B.bgs_render_workspace_bytes(f, base), dtype=torch.uint8, device=dev)
    up = torch.ones(3, H, W, device=dev)
    bf, bb, fms, bms = B.bgs_autotune(f, base, out, up, {"records": B.grad_records(P, dev)}, ws)
    assert fms > 0 and bms > 0
    assert bb.flags & B.FLAG_PACKED_GRADS and not bf.flags & B.FLAG_PACKED_GRADS
