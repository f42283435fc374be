"""bgs_render_fwd_noalloc (the forward for callers that cannot allocate: its
work queue lives in a device array inside the library) through the C ABI,
against bgs_render_fwd with a caller workspace on the same inputs: outputs
identical bit for bit, on two calls in a row with the second frame smaller
than the first (the array keeps the first call's queue), for every balanced
variant and the static ones.  A frame whose queue exceeds the array is
refused before any work is queued.  Outputs are poisoned before each call."""
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

VARIANTS = [("pixel", 16, "cost"), ("pixel", 16, "raster"), ("pixel", 8, "cost"), ("pixel", 32, "cost"),
            ("hybrid", 8, "cost"), ("gauss", 8, "cost"), ("static", 16, "raster"), ("static_wave", 16, "raster")]


def _outs(H, W):
    from paper_2412_17378_amd.pipeline import poison_fwd
    out = dict(color=torch.empty(3, H, W, device="cuda"), alpha=torch.empty(H, W, device="cuda"),
               depth=torch.empty(H, W, device="cuda"), final_T=torch.empty(H, W, device="cuda"),
               n_contrib=torch.empty(H, W, dtype=torch.int32, device="cuda"))
    poison_fwd(out)
    return out


@pytest.mark.parametrize("variant,sub,order", VARIANTS)
def test_noalloc_forward_matches_workspace_forward(variant, sub, order):
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd import bgs as B
    rast = Rasterizer("cuda")
    big = rast.prepare_scene(scenes.make("0"))
    small = rast.prepare_scene(scenes.scene_tiny(n=300, seed=12, width=83, height=45, log_scale_mu=-2.5))
    for name, prep in (("scene 0 (128x128)", big), ("tiny 83x45", small)):
        print(f"[noalloc] {name} cfg={variant}/{sub}/{order}", flush=True)
        H, W = prep.height, prep.width
        cfg = make_cfg(variant, sub, order, (0.1, 0.2, 0.3))
        f = prep.frame()
        ref = _outs(H, W)
        ws = torch.empty(B.bgs_render_workspace_bytes(f, cfg), dtype=torch.uint8, device="cuda")
        B.bgs_render_fwd(f, cfg, ref["color"], ref["alpha"], ref["depth"], ref["final_T"], ref["n_contrib"], ws)
        got = _outs(H, W)
        B.bgs_render_fwd_noalloc(f, cfg, got["color"], got["alpha"], got["depth"], got["final_T"], got["n_contrib"])
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], got[k]), (name, k)
        assert int(got["n_contrib"].min()) >= 0


def test_noalloc_refuses_a_queue_beyond_its_array():
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    cap = B.bgs_render_fwd_noalloc_max_bytes()
    assert 0 < cap <= 4 << 20
    buf = torch.zeros(64, device="cuda")
    ids = torch.zeros(64, dtype=torch.int32, device="cuda")
    # 8192 x 8192 pixels = 262 144 tiles: the queue needs more than the array
    # holds; the call must refuse before it reads any of these (small) arrays
    f = B.Frame()
    f.width, f.height, f.tile = 8192, 8192, B.TILE
    f.ranges, f.point_list = B._ptr(ids), B._ptr(ids)
    f.means2D, f.conic_opacity, f.rgb, f.depth = B._ptr(buf), B._ptr(buf), B._ptr(buf), B._ptr(buf)
    out = torch.empty(1, device="cuda")
    n = torch.empty(1, dtype=torch.int32, device="cuda")
    st = B.lib().bgs_render_fwd_noalloc(B.C.byref(f), B.C.byref(make_cfg("pixel", 16, "cost")), B._ptr(out),
                                        B._ptr(out), B._ptr(out), B._ptr(out), B._ptr(n), None)
    assert st == B.BGS_ECAPACITY, st
    assert "bytes of queue state" in B.lib().bgs_last_error().decode()
