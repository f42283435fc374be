"""The task pool of the balanced kernels (Alg. 1; Sec. 4.1, 4.3) audited
through the C ABI: with bgs_render_cfg.item_claims set, every work item of a
render -- 8x8 sub-tiles, 16x16 tiles or 32x32 blocks -- is claimed by exactly
one wave exactly once (no item dropped, none rendered twice, no claim outside
the item range), for the forward and the backward, raster and cost order.
The queue state at the end must be what the claim loop implies: the item
count as dealt, and every one of the 64 fetch counters at or past its queue's
size (a wave leaves only once every queue is drained).  Forward outputs are
poisoned before each render, so a pixel no item wrote shows up as NaN / -1."""
import numpy as np
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

NQ, QSTRIDE = 64, 32
FWD = [("pixel", 8, "raster"), ("pixel", 8, "cost"), ("pixel", 16, "raster"), ("pixel", 16, "cost"),
       ("pixel", 32, "cost"), ("pixel", 32, "raster"), ("hybrid", 8, "cost"), ("gauss", 8, "cost")]
BWD = [v for v in FWD if v[0] == "pixel"]


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _scene(name):
    if name == "ragged":
        return scenes.scene_tiny(n=400, seed=3, width=83, height=45, log_scale_mu=-2.5)
    return scenes.make(name)


def _n_items(W, H, sub):
    tx, ty = (W + 15) // 16, (H + 15) // 16
    return {8: 4 * tx * ty, 16: tx * ty, 32: ((tx + 1) // 2) * ((ty + 1) // 2)}[sub]


def _check_queue(rast, claims, n_items, what):
    c = claims.cpu().numpy()
    assert np.all(c[:n_items] == 1), (what, "claims != 1 at", np.nonzero(c[:n_items] != 1)[0][:8],
                                      c[:n_items][c[:n_items] != 1][:8])
    assert np.all(c[n_items:] == 0), (what, "claim beyond the items")
    ws = rast.ws.get("render", 0).view(torch.int32)[:NQ * QSTRIDE + 1].cpu().numpy().astype(np.int64)
    n = int(ws[NQ * QSTRIDE])
    assert n == n_items, (what, n, n_items)
    ctr = ws[0:NQ * QSTRIDE:QSTRIDE]
    size = np.array([(n - q - 1) // NQ + 1 if n > q else 0 for q in range(NQ)])
    assert np.all(ctr >= size), (what, "a queue was not drained", ctr - size)
    # every counter step past the size is one failed claim of one wave
    assert int((ctr - size).sum()) <= 256 * 32 * 2 * NQ, (what, int((ctr - size).sum()))


@pytest.mark.parametrize("name", ["ragged", "0", "1"])
@pytest.mark.parametrize("variant,sub,order", FWD)
def test_forward_claims_every_item_once(rast, name, variant, sub, order):
    from paper_2412_17378_amd import make_cfg
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    print(f"[queue] fwd case={name} cfg={variant}/{sub}/{order}", flush=True)
    prep = rast.prepare_scene(s)
    n = _n_items(W, H, sub)
    claims = torch.zeros(n + 64, dtype=torch.int32, device="cuda")
    cfg = make_cfg(variant, sub, order, tuple(s.bg))
    cfg.item_claims = claims.data_ptr()
    out = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    _check_queue(rast, claims, n, f"fwd {name} {variant}/{sub}/{order}")
    for k in ("color", "alpha", "depth", "final_T"):
        assert bool(torch.isfinite(out[k]).all()), k
    assert int(out["n_contrib"].min()) >= 0


@pytest.mark.parametrize("name", ["ragged", "0", "1"])
@pytest.mark.parametrize("variant,sub,order", BWD)
def test_backward_claims_every_item_once(rast, name, variant, sub, order):
    from paper_2412_17378_amd import make_cfg
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    print(f"[queue] bwd case={name} cfg={variant}/{sub}/{order}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg(variant, sub, order, tuple(s.bg))
    fwd = rast.render_fwd(prep, cfg)
    n = _n_items(W, H, sub)
    claims = torch.zeros(n + 64, dtype=torch.int32, device="cuda")
    cfg.item_claims = claims.data_ptr()
    gC = torch.randn(3, H, W, device="cuda")
    rast.render_bwd(prep, cfg, fwd, gC)
    torch.cuda.synchronize()
    _check_queue(rast, claims, n, f"bwd {name} {variant}/{sub}/{order}")


def test_static_variants_take_no_claims(rast):
    from paper_2412_17378_amd import make_cfg
    s = _scene("0")
    prep = rast.prepare_scene(s)
    claims = torch.zeros(1024, dtype=torch.int32, device="cuda")
    for v in (("static", 16, "raster"), ("static_wave", 16, "raster")):
        cfg = make_cfg(*v)
        cfg.item_claims = claims.data_ptr()
        fwd = rast.render_fwd(prep, cfg)
        rast.render_bwd(prep, cfg, fwd, torch.randn(3, prep.height, prep.width, device="cuda"))
    torch.cuda.synchronize()
    assert int(claims.abs().sum()) == 0


@pytest.mark.parametrize("name", ["0", "1"])
def test_split_walks_claim_both_parts_once(rast, name):
    """Split backward walks: every tile is claimed once at claims[tile] (its
    whole walk, or the lower part), and the upper part of exactly the tiles
    whose walk reaches 128 entries once at claims[n_tiles + tile]."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost", tuple(s.bg), flags=B.FLAG_SPLIT_WALKS)
    fwd = rast.render_fwd(prep, cfg)
    nt = B.n_tiles(W, H)
    claims = torch.zeros(2 * nt + 64, dtype=torch.int32, device="cuda")
    cfg.item_claims = claims.data_ptr()
    print(f"[queue] split case={name}", flush=True)
    rast.render_bwd(prep, cfg, fwd, torch.randn(3, H, W, device="cuda"))
    torch.cuda.synchronize()
    # each tile's walk: the deepest n_contrib of its pixels, within its list
    nc = fwd["n_contrib"].cpu().numpy().astype(np.int64)
    rg = prep.ranges.cpu().numpy().astype(np.int64)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    pad = np.zeros((TY * 16, TX * 16), np.int64)
    pad[:H, :W] = nc
    walk = pad.reshape(TY, 16, TX, 16).max(axis=(1, 3)).ravel()
    walk = np.minimum(walk, rg[:, 1] - rg[:, 0])
    split = walk >= 128
    c = claims.cpu().numpy()
    assert np.all(c[:nt] == 1), np.nonzero(c[:nt] != 1)[0][:8]
    np.testing.assert_array_equal(c[nt:2 * nt], split.astype(np.int32))
    assert np.all(c[2 * nt:] == 0)
    n = int(rast.ws.get("render", 0).view(torch.int32)[NQ * QSTRIDE].item())
    assert n == nt + int(split.sum()), (n, nt, int(split.sum()))
    print(f"[queue] split case={name}: {int(split.sum())} of {nt} tiles split", flush=True)
    if name == "1":
        assert split.any()
