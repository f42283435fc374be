"""The task pool of the balanced kernels (Alg. 1; Sec. 4.1, 4.3) audited
through the C ABI: with bgs_render_cfg.item_claims set, every work item of a
render -- 8x8 sub-tiles, 16x16 tiles or 32x32 blocks -- is claimed by exactly
one wave exactly once (no item dropped, none rendered twice, no claim outside
the item range), for the forward and the backward, raster and cost order,
with the dealt items taken by persistent waves from the 64 fetch counters or
dispatched as a plain grid in rank order.  The queue state at the end must be
what the dispatch implies: the item count as dealt; with persistent waves
every one of the 64 fetch counters at or past its queue's size (a wave
leaves only once every queue is drained), with the grid all counters still
at zero.  Forward outputs are poisoned before each render, so a pixel no item
wrote shows up as NaN / -1."""
import numpy as np
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

NQ, QSTRIDE = 64, 32
# (variant, sub-tile, order, persistent task pool); sub-tile 8 always runs persistent waves
FWD = [("pixel", 8, "raster", True), ("pixel", 8, "cost", True), ("pixel", 16, "raster", False),
       ("pixel", 16, "cost", False), ("pixel", 16, "raster", True), ("pixel", 16, "cost", True),
       ("pixel", 32, "cost", False), ("pixel", 32, "raster", True), ("hybrid", 8, "cost", True),
       ("gauss", 8, "cost", True)]
BWD = [v for v in FWD if v[0] == "pixel"]


def _cfg(v, bg, flags=0):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    return make_cfg(*v[:3], bg, flags=flags | (B.FLAG_PERSISTENT if v[3] and v[1] != 8 else 0))


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _scene(name):
    if name == "ragged":
        return scenes.scene_tiny(n=400, seed=3, width=83, height=45, log_scale_mu=-2.5)
    return scenes.make(name)


N_UNITS = 15  # parts of a tile's work a wave-per-tile item may cover (include/bgs.h, item_claims)
# the ways a tile's work may be dealt: whole; two walk parts; four blocks; four blocks in two parts
PARTITIONS = [{0}, {1, 2}, {3, 4, 5, 6}, set(range(7, 15))]


def _n_items(W, H, sub):
    tx, ty = (W + 15) // 16, (H + 15) // 16
    return {8: 4 * tx * ty, 16: N_UNITS * tx * ty, 32: ((tx + 1) // 2) * ((ty + 1) // 2)}[sub]


def _check_queue(rast, claims, n_slots, what, nt=None, pool=True):
    """Every dealt item claimed exactly once.  For wave-per-tile queues (nt
    given) the claims are per (tile, unit): each tile's claimed units must be
    exactly one of the partitions of its work.  Then the queue state: the item
    count as dealt; with the persistent pool every counter at or past its
    queue's size, with the dispatched grid every counter untouched."""
    c = claims.cpu().numpy()
    assert np.all(c[n_slots:] == 0), (what, "claim beyond the items")
    if nt is None:
        assert np.all(c[:n_slots] == 1), (what, "claims != 1 at", np.nonzero(c[:n_slots] != 1)[0][:8],
                                          c[:n_slots][c[:n_slots] != 1][:8])
        n_dealt = n_slots
    else:
        per = c[:N_UNITS * nt].reshape(N_UNITS, nt)
        assert per.max() <= 1, (what, "an item claimed twice")
        for t in range(nt):
            got = set(np.nonzero(per[:, t])[0].tolist())
            assert got in PARTITIONS, (what, "tile", t, "claimed units", sorted(got))
        n_dealt = int(per.sum())
    ws = rast.ws.get("render", 0).view(torch.int32)[:NQ * QSTRIDE + 2].cpu().numpy().astype(np.int64)
    n, nw = int(ws[NQ * QSTRIDE]), int(ws[NQ * QSTRIDE + 1])
    assert n == n_dealt, (what, n, n_dealt)
    ctr = ws[0:NQ * QSTRIDE:QSTRIDE]
    if not pool:
        assert np.all(ctr == 0), (what, "a fetch counter moved under grid dispatch")
        return n_dealt
    size = np.array([(n - q - 1) // NQ + 1 if n > q else 0 for q in range(NQ)])
    first = np.array([(nw - q - 1) // NQ + 1 if nw > q else 0 for q in range(NQ)])  # taken without a claim
    assert np.all(ctr + first >= size), (what, "a queue was not drained", ctr + first - size)
    # every counter step past the size is one failed claim of one wave
    assert int(np.maximum(ctr + first - size, 0).sum()) <= nw * NQ, (what, int((ctr + first - size).sum()))
    return n_dealt


@pytest.mark.parametrize("name", ["ragged", "0", "1", "1-hotspot"])
@pytest.mark.parametrize("v", FWD)
def test_forward_claims_every_item_once(rast, name, v):
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    sub = v[1]
    print(f"[queue] fwd case={name} cfg={v}", flush=True)
    prep = rast.prepare_scene(s)
    n = _n_items(W, H, sub)
    claims = torch.zeros(n + 64, dtype=torch.int32, device="cuda")
    cfg = _cfg(v, tuple(s.bg))
    cfg.item_claims = claims.data_ptr()
    out = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    nt = (W + 15) // 16 * ((H + 15) // 16) if sub == 16 else None
    _check_queue(rast, claims, n, f"fwd {name} {v}", nt, pool=v[3])
    for k in ("color", "alpha", "depth", "final_T"):
        assert bool(torch.isfinite(out[k]).all()), k
    assert int(out["n_contrib"].min()) >= 0


@pytest.mark.parametrize("name", ["ragged", "0", "1"])
@pytest.mark.parametrize("v", BWD)
def test_backward_claims_every_item_once(rast, name, v):
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    sub = v[1]
    print(f"[queue] bwd case={name} cfg={v}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = _cfg(v, tuple(s.bg))
    fwd = rast.render_fwd(prep, cfg)
    n = _n_items(W, H, sub)
    claims = torch.zeros(n + 64, dtype=torch.int32, device="cuda")
    cfg.item_claims = claims.data_ptr()
    gC = torch.randn(3, H, W, device="cuda")
    rast.render_bwd(prep, cfg, fwd, gC)
    torch.cuda.synchronize()
    nt = (W + 15) // 16 * ((H + 15) // 16) if sub == 16 else None
    _check_queue(rast, claims, n, f"bwd {name} {v}", nt, pool=v[3])


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


@pytest.mark.parametrize("name", ["0", "1", "1-hotspot"])
@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("pool", [False, True])
def test_backward_units_follow_the_walks(rast, name, split, pool):
    """Cost-ordered wave-per-tile backward: each tile's work is dealt as the
    units its walk (the deepest n_contrib, within its list) calls for -- four
    blocks from 512 entries on, and with split walks two parts from 128 on --
    and every unit is claimed exactly once."""
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    W, H = s.cameras[0].width, s.cameras[0].height
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost", tuple(s.bg),
                   flags=(B.FLAG_SPLIT_WALKS if split else 0) | (B.FLAG_PERSISTENT if pool else 0))
    fwd = rast.render_fwd(prep, cfg)
    nt = B.n_tiles(W, H)
    claims = torch.zeros(N_UNITS * nt + 64, dtype=torch.int32, device="cuda")
    cfg.item_claims = claims.data_ptr()
    print(f"[queue] units case={name} split={split}", flush=True)
    rast.render_bwd(prep, cfg, fwd, torch.randn(3, H, W, device="cuda"))
    torch.cuda.synchronize()
    _check_queue(rast, claims, N_UNITS * nt, f"bwd units {name} split={split} pool={pool}", nt, pool=pool)
    # the walk of each tile: the deepest n_contrib of its pixels, within its list
    nc = fwd["n_contrib"].cpu().numpy().astype(np.int64)
    rg = prep.ranges.cpu().numpy().astype(np.int64)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    pad = np.zeros((TY * 16, TX * 16), np.int64)
    pad[:H, :W] = nc
    walk = np.minimum(pad.reshape(TY, 16, TX, 16).max(axis=(1, 3)).ravel(), rg[:, 1] - rg[:, 0])
    per = claims[:N_UNITS * nt].cpu().numpy().reshape(N_UNITS, nt)
    blocks, parts = walk >= 512, (walk >= 128) & split
    expect = np.where(blocks & parts, 3, np.where(blocks, 2, np.where(parts, 1, 0)))
    got = np.array([next(i for i, P in enumerate(PARTITIONS) if set(np.nonzero(per[:, t])[0].tolist()) == P)
                    for t in range(nt)])
    np.testing.assert_array_equal(got, expect)
    print(f"[queue] units case={name} split={split}: {int(blocks.sum())} tiles as blocks, {int(parts.sum())} "
          f"split of {nt}", flush=True)
    if name == "1-hotspot":
        assert blocks.any()
