"""Capped tile lists (bgs_tile_lists max_per_tile = K) and the forward's
overflow report (bgs_render_cfg.list_cap / list_overflow).

* Lists: each capped list is the first min(L, K) entries of the oracle's
  whole list, bit for bit, at its tile's fixed slot; M counts the kept
  entries; a capacity below n_tiles K is refused before any work.
* Forward: every variant raises the flag when some pixel examines more than
  K entries of a tile list (it cannot have stopped inside the capped list),
  never when K exceeds every pixel's examined count, and whenever the flag
  stays clear the images equal the whole lists' bit for bit.
* FrameStep with a cap ("auto" and forced): the same images as the uncapped
  step bit for bit, gradients to the accumulation order, also as a replayed
  hipGraph; a cap below the pixels' depth reports the overflow.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import to_np
from workloads import scenes

pytestmark = pytest.mark.gpu

VARIANTS = [("static", 16, "raster"), ("pixel", 8, "cost"), ("pixel", 16, "cost"), ("hybrid", 8, "cost"),
            ("gauss", 8, "cost")]


def _scene(name):
    if name == "sh3-tiny":
        return scenes.scene_tiny(n=200, seed=11, width=80, height=56, sh_degree=3)
    return scenes.make(name)


def _lists(B, W, H, P, pr, K, cap):
    if K <= 2048:  # fixed per-tile slots
        cap = max(cap, K * B.n_tiles(W, H))
    dev = pr["means2D"].device
    n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    ranges = torch.full((B.n_tiles(W, H), 2), 7, dtype=torch.int32, device=dev)
    pl = torch.full((cap,), -5, dtype=torch.int32, device=dev)
    ws = torch.empty(B.bgs_tile_lists_workspace_bytes(W, H, P, cap), dtype=torch.uint8, device=dev)
    assert B.bgs_tile_lists(W, H, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"], pl, ranges, n_dev,
                            ws, max_per_tile=K)
    return pl, ranges, n_dev


@pytest.mark.parametrize("name", ["tiny-300", "0", "sh3-tiny"])
def test_capped_lists_are_prefixes(name):
    from paper_2412_17378_amd import Rasterizer
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    cam = s.cameras[0]
    W, H = cam.width, cam.height
    rast = Rasterizer("cuda", poison_outputs=True)
    pr = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    ob = oracle.bin_sort_ranges(W, H, to_np(pr["means2D"]), to_np(pr["radius"]), to_np(pr["depth"]))
    orr, opl = ob["ranges"], ob["point_list"]
    L = (orr[:, 1] - orr[:, 0]).astype(np.int64)
    for K in (1, 7, 64, int(L.max()), int(L.max()) + 5, 2049, 5000):
        print(f"[capped] lists case={name} K={K}", flush=True)
        pl, ranges, n_dev = _lists(B, W, H, s.P, pr, K, int(ob["n_pairs"]))
        torch.cuda.synchronize()
        rg = to_np(ranges)
        assert int(n_dev.item()) == int(np.minimum(L, K).sum())
        np.testing.assert_array_equal(rg[:, 1] - rg[:, 0], np.minimum(L, K))
        got = to_np(pl)
        for t in np.nonzero(L)[0]:
            assert K > 2048 or rg[t, 0] == t * K
            np.testing.assert_array_equal(got[rg[t, 0]:rg[t, 1]], opl[orr[t, 0]:orr[t, 0] + min(L[t], K)])
    # too small a capacity for the fixed slots: refused, nothing written
    nt = B.n_tiles(W, H)
    K = min(2048, int(ob["n_pairs"]) // nt + 64)
    cap = nt * K - 1  # holds the whole lists, one short of the fixed slots
    n_dev = torch.full((1,), 3, dtype=torch.int64, device=pr["means2D"].device)
    ranges = torch.full((nt, 2), 7, dtype=torch.int32, device=n_dev.device)
    pl = torch.full((cap,), -5, dtype=torch.int32, device=n_dev.device)
    ws = torch.empty(B.bgs_tile_lists_workspace_bytes(W, H, s.P, cap), dtype=torch.uint8, device=n_dev.device)
    assert not B.bgs_tile_lists(W, H, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"], pl, ranges,
                                n_dev, ws, max_per_tile=K)
    torch.cuda.synchronize()
    assert bool(torch.all(ranges == 7)) and int(n_dev.item()) == 3 and bool(torch.all(pl == -5))


def test_capped_compact_lists_full_size():
    """K above 2048 goes through the segment split and keeps the lists
    compact: on the 1080p scene (lists up to 95 k) each capped list is the
    prefix of the whole list the same builder writes (whole lists are checked
    against the oracle elsewhere), ranges are packed front to back."""
    from paper_2412_17378_amd import Rasterizer
    from paper_2412_17378_amd import bgs as B
    s = scenes.make("1")
    cam = s.cameras[0]
    W, H = cam.width, cam.height
    rast = Rasterizer("cuda", poison_outputs=True)
    pr = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    whole_pl, whole_rg, n_whole = _lists(B, W, H, s.P, pr, 0, 160_000_000)
    torch.cuda.synchronize()
    M = int(n_whole.item())
    wr = to_np(whole_rg)
    L = (wr[:, 1] - wr[:, 0]).astype(np.int64)
    wpl = to_np(whole_pl[:M])
    del whole_pl
    for K in (2049, 3000):
        print(f"[capped] compact K={K}", flush=True)
        pl, ranges, n_dev = _lists(B, W, H, s.P, pr, K, M)
        torch.cuda.synchronize()
        keep = np.minimum(L, K)
        assert int(n_dev.item()) == int(keep.sum())
        rg = to_np(ranges)
        np.testing.assert_array_equal(rg[:, 1] - rg[:, 0], keep)
        start = np.concatenate([[0], np.cumsum(keep)[:-1]])
        np.testing.assert_array_equal(rg[keep > 0, 0], start[keep > 0])
        got = to_np(pl[:int(keep.sum())])
        for t in np.nonzero(L)[0]:
            np.testing.assert_array_equal(got[rg[t, 0]:rg[t, 1]], wpl[wr[t, 0]:wr[t, 0] + keep[t]])


@pytest.mark.parametrize("name", ["0", "tiny-300"])
def test_capped_render_and_overflow_flag(name):
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    cam = s.cameras[0]
    W, H = cam.width, cam.height
    rast = Rasterizer("cuda", poison_outputs=True)
    prep = rast.prepare_scene(s)
    pr = dict(means2D=prep.means2D, radius=prep.radius, depth=prep.depth, tiles_touched=prep.tiles_touched)
    torch.cuda.synchronize()
    m2, co = to_np(prep.means2D), to_np(prep.conic_opacity)
    of = oracle.render_fwd(W, H, to_np(prep.ranges), to_np(prep.point_list), m2, co, to_np(prep.rgb),
                           to_np(prep.depth), bg=tuple(s.bg))
    ex = of["n_examined"]
    deepest = int(ex.max())
    dev = torch.device("cuda")
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    for K in (4, max(1, deepest // 2), deepest, deepest + 1):
        pl, ranges, _ = _lists(B, W, H, s.P, pr, K, prep.n_pairs)
        frame = B.make_frame(W, H, ranges, pl, prep.means2D, prep.conic_opacity, prep.rgb, prep.depth)
        for v in VARIANTS:
            print(f"[capped] render case={name} K={K} cfg={v}", flush=True)
            whole = rast.render_fwd(prep, make_cfg(*v, tuple(s.bg)))
            cfg = make_cfg(*v, tuple(s.bg))
            cfg.list_cap, cfg.list_overflow = K, flag.data_ptr()
            flag.zero_()
            out = {k: torch.empty_like(t) for k, t in whole.items()}
            ws = torch.empty(B.bgs_render_workspace_bytes(frame, cfg), dtype=torch.uint8, device=dev)
            B.bgs_render_fwd(frame, cfg, out["color"], out["alpha"], out["depth"], out["final_T"], out["n_contrib"],
                             ws)
            torch.cuda.synchronize()
            raised = bool(flag.item())
            if deepest > K:
                assert raised, (K, v)  # a pixel examines past the cap: it cannot stop inside
            if K > deepest:
                assert not raised, (K, v)
            if not raised:
                for k in whole:
                    assert torch.equal(whole[k], out[k]), (K, v, k)


def _params(s, dev):
    return {k: torch.from_numpy(getattr(s, k)).to(dev).contiguous()
            for k in ("means3D", "log_scales", "quats", "opacity", "colors")}


@pytest.mark.parametrize("name", ["1", "3-early", "2"])
def test_frame_step_capped(name):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd.pipeline import FrameStep
    dev = torch.device("cuda")
    s = scenes.make(name)
    cam = s.cameras[0]
    params = _params(s, dev)
    up = torch.from_numpy(s.upstream()["dL_dcolor"]).to(dev)
    fc = make_cfg("static", 16, "raster", tuple(s.bg))
    bc = make_cfg("pixel", 16, "cost", tuple(s.bg))
    print(f"[capped] frame step scene={name}", flush=True)
    whole = FrameStep(cam, params, s.sh_degree, up, fc, bc, poison_outputs=True)
    whole.run()
    torch.cuda.synchronize()
    ref_f = {k: v.clone() for k, v in whole.fwd.items()}
    ref_g = {k: v.clone() for k, v in whole.grads.items()}
    M = whole.n_pairs()
    del whole
    capped = FrameStep(cam, params, s.sh_degree, up, fc, bc, list_cap="auto", poison_outputs=True)
    K = capped.list_cap
    print(f"[capped] scene={name} K={K} M={M}", flush=True)
    assert K > 0 and capped.M_whole == M

    def same():
        for k in ref_f:
            assert torch.equal(ref_f[k], capped.fwd[k]), k
        for k in ref_g:
            scale = float(ref_g[k].abs().max()) + 1e-30
            assert float((ref_g[k] - capped.grads[k]).abs().max()) <= 1e-4 * scale, k

    capped.run()
    assert not capped.overflowed()
    assert capped.n_pairs() < M
    same()
    graph = capped.capture()
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert not capped.overflowed()
        same()
    del graph
    capped.set_list_cap(8)
    capped.run()
    assert capped.overflowed()
    capped.run()
    assert capped.overflowed()  # the report holds until cleared
    capped.clear_overflow()
    assert not capped.overflowed()
    capped.set_list_cap(None)
    capped.run()
    assert not capped.overflowed() and capped.n_pairs() == M
    same()
