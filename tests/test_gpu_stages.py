"""GPU parity of the pre-render stages (project, bin, sort, ranges) against the
FP64 oracle, through the C ABI.

* project: fp32 vs fp64 within 1e-4 relative (s = RMS per quantity); integer
  radius and tile counts exact except where the oracle's real-valued extent
  or square edge sits within 1e-4 px of a rounding boundary.
* bin/sort/ranges, stage-isolated: the oracle's binning fed the GPU's own
  fp32 splats must give the identical point list and ranges, bit for bit.
* end to end: per-tile lists from the fp64 projection equal the GPU's except
  for Gaussians flagged as above or with a depth gap < 1e-6 relative.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import check_close, rms, to_np
from workloads import scenes

pytestmark = pytest.mark.gpu

CASES = ["tiny-40", "tiny-300", "0", "sh3-tiny"]


def _scene(name):
    if name == "sh3-tiny":
        return scenes.scene_tiny(n=200, seed=11, width=80, height=56, sh_degree=3)
    return scenes.make(name)


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _near_boundary(orc_pr, cam, tol=1e-4):
    """Gaussians whose integer quantities the fp32 path may round differently."""
    ext = orc_pr["extent"]
    r = np.ceil(ext)
    flag = np.abs(ext - np.round(ext)) < tol * np.maximum(1.0, ext)
    for k in (0, 1):
        c = orc_pr["means2D"][:, k]
        for e in (c - r, c + r):
            flag |= np.abs(e / 16.0 - np.round(e / 16.0)) * 16.0 < tol * np.maximum(1.0, np.abs(e))
    return flag


@pytest.mark.parametrize("name", CASES)
def test_project_parity(rast, name):
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[project] case={name} P={s.P}", flush=True)
    g = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    o = oracle.project_scene(s)
    vis = o["radius"] > 0
    flag = _near_boundary(o, cam)
    assert np.array_equal(to_np(g["radius"]) > 0, vis)
    ok = vis & ~flag
    assert np.array_equal(to_np(g["radius"])[ok], o["radius"][ok])
    check_close(to_np(g["means2D"])[vis], o["means2D"][vis], rms(o["means2D"][vis]), "means2D")
    check_close(to_np(g["depth"])[vis], o["depth"][vis], rms(o["depth"][vis]), "depth")
    check_close(to_np(g["rgb"])[vis], o["rgb"][vis], max(rms(o["rgb"][vis]), 1e-6), "rgb")
    co = o["conic_opacity"][vis]
    for k in range(3):
        check_close(to_np(g["conic_opacity"])[vis, k], co[:, k], rms(co[:, k]), f"conic[{k}]")
    np.testing.assert_array_equal(to_np(g["conic_opacity"])[vis, 3], s.opacity[vis])
    # tile counts from the oracle's own binning
    tid, gid = oracle.bin_pairs(cam.width, cam.height, o["means2D"], o["radius"])
    cnt = np.bincount(gid, minlength=s.P)
    assert np.array_equal(to_np(g["tiles_touched"])[ok], cnt[ok])


@pytest.mark.parametrize("method", ["fused", "sort"])
@pytest.mark.parametrize("name", CASES)
def test_bin_sort_ranges_bit_exact(rast, name, method):
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[bin] case={name} method={method} P={s.P}", flush=True)
    prep = rast.prepare_scene(s, method=method)
    torch.cuda.synchronize()
    ob = oracle.bin_sort_ranges(cam.width, cam.height, to_np(prep.means2D), to_np(prep.radius), to_np(prep.depth))
    assert prep.n_pairs == ob["n_pairs"]
    np.testing.assert_array_equal(to_np(prep.point_list), ob["point_list"])
    if prep.tile_keys is not None:
        np.testing.assert_array_equal(to_np(prep.tile_keys), ob["tile_ids"])
    np.testing.assert_array_equal(to_np(prep.ranges), ob["ranges"])


@pytest.mark.parametrize("name", CASES)
def test_lists_end_to_end(rast, name):
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[lists] case={name} P={s.P}", flush=True)
    prep = rast.prepare_scene(s)
    torch.cuda.synchronize()
    o = oracle.project_scene(s)
    ob = oracle.bin_sort_ranges(cam.width, cam.height, o["means2D"], o["radius"], o["depth"])
    flag = _near_boundary(o, cam)
    d = o["depth"]
    order = np.argsort(d)
    ds = d[order]
    close = np.zeros(s.P, bool)
    gap = np.abs(np.diff(ds)) < 1e-6 * np.maximum(ds[1:], 1e-30)
    close[order[1:][gap]] = True
    close[order[:-1][gap]] = True
    flag |= close
    rg_g, pl_g = to_np(prep.ranges), to_np(prep.point_list)
    mism = set()
    for t in range(rg_g.shape[0]):
        a = list(pl_g[rg_g[t, 0]:rg_g[t, 1]])
        b = list(ob["point_list"][ob["ranges"][t, 0]:ob["ranges"][t, 1]])
        if a != b:
            mism |= set(a) ^ set(b)
            if set(a) == set(b):  # same members, different order: a depth tie
                mism |= {x for x, y in zip(a, b) if x != y}
    unexplained = [m for m in mism if not flag[m]]
    assert not unexplained, unexplained[:10]


@pytest.mark.parametrize("name", ["0", "tiny-300"])
def test_fused_lists_overflow(rast, name):
    """A capacity below M: the call returns without waiting, writes nothing to
    the point list, writes every range empty and puts M (overflow of the tile
    lists) or a lower bound of M above the capacity (overflow already of the
    coarse lists) in n_pairs; the same buffers with capacity M then hold the
    oracle's lists."""
    from paper_2412_17378_amd import bgs as B
    s = _scene(name)
    cam = s.cameras[0]
    W, H = cam.width, cam.height
    pr = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    ob = oracle.bin_sort_ranges(W, H, to_np(pr["means2D"]), to_np(pr["radius"]), to_np(pr["depth"]))
    M = int(ob["n_pairs"])
    assert M > 8
    dev = torch.device("cuda")
    n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    ranges = torch.full((B.n_tiles(W, H), 2), 7, dtype=torch.int32, device=dev)
    for cap in (M - 1, M // 8, 1, M):
        print(f"[lists-overflow] case={name} M={M} capacity={cap}", flush=True)
        pl = torch.full((cap,), -5, dtype=torch.int32, device=dev)
        ws = torch.empty(B.bgs_tile_lists_workspace_bytes(W, H, s.P, cap), dtype=torch.uint8, device=dev)
        B.bgs_tile_lists(W, H, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"], pl, ranges, n_dev, ws)
        torch.cuda.synchronize()
        n = int(n_dev.item())
        if cap < M:
            assert cap < n <= M, (cap, n, M)
            if cap == M - 1:
                assert n == M
            assert bool(torch.all(pl == -5))
            assert bool(torch.all(ranges == 0))
        else:
            assert n == M
            np.testing.assert_array_equal(to_np(pl), ob["point_list"])
            np.testing.assert_array_equal(to_np(ranges), ob["ranges"])
