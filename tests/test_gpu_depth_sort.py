"""The fused list builder's depth order, whole, through bgs_tile_lists.

Every Gaussian sits at the centre of a one-tile image (radius 1), so the
tile's list is the depth order of all listed Gaussians: ids sorted by depth,
equal depths in id order (a stable sort, the definition the renderer's
front-to-back order rests on).  Unlisted Gaussians (tiles_touched 0) take no
place in it.  Cases: many sort blocks (300 k items, 147 blocks of 2048: every
block's offsets come from the blocks before it), a ragged block count, a
single item, keys whose high bytes are all equal (identity passes), keys
that are all equal (the list keeps id order), and depths spread over many
binades (every byte sorts).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _depths(kind, P, rng):
    if kind == "spread":  # log-uniform over 1e-3 .. 1e4, with repeats: every key byte varies
        d = np.exp(rng.uniform(np.log(1e-3), np.log(1e4), P)).astype(np.float32)
        rep = rng.random(P) < 0.2
        d[rep] = rng.choice(d[:64], rep.sum())
        return d
    if kind == "narrow":  # 1 .. 1.0001: the two high bytes are the same in every key
        return (1.0 + rng.uniform(0.0, 1e-4, P)).astype(np.float32)
    if kind == "equal":
        return np.full(P, 2.5, np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("P,kind", [(300_000, "spread"), (300_000, "narrow"), (2049, "spread"), (1, "spread"),
                                    (40_000, "equal")])
def test_depth_order_of_one_tile(P, kind):
    from paper_2412_17378_amd import bgs as B
    dev = torch.device("cuda")
    rng = np.random.default_rng(P + len(kind))
    depth = _depths(kind, P, rng)
    listed = rng.random(P) >= 0.1
    if P == 1:
        listed[:] = True
    print(f"[depth-sort] P={P} depths={kind} listed={int(listed.sum())}", flush=True)
    means2D = torch.full((P, 2), 8.0, device=dev)
    radius = torch.from_numpy(np.where(listed, 1, 0).astype(np.int32)).to(dev)
    touched = torch.from_numpy(listed.astype(np.int32)).to(dev)
    d = torch.from_numpy(depth).to(dev)
    point_list = torch.full((P,), -1, dtype=torch.int32, device=dev)
    ranges = torch.full((1, 2), -1, dtype=torch.int32, device=dev)
    n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(B.bgs_tile_lists_workspace_bytes(16, 16, P, P), dtype=torch.uint8, device=dev)
    ws.fill_(0xA5)  # stale scratch: nothing may rely on a cleared workspace
    for rep in range(2):  # a second build on the same workspace
        assert B.bgs_tile_lists(16, 16, means2D, radius, d, touched, point_list, ranges, n_dev, ws)
        torch.cuda.synchronize()
        ids = np.flatnonzero(listed)
        want = ids[np.argsort(depth[ids], kind="stable")]
        M = int(n_dev.item())
        assert M == want.size
        assert ranges.cpu().numpy().tolist() == [[0, M]]
        np.testing.assert_array_equal(point_list.cpu().numpy()[:M], want)
