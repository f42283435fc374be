"""Parity at the benchmark's full size (1920x1080, 500k Gaussians, balanced
pixel-wise kernels, cost-ordered queue) on sampled outputs the oracle computes
window by window: the per-tile lists of the windows' tiles bit for bit, the
forward images inside the windows, and per-Gaussian gradients with the
upstream gradient cropped to the windows on both sides.  Also the any-size
property that the static and balanced forward kernels agree bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from parity import MARGIN, compare_forward, compare_grads, oracle_bwd_from_gpu, oracle_render_from_gpu, to_np
from workloads import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    from paper_2412_17378_amd import Rasterizer, make_cfg
    s = scenes.make("1")
    rast = Rasterizer("cuda", poison_outputs=True)
    print(f"[full] scene 1 P={s.P}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 8, "cost")
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    rg = to_np(prep.ranges)
    lens = rg[:, 1] - rg[:, 0]
    heavy = int(np.argmax(lens))
    TX = (1920 + 15) // 16
    rng = np.random.default_rng(3)
    wins = [(int(heavy % TX) * 16, int(heavy // TX) * 16, int(heavy % TX) * 16 + 32, int(heavy // TX) * 16 + 32)]
    wins = [(x0, y0, min(x1, 1920), min(y1, 1080)) for x0, y0, x1, y1 in wins]

    def overlaps(a, b):
        return not (a[2] <= b[0] or b[2] <= a[0] or a[3] <= b[1] or b[3] <= a[1])

    while len(wins) < 4:  # pairwise disjoint windows, so the oracle's per-window sums add up
        x0 = int(rng.integers(0, 1920 - 48)) // 16 * 16
        y0 = int(rng.integers(0, 1080 - 48)) // 16 * 16
        w = (x0, y0, x0 + 48, y0 + 48)
        if not any(overlaps(w, v) for v in wins):
            wins.append(w)
    return s, rast, prep, cfg, fwd, wins


def test_full_lists_in_windows(full):
    s, rast, prep, cfg, fwd, wins = full
    pl, rg = to_np(prep.point_list), to_np(prep.ranges)
    TX = 120
    for (x0, y0, x1, y1) in wins:
        tw = [x0 // 16, y0 // 16, (x1 + 15) // 16, (y1 + 15) // 16]
        ob = oracle.bin_sort_ranges(1920, 1080, to_np(prep.means2D), to_np(prep.radius), to_np(prep.depth),
                                    window=tw)
        for ty in range(tw[1], tw[3]):
            for tx in range(tw[0], tw[2]):
                t = ty * TX + tx
                a = pl[rg[t, 0]:rg[t, 1]]
                b = ob["point_list"][ob["ranges"][t, 0]:ob["ranges"][t, 1]]
                np.testing.assert_array_equal(a, b)


def test_full_forward_in_windows(full):
    s, rast, prep, cfg, fwd, wins = full
    for w in wins:
        orc = oracle_render_from_gpu(prep, window=w)
        compare_forward(fwd, orc, window=w, name=f"full fwd {w}")


@pytest.mark.parametrize("variant,sub", [("gauss", 8), ("hybrid", 8), ("pixel", 16)])
def test_full_other_variants_in_windows(full, variant, sub):
    from paper_2412_17378_amd import make_cfg
    s, rast, prep, cfg, fwd, wins = full
    out = rast.render_fwd(prep, make_cfg(variant, sub, "cost"))
    torch.cuda.synchronize()
    for w in wins[:2]:
        orc = oracle_render_from_gpu(prep, window=w)
        compare_forward(out, orc, window=w, name=f"full {variant}/{sub} {w}")


def test_full_static_equals_balanced(full):
    from paper_2412_17378_amd import make_cfg
    s, rast, prep, cfg, fwd, wins = full
    st = rast.render_fwd(prep, make_cfg("static"))
    wide = rast.render_fwd(prep, make_cfg("pixel", 16, "cost"))
    torch.cuda.synchronize()
    for k in fwd:
        assert torch.equal(st[k], fwd[k]), k
        assert torch.equal(wide[k], fwd[k]), ("wide", k)


def test_full_backward_cropped(full):
    s, rast, prep, cfg, fwd, wins = full
    H, W = 1080, 1920
    rng = np.random.default_rng(17)
    gC = np.zeros((3, H, W), np.float32)
    flagged_total = 0
    for (x0, y0, x1, y1) in wins:
        gC[:, y0:y1, x0:x1] = rng.standard_normal((3, y1 - y0, x1 - x0))
    for w in wins:
        orc = oracle_render_from_gpu(prep, window=w)
        x0, y0, x1, y1 = w
        m = orc["margin"][y0:y1, x0:x1] < MARGIN
        flagged_total += int(m.sum())
        gC[:, y0:y1, x0:x1][:, m] = 0.0
    from paper_2412_17378_amd import make_cfg
    runs = []
    from paper_2412_17378_amd import bgs as B
    for c in (cfg, make_cfg("pixel", 16, "cost"), make_cfg("pixel", 16, "cost", flags=B.FLAG_SPLIT_WALKS),
              make_cfg("static_wave", 16, "raster"), make_cfg("static")):
        print(f"[full-bwd] cfg variant={c.variant} sub={c.subtile}", flush=True)
        runs.append((c, rast.render_bwd(prep, c, fwd, torch.from_numpy(gC).cuda())))
    torch.cuda.synchronize()
    acc = None
    for w in wins:
        o = oracle_bwd_from_gpu(prep, gC, window=w)
        if acc is None:
            acc = o
        else:
            for k in ("means2D", "conic", "opacity", "rgb", "depth"):
                acc["mag"][k] = acc["mag"][k] + o["mag"][k]
                acc[k] = acc[k] + o[k]
    for c, grads in runs:
        compare_grads(grads, acc, name=f"full bwd variant={c.variant} sub={c.subtile} flags={c.flags}")
