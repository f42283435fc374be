"""The benchmark's timed step checked against the oracle directly, at full
size: scene "1" (1920x1080, 500k Gaussians) through pipeline.FrameStep with
tile lists capped at the automatically chosen K (list_cap="auto") and the
forward / backward kernel pairs the autotuner chooses between, eagerly and as
replays of the captured hipGraph.  The oracle builds its own whole,
uncapped lists for the window tiles from the GPU's projected splats, renders
the windows, and differentiates them with the upstream gradient cropped to
the windows; outputs are poisoned before every step, so nothing passes on
values left from an earlier step."""
import numpy as np
import pytest
import torch

import oracle
from parity import MARGIN, compare_forward, compare_grads, to_np
from workloads import scenes

pytestmark = pytest.mark.gpu

PAIRS = [(("static", 16, "raster"), ("pixel", 16, "cost")),
         (("pixel", 16, "cost"), ("pixel", 16, "cost")),
         (("pixel", 16, "raster"), ("pixel", 16, "cost", "split")),
         (("pixel", 32, "cost"), ("pixel", 32, "cost")),
         (("static_wave", 16, "raster"), ("static_wave", 16, "raster"))]


def _params(s, dev):
    return {k: torch.from_numpy(getattr(s, k)).to(dev).contiguous()
            for k in ("means3D", "log_scales", "quats", "opacity", "colors")}


@pytest.fixture(scope="module")
def ref():
    from paper_2412_17378_amd import Rasterizer
    s = scenes.make("1")
    cam = s.cameras[0]
    W, H = cam.width, cam.height
    rast = Rasterizer("cuda")
    pr = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    m2, co, rgb, dp, rad = (to_np(pr[k]) for k in ("means2D", "conic_opacity", "rgb", "depth", "radius"))
    TX = (W + 15) // 16
    # the tile with the longest list (located with the GPU's own lists; the
    # reference lists below are the oracle's) and three random windows,
    # pairwise disjoint
    lens = to_np(rast.bin_sort_ranges(W, H, pr).ranges)
    heavy = int(np.argmax(lens[:, 1] - lens[:, 0]))
    del lens
    hx, hy = heavy % TX * 16, heavy // TX * 16
    wins = [(hx, hy, min(hx + 32, W), min(hy + 32, H))]
    rng = np.random.default_rng(21)

    def overlaps(a, b):
        return not (a[2] <= b[0] or b[2] <= a[0] or a[3] <= b[1] or b[3] <= a[1])

    while len(wins) < 4:
        x0 = int(rng.integers(0, W - 48)) // 16 * 16
        y0 = int(rng.integers(0, H - 48)) // 16 * 16
        w = (x0, y0, x0 + 48, y0 + 48)
        if not any(overlaps(w, v) for v in wins):
            wins.append(w)
    gC = np.zeros((3, H, W), np.float32)
    orcs = []
    for (x0, y0, x1, y1) in wins:
        tw = [x0 // 16, y0 // 16, (x1 + 15) // 16, (y1 + 15) // 16]
        ob = oracle.bin_sort_ranges(W, H, m2, rad, dp, window=tw)
        o = oracle.render_fwd(W, H, ob["ranges"], ob["point_list"], m2, co, rgb, dp, bg=tuple(s.bg),
                              window=(x0, y0, x1, y1))
        orcs.append((ob, o))
        g = rng.standard_normal((3, y1 - y0, x1 - x0)).astype(np.float32)
        g[:, o["margin"][y0:y1, x0:x1] < MARGIN] = 0.0
        gC[:, y0:y1, x0:x1] = g
    acc = None
    for w, (ob, _) in zip(wins, orcs):
        b = oracle.render_bwd(W, H, ob["ranges"], ob["point_list"], m2, co, rgb, dp, gC, bg=tuple(s.bg), window=w)
        if acc is None:
            acc = b
        else:
            for k in ("means2D", "conic", "opacity", "rgb", "depth"):
                acc[k] = acc[k] + b[k]
                acc["mag"][k] = acc["mag"][k] + b["mag"][k]
    return s, wins, orcs, gC, acc


@pytest.mark.parametrize("fwd,bwd", PAIRS)
def test_timed_step_against_oracle(ref, fwd, bwd):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd.pipeline import FrameStep
    s, wins, orcs, gC, acc = ref
    dev = torch.device("cuda")
    cam = s.cameras[0]
    print(f"[timed] fwd={fwd} bwd={bwd}", flush=True)
    from paper_2412_17378_amd import bgs as B
    bc = make_cfg(*bwd[:3], tuple(s.bg), flags=B.FLAG_SPLIT_WALKS if "split" in bwd[3:] else 0)
    step = FrameStep(cam, _params(s, dev), s.sh_degree, torch.from_numpy(gC).to(dev), make_cfg(*fwd, tuple(s.bg)),
                     bc, list_cap="auto", poison_outputs=True)
    assert 0 < step.list_cap <= 2048, step.list_cap

    def check(what):
        assert not step.overflowed(), what
        for w, (_, o) in zip(wins, orcs):
            compare_forward(step.fwd, o, window=w, name=f"timed {what} {fwd} {w}")
        compare_grads(step.grads, acc, name=f"timed {what} {fwd}/{bwd}")

    step.run()
    torch.cuda.synchronize()
    check("eager")
    graph = step.capture()
    for r in range(2):
        graph.replay()
        torch.cuda.synchronize()
        check(f"replay {r}")
    del graph
