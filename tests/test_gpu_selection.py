"""Self-adaptive selection (Sec. 4.4) across a changing workload.

AdaptiveSelector (re-tuning on every frame here) is fed the training-stage
frames 3-early -> 3-mid -> 3-late and then the hot-spot frame (scene 1 with a
late, dense cluster in front: one tile holding thousands of entries, the
case where the per-tile critical path dominates).  Each stage's candidates
are also timed independently by the test.  Asserted:

* every pick is within 10% of the fastest candidate this test measures on
  that stage (the pick follows the measured times);
* where the times cross -- an earlier stage's pick is at least 1.5x slower
  than the best on a later stage -- the later pick differs (on the hot spot
  the grid-static kernels the early stages pick fall far behind);
* the backward picks split walks on the hot spot, whose deepest walk is
  many times the mean.
"""
import numpy as np
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

STAGES = ["3-early", "3-mid", "3-late", "1-hotspot"]
# the autotuner's candidates (variant, sub-tile, order, flags: 2 split walks, 8 persistent pool)
FWD = [("static", 16, "raster", 0), ("static_wave", 16, "raster", 0), ("pixel", 8, "raster", 0),
       ("pixel", 8, "cost", 0), ("pixel", 16, "raster", 0), ("pixel", 16, "cost", 0), ("pixel", 16, "cost", 8),
       ("pixel", 32, "cost", 0), ("hybrid", 8, "cost", 0), ("gauss", 8, "cost", 0)]
BWD = [("static", 16, "raster", 0), ("static_wave", 16, "raster", 0), ("pixel", 8, "raster", 0),
       ("pixel", 8, "cost", 0), ("pixel", 16, "raster", 0), ("pixel", 16, "cost", 0), ("pixel", 16, "cost", 8),
       ("pixel", 16, "cost", 2), ("pixel", 32, "cost", 0)]


def _median_ms(fn, n=5):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(n):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def test_selection_follows_the_workload():
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd import bgs as B
    from paper_2412_17378_amd.pipeline import AdaptiveSelector
    rast = Rasterizer("cuda")
    sel = AdaptiveSelector(rast, make_cfg("pixel", 16, "cost"), interval=1)
    seq = []
    for name in STAGES:
        s = scenes.make(name)
        print(f"[select] stage={name} P={s.P}", flush=True)
        prep = rast.prepare_scene(s)
        bg = tuple(s.bg)
        sel.base = make_cfg("pixel", 16, "cost", bg)
        up = torch.ones(3, prep.height, prep.width, device="cuda")
        fcfg, bcfg = sel.select(prep, up)
        pick_f, pick_b = B.cfg_name(fcfg), B.cfg_name(bcfg)
        out = rast.render_fwd(prep, make_cfg("static", 16, "raster", bg))
        tf = {}
        for v in FWD:
            c = make_cfg(*v[:3], bg, flags=v[3])
            tf[B.cfg_name(c)] = _median_ms(lambda: rast.render_fwd(prep, c, out=out))
        rast.render_fwd(prep, make_cfg("static", 16, "raster", bg), out=out)
        grads = dict(means2D=torch.zeros(prep.P, 2, device="cuda"), conic_opacity=torch.zeros(prep.P, 4, device="cuda"),
                     rgb=torch.zeros(prep.P, 3, device="cuda"), depth=None)
        tb = {}
        for v in BWD:
            c = make_cfg(*v[:3], bg, flags=v[3])
            tb[B.cfg_name(c)] = _median_ms(lambda: rast.render_bwd(prep, c, out, up, grads=grads))
        print(f"[select] {name}: picks forward {pick_f}, backward {pick_b}; fastest measured forward "
              f"{min(tf, key=tf.get)} {min(tf.values()):.3f} ms (pick {tf[pick_f]:.3f}), backward "
              f"{min(tb, key=tb.get)} {min(tb.values()):.3f} ms (pick {tb[pick_b]:.3f})", flush=True)
        seq.append((name, pick_f, pick_b, tf, tb))
        assert tf[pick_f] <= 1.10 * min(tf.values()), (name, pick_f, tf)
        assert tb[pick_b] <= 1.10 * min(tb.values()), (name, pick_b, tb)
        del prep, out, grads
        torch.cuda.empty_cache()
    print("[select] sequence: " + " -> ".join(f"{n} ({f} / {b})" for n, f, b, _, _ in seq), flush=True)
    changed = 0
    for i, (_, pf0, pb0, _, _) in enumerate(seq):
        for name, pf1, pb1, tf, tb in seq[i + 1:]:
            if tf[pf0] >= 1.5 * min(tf.values()):  # an earlier pick fell behind here: the pick moved
                assert pf1 != pf0, (name, pf0, tf)
                changed += 1
            if tb[pb0] >= 1.5 * min(tb.values()):
                assert pb1 != pb0, (name, pb0, tb)
                changed += 1
    assert changed >= 1, "no stage made an earlier pick fall behind"
    assert seq[-1][2].endswith("/split"), seq[-1][2]
