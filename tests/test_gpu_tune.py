"""The measured variant selection (bgs_autotune, the adaptive selection of
Sec. 4.4): valid winners, the per-workload cache file, and correct results
with the chosen kernels."""
import numpy as np
import pytest
import torch

from parity import compare_forward, oracle_render_from_gpu
from workloads import scenes

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_parity(tmp_path):
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd import bgs as B
    s = scenes.make("0")
    rast = Rasterizer("cuda", poison_outputs=True)
    prep = rast.prepare_scene(s)
    g = torch.from_numpy(s.upstream()["dL_dcolor"]).cuda()
    cache = str(tmp_path / "tune.txt")
    base = make_cfg("pixel", 8, "cost", (0.1, 0.2, 0.3))
    print("[tune] first call", flush=True)
    f1, b1, fms, bms = rast.autotune(prep, base, g, cache)
    torch.cuda.synchronize()
    for c in (f1, b1):
        assert c.variant in B.VARIANTS.values()
        assert (c.variant == B.STATIC) or c.subtile in (8, 16)
        assert tuple(round(x, 6) for x in c.bg) == (0.1, 0.2, 0.3)
        assert not c.wg_trace and not c.n_examined
    assert fms > 0 and bms > 0
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith(f"{s.cameras[0].width}x{s.cameras[0].height}:")
    print("[tune] cached call", flush=True)
    f2, b2, fms2, bms2 = rast.autotune(prep, base, g, cache)
    assert (f2.variant, f2.subtile, f2.order) == (f1.variant, f1.subtile, f1.order)
    assert (b2.variant, b2.subtile, b2.order) == (b1.variant, b1.subtile, b1.order)
    assert abs(fms2 - fms) < 1e-3 * fms and abs(bms2 - bms) < 1e-3 * bms
    assert len(open(cache).read().strip().splitlines()) == 1  # a hit appends nothing
    # the winners render the oracle's image
    out = rast.render_fwd(prep, f1)
    torch.cuda.synchronize()
    compare_forward(out, oracle_render_from_gpu(prep, bg=(0.1, 0.2, 0.3)), name="tuned forward")


def test_adaptive_selector_retunes_on_interval():
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd.pipeline import AdaptiveSelector
    s = scenes.make("0")
    rast = Rasterizer("cuda", poison_outputs=True)
    prep = rast.prepare_scene(s)
    sel = AdaptiveSelector(rast, make_cfg("pixel", 8, "cost"), interval=2)
    calls = []
    orig = rast.autotune

    def counting(*a, **k):
        calls.append(1)
        return orig(*a, **k)

    rast.autotune = counting
    for _ in range(5):
        f, b = sel.select(prep)
    assert len(calls) == 3  # calls 0, 2 and 4
    assert f.variant in (0, 1, 2, 3)
