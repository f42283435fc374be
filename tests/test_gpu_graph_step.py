"""The whole training-shaped step (project -> tile lists -> queue ->
render_fwd -> queue -> render_bwd) captured once as a hipGraph
(pipeline.FrameStep.capture) and replayed: every replay, with eager GPU work
and synchronizations between replays, must give the eager step's images bit
for bit and its gradients to the accumulation order; after an in-place
change of the parameters a replay must render the changed scene like an
eager step does."""
import numpy as np
import pytest
import torch

from workloads import scenes

pytestmark = pytest.mark.gpu

CFGS = [("pixel", 16, "cost"), ("static", 16, "raster"), ("pixel", 8, "cost")]


def _params(s, dev):
    return {k: torch.from_numpy(getattr(s, k)).to(dev).contiguous()
            for k in ("means3D", "log_scales", "quats", "opacity", "colors")}


def _snapshot(step):
    return {k: v.clone() for k, v in step.fwd.items()}, {k: v.clone() for k, v in step.grads.items()}


def _same(a, b, what):
    fa, ga = a
    fb, gb = b
    for k in fa:
        assert torch.equal(fa[k], fb[k]), (what, k)
    for k in ga:
        scale = float(ga[k].abs().max()) + 1e-30
        assert float((ga[k] - gb[k]).abs().max()) <= 1e-4 * scale, (what, k)


@pytest.mark.parametrize("name", ["0", "3-early"])
@pytest.mark.parametrize("binning", ["square", "ellipse"])
@pytest.mark.parametrize("cfg", CFGS)
def test_graph_step_replays(name, binning, cfg):
    from paper_2412_17378_amd import make_cfg
    from paper_2412_17378_amd.pipeline import FrameStep
    dev = torch.device("cuda")
    s = scenes.make(name)
    cam = s.cameras[0]
    print(f"[graph-step] scene={name} binning={binning} cfg={cfg}", flush=True)
    params = _params(s, dev)
    up = torch.from_numpy(s.upstream()["dL_dcolor"]).to(dev)
    c = make_cfg(*cfg, tuple(s.bg))
    step = FrameStep(cam, params, s.sh_degree, up, c, c, binning=binning, poison_outputs=True)
    step.run()
    torch.cuda.synchronize()
    assert step.n_pairs() <= step.capacity
    eager = _snapshot(step)
    graph = step.capture()
    torch.cuda.synchronize()
    rng = torch.Generator(device=dev).manual_seed(0)
    for r in range(3):
        junk = torch.randn(4096, device=dev, generator=rng) @ torch.randn(4096, 16, device=dev, generator=rng)
        torch.cuda.synchronize()
        del junk
        graph.replay()
        torch.cuda.synchronize()
        _same(eager, _snapshot(step), f"replay {r}")
    # the graph reads the parameters each replay: change them in place
    params["opacity"].mul_(0.5)
    graph.replay()
    torch.cuda.synchronize()
    replayed = _snapshot(step)
    step.run()
    torch.cuda.synchronize()
    _same(_snapshot(step), replayed, "after the in-place update")
    assert not torch.equal(replayed[0]["alpha"], eager[0]["alpha"])
    del graph
