"""Deterministic-order backward (bgs_render_bwd_det): gradients identical
bit for bit from run to run (the atomic backward's are not, in general),
equal to the oracle's within the backward tolerance, and to the atomic
backward's up to fp32 rounding; capacity and configuration errors."""
import numpy as np
import pytest
import torch

from parity import MARGIN, compare_grads, oracle_bwd_from_gpu, oracle_render_from_gpu
from workloads import scenes

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "sh3":
        return scenes.scene_tiny(n=200, seed=11, width=80, height=56, sh_degree=3)
    return scenes.make(name)


@pytest.fixture(scope="module")
def rast():
    from paper_2412_17378_amd import Rasterizer
    return Rasterizer("cuda", poison_outputs=True)


def _upstream(s, orc_f, seed=5):
    cam = s.cameras[0]
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    gA = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    gD = rng.standard_normal((cam.height, cam.width)).astype(np.float32)
    if orc_f is not None:
        flagged = orc_f["margin"] < MARGIN
        for g in (gC, gA[None], gD[None]):
            g[:, flagged] = 0.0
    return gC, gA, gD


@pytest.mark.parametrize("name", ["tiny-300", "0", "sh3"])
def test_det_backward_parity_and_repeatability(rast, name):
    from paper_2412_17378_amd import make_cfg
    s = _scene(name)
    bg = (0.3, 0.1, 0.2)
    print(f"[det-bwd] case={name}", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost", bg)
    fwd = rast.render_fwd(prep, cfg)
    torch.cuda.synchronize()
    orc_f = oracle_render_from_gpu(prep, bg=bg)
    gC, gA, gD = _upstream(s, orc_f)
    dev = torch.device("cuda")
    up = [torch.from_numpy(g).to(dev) for g in (gC, gA, gD)]
    runs = [rast.render_bwd_det(prep, cfg, fwd, *up) for _ in range(3)]
    torch.cuda.synchronize()
    for r in runs[1:]:
        for k in runs[0]:
            assert torch.equal(runs[0][k], r[k]), k
    orc = oracle_bwd_from_gpu(prep, gC, gA, gD, bg=bg)
    compare_grads(runs[0], orc, name=f"det {name}")
    atomic = rast.render_bwd(prep, cfg, fwd, *up)
    torch.cuda.synchronize()
    for k in atomic:
        a, b = atomic[k], runs[0][k]
        assert float((a - b).abs().max()) <= 1e-4 * (float(a.abs().max()) + 1e-30), k


def test_det_backward_full_size_repeatable(rast):
    """1920x1080, 100k Gaussians: identical from run to run, close to the
    atomic backward."""
    from paper_2412_17378_amd import make_cfg
    s = scenes.make("3-early")
    print("[det-bwd] scene 3-early", flush=True)
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost")
    fwd = rast.render_fwd(prep, cfg)
    gC, gA, gD = _upstream(s, None)
    dev = torch.device("cuda")
    up = [torch.from_numpy(gC).to(dev), None, None]
    a = rast.render_bwd_det(prep, cfg, fwd, *up)
    b = rast.render_bwd_det(prep, cfg, fwd, *up)
    atomic = rast.render_bwd(prep, cfg, fwd, *up)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
        scale = float(atomic[k].abs().max()) + 1e-30
        assert float((a[k] - atomic[k]).abs().max()) <= 1e-4 * scale, k


def test_det_backward_capacity_and_config(rast):
    from paper_2412_17378_amd import bgs as B
    from paper_2412_17378_amd import make_cfg
    s = scenes.make("0")
    prep = rast.prepare_scene(s)
    cfg = make_cfg("pixel", 16, "cost")
    fwd = rast.render_fwd(prep, cfg)
    dev = torch.device("cuda")
    gC = torch.from_numpy(_upstream(s, None)[0]).to(dev)
    P = prep.P
    grads = {k: torch.zeros(P, n, device=dev) for k, n in (("means2D", 2), ("conic_opacity", 4), ("rgb", 3))}
    f = prep.frame()
    ws = torch.empty(B.bgs_render_bwd_det_workspace_bytes(f, P, 1), dtype=torch.uint8, device=dev)
    with pytest.raises(B.BgsError) as ei:
        B.bgs_render_bwd_det(f, cfg, P, fwd["final_T"], fwd["n_contrib"], gC, None, None, grads["means2D"],
                             grads["conic_opacity"], grads["rgb"], None, 1, ws)
    assert ei.value.status == B.BGS_ECAPACITY and ei.value.n_occ > 1
    for g in grads.values():  # nothing written
        assert float(g.abs().max()) == 0.0
    ws = torch.empty(B.bgs_render_bwd_det_workspace_bytes(f, P, ei.value.n_occ), dtype=torch.uint8, device=dev)
    assert B.bgs_render_bwd_det(f, cfg, P, fwd["final_T"], fwd["n_contrib"], gC, None, None, grads["means2D"],
                                grads["conic_opacity"], grads["rgb"], None, ei.value.n_occ, ws) == ei.value.n_occ
    with pytest.raises(B.BgsError) as ei2:
        B.bgs_render_bwd_det(f, make_cfg("pixel", 8, "cost"), P, fwd["final_T"], fwd["n_contrib"], gC, None, None,
                             grads["means2D"], grads["conic_opacity"], grads["rgb"], None, 1 << 20, ws)
    assert ei2.value.status == B.BGS_EUNSUPPORTED
