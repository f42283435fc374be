"""A training loop through the whole differentiable path (projection, tile
lists, render, render backward, projection backward) with the measured
kernel selection re-run every few iterations: perturbed Gaussians are fitted
to images of the unperturbed ones from four orbit views."""
import numpy as np
import pytest
import torch

from workloads import scenes
from workloads.scenes import _orbit_camera

pytestmark = pytest.mark.gpu


def test_fit_with_adaptive_selection():
    from paper_2412_17378_amd import Rasterizer, make_cfg
    from paper_2412_17378_amd.pipeline import AdaptiveSelector, fit, render_gaussians
    s = scenes.scene_tiny(n=300, seed=31, width=80, height=64, log_scale_mu=-2.5)
    cams = [_orbit_camera(80, 64, az=a, el=0.15 * (-1) ** k, radius=4.0, centre=(0.0, 0.0, 4.0))
            for k, a in enumerate((0.0, 0.5, -0.5, 1.0))]
    rast = Rasterizer("cuda", poison_outputs=True)
    dev = torch.device("cuda")
    true = {k: torch.from_numpy(np.ascontiguousarray(getattr(s, k))).to(dev)
            for k in ("means3D", "log_scales", "quats", "opacity", "colors")}
    with torch.no_grad():
        targets = [render_gaussians(*true.values(), c, s.sh_degree, rast)[0].clone() for c in cams]
    rng = np.random.default_rng(8)
    start = {k: v.clone() for k, v in true.items()}
    start["means3D"] += torch.from_numpy(rng.normal(0, 0.03, s.means3D.shape).astype(np.float32)).to(dev)
    start["log_scales"] += torch.from_numpy(rng.normal(0, 0.2, s.log_scales.shape).astype(np.float32)).to(dev)
    start["colors"] = torch.full_like(start["colors"], 0.5)
    start["opacity"] = torch.full_like(start["opacity"], 0.5)
    params = {k: v.clone().requires_grad_(True) for k, v in start.items()}
    sel = AdaptiveSelector(rast, make_cfg("pixel", 8, "cost"), interval=25)
    tunes = []
    orig = rast.autotune

    def counting(*a, **k):
        tunes.append(1)
        return orig(*a, **k)

    rast.autotune = counting
    print("[train] fitting", flush=True)
    losses = fit(params, cams, targets, s.sh_degree, rast, iters=120, lr=1e-2, selector=sel)
    print(f"[train] loss {losses[0]:.5f} -> {np.mean(losses[-8:]):.5f}, {len(tunes)} selections", flush=True)
    assert np.all(np.isfinite(losses))
    assert np.mean(losses[-8:]) < 0.25 * np.mean(losses[:4]), (losses[:4], losses[-8:])
    assert len(tunes) == 5  # iterations 0, 25, 50, 75, 100
