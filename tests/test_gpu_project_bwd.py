"""GPU parity of bgs_project_bwd (the projection's derivative) against the
FP64 oracle, on the same inputs and upstream gradients, and of the full
differentiable render from the 3D parameters (Render3DFn) against the
oracle chain render_bwd -> project_bwd on the GPU path's own lists.
Tolerance per element of each gradient: |x - y| <= 1e-4 max(|y|, RMS(y))
plus 32 times the oracle's own change under one-ulp perturbations of the
FP32 inputs (the problem's conditioning at input precision)."""
import numpy as np
import pytest
import torch

import oracle
from parity import check_close, oracle_bwd_from_gpu, rms, to_np
from workloads import scenes
from workloads.scenes import _orbit_camera

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "orbit-sh3":  # rotated camera, SH degree 3
        s = scenes.scene_tiny(n=400, seed=21, width=96, height=64, sh_degree=3)
        s.cameras = [_orbit_camera(96, 64, az=0.4, el=0.2, radius=4.0, centre=(0.0, 0.0, 4.0))]
        return s
    if name == "rgb":
        return scenes.scene_tiny(n=400, seed=22, width=96, height=64)
    return scenes.make(name)


ULP_K = 32  # FP32 pipeline rounding modelled as up to 32 one-ulp input perturbations


def _ulp_sensitivity(cam, s, grads):
    """Per element, the largest change of the oracle's projection gradient
    when every FP32 input (means, log-scales, quaternions, colours) moves by
    one ulp with random signs (two draws): the conditioning of the problem at
    the inputs' own precision, which no FP32 evaluation can beat."""
    gm, gco, gr, gd = grads
    base = oracle.project_bwd(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree, gm, gco, gr, gd)
    sens = {k: np.zeros_like(v) for k, v in base.items()}
    rng = np.random.default_rng(77)
    for _ in range(2):
        pert = []
        for a in (s.means3D, s.log_scales, s.quats, s.colors):
            sign = rng.choice(np.array([-1.0, 1.0], np.float32), size=a.shape)
            pert.append(np.nextafter(a, a + sign * np.float32(1.0)).astype(np.float32))
        o = oracle.project_bwd(cam, pert[0], pert[1], pert[2], s.opacity, pert[3], s.sh_degree, gm, gco, gr, gd)
        for k in sens:
            sens[k] = np.maximum(sens[k], np.abs(o[k] - base[k]))
    return base, sens


def _compare(gpu, orc, sens, name, names=("means3D", "log_scales", "quats", "opacity", "colors")):
    """|x - y| <= 1e-4 max(|y|, RMS(y)) + 32 s, s the oracle's own one-ulp sensitivity."""
    for k in names:
        y = orc[k].reshape(-1)
        x = to_np(gpu[k]).reshape(-1)
        floor = np.maximum(np.abs(y), max(rms(y), 1e-30)) + ULP_K * sens[k].reshape(-1) / 1e-4
        check_close(x, y, floor, f"{name} d{k}")


@pytest.mark.parametrize("name", ["2", "3-early", "4"])
def test_project_forward_parity_full_size(name):
    """The forward projection on the full anisotropic scenes (needle-shaped
    Gaussians included): conic, means2D, depth, rgb per element within
    1e-4 max(|y|, RMS(y))."""
    from paper_2412_17378_amd import Rasterizer
    s = scenes.scene4(n_views=32) if name == "4" else scenes.make(name)
    cam = s.cameras[4 if name == "4" else 0]
    print(f"[proj-fwd] case={name} P={s.P}", flush=True)
    rast = Rasterizer("cuda", poison_outputs=True)
    g = rast.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    torch.cuda.synchronize()
    o = oracle.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree)
    vis = o["radius"] > 0
    assert np.array_equal(to_np(g["radius"]) > 0, vis)
    co = o["conic_opacity"][vis]
    for k in range(3):
        check_close(to_np(g["conic_opacity"])[vis, k], co[:, k], rms(co[:, k]), f"{name} conic[{k}]")
    check_close(to_np(g["means2D"])[vis], o["means2D"][vis], rms(o["means2D"][vis]), f"{name} means2D")
    check_close(to_np(g["depth"])[vis], o["depth"][vis], rms(o["depth"][vis]), f"{name} depth")
    check_close(to_np(g["rgb"])[vis], o["rgb"][vis], max(rms(o["rgb"][vis]), 1e-6), f"{name} rgb")


@pytest.mark.parametrize("name", ["rgb", "orbit-sh3", "0", "2", "3-early"])
def test_project_bwd_parity(name):
    from paper_2412_17378_amd import Rasterizer
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[proj-bwd] case={name} P={s.P}", flush=True)
    rast = Rasterizer("cuda", poison_outputs=True)
    rng = np.random.default_rng(5)
    P = s.P
    gm = rng.standard_normal((P, 2)).astype(np.float32)
    gco = (rng.standard_normal((P, 4)) * np.array([1e-2, 1e-2, 1e-2, 1.0])).astype(np.float32)
    gr = rng.standard_normal((P, 3)).astype(np.float32)
    gd = rng.standard_normal(P).astype(np.float32)
    dev = torch.device("cuda")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = rast.project_bwd(cam, s.means3D, s.log_scales, s.quats, s.colors, s.sh_degree, T(gm), T(gco), T(gr), T(gd))
    torch.cuda.synchronize()
    o, sens = _ulp_sensitivity(cam, s, (gm, gco, gr, gd))
    _compare(g, o, sens, name)


@pytest.mark.parametrize("name", ["orbit-sh3", "0"])
def test_render3d_gradients(name):
    """Loss on the rendered image -> gradients of the 3D parameters, against the
    oracle's render_bwd (on the GPU's own lists and splats) and project_bwd."""
    from paper_2412_17378_amd import Rasterizer, make_cfg, render_gaussians
    s = _scene(name)
    cam = s.cameras[0]
    print(f"[render3d] case={name} P={s.P}", flush=True)
    rast = Rasterizer("cuda", poison_outputs=True)
    dev = torch.device("cuda")
    params = [torch.from_numpy(np.ascontiguousarray(getattr(s, k))).to(dev).requires_grad_(True)
              for k in ("means3D", "log_scales", "quats", "opacity", "colors")]
    color, alpha, depth = render_gaussians(*params, cam, s.sh_degree, rast)
    rng = np.random.default_rng(3)
    gC = rng.standard_normal(tuple(color.shape)).astype(np.float32)
    prep = rast.prepare(cam, *[p.detach() for p in params], s.sh_degree)
    orc_f = oracle.render_fwd(cam.width, cam.height, to_np(prep.ranges), to_np(prep.point_list),
                              to_np(prep.means2D), to_np(prep.conic_opacity), to_np(prep.rgb), to_np(prep.depth))
    gC[:, orc_f["margin"] < 1e-4] = 0.0  # no upstream gradient at near-threshold pixels
    (color * torch.from_numpy(gC).to(dev)).sum().backward()
    torch.cuda.synchronize()
    ob = oracle_bwd_from_gpu(prep, gC)
    gco = np.concatenate([ob["conic"], ob["opacity"][:, None]], 1)
    o = oracle.project_bwd(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, s.sh_degree, ob["means2D"],
                           gco, ob["rgb"], ob["depth"])
    got = dict(zip(("means3D", "log_scales", "quats", "opacity", "colors"), [p.grad for p in params]))
    # the chain inherits the render gradient's tolerance scale (sums over pixels)
    for k in got:
        y = o[k].reshape(-1)
        x = to_np(got[k]).reshape(-1)
        check_close(x, y, max(rms(y), 1e-30), f"{name} render3d d{k}", rtol=1e-3)


@pytest.mark.parametrize("n", [700, 1000])
@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_project_sh_degrees_staged(deg, offset, n):
    """Every SH degree through the per-degree kernels (degrees >= 1 stage the
    colour rows of a 256-Gaussian workgroup through LDS): P not a multiple of
    256, colour arrays 16-byte aligned (offset 0) and not (offset one float).
    Forward colour and backward gradients against the oracle; the words
    around the colour-gradient run stay untouched."""
    from paper_2412_17378_amd import bgs as B
    s = scenes.scene_tiny(n=n, seed=31 + deg, width=96, height=64, sh_degree=deg)
    cam = s.cameras[0]
    P = s.P
    print(f"[proj-sh] degree={deg} offset={offset} P={P}", flush=True)
    dev = torch.device("cuda")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ncol = 3 * (deg + 1) ** 2
    cbuf = torch.zeros(P * ncol + 8, device=dev)
    colors = cbuf[offset:offset + P * ncol]
    colors.copy_(T(s.colors.reshape(-1)))
    f = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
             rgb=torch.zeros(P, 3, device=dev), depth=torch.zeros(P, device=dev),
             radius=torch.zeros(P, dtype=torch.int32, device=dev), tt=torch.zeros(P, dtype=torch.int32, device=dev))
    B.bgs_project(cam, T(s.means3D), T(s.log_scales), T(s.quats), T(s.opacity), colors, deg, f["means2D"],
                  f["conic_opacity"], f["rgb"], f["depth"], f["radius"], f["tt"])
    rng = np.random.default_rng(9)
    gm = rng.standard_normal((P, 2)).astype(np.float32)
    gco = (rng.standard_normal((P, 4)) * np.array([1e-2, 1e-2, 1e-2, 1.0])).astype(np.float32)
    gr = rng.standard_normal((P, 3)).astype(np.float32)
    gd = rng.standard_normal(P).astype(np.float32)
    gbuf = torch.full((P * ncol + 8,), float("nan"), device=dev)
    out = dict(means3D=torch.zeros(P, 3, device=dev), log_scales=torch.zeros(P, 3, device=dev),
               quats=torch.zeros(P, 4, device=dev), opacity=torch.zeros(P, device=dev),
               colors=gbuf[offset:offset + P * ncol])
    B.bgs_project_bwd(cam, T(s.means3D), T(s.log_scales), T(s.quats), colors, deg, T(gm), T(gco), T(gr), T(gd), out)
    torch.cuda.synchronize()
    o = oracle.project(cam, s.means3D, s.log_scales, s.quats, s.opacity, s.colors, deg)
    vis = o["radius"] > 0
    assert vis.sum() > P // 2
    assert np.array_equal(to_np(f["radius"]) > 0, vis)
    check_close(to_np(f["rgb"])[vis], o["rgb"][vis], max(rms(o["rgb"][vis]), 1e-6), f"deg {deg} rgb")
    ob, sens = _ulp_sensitivity(cam, s, (gm, gco, gr, gd))
    gpu = dict(out)
    gpu["colors"] = out["colors"].reshape(s.colors.shape)
    _compare(gpu, ob, sens, f"deg {deg} offset {offset}")
    g = to_np(gbuf)
    assert np.all(np.isnan(g[:offset])) and np.all(np.isnan(g[offset + P * ncol:]))
