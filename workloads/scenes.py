"""Seeded synthetic scenes shaped like the workloads the rasterizer is measured on.

This module only draws random numbers and lays them out; it holds none of the
rasterizer's arithmetic (no projection, binning, blending or derivatives), so
both the FP64 oracle and the HIP path can consume its output.

Every scene is a set of 3D Gaussians (means, log-scales, unit quaternions
(w, x, y, z), opacities, colours or SH coefficients) plus one or more pinhole
cameras (world->camera rotation R, translation t, intrinsics).  Image pixel
(px, py) is sampled at integer coordinates; the principal point is (W/2, H/2).

Recipes (sizes follow the five measured workloads; seeds are 17378 + id):

  "0"   128x128, f=128, 2 000 Gaussians; means U([-1,1]^2 x [3,5]); log-scales
        N(-3, 0.5); opacity sigmoid(N(0,1)); RGB U[0,1]; black background.
  "1"   1920x1080, f=1920, 500 000 Gaussians: 69% as "0"; 30% clustered with
        x in 0.25 +- 0.448, y in 0.10 +- 0.251 (a 430x241 px window at z=4, i.e.
        5% of the screen), z in [3,5]; 1% large with log-scales N(-0.5, 0.3).
  "2"   1600x1064, f=1600, 3 000 000 Gaussians; SH degree 3 (16 coefficients per
        channel): DC U(-0.5/C0, 0.5/C0) with C0 = 1/(2 sqrt(pi)), the rest
        N(0, 0.2); anisotropic log-scales N(-4, 1); opacity sigmoid(N(-1, 1.5)).
  "3-early" / "3-mid" / "3-late"
        1920x1080 stage sweep: 100k N(-1,0.5) uniform; 1M N(-3,0.8) with 50%
        clustered as "1"; 6M N(-5,0.7) in 8 depth layers z = 3.2 .. 4.8.
  "4"   32 orbit views (radius 4 about (0,0,4), elevation +-15 deg) of a 2M
        Gaussian scene distributed as "2", resolutions cycling 640x360 ..
        1920x1080 with f = W.
  "1-translucent"
        supplementary stress variant of "1": every opacity U[0.02, 0.03], so
        few pixels reach the transmittance cut-off and per-pixel work follows
        the per-tile list length.  Reported beside "1", never instead of it.
  "1-hotspot"
        supplementary stress variant of "1" with a hot spot: 3 000 more faint
        Gaussians (log-scales N(-4.3, 0.1), opacity U[0.006, 0.009]) at z in
        [2.2, 2.8], in front of the scene box, all projecting within 6 px of
        pixel (730, 930) -- a few tiles near the bottom of the frame, late in
        raster order, whose pixels each walk thousands of faint entries before
        stopping, so the heaviest tile outweighs a SIMD's fair share (tail
        ratio R > 1).  Reported beside "1", never instead of it.
  "tiny-N"
        small scenes for brute-force checks (N Gaussians, 48x40 image, f=48).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 17378

# 1/(2 sqrt(pi)): amplitude of the constant real spherical harmonic.  Used only
# to scale the random DC coefficients so the DC colour is uniform in [0, 1].
_SH_C0 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # [3,3] float64, world -> camera rotation (rows = camera axes)
    t: np.ndarray          # [3] float64, camera = R @ world + t
    znear: float = 0.2


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    means3D: np.ndarray     # [P,3] f32
    log_scales: np.ndarray  # [P,3] f32
    quats: np.ndarray       # [P,4] f32, (w,x,y,z), unit norm
    opacity: np.ndarray     # [P]   f32 in (0,1)
    colors: np.ndarray      # [P,3] f32 RGB when sh_degree < 0, else [P,(d+1)^2,3] SH coefficients
    sh_degree: int          # -1: colours given directly; 0..3: SH degree
    cameras: List[Camera]
    bg: np.ndarray          # [3] f32

    @property
    def P(self) -> int:
        return int(self.means3D.shape[0])

    def upstream(self, view: int = 0, seed_offset: int = 1) -> dict:
        """Random upstream gradients dL/d(out_color) ~ N(0,1) per channel, [3,H,W] f32."""
        cam = self.cameras[view]
        rng = np.random.default_rng(self.seed * 1000 + 7 * view + seed_offset)
        g = rng.standard_normal((3, cam.height, cam.width), dtype=np.float32)
        return {"dL_dcolor": g}


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _quats(rng, n):
    q = rng.standard_normal((n, 4)).astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _uniform_box(rng, n, xlo=-1.0, xhi=1.0, ylo=-1.0, yhi=1.0, zlo=3.0, zhi=5.0):
    m = np.empty((n, 3), np.float64)
    m[:, 0] = rng.uniform(xlo, xhi, n)
    m[:, 1] = rng.uniform(ylo, yhi, n)
    m[:, 2] = rng.uniform(zlo, zhi, n)
    return m


def _clustered(rng, n):
    return _uniform_box(rng, n, 0.25 - 0.448, 0.25 + 0.448, 0.10 - 0.251, 0.10 + 0.251)


def _axis_camera(w, h, f):
    return Camera(width=w, height=h, fx=float(f), fy=float(f), cx=w / 2.0, cy=h / 2.0,
                  R=np.eye(3), t=np.zeros(3))


def _orbit_camera(w, h, az, el, radius=4.0, centre=(0.0, 0.0, 4.0)):
    c0 = np.asarray(centre, np.float64)
    pos = c0 + radius * np.array([math.sin(az) * math.cos(el), math.sin(el),
                                  -math.cos(az) * math.cos(el)])
    fwd = c0 - pos
    fwd /= np.linalg.norm(fwd)
    down_hint = np.array([0.0, 1.0, 0.0])
    right = np.cross(down_hint, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ pos
    return Camera(width=w, height=h, fx=float(w), fy=float(w), cx=w / 2.0, cy=h / 2.0, R=R, t=t)


def _sh_coeffs(rng, n, degree=3):
    k = (degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (n, k, 3)).astype(np.float32)
    sh[:, 0, :] = rng.uniform(-0.5 / _SH_C0, 0.5 / _SH_C0, (n, 3)).astype(np.float32)
    return sh


def _finish(name, seed, means, log_scales, quats, opacity, colors, sh_degree, cameras):
    return Scene(name=name, seed=seed,
                 means3D=np.ascontiguousarray(means, np.float32),
                 log_scales=np.ascontiguousarray(log_scales, np.float32),
                 quats=np.ascontiguousarray(quats, np.float32),
                 opacity=np.ascontiguousarray(opacity, np.float32),
                 colors=np.ascontiguousarray(colors, np.float32),
                 sh_degree=sh_degree, cameras=cameras,
                 bg=np.zeros(3, np.float32))


def _base_params(rng, n, ls_mu, ls_sd):
    return (rng.normal(ls_mu, ls_sd, (n, 3)), _quats(rng, n),
            _sigmoid(rng.standard_normal(n)), rng.uniform(0.0, 1.0, (n, 3)))


def scene0(seed: Optional[int] = None) -> Scene:
    seed = SEED_BASE + 0 if seed is None else seed
    rng = _rng(seed)
    n = 2000
    means = _uniform_box(rng, n)
    ls, q, op, rgb = _base_params(rng, n, -3.0, 0.5)
    return _finish("0", seed, means, ls, q, op, rgb, -1, [_axis_camera(128, 128, 128)])


def _scene1_arrays(rng, n_total):
    n_cl = int(round(0.30 * n_total))
    n_lg = int(round(0.01 * n_total))
    n_bs = n_total - n_cl - n_lg
    means = np.concatenate([_uniform_box(rng, n_bs), _clustered(rng, n_cl), _uniform_box(rng, n_lg)])
    ls = np.concatenate([rng.normal(-3.0, 0.5, (n_bs + n_cl, 3)), rng.normal(-0.5, 0.3, (n_lg, 3))])
    q = _quats(rng, n_total)
    op = _sigmoid(rng.standard_normal(n_total))
    rgb = rng.uniform(0.0, 1.0, (n_total, 3))
    # interleave the three populations so that input order carries no structure
    perm = rng.permutation(n_total)
    return means[perm], ls[perm], q, op, rgb


def scene1(seed: Optional[int] = None, n_total: int = 500_000) -> Scene:
    seed = SEED_BASE + 1 if seed is None else seed
    rng = _rng(seed)
    means, ls, q, op, rgb = _scene1_arrays(rng, n_total)
    return _finish("1", seed, means, ls, q, op, rgb, -1, [_axis_camera(1920, 1080, 1920)])


def scene1_translucent(seed: Optional[int] = None, n_total: int = 500_000) -> Scene:
    seed = SEED_BASE + 101 if seed is None else seed
    rng = _rng(seed)
    means, ls, q, _, rgb = _scene1_arrays(rng, n_total)
    op = rng.uniform(0.02, 0.03, n_total)
    return _finish("1-translucent", seed, means, ls, q, op, rgb, -1, [_axis_camera(1920, 1080, 1920)])


def scene1_hotspot(seed: Optional[int] = None, n_total: int = 500_000, n_hot: int = 3_000) -> Scene:
    seed = SEED_BASE + 102 if seed is None else seed
    rng = _rng(seed)
    means, ls, q, op, rgb = _scene1_arrays(rng, n_total)
    # in front of the scene box, all projecting within +-6 px of pixel (730, 930)
    z = rng.uniform(2.2, 2.8, n_hot)
    u = 730.0 + rng.uniform(-6.0, 6.0, n_hot)
    v = 930.0 + rng.uniform(-6.0, 6.0, n_hot)
    hot = np.stack([(u + 0.5 - 960.0) * z / 1920.0, (v + 0.5 - 540.0) * z / 1920.0, z], axis=1)
    means = np.concatenate([means, hot])
    ls = np.concatenate([ls, rng.normal(-4.3, 0.1, (n_hot, 3))])
    q = np.concatenate([q, _quats(rng, n_hot)])
    op = np.concatenate([op, rng.uniform(0.006, 0.009, n_hot)])
    rgb = np.concatenate([rgb, rng.uniform(0.0, 1.0, (n_hot, 3))])
    return _finish("1-hotspot", seed, means, ls, q, op, rgb, -1, [_axis_camera(1920, 1080, 1920)])


def _scene2_arrays(rng, n):
    means = _uniform_box(rng, n)
    ls = rng.normal(-4.0, 1.0, (n, 3))
    q = _quats(rng, n)
    op = _sigmoid(rng.normal(-1.0, 1.5, n))
    sh = _sh_coeffs(rng, n, 3)
    return means, ls, q, op, sh


def scene2(seed: Optional[int] = None, n: int = 3_000_000) -> Scene:
    seed = SEED_BASE + 2 if seed is None else seed
    rng = _rng(seed)
    means, ls, q, op, sh = _scene2_arrays(rng, n)
    return _finish("2", seed, means, ls, q, op, sh, 3, [_axis_camera(1600, 1064, 1600)])


def scene3(stage: str, seed: Optional[int] = None) -> Scene:
    seed = SEED_BASE + 3 if seed is None else seed
    rng = _rng(seed + {"early": 0, "mid": 10, "late": 20}[stage])
    if stage == "early":
        n = 100_000
        means = _uniform_box(rng, n)
        ls = rng.normal(-1.0, 0.5, (n, 3))
    elif stage == "mid":
        n = 1_000_000
        h = n // 2
        means = np.concatenate([_uniform_box(rng, n - h), _clustered(rng, h)])
        means = means[rng.permutation(n)]
        ls = rng.normal(-3.0, 0.8, (n, 3))
    elif stage == "late":
        n = 6_000_000
        layers = np.linspace(3.2, 4.8, 8)
        means = _uniform_box(rng, n)
        means[:, 2] = layers[rng.integers(0, 8, n)] + rng.normal(0.0, 0.02, n)
        ls = rng.normal(-5.0, 0.7, (n, 3))
    else:
        raise ValueError(stage)
    q = _quats(rng, n)
    op = _sigmoid(rng.standard_normal(n))
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    return _finish("3-" + stage, seed, means, ls, q, op, rgb, -1, [_axis_camera(1920, 1080, 1920)])


RESOLUTIONS_4 = [(640, 360), (960, 540), (1280, 720), (1600, 900), (1920, 1080)]


def scene4(seed: Optional[int] = None, n: int = 2_000_000, n_views: int = 32) -> Scene:
    seed = SEED_BASE + 4 if seed is None else seed
    rng = _rng(seed)
    means, ls, q, op, sh = _scene2_arrays(rng, n)
    cams = []
    for i in range(n_views):
        w, h = RESOLUTIONS_4[i % len(RESOLUTIONS_4)]
        az = 2.0 * math.pi * i / n_views
        el = math.radians(15.0) * (1.0 if i % 2 == 0 else -1.0)
        cams.append(_orbit_camera(w, h, az, el))
    return _finish("4", seed, means, ls, q, op, sh, 3, cams)


def scene_tiny(n: int = 24, seed: int = 5, width: int = 48, height: int = 40, sh_degree: int = -1,
               log_scale_mu: float = -2.0) -> Scene:
    rng = _rng(SEED_BASE + 1000 + seed)
    means = _uniform_box(rng, n, -0.5, 0.5, -0.45, 0.45, 3.0, 5.0)
    ls = rng.normal(log_scale_mu, 0.4, (n, 3))
    q = _quats(rng, n)
    op = _sigmoid(rng.standard_normal(n))
    if sh_degree < 0:
        col = rng.uniform(0.0, 1.0, (n, 3))
    else:
        col = _sh_coeffs(rng, n, sh_degree)
    return _finish(f"tiny-{n}", SEED_BASE + 1000 + seed, means, ls, q, op, col, sh_degree,
                   [_axis_camera(width, height, width)])


def make(name: str, **kw) -> Scene:
    """Build a scene by workload name ("0", "1", "2", "3-early", "3-mid", "3-late", "4",
    "1-translucent", "1-hotspot", "tiny-N")."""
    if name == "0":
        return scene0(**kw)
    if name == "1":
        return scene1(**kw)
    if name == "1-translucent":
        return scene1_translucent(**kw)
    if name == "1-hotspot":
        return scene1_hotspot(**kw)
    if name == "2":
        return scene2(**kw)
    if name.startswith("3-"):
        return scene3(name[2:], **kw)
    if name == "4":
        return scene4(**kw)
    if name.startswith("tiny-"):
        return scene_tiny(int(name[5:]), **kw)
    raise ValueError(f"unknown scene {name!r}")
