"""FP64 CPU oracle of the 3DGS tile-rasterizer path (project -> bin -> sort ->
ranges -> render forward / backward), written from Balanced 3DGS (arXiv
2412.17378) Sec. 2.1, Eq. (1)-(4) and the per-pixel skip / stop rules of its
detailed naive render loop (Appendix).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline leg use this package.  It shares no code with the HIP library.

Thin ctypes layer over ``liborc.so`` (built from ``orc.c`` by ``build.py``).
Arrays are numpy; floating inputs are widened to float64 and every result is
float64 (int32 for indices and counts).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

TILE = 16


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("znear", C.c_double)]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.library_path()
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.orc_project.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_project.restype = C.c_int
        L.orc_project_bwd.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_project_bwd.restype = C.c_int
        L.orc_bin.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp]
        L.orc_bin.restype = i64
        L.orc_bin_exact.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp, vp]
        L.orc_bin_exact.restype = i64
        L.orc_rect_min_q.argtypes = [C.c_double] * 7
        L.orc_rect_min_q.restype = C.c_double
        L.orc_bin_q_limit.argtypes = [C.c_double]
        L.orc_bin_q_limit.restype = C.c_double
        L.orc_sort.argtypes = [i64, vp, vp, vp]
        L.orc_sort.restype = C.c_int
        L.orc_ranges.argtypes = [i64, vp, i32, vp]
        L.orc_ranges.restype = C.c_int
        L.orc_render_fwd.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_render_fwd.restype = i64
        L.orc_render_bwd.argtypes = [i32, i32, i32] + [vp] * 21
        L.orc_render_bwd.restype = i64
        L.orc_sh_basis.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double]
        L.orc_sh_basis.restype = C.c_double
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().orc_num_threads())


def sh_basis(l: int, m: int, d) -> float:
    return float(lib().orc_sh_basis(l, m, float(d[0]), float(d[1]), float(d[2])))


def _camera(cam) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = t[k]
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def _i32(a):
    return np.ascontiguousarray(a, np.int32)


def project(cam, means3D, log_scales, quats, opacity, colors, sh_degree: int) -> dict:
    """Eq. (1)-(3) per Gaussian.  Returns means2D [P,2], conic_opacity [P,4]
    (a, b, c, o), rgb [P,3], depth [P], radius [P] int32 (0 = culled),
    extent [P] (3 sqrt(lambda_max) before rounding up), cov2d [P,3]."""
    P = int(np.asarray(means3D).shape[0])
    m3, ls, q, op, col = _f32(means3D), _f32(log_scales), _f32(quats), _f32(opacity), _f32(colors)
    out = dict(means2D=np.zeros((P, 2)), conic_opacity=np.zeros((P, 4)), rgb=np.zeros((P, 3)),
               depth=np.zeros(P), radius=np.zeros(P, np.int32), extent=np.zeros(P), cov2d=np.zeros((P, 3)))
    cc = _camera(cam)
    rc = lib().orc_project(C.byref(cc), P, _p(m3), _p(ls), _p(q), _p(op), _p(col), int(sh_degree),
                           _p(out["means2D"]), _p(out["conic_opacity"]), _p(out["rgb"]), _p(out["depth"]),
                           _p(out["radius"]), _p(out["extent"]), _p(out["cov2d"]))
    if rc != 0:
        raise ValueError("orc_project failed")
    return out


def project_bwd(cam, means3D, log_scales, quats, opacity, colors, sh_degree: int, dL_dmeans2D,
                dL_dconic_opacity, dL_drgb, dL_ddepth=None) -> dict:
    """Derivative of :func:`project`: from the gradients of its outputs
    (means2D, conic_opacity, rgb, depth) to those of its inputs.  Returns
    means3D [P,3], log_scales [P,3], quats [P,4], opacity [P], colors (shape
    of the colour input); zeros for culled Gaussians."""
    P = int(np.asarray(means3D).shape[0])
    m3, ls, q, op, col = _f32(means3D), _f32(log_scales), _f32(quats), _f32(opacity), _f32(colors)
    gm, gco, gr = _f64(dL_dmeans2D), _f64(dL_dconic_opacity), _f64(dL_drgb)
    gd = None if dL_ddepth is None else _f64(dL_ddepth)
    out = dict(means3D=np.zeros((P, 3)), log_scales=np.zeros((P, 3)), quats=np.zeros((P, 4)),
               opacity=np.zeros(P), colors=np.zeros(col.shape))
    cc = _camera(cam)
    rc = lib().orc_project_bwd(C.byref(cc), P, _p(m3), _p(ls), _p(q), _p(op), _p(col), int(sh_degree), _p(gm),
                               _p(gco), _p(gr), _p(gd), _p(out["means3D"]), _p(out["log_scales"]),
                               _p(out["quats"]), _p(out["opacity"]), _p(out["colors"]))
    if rc != 0:
        raise ValueError("orc_project_bwd failed")
    return out


def project_scene(scene, view: int = 0) -> dict:
    return project(scene.cameras[view], scene.means3D, scene.log_scales, scene.quats, scene.opacity,
                   scene.colors, scene.sh_degree)


def n_tiles(width: int, height: int, tile: int = TILE) -> int:
    return ((width + tile - 1) // tile) * ((height + tile - 1) // tile)


def bin_pairs(width, height, means2D, radius, tile: int = TILE, window: Optional[Sequence[int]] = None,
              conic_opacity=None):
    """(tile id, Gaussian id) pairs in input order, unsorted.  With
    conic_opacity [P,4] the exact ellipse-tile rule filters the square rule's
    pairs (orc_bin_exact)."""
    m2, r = _f64(means2D), _i32(radius)
    P = int(r.shape[0])
    win = None if window is None else _i32(window)
    if conic_opacity is None:
        def run(t, g):
            return lib().orc_bin(width, height, tile, P, _p(m2), _p(r), _p(win), t, g)
    else:
        co = _f64(conic_opacity)

        def run(t, g):
            return lib().orc_bin_exact(width, height, tile, P, _p(m2), _p(r), _p(co), _p(win), t, g)
    M = run(None, None)
    tid = np.zeros(max(M, 1), np.int32)
    gid = np.zeros(max(M, 1), np.int32)
    M2 = run(_p(tid), _p(gid))
    assert M == M2
    return tid[:M].copy(), gid[:M].copy()


def rect_min_q(a, b, c, lx, hx, ly, hy) -> float:
    """min of a x^2 + 2 b x y + c y^2 over [lx, hx] x [ly, hy]."""
    return float(lib().orc_rect_min_q(a, b, c, lx, hx, ly, hy))


def bin_q_limit(opacity) -> float:
    """Upper bound on q of the exact binning rule (negative: never blends)."""
    return float(lib().orc_bin_q_limit(float(opacity)))


def sort_pairs(tile_ids, gauss_ids, depth):
    tid, gid = _i32(tile_ids).copy(), _i32(gauss_ids).copy()
    d = _f64(depth)
    if lib().orc_sort(int(tid.shape[0]), _p(tid), _p(gid), _p(d)) != 0:
        raise MemoryError("orc_sort")
    return tid, gid


def ranges(sorted_tile_ids, n_tiles_: int):
    tid = _i32(sorted_tile_ids)
    out = np.zeros((n_tiles_, 2), np.int32)
    if lib().orc_ranges(int(tid.shape[0]), _p(tid), n_tiles_, _p(out)) != 0:
        raise ValueError("tile id out of range")
    return out


def bin_sort_ranges(width, height, means2D, radius, depth, tile: int = TILE, window=None, conic_opacity=None) -> dict:
    tid, gid = bin_pairs(width, height, means2D, radius, tile, window, conic_opacity)
    tid, gid = sort_pairs(tid, gid, depth)
    return dict(tile_ids=tid, point_list=gid, ranges=ranges(tid, n_tiles(width, height, tile)),
                n_pairs=int(tid.shape[0]))


def render_fwd(width, height, ranges_, point_list, means2D, conic_opacity, rgb, depth, bg=(0, 0, 0),
               tile: int = TILE, window: Optional[Sequence[int]] = None) -> dict:
    """Eq. (4) per pixel with the skip / stop rules.  Outputs are planar:
    color [3,H,W], alpha/depth/final_T/margin [H,W], n_contrib/n_examined/
    n_blended [H,W] (n_blended: entries blended, the pixel's contributors).
    ``blends`` = examined entries, ``contributors`` = blended entries, summed
    over the pixels.  Pixels outside ``window`` = (x0, y0, x1, y1) stay zero."""
    H, W = int(height), int(width)
    rg, pl = _i32(ranges_), _i32(point_list)
    m2, co, cl, dp, b = _f64(means2D), _f64(conic_opacity), _f64(rgb), _f64(depth), _f64(bg)
    win = None if window is None else _i32(window)
    out = dict(color=np.zeros((3, H, W)), alpha=np.zeros((H, W)), depth=np.zeros((H, W)),
               final_T=np.zeros((H, W)), n_contrib=np.zeros((H, W), np.int32),
               n_examined=np.zeros((H, W), np.int64), n_blended=np.zeros((H, W), np.int32),
               margin=np.full((H, W), np.inf))
    tot = lib().orc_render_fwd(W, H, tile, _p(rg), _p(pl), _p(m2), _p(co), _p(cl), _p(dp), _p(b), _p(win),
                               _p(out["color"]), _p(out["alpha"]), _p(out["depth"]), _p(out["final_T"]),
                               _p(out["n_contrib"]), _p(out["n_examined"]), _p(out["n_blended"]),
                               _p(out["margin"]))
    out["blends"] = int(tot)
    out["contributors"] = int(out["n_blended"].sum(dtype=np.int64))
    return out


def render_bwd(width, height, ranges_, point_list, means2D, conic_opacity, rgb, depth, dL_dcolor,
               dL_dalpha=None, dL_ddepth=None, bg=(0, 0, 0), tile: int = TILE,
               window: Optional[Sequence[int]] = None) -> dict:
    """Exact derivative of :func:`render_fwd` (decisions frozen) for
    L = <dL_dcolor, color> + <dL_dalpha, alpha> + <dL_ddepth, depth>.
    ``mag`` holds, per gradient element, the sum of the absolute values of
    its per-pixel terms."""
    H, W = int(height), int(width)
    rg, pl = _i32(ranges_), _i32(point_list)
    m2, co, cl, dp, b = _f64(means2D), _f64(conic_opacity), _f64(rgb), _f64(depth), _f64(bg)
    P = int(m2.shape[0])
    gC = _f64(dL_dcolor)
    gA = None if dL_dalpha is None else _f64(dL_dalpha)
    gD = None if dL_ddepth is None else _f64(dL_ddepth)
    win = None if window is None else _i32(window)
    out = dict(means2D=np.zeros((P, 2)), conic=np.zeros((P, 3)), opacity=np.zeros(P), rgb=np.zeros((P, 3)),
               depth=np.zeros(P))
    mag = {k: np.zeros_like(v) for k, v in out.items()}
    tot = lib().orc_render_bwd(W, H, tile, _p(rg), _p(pl), _p(m2), _p(co), _p(cl), _p(dp), _p(b), _p(win),
                               _p(gC), _p(gA), _p(gD), _p(out["means2D"]), _p(out["conic"]), _p(out["opacity"]),
                               _p(out["rgb"]), _p(out["depth"]), _p(mag["means2D"]), _p(mag["conic"]),
                               _p(mag["opacity"]), _p(mag["rgb"]), _p(mag["depth"]))
    out["blends"] = int(tot)
    out["mag"] = mag
    return out
