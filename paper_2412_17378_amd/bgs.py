"""ctypes binding of libbgs.so (include/bgs.h): the same entry points, taking
torch CUDA tensors.  Argument marshalling only: every step runs in the HIP
library; this module checks shapes/dtypes, passes device pointers and the
current HIP stream, and turns a non-OK status into BgsError.

The library must be built (``python -m paper_2412_17378_amd.build``); when it
is missing, importing the binding's loader raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbgs.so")

BGS_OK, BGS_EINVAL, BGS_ECAPACITY, BGS_EHIP, BGS_EUNSUPPORTED, BGS_EINTERNAL = 0, -1, -2, -3, -4, -5
STATIC, BALANCED_PIXEL, BALANCED_GAUSS, BALANCED_HYBRID, STATIC_WAVE = 0, 1, 2, 3, 4
ORDER_RASTER, ORDER_COST = 0, 1
FLAG_QUEUE_READY = 1
FLAG_SPLIT_WALKS = 2
FLAG_PACKED_GRADS = 4
FLAG_PERSISTENT = 8
GRAD_RECORD = 16  # floats per Gaussian in packed gradients: conic+opacity 0-3, means2D 4-5, rgb 6-8, depth 9
TILE = 16

VARIANTS = {"static": STATIC, "pixel": BALANCED_PIXEL, "gauss": BALANCED_GAUSS, "hybrid": BALANCED_HYBRID,
            "static_wave": STATIC_WAVE}
ORDERS = {"raster": ORDER_RASTER, "cost": ORDER_COST}


class BgsError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("znear", C.c_float)]


class Frame(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tile", C.c_int32),
                ("ranges", C.c_void_p), ("point_list", C.c_void_p), ("means2D", C.c_void_p),
                ("conic_opacity", C.c_void_p), ("rgb", C.c_void_p), ("depth", C.c_void_p)]


class ViewIO(C.Structure):
    _fields_ = [("P", C.c_int64), ("out_color", C.c_void_p), ("out_alpha", C.c_void_p), ("out_depth", C.c_void_p),
                ("final_T", C.c_void_p), ("n_contrib", C.c_void_p), ("dL_dcolor", C.c_void_p),
                ("dL_dalpha", C.c_void_p), ("dL_ddepth", C.c_void_p), ("dL_dmeans2D", C.c_void_p),
                ("dL_dconic_opacity", C.c_void_p), ("dL_drgb", C.c_void_p), ("dL_ddepths", C.c_void_p)]


class RenderCfg(C.Structure):
    _fields_ = [("variant", C.c_int32), ("subtile", C.c_int32), ("order", C.c_int32), ("flags", C.c_int32),
                ("bg", C.c_float * 3), ("wg_trace", C.c_void_p), ("wg_trace_cap", C.c_int64),
                ("n_examined", C.c_void_p), ("list_cap", C.c_uint32), ("list_overflow", C.c_void_p),
                ("item_claims", C.c_void_p), ("split_color", C.c_void_p), ("split_depth", C.c_void_p)]


_LIB = None
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2412_17378_amd.build`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "bgs_last_error": ([], C.c_char_p),
            "bgs_version": ([], C.c_char_p),
            "bgs_project": ([_vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
                            C.c_int),
            "bgs_project_bwd": ([_vp, _i64, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp], C.c_int),
            "bgs_project_bwd_packed": ([_vp, _i64, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
                                       C.c_int),
            "bgs_bin_workspace_bytes": ([_i64], _sz),
            "bgs_bin": ([_i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp], C.c_int),
            "bgs_sort_workspace_bytes": ([_i64], _sz),
            "bgs_sort": ([_vp, _vp, _vp, _vp, _i64, _i32, _vp, _sz, _vp], C.c_int),
            "bgs_ranges": ([_vp, _i64, _i32, _vp, _vp], C.c_int),
            "bgs_tile_lists_workspace_bytes": ([_i32, _i32, _i64, _i64], _sz),
            "bgs_tile_lists": ([_i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, C.c_uint32, _vp, _vp, _vp,
                                _sz, _vp], C.c_int),
            "bgs_tile_lists_exact": ([_i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, C.c_uint32, _vp, _vp,
                                      _vp, _sz, _vp], C.c_int),
            "bgs_render_workspace_bytes": ([_vp, _vp], _sz),
            "bgs_queue_build": ([_vp, _vp, _vp, _vp, _sz, _vp], C.c_int),
            "bgs_render_fwd": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], C.c_int),
            "bgs_render_fwd_noalloc": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
            "bgs_render_fwd_noalloc_max_bytes": ([], _sz),
            "bgs_render_bwd": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], C.c_int),
            "bgs_render_bwd_det_workspace_bytes": ([_vp, _i64, _i64], _sz),
            "bgs_render_bwd_det": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _sz,
                                    _vp], C.c_int),
            "bgs_autotune": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, C.c_char_p, _vp, _vp,
                              _vp, _vp, _vp], C.c_int),
            "bgs_plan_create": ([_vp, _i32, _vp, _vp, _vp, _vp, _vp], C.c_int),
            "bgs_plan_launch": ([_vp, _vp], C.c_int),
            "bgs_plan_destroy": ([_vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def exported_symbols():
    """Names the header declares (used by the load test)."""
    return ["bgs_last_error", "bgs_version", "bgs_project", "bgs_project_bwd", "bgs_project_bwd_packed",
            "bgs_bin_workspace_bytes", "bgs_bin",
            "bgs_sort_workspace_bytes", "bgs_sort", "bgs_ranges", "bgs_tile_lists_workspace_bytes", "bgs_tile_lists",
            "bgs_tile_lists_exact", "bgs_render_workspace_bytes", "bgs_queue_build", "bgs_autotune", "bgs_plan_create", "bgs_plan_launch",
            "bgs_plan_destroy",
            "bgs_render_fwd", "bgs_render_fwd_noalloc", "bgs_render_fwd_noalloc_max_bytes", "bgs_render_bwd",
            "bgs_render_bwd_det_workspace_bytes", "bgs_render_bwd_det"]


def _check(fn: str, st: int):
    if st != BGS_OK:
        raise BgsError(fn, st, lib().bgs_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _expect(t, shape, dtype, name):
    if t is None:
        return
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        raise ValueError(f"{name}: expected {tuple(shape)} {dtype}, got {tuple(t.shape)} {t.dtype}")


def make_camera(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(x) for x in list(getattr(cam.R, "reshape")(9))]
    t = [float(x) for x in list(getattr(cam.t, "reshape")(3))]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = t[k]
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def make_cfg(variant="pixel", subtile: int = 8, order="raster", bg=(0.0, 0.0, 0.0), flags: int = 0) -> RenderCfg:
    c = RenderCfg()
    c.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    c.subtile = int(subtile)
    c.order = ORDERS[order] if isinstance(order, str) else int(order)
    c.flags = int(flags)
    for k in range(3):
        c.bg[k] = float(bg[k])
    return c


def copy_cfg(c: RenderCfg) -> RenderCfg:
    d = RenderCfg()
    C.pointer(d)[0] = c
    return d


def with_forward_outputs(c: RenderCfg, out_color, out_depth) -> RenderCfg:
    """A copy of a backward configuration that carries the forward's outputs
    (needed by split walks, FLAG_SPLIT_WALKS); other configurations are
    returned unchanged."""
    if not c.flags & FLAG_SPLIT_WALKS:
        return c
    d = copy_cfg(c)
    d.split_color, d.split_depth = _ptr(out_color), _ptr(out_depth)
    return d


def n_tiles(width: int, height: int) -> int:
    return ((width + TILE - 1) // TILE) * ((height + TILE - 1) // TILE)


def tile_lists_supported(width: int, height: int) -> bool:
    """Whether bgs_tile_lists handles this tile grid (see include/bgs.h)."""
    tx, ty = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
    gx, gy = (tx + 7) // 8, (ty + 7) // 8  # groups of 8x8 tiles
    return gx * gy <= 8192 and (gx + 1) * (gy + 1) * 4 <= 65536 and tx <= 65535 and ty <= 65535


_DUMMY = {}


def _nonempty(t: torch.Tensor) -> torch.Tensor:
    """An empty array still has to be passed as a valid, aligned device
    pointer (nothing is read through it)."""
    if t.numel() > 0:
        return t
    d = _DUMMY.get(t.device)
    if d is None:
        d = _DUMMY[t.device] = torch.zeros(64, dtype=torch.float32, device=t.device)
    return d


def make_frame(width, height, ranges, point_list, means2D, conic_opacity, rgb, depth) -> Frame:
    P = means2D.shape[0]
    _expect(ranges, (n_tiles(width, height), 2), torch.int32, "ranges")
    _expect(means2D, (P, 2), torch.float32, "means2D")
    _expect(conic_opacity, (P, 4), torch.float32, "conic_opacity")
    _expect(rgb, (P, 3), torch.float32, "rgb")
    _expect(depth, (P,), torch.float32, "depth")
    if point_list.dtype != torch.int32 or point_list.dim() != 1:
        raise ValueError("point_list must be a 1-D int32 tensor")
    f = Frame()
    f.width, f.height, f.tile = int(width), int(height), TILE
    f.ranges, f.point_list = _ptr(ranges), _ptr(_nonempty(point_list))
    f.means2D, f.conic_opacity = _ptr(_nonempty(means2D)), _ptr(_nonempty(conic_opacity))
    f.rgb, f.depth = _ptr(_nonempty(rgb)), _ptr(_nonempty(depth))
    return f


# ------------------------------------------------------------------ calls
def bgs_project(cam, means3D, log_scales, quats, opacity, colors, sh_degree: int, means2D, conic_opacity, rgb,
                depth, radius, tiles_touched, stream=None):
    P = means3D.shape[0]
    _expect(means3D, (P, 3), torch.float32, "means3D")
    _expect(log_scales, (P, 3), torch.float32, "log_scales")
    _expect(quats, (P, 4), torch.float32, "quats")
    _expect(opacity, (P,), torch.float32, "opacity")
    ncol = 3 if sh_degree < 0 else 3 * (sh_degree + 1) ** 2
    if colors.numel() != P * ncol or colors.dtype != torch.float32:
        raise ValueError("colors: wrong size or dtype")
    _expect(means2D, (P, 2), torch.float32, "means2D")
    _expect(conic_opacity, (P, 4), torch.float32, "conic_opacity")
    _expect(radius, (P,), torch.int32, "radius")
    _expect(tiles_touched, (P,), torch.int32, "tiles_touched")
    c = make_camera(cam) if not isinstance(cam, Camera) else cam
    _check("bgs_project", lib().bgs_project(C.byref(c), P, _ptr(means3D), _ptr(log_scales), _ptr(quats),
                                            _ptr(opacity), _ptr(colors), int(sh_degree), TILE, _ptr(means2D),
                                            _ptr(conic_opacity), _ptr(rgb), _ptr(depth), _ptr(radius),
                                            _ptr(tiles_touched), _stream(stream)))


def bgs_project_bwd(cam, means3D, log_scales, quats, colors, sh_degree: int, dL_dmeans2D, dL_dconic_opacity,
                    dL_drgb, dL_ddepth, out: dict, stream=None):
    """Writes out["means3D"|"log_scales"|"quats"|"opacity"|"colors"] (the
    gradients of the projection inputs)."""
    P = means3D.shape[0]
    _expect(dL_dmeans2D, (P, 2), torch.float32, "dL_dmeans2D")
    _expect(dL_dconic_opacity, (P, 4), torch.float32, "dL_dconic_opacity")
    _expect(dL_drgb, (P, 3), torch.float32, "dL_drgb")
    if dL_ddepth is not None:
        _expect(dL_ddepth, (P,), torch.float32, "dL_ddepth")
    _expect(out["quats"], (P, 4), torch.float32, "dL_dquats")
    if out["colors"].numel() != colors.numel():
        raise ValueError("dL_dcolors: wrong size")
    c = make_camera(cam) if not isinstance(cam, Camera) else cam
    _check("bgs_project_bwd", lib().bgs_project_bwd(
        C.byref(c), P, _ptr(means3D), _ptr(log_scales), _ptr(quats), _ptr(colors), int(sh_degree),
        _ptr(dL_dmeans2D), _ptr(dL_dconic_opacity), _ptr(dL_drgb), _ptr(dL_ddepth), _ptr(out["means3D"]),
        _ptr(out["log_scales"]), _ptr(out["quats"]), _ptr(out["opacity"]), _ptr(out["colors"]), _stream(stream)))


def grad_records(P: int, device) -> torch.Tensor:
    """Zeroed packed-gradient records [P][16] (64-byte aligned: torch's
    device allocations are)."""
    return torch.zeros(P, GRAD_RECORD, dtype=torch.float32, device=device)


def record_views(rec: torch.Tensor) -> dict:
    """The four screen-space gradients inside packed records (strided views)."""
    return {"means2D": rec[:, 4:6], "conic_opacity": rec[:, 0:4], "rgb": rec[:, 6:9], "depth": rec[:, 9]}


def bgs_project_bwd_packed(cam, means3D, log_scales, quats, colors, sh_degree: int, dL_drecords, out: dict,
                           stream=None):
    """bgs_project_bwd reading packed gradient records [P][16]."""
    P = means3D.shape[0]
    _expect(dL_drecords, (P, GRAD_RECORD), torch.float32, "dL_drecords")
    _expect(out["quats"], (P, 4), torch.float32, "dL_dquats")
    if out["colors"].numel() != colors.numel():
        raise ValueError("dL_dcolors: wrong size")
    c = make_camera(cam) if not isinstance(cam, Camera) else cam
    _check("bgs_project_bwd_packed", lib().bgs_project_bwd_packed(
        C.byref(c), P, _ptr(means3D), _ptr(log_scales), _ptr(quats), _ptr(colors), int(sh_degree),
        _ptr(dL_drecords), _ptr(out["means3D"]), _ptr(out["log_scales"]), _ptr(out["quats"]), _ptr(out["opacity"]),
        _ptr(out["colors"]), _stream(stream)))


def bgs_bin_workspace_bytes(P: int) -> int:
    return int(lib().bgs_bin_workspace_bytes(int(P)))


def bgs_bin(width, height, means2D, radius, depth, tiles_touched, keys, values, ws, stream=None) -> int:
    """Returns the pair count M.  Synchronizes the stream.  Raises BgsError
    with status BGS_ECAPACITY (and .n_pairs) when keys/values are too small."""
    P = means2D.shape[0]
    n = C.c_int64(0)
    cap = 0 if keys is None else keys.numel()
    st = lib().bgs_bin(int(width), int(height), TILE, P, _ptr(means2D), _ptr(radius), _ptr(depth),
                       _ptr(tiles_touched), _ptr(keys) if cap else None, _ptr(values) if cap else None, cap,
                       C.byref(n), _ptr(ws), ws.numel(), _stream(stream))
    if st == BGS_ECAPACITY:
        e = BgsError("bgs_bin", st, lib().bgs_last_error().decode())
        e.n_pairs = int(n.value)
        raise e
    _check("bgs_bin", st)
    return int(n.value)


def bgs_sort_workspace_bytes(n: int) -> int:
    return int(lib().bgs_sort_workspace_bytes(int(n)))


def bgs_sort(keys_in, values_in, keys_out, values_out, n: int, key_bits: int, ws, stream=None):
    _check("bgs_sort", lib().bgs_sort(_ptr(keys_in), _ptr(values_in), _ptr(keys_out), _ptr(values_out), int(n),
                                      int(key_bits), _ptr(ws), ws.numel(), _stream(stream)))


def bgs_ranges(sorted_keys, n: int, n_tiles_: int, ranges, stream=None):
    _check("bgs_ranges", lib().bgs_ranges(_ptr(sorted_keys) if n > 0 else None, int(n), int(n_tiles_),
                                          _ptr(ranges), _stream(stream)))


def bgs_tile_lists_workspace_bytes(width: int, height: int, P: int, capacity: int) -> int:
    return int(lib().bgs_tile_lists_workspace_bytes(int(width), int(height), int(P), int(capacity)))


def bgs_tile_lists(width, height, means2D, radius, depth, tiles_touched, point_list, ranges, n_pairs_dev, ws,
                   stream=None, conic_opacity=None, max_per_tile: int = 0) -> bool:
    """Asynchronous: n_pairs_dev (int64 [>=1] device tensor) receives M, or a
    lower bound of M above the capacity (point_list.numel()) on overflow, in
    which case every range is empty; the caller compares n_pairs_dev with the
    capacity when convenient and grows.  Returns False on BGS_ECAPACITY.
    With conic_opacity ([P,4] float32) the lists use exact ellipse-tile
    binning (bgs_tile_lists_exact).  max_per_tile > 0 keeps the first
    max_per_tile entries of each tile's list (see include/bgs.h)."""
    cap = 0 if point_list is None else point_list.numel()
    _expect(ranges, (n_tiles(width, height), 2), torch.int32, "ranges")
    P = means2D.shape[0]
    K = int(max_per_tile)
    if not 0 <= K < 1 << 32:
        raise ValueError("max_per_tile must be in [0, 2^32)")
    if conic_opacity is None:
        st = lib().bgs_tile_lists(int(width), int(height), TILE, P, _ptr(means2D), _ptr(radius), _ptr(depth),
                                  _ptr(tiles_touched), _ptr(point_list) if cap else None, cap, K, _ptr(ranges),
                                  _ptr(n_pairs_dev), _ptr(ws), ws.numel(), _stream(stream))
    else:
        _expect(conic_opacity, (P, 4), torch.float32, "conic_opacity")
        st = lib().bgs_tile_lists_exact(int(width), int(height), TILE, P, _ptr(means2D), _ptr(conic_opacity),
                                        _ptr(radius), _ptr(depth), _ptr(tiles_touched),
                                        _ptr(point_list) if cap else None, cap, K, _ptr(ranges), _ptr(n_pairs_dev),
                                        _ptr(ws), ws.numel(), _stream(stream))
    if st == BGS_ECAPACITY:
        return False
    _check("bgs_tile_lists", st)
    return True


def bgs_render_workspace_bytes(frame: Frame, cfg: RenderCfg) -> int:
    return int(lib().bgs_render_workspace_bytes(C.byref(frame), C.byref(cfg)))


def bgs_queue_build(frame: Frame, cfg: RenderCfg, n_contrib, ws, stream=None):
    _check("bgs_queue_build", lib().bgs_queue_build(C.byref(frame), C.byref(cfg), _ptr(n_contrib), _ptr(ws),
                                                    ws.numel(), _stream(stream)))


def bgs_render_fwd(frame: Frame, cfg: RenderCfg, out_color, out_alpha, out_depth, final_T, n_contrib, ws,
                   stream=None):
    H, W = frame.height, frame.width
    _expect(out_color, (3, H, W), torch.float32, "out_color")
    for t, nm in ((out_alpha, "out_alpha"), (out_depth, "out_depth"), (final_T, "final_T")):
        _expect(t, (H, W), torch.float32, nm)
    _expect(n_contrib, (H, W), torch.int32, "n_contrib")
    _check("bgs_render_fwd", lib().bgs_render_fwd(C.byref(frame), C.byref(cfg), _ptr(out_color), _ptr(out_alpha),
                                                  _ptr(out_depth), _ptr(final_T), _ptr(n_contrib), _ptr(ws),
                                                  ws.numel(), _stream(stream)))


def bgs_render_fwd_noalloc(frame: Frame, cfg: RenderCfg, out_color, out_alpha, out_depth, final_T, n_contrib,
                           stream=None):
    """bgs_render_fwd with the queue in the library's own device array (no
    workspace, nothing allocated)."""
    H, W = frame.height, frame.width
    _expect(out_color, (3, H, W), torch.float32, "out_color")
    for t, nm in ((out_alpha, "out_alpha"), (out_depth, "out_depth"), (final_T, "final_T")):
        _expect(t, (H, W), torch.float32, nm)
    _expect(n_contrib, (H, W), torch.int32, "n_contrib")
    _check("bgs_render_fwd_noalloc",
           lib().bgs_render_fwd_noalloc(C.byref(frame), C.byref(cfg), _ptr(out_color), _ptr(out_alpha),
                                        _ptr(out_depth), _ptr(final_T), _ptr(n_contrib), _stream(stream)))


def bgs_render_fwd_noalloc_max_bytes() -> int:
    return int(lib().bgs_render_fwd_noalloc_max_bytes())


def bgs_autotune(frame: Frame, base: RenderCfg, out: dict, dL_dcolor, grads: Optional[dict], ws,
                 cache_path: Optional[str] = None, stream=None):
    """Returns (best_fwd, best_bwd, fwd_ms, bwd_ms); out / grads are scratch.
    With FLAG_PACKED_GRADS in base, grads is {"records": [P][16] records}."""
    bf, bb = RenderCfg(), RenderCfg()
    fms, bms = C.c_float(0), C.c_float(0)
    g = grads or {}
    if "records" in g:
        g = {"means2D": g["records"]}
    _check("bgs_autotune", lib().bgs_autotune(
        C.byref(frame), C.byref(base), _ptr(out["color"]), _ptr(out["alpha"]), _ptr(out["depth"]),
        _ptr(out["final_T"]), _ptr(out["n_contrib"]), _ptr(dL_dcolor) if grads is not None else None,
        _ptr(g.get("means2D")), _ptr(g.get("conic_opacity")), _ptr(g.get("rgb")), _ptr(ws), ws.numel(),
        None if cache_path is None else cache_path.encode(), C.byref(bf), C.byref(bb), C.byref(fms), C.byref(bms),
        _stream(stream)))
    return bf, bb, float(fms.value), float(bms.value)


def make_view_io(P, out: dict, dL_dcolor, grads: dict, dL_dalpha=None, dL_ddepth=None) -> ViewIO:
    v = ViewIO()
    v.P = int(P)
    v.out_color, v.out_alpha, v.out_depth = _ptr(out["color"]), _ptr(out["alpha"]), _ptr(out["depth"])
    v.final_T, v.n_contrib = _ptr(out["final_T"]), _ptr(out["n_contrib"])
    v.dL_dcolor, v.dL_dalpha, v.dL_ddepth = _ptr(dL_dcolor), _ptr(dL_dalpha), _ptr(dL_ddepth)
    v.dL_dmeans2D = _ptr(_nonempty(grads["means2D"]))
    v.dL_dconic_opacity = _ptr(_nonempty(grads["conic_opacity"]))
    v.dL_drgb = _ptr(_nonempty(grads["rgb"]))
    v.dL_ddepths = None if grads.get("depth") is None else _ptr(_nonempty(grads["depth"]))
    return v


def bgs_plan_create(frames, ios, cfg: RenderCfg, cfg_bwd: RenderCfg = None, stream=None) -> C.c_void_p:
    n = len(frames)
    fa = (Frame * n)(*frames)
    ia = (ViewIO * n)(*ios)
    h = C.c_void_p()
    _check("bgs_plan_create", lib().bgs_plan_create(C.byref(h), n, fa, ia, C.byref(cfg),
                                                    None if cfg_bwd is None else C.byref(cfg_bwd), _stream(stream)))
    return h


def bgs_plan_launch(plan, stream=None):
    _check("bgs_plan_launch", lib().bgs_plan_launch(plan, _stream(stream)))


def bgs_plan_destroy(plan):
    lib().bgs_plan_destroy(plan)


def cfg_name(c: RenderCfg) -> str:
    names = {v: k for k, v in VARIANTS.items()}
    base = f"{names.get(c.variant, c.variant)}{c.subtile}/{'cost' if c.order == ORDER_COST else 'raster'}"
    return base + ("/split" if c.flags & FLAG_SPLIT_WALKS else "") + ("/persistent" if c.flags & FLAG_PERSISTENT
                                                                      else "")


def bgs_render_bwd_det_workspace_bytes(frame: Frame, P: int, max_occ: int) -> int:
    return int(lib().bgs_render_bwd_det_workspace_bytes(C.byref(frame), int(P), int(max_occ)))


def bgs_render_bwd_det(frame: Frame, cfg: RenderCfg, P: int, final_T, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth,
                       dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepths, max_occ: int, ws, stream=None) -> int:
    """Deterministic-order backward (see include/bgs.h); returns the number of
    walked (tile, entry) pairs.  Raises BgsError (status BGS_ECAPACITY, with
    .n_occ set) when they exceed max_occ."""
    H, W = frame.height, frame.width
    _expect(final_T, (H, W), torch.float32, "final_T")
    _expect(n_contrib, (H, W), torch.int32, "n_contrib")
    _expect(dL_dcolor, (3, H, W), torch.float32, "dL_dcolor")
    _expect(dL_dalpha, (H, W), torch.float32, "dL_dalpha")
    _expect(dL_ddepth, (H, W), torch.float32, "dL_ddepth")
    n = C.c_int64(0)
    st = lib().bgs_render_bwd_det(C.byref(frame), C.byref(cfg), int(P), _ptr(final_T), _ptr(n_contrib),
                                  _ptr(dL_dcolor), _ptr(dL_dalpha), _ptr(dL_ddepth),
                                  *[None if t is None else _ptr(_nonempty(t))
                                    for t in (dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepths)], int(max_occ),
                                  C.byref(n), _ptr(ws), ws.numel(), _stream(stream))
    if st != BGS_OK:
        e = BgsError("bgs_render_bwd_det", st, lib().bgs_last_error().decode(errors="replace"))
        e.n_occ = n.value
        raise e
    return n.value


def bgs_render_bwd(frame: Frame, cfg: RenderCfg, final_T, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dmeans2D,
                   dL_dconic_opacity, dL_drgb, dL_ddepths, ws, stream=None):
    H, W = frame.height, frame.width
    _expect(final_T, (H, W), torch.float32, "final_T")
    _expect(n_contrib, (H, W), torch.int32, "n_contrib")
    _expect(dL_dcolor, (3, H, W), torch.float32, "dL_dcolor")
    _expect(dL_dalpha, (H, W), torch.float32, "dL_dalpha")
    _expect(dL_ddepth, (H, W), torch.float32, "dL_ddepth")
    opt = lambda t: None if t is None else _ptr(_nonempty(t))  # noqa: E731 (packed: the last three are None)
    _check("bgs_render_bwd", lib().bgs_render_bwd(C.byref(frame), C.byref(cfg), _ptr(final_T), _ptr(n_contrib),
                                                  _ptr(dL_dcolor), _ptr(dL_dalpha), _ptr(dL_ddepth),
                                                  opt(dL_dmeans2D), opt(dL_dconic_opacity), opt(dL_drgb),
                                                  opt(dL_ddepths), _ptr(ws), ws.numel(), _stream(stream)))
