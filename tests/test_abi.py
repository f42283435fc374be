"""CPU checks of the boundary: libbgs.so loads and exports every entry point
include/bgs.h declares; invalid arguments come back as status codes (no GPU
work is launched by these calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bgs_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_2412_17378_amd import bgs
    if not os.path.exists(bgs.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return bgs.lib()


def test_header_declares_the_pipeline():
    names = _declared()
    for n in ("bgs_project", "bgs_bin", "bgs_sort", "bgs_ranges", "bgs_queue_build", "bgs_render_fwd",
              "bgs_render_bwd"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_invalid_arguments_are_status_codes():
    from paper_2412_17378_amd import bgs as B
    L = _lib()
    cam = B.Camera()
    cam.width, cam.height = 0, 10
    st = L.bgs_project(ctypes.byref(cam), 1, None, None, None, None, None, -1, 16, None, None, None, None, None,
                       None, None)
    assert st == B.BGS_EINVAL
    assert b"image size" in L.bgs_last_error()
    cam.width = 10
    st = L.bgs_project(ctypes.byref(cam), 1, None, None, None, None, None, -1, 8, None, None, None, None, None,
                       None, None)
    assert st == B.BGS_EUNSUPPORTED
    st = L.bgs_render_fwd(None, None, None, None, None, None, None, None, 0, None)
    assert st == B.BGS_EINVAL
    f = B.Frame()
    f.width, f.height, f.tile = 32, 32, 16
    cfg = B.make_cfg("pixel", 8)
    st = L.bgs_render_fwd(ctypes.byref(f), ctypes.byref(cfg), None, None, None, None, None, None, 0, None)
    assert st == B.BGS_EINVAL  # null frame arrays
    st = L.bgs_sort(None, None, None, None, 10, 0, None, 0, None)
    assert st == B.BGS_EINVAL
    assert L.bgs_render_workspace_bytes(ctypes.byref(f), ctypes.byref(cfg)) > 0
    # the work counter is only written by the wave-per-tile forward
    cfg.n_examined = 1
    st = L.bgs_render_fwd(ctypes.byref(f), ctypes.byref(cfg), None, None, None, None, None, None, 0, None)
    assert st == B.BGS_EINVAL  # (null frame arrays are checked first)
    # split walks: need the forward's colour and depth, and the wave-per-tile cost-ordered backward
    buf = (ctypes.c_float * 64)()
    f2 = B.Frame()
    f2.width, f2.height, f2.tile = 32, 32, 16
    f2.ranges = f2.point_list = f2.means2D = f2.rgb = f2.depth = ctypes.addressof(buf)
    f2.conic_opacity = (ctypes.addressof(buf) + 15) // 16 * 16
    f2.means2D = (ctypes.addressof(buf) + 7) // 8 * 8
    p = ctypes.addressof(buf)
    sc = B.make_cfg("pixel", 16, "cost", flags=B.FLAG_SPLIT_WALKS)
    st = L.bgs_render_bwd(ctypes.byref(f2), ctypes.byref(sc), p, p, p, None, None, p, p, p, None, p, 1 << 16, None)
    assert st == B.BGS_EINVAL and b"split" in L.bgs_last_error()
    sc = B.make_cfg("pixel", 8, "cost", flags=B.FLAG_SPLIT_WALKS)
    st = L.bgs_render_bwd(ctypes.byref(f2), ctypes.byref(sc), p, p, p, None, None, p, p, p, None, p, 1 << 16, None)
    assert st == B.BGS_EUNSUPPORTED
    # packed gradient records: one 64-byte aligned array in dL_dmeans2D, the other three null
    pc = B.make_cfg("static", flags=B.FLAG_PACKED_GRADS)
    a64 = (ctypes.addressof(buf) + 63) // 64 * 64
    st = L.bgs_render_bwd(ctypes.byref(f2), ctypes.byref(pc), p, p, p, None, None, a64, p, p, None, p, 1 << 16, None)
    assert st == B.BGS_EINVAL and b"packed" in L.bgs_last_error()
    st = L.bgs_render_bwd(ctypes.byref(f2), ctypes.byref(pc), p, p, p, None, None, a64 + 4, None, None, None, p,
                          1 << 16, None)
    assert st == B.BGS_EINVAL and b"64-byte" in L.bgs_last_error()
    st = L.bgs_render_bwd_det(ctypes.byref(f2), ctypes.byref(B.make_cfg("pixel", 16, "cost",
                                                                        flags=B.FLAG_PACKED_GRADS)),
                              1, p, p, p, None, None, a64, p, None, None, 0, ctypes.byref(ctypes.c_int64()), p,
                              1 << 16, None)
    assert st == B.BGS_EINVAL and b"packed" in L.bgs_last_error()
    cam.width = cam.height = 8
    st = L.bgs_project_bwd_packed(ctypes.byref(cam), 1, p, p, p, p, -1, None, p, p, a64, p, p, None)
    assert st == B.BGS_EINVAL and b"null" in L.bgs_last_error()
    st = L.bgs_project_bwd_packed(ctypes.byref(cam), 1, p, p, p, p, -1, a64 + 16, p, p, a64, p, p, None)
    assert st == B.BGS_EINVAL and b"64-byte" in L.bgs_last_error()
    # exact binning keeps a Gaussian's tile rows in one LDS buffer: at most 1024 tile rows
    a16 = (ctypes.addressof(buf) + 15) // 16 * 16
    st = L.bgs_tile_lists_exact(16, 16 * 1025, 16, 1, p, a16, p, p, p, p, 1, 0, p, p, p, 1 << 16, None)
    assert st == B.BGS_EUNSUPPORTED and b"16384" in L.bgs_last_error()
    st = L.bgs_autotune(None, None, None, None, None, None, None, None, None, None, None, None, 0, None, None, None,
                        None, None, None)
    assert st == B.BGS_EINVAL
    plan = ctypes.c_void_p()
    st = L.bgs_plan_create(ctypes.byref(plan), 0, None, None, None, None, None)
    assert st == B.BGS_EINVAL
    L.bgs_plan_destroy(None)  # accepted


def test_version():
    assert _lib().bgs_version().startswith(b"bgs")
