"""The rasterizer pipeline over the C ABI: project -> bin -> sort -> ranges ->
render_fwd / render_bwd, plus the differentiable render as a
torch.autograd.Function.

torch provides device memory (outputs, workspaces) and the stream; every
step of the path runs in libbgs.so.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import bgs as B


@dataclasses.dataclass
class Prepared:
    """Screen-space splats and per-tile sorted lists of one view."""
    width: int
    height: int
    means2D: torch.Tensor        # [P,2] f32
    conic_opacity: torch.Tensor  # [P,4] f32
    rgb: torch.Tensor            # [P,3] f32
    depth: torch.Tensor          # [P] f32
    radius: torch.Tensor         # [P] i32
    tiles_touched: torch.Tensor  # [P] i32
    n_pairs: int
    tile_keys: Optional[torch.Tensor]  # [n_pairs] i32 sorted tile ids (sort method only)
    point_list: torch.Tensor     # [n_pairs] i32
    ranges: torch.Tensor         # [n_tiles,2] i32

    @property
    def P(self) -> int:
        return int(self.means2D.shape[0])

    def frame(self) -> B.Frame:
        return B.make_frame(self.width, self.height, self.ranges, self.point_list, self.means2D,
                            self.conic_opacity, self.rgb, self.depth)


class Workspace:
    """Grow-only device byte buffers, one per role."""

    def __init__(self, device):
        self.device = device
        self._bufs = {}

    def get(self, role: str, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        b = self._bufs.get(role)
        if b is None or b.numel() < nbytes:
            b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._bufs[role] = b
        return b


def key_bits_for(n_tiles: int) -> int:
    return max(1, int(n_tiles - 1).bit_length())


def poison_fwd(out: dict) -> None:
    """Fill forward outputs with values no render writes (NaN, and -1 for
    n_contrib), so that a pixel a kernel never wrote stays visible."""
    for k, t in out.items():
        t.fill_(-1 if k == "n_contrib" else float("nan"))


class Rasterizer:
    def __init__(self, device: str = "cuda", reuse_pairs: bool = False, lists_method: str = "fused",
                 binning: str = "square", poison_outputs: bool = False):
        """reuse_pairs: the sorted lists of a prepared frame live in buffers
        that the next prepare() overwrites (no per-frame allocation); off by
        default so that several prepared frames can coexist.  binning:
        "square" (the 3-sigma square tile rule) or "ellipse" (exact
        ellipse-tile binning: shorter lists, the same renders; fused lists
        only).  poison_outputs: a debugging aid that fills the forward outputs
        with NaN (n_contrib with -1) before every render, so a work item the
        kernel drops cannot pass on values a buffer held before."""
        if binning not in ("square", "ellipse"):
            raise ValueError(f"unknown binning {binning!r}")
        B.lib()
        self.device = torch.device(device)
        self.ws = Workspace(self.device)
        self.pair_capacity = 0
        self.reuse_pairs = reuse_pairs
        self.lists_method = lists_method
        self.binning = binning
        self.poison_outputs = poison_outputs

    def _t(self, a, dtype=torch.float32):
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(a, dtype=dtype).to(self.device).contiguous()

    def project(self, cam, means3D, log_scales, quats, opacity, colors, sh_degree: int) -> dict:
        means3D, log_scales, quats = self._t(means3D), self._t(log_scales), self._t(quats)
        opacity, colors = self._t(opacity), self._t(colors)
        P = means3D.shape[0]
        dev = self.device
        out = dict(means2D=torch.empty(P, 2, device=dev), conic_opacity=torch.empty(P, 4, device=dev),
                   rgb=torch.empty(P, 3, device=dev), depth=torch.empty(P, device=dev),
                   radius=torch.empty(P, dtype=torch.int32, device=dev),
                   tiles_touched=torch.empty(P, dtype=torch.int32, device=dev))
        B.bgs_project(cam, means3D, log_scales, quats, opacity, colors, sh_degree, out["means2D"],
                      out["conic_opacity"], out["rgb"], out["depth"], out["radius"], out["tiles_touched"])
        return out

    def project_bwd(self, cam, means3D, log_scales, quats, colors, sh_degree: int, dL_dmeans2D, dL_dconic_opacity,
                    dL_drgb, dL_ddepth=None) -> dict:
        """Gradients of the projection inputs (bgs_project_bwd)."""
        means3D, log_scales, quats, colors = self._t(means3D), self._t(log_scales), self._t(quats), self._t(colors)
        P = means3D.shape[0]
        dev = self.device
        out = dict(means3D=torch.empty(P, 3, device=dev), log_scales=torch.empty(P, 3, device=dev),
                   quats=torch.empty(P, 4, device=dev), opacity=torch.empty(P, device=dev),
                   colors=torch.empty_like(colors))
        B.bgs_project_bwd(cam, means3D, log_scales, quats, colors, sh_degree, dL_dmeans2D.contiguous(),
                          dL_dconic_opacity.contiguous(), dL_drgb.contiguous(),
                          None if dL_ddepth is None else dL_ddepth.contiguous(), out)
        return out

    def bin_sort_ranges(self, width: int, height: int, pr: dict, method: Optional[str] = None) -> Prepared:
        """Per-tile depth-ordered lists.  method "fused" = bgs_tile_lists (one
        counting pass), "sort" = bgs_bin + bgs_sort + bgs_ranges; default: fused
        when the tile grid allows it."""
        P = pr["means2D"].shape[0]
        dev = self.device
        nt = B.n_tiles(width, height)
        method = method or self.lists_method
        if method == "fused" and not B.tile_lists_supported(width, height):
            method = "sort"
        if self.binning == "ellipse" and method != "fused":
            raise ValueError("ellipse binning needs the fused list builder (bgs_tile_lists_exact)")
        ranges = torch.empty(nt, 2, dtype=torch.int32, device=dev)

        def pair_bufs(cap):
            return [self.ws.get(r, 4 * cap).view(torch.int32)[:cap] for r in ("keys", "vals", "skeys", "svals")]

        if method == "fused":
            n_dev = self.ws.get("n_pairs", 8).view(torch.int64)[:1]
            while True:
                cap = self.pair_capacity
                ws = self.ws.get("lists", B.bgs_tile_lists_workspace_bytes(width, height, P, cap))
                pl = self.ws.get("svals", 4 * cap).view(torch.int32)[:cap]
                B.bgs_tile_lists(width, height, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"],
                                 pl if cap else None, ranges, n_dev, ws,
                                 conic_opacity=pr["conic_opacity"] if self.binning == "ellipse" else None)
                M = int(n_dev.item())
                if M <= cap:
                    break
                # grow with headroom and build again
                self.pair_capacity = int(M * 1.25) + 1024
            skeys, svals = None, pl
        else:
            ws = self.ws.get("bin", B.bgs_bin_workspace_bytes(P))
            cap = self.pair_capacity
            keys, vals, skeys, svals = pair_bufs(cap)
            try:
                M = B.bgs_bin(width, height, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"],
                              keys if cap else None, vals if cap else None, ws)
            except B.BgsError as e:
                if e.status != B.BGS_ECAPACITY:
                    raise
                # grow with headroom and emit again
                self.pair_capacity = cap = int(e.n_pairs * 1.25) + 1024
                keys, vals, skeys, svals = pair_bufs(cap)
                M = B.bgs_bin(width, height, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"], keys,
                              vals, ws)
            if M > 0:
                sws = self.ws.get("sort", B.bgs_sort_workspace_bytes(M))
                B.bgs_sort(keys, vals, skeys, svals, M, key_bits_for(nt), sws)
            B.bgs_ranges(skeys, M, nt, ranges)
        if not self.reuse_pairs:
            svals = svals[:M].clone()
            skeys = None if skeys is None else skeys[:M].clone()
        return Prepared(width=width, height=height, means2D=pr["means2D"], conic_opacity=pr["conic_opacity"],
                        rgb=pr["rgb"], depth=pr["depth"], radius=pr["radius"], tiles_touched=pr["tiles_touched"],
                        n_pairs=M, tile_keys=None if skeys is None else skeys[:M], point_list=svals[:M],
                        ranges=ranges)

    def prepare(self, cam, means3D, log_scales, quats, opacity, colors, sh_degree: int,
                method: Optional[str] = None) -> Prepared:
        pr = self.project(cam, means3D, log_scales, quats, opacity, colors, sh_degree)
        return self.bin_sort_ranges(int(cam.width), int(cam.height), pr, method)

    def prepare_scene(self, scene, view: int = 0, method: Optional[str] = None) -> Prepared:
        return self.prepare(scene.cameras[view], scene.means3D, scene.log_scales, scene.quats, scene.opacity,
                            scene.colors, scene.sh_degree, method)

    def render_fwd(self, prep: Prepared, cfg: B.RenderCfg, out: Optional[dict] = None) -> dict:
        H, W = prep.height, prep.width
        dev = self.device
        if out is None:
            out = dict(color=torch.empty(3, H, W, device=dev), alpha=torch.empty(H, W, device=dev),
                       depth=torch.empty(H, W, device=dev), final_T=torch.empty(H, W, device=dev),
                       n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
        if self.poison_outputs:
            poison_fwd(out)
        f = prep.frame()
        ws = self.ws.get("render", B.bgs_render_workspace_bytes(f, cfg))
        B.bgs_render_fwd(f, cfg, out["color"], out["alpha"], out["depth"], out["final_T"], out["n_contrib"], ws)
        return out

    def count_examined(self, prep: Prepared, bg=(0.0, 0.0, 0.0)) -> torch.Tensor:
        """Per-pixel number of list entries the sequential forward loop
        examines (the forward's algorithmic work), int32 [H, W], from one
        forward with the wave-per-tile kernel."""
        H, W = prep.height, prep.width
        n = torch.empty(H, W, dtype=torch.int32, device=self.device)
        cfg = B.make_cfg("pixel", 16, "cost", bg)
        cfg.n_examined = n.data_ptr()
        self.render_fwd(prep, cfg)
        return n

    def render_bwd(self, prep: Prepared, cfg: B.RenderCfg, fwd: dict, dL_dcolor, dL_dalpha=None, dL_ddepth=None,
                   grads: Optional[dict] = None, want_depth: bool = True) -> dict:
        """Gradients of the 2D splats (added into `grads` when given).  With
        FLAG_PACKED_GRADS in cfg they go into one [P][16] record array
        (grads["records"]), and the returned dict also holds its views."""
        P = prep.P
        dev = self.device
        packed = bool(cfg.flags & B.FLAG_PACKED_GRADS)
        if grads is None:
            if packed:
                rec = B.grad_records(P, dev)
                grads = dict(B.record_views(rec), records=rec)
            else:
                grads = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
                             rgb=torch.zeros(P, 3, device=dev),
                             depth=torch.zeros(P, device=dev) if want_depth else None)
        f = prep.frame()
        ws = self.ws.get("render", B.bgs_render_workspace_bytes(f, cfg))
        if cfg.flags & B.FLAG_SPLIT_WALKS:  # split walks read the forward's colour and depth
            cfg = B.with_forward_outputs(cfg, fwd["color"], fwd["depth"])
        outs = ((grads["records"], None, None, None) if packed else
                (grads["means2D"], grads["conic_opacity"], grads["rgb"], grads["depth"]))
        B.bgs_render_bwd(f, cfg, fwd["final_T"], fwd["n_contrib"], dL_dcolor, dL_dalpha, dL_ddepth, *outs, ws)
        return grads

    def render_bwd_det(self, prep: Prepared, cfg: B.RenderCfg, fwd: dict, dL_dcolor, dL_dalpha=None, dL_ddepth=None,
                       grads: Optional[dict] = None) -> dict:
        """Deterministic-order backward (bgs_render_bwd_det; cfg must be the
        pixel-wise variant with subtile 16): the same gradients up to fp32
        rounding, identical from run to run.  The slot capacity grows on
        demand (one retry)."""
        P = prep.P
        dev = self.device
        packed = bool(cfg.flags & B.FLAG_PACKED_GRADS)
        if grads is None:
            if packed:
                rec = B.grad_records(P, dev)
                grads = dict(B.record_views(rec), records=rec)
            else:
                grads = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
                             rgb=torch.zeros(P, 3, device=dev), depth=torch.zeros(P, device=dev))
        outs = ((grads["records"], None, None, None) if packed else
                (grads["means2D"], grads["conic_opacity"], grads["rgb"], grads["depth"]))
        f = prep.frame()
        cap = getattr(self, "det_capacity", 1 << 20)
        for _ in range(2):
            ws = self.ws.get("render_det", B.bgs_render_bwd_det_workspace_bytes(f, P, cap))
            try:
                B.bgs_render_bwd_det(f, cfg, P, fwd["final_T"], fwd["n_contrib"], dL_dcolor, dL_dalpha, dL_ddepth,
                                     *outs, cap, ws)
                self.det_capacity = cap
                return grads
            except B.BgsError as e:
                if e.status != B.BGS_ECAPACITY:
                    raise
                cap = int(e.n_occ * 1.25) + 1024  # nothing was written: grow and run again
        raise RuntimeError("bgs_render_bwd_det: capacity did not converge")


    def autotune(self, prep: Prepared, base: B.RenderCfg, dL_dcolor=None, cache_path: Optional[str] = None):
        """Time the kernel variants on this frame (bgs_autotune) and return
        (best_fwd_cfg, best_bwd_cfg, fwd_ms, bwd_ms)."""
        H, W, P, dev = prep.height, prep.width, prep.P, self.device
        out = dict(color=torch.empty(3, H, W, device=dev), alpha=torch.empty(H, W, device=dev),
                   depth=torch.empty(H, W, device=dev), final_T=torch.empty(H, W, device=dev),
                   n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
        grads = None
        if dL_dcolor is not None:
            grads = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
                         rgb=torch.zeros(P, 3, device=dev))
        f = prep.frame()
        ws = self.ws.get("render", B.bgs_render_workspace_bytes(f, base))
        return B.bgs_autotune(f, base, out, dL_dcolor, grads, ws, cache_path)


class BatchedPlan:
    """Forward + backward over several prepared views in one hipGraph launch
    (bgs_plan_*): one cross-view work queue, one persistent launch each way.
    Owns the per-view outputs (`outs[v]`) and gradients (`grads[v]`), which
    every launch overwrites."""

    def __init__(self, rast: Rasterizer, preps, upstream, cfg: B.RenderCfg, cfg_bwd: B.RenderCfg = None):
        self.preps = list(preps)
        self.upstream = [u.contiguous() for u in upstream]
        dev = rast.device
        self.outs, self.grads, frames, ios = [], [], [], []
        for prep, g in zip(self.preps, self.upstream):
            H, W, P = prep.height, prep.width, prep.P
            out = dict(color=torch.empty(3, H, W, device=dev), alpha=torch.empty(H, W, device=dev),
                       depth=torch.empty(H, W, device=dev), final_T=torch.empty(H, W, device=dev),
                       n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
            grads = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
                         rgb=torch.zeros(P, 3, device=dev), depth=torch.zeros(P, device=dev))
            self.outs.append(out)
            self.grads.append(grads)
            frames.append(prep.frame())
            ios.append(B.make_view_io(P, out, g, grads))
        self.handle = B.bgs_plan_create(frames, ios, cfg, cfg_bwd)

    def launch(self):
        B.bgs_plan_launch(self.handle)

    def poison(self):
        """Fill every view's forward outputs with NaN (n_contrib with -1), so
        a pixel the next launch does not write stays visible."""
        for out in self.outs:
            poison_fwd(out)

    def close(self):
        if self.handle is not None:
            B.bgs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameStep:
    """One training-shaped step on one view with every buffer allocated up
    front and no host synchronization: project -> tile lists (bgs_tile_lists,
    or bgs_tile_lists_exact with binning="ellipse") -> queue -> render_fwd ->
    gradients zeroed -> queue -> render_bwd, on the current stream.  The pair
    capacity is sized once by a synchronous build (headroom for later steps);
    should a later step need more, its lists come out empty and n_pairs()
    (a host read) exceeds capacity.  Because nothing in the step waits for
    the GPU or allocates, capture() can record it once as a hipGraph that
    replays the whole step with a single launch.

    params: means3D [P,3], log_scales [P,3], quats [P,4], opacity [P],
    colors [P,3] or [P,K,3] (device tensors, read each step, so they may be
    updated in place between steps).  Outputs: self.pr (projection),
    self.fwd (images), self.grads (gradients of the 2D splats).

    poison_outputs: fill the forward outputs with NaN (n_contrib -1) at the
    start of every step, also inside a captured graph (a debugging aid).

    packed_grads: the backward accumulates into one [P][16] array of gradient
    records (FLAG_PACKED_GRADS; self.grad_records), one cache line per
    Gaussian for the ten atomic adds of a list entry, and self.grads holds
    strided views of it; False: four separate arrays.

    list_cap: None builds whole tile lists.  An int K keeps the first K
    entries of each tile's list (bgs_tile_lists max_per_tile); "auto" picks K
    from one uncapped step (twice the deepest contributor, rounded up) and
    doubles it until a capped step runs without overflow.  With a cap, a
    step's outputs equal the uncapped step's unless overflowed() (a host
    read) reports that a pixel ran off a capped list; the caller then
    rebuilds with set_list_cap (larger K, or None) and runs the step again.
    The report covers every step since the cap was set or clear_overflow()
    was called (the flag is not cleared per step), so checking every few
    steps misses none."""

    def __init__(self, cam, params: dict, sh_degree: int, dL_dcolor, fcfg: B.RenderCfg, bcfg: B.RenderCfg,
                 binning: str = "square", headroom: float = 1.25, list_cap=None, poison_outputs: bool = False,
                 packed_grads: bool = True):
        if binning not in ("square", "ellipse"):
            raise ValueError(f"unknown binning {binning!r}")
        W, H = int(cam.width), int(cam.height)
        if not B.tile_lists_supported(W, H):
            raise ValueError("FrameStep needs the fused list builder (tile grid too large)")
        self.cam, self.params, self.sh_degree = cam, params, int(sh_degree)
        self.W, self.H, self.binning = W, H, binning
        self.poison_outputs = poison_outputs
        self.dL_dcolor = dL_dcolor.contiguous()
        dev = self.dL_dcolor.device
        P = params["means3D"].shape[0]
        self.P = P
        self.fcfg, self.bcfg = fcfg, bcfg
        self.fcfg_ready = B.make_cfg(fcfg.variant, fcfg.subtile, fcfg.order, tuple(fcfg.bg),
                                     flags=B.FLAG_QUEUE_READY | (fcfg.flags & B.FLAG_PERSISTENT))
        self.packed_grads = bool(packed_grads)
        self.bcfg_ready = B.make_cfg(bcfg.variant, bcfg.subtile, bcfg.order, tuple(bcfg.bg),
                                     flags=B.FLAG_QUEUE_READY | (bcfg.flags & (B.FLAG_SPLIT_WALKS | B.FLAG_PERSISTENT)) |
                                     (B.FLAG_PACKED_GRADS if self.packed_grads else 0))
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        self.list_cap = 0
        self.pr = dict(means2D=torch.empty(P, 2, device=dev), conic_opacity=torch.empty(P, 4, device=dev),
                       rgb=torch.empty(P, 3, device=dev), depth=torch.empty(P, device=dev),
                       radius=torch.empty(P, dtype=torch.int32, device=dev),
                       tiles_touched=torch.empty(P, dtype=torch.int32, device=dev))
        self.fwd = dict(color=torch.empty(3, H, W, device=dev), alpha=torch.empty(H, W, device=dev),
                        depth=torch.empty(H, W, device=dev), final_T=torch.empty(H, W, device=dev),
                        n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev))
        # split walks read the forward's colour and depth
        self.bcfg_ready.split_color = self.fwd["color"].data_ptr()
        self.bcfg_ready.split_depth = self.fwd["depth"].data_ptr()
        if self.packed_grads:
            self.grad_records = B.grad_records(P, dev)
            self.grads = B.record_views(self.grad_records)
            self._grad_list = [self.grad_records]
        else:
            # separate allocations, zeroed by one multi-tensor fill
            self.grad_records = None
            self.grads = dict(means2D=torch.zeros(P, 2, device=dev), conic_opacity=torch.zeros(P, 4, device=dev),
                              rgb=torch.zeros(P, 3, device=dev), depth=torch.zeros(P, device=dev))
            self._grad_list = list(self.grads.values())
        self.ranges = torch.empty(B.n_tiles(W, H), 2, dtype=torch.int32, device=dev)
        self.n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        # size the pair buffers: build the lists until the capacity holds M
        self._project()
        cap = 0
        while True:
            self._alloc_lists(cap)
            self._lists()
            M = int(self.n_dev.item())
            if M <= cap:
                break
            cap = int(M * headroom) + 1024
        self.capacity = cap
        self.frame = B.make_frame(W, H, self.ranges, self.point_list, self.pr["means2D"], self.pr["conic_opacity"],
                                  self.pr["rgb"], self.pr["depth"])
        rb = max(B.bgs_render_workspace_bytes(self.frame, fcfg), B.bgs_render_workspace_bytes(self.frame, bcfg))
        self.rws = torch.empty(rb, dtype=torch.uint8, device=dev)
        self.M_whole = M
        self.whole_list_len = (self.ranges[:, 1] - self.ranges[:, 0]).clone()  # of the sizing build's whole lists
        if list_cap == "auto":
            self.run()
            deepest = int(self.fwd["n_contrib"].max().item())
            longest = int((self.ranges[:, 1] - self.ranges[:, 0]).max().item())
            K = (2 * deepest + 64 + 63) // 64 * 64
            while K < longest and (K > 2048 or K * B.n_tiles(W, H) <= self.capacity):
                self.set_list_cap(K)
                self.run()
                if not self.overflowed():
                    break
                K *= 2
            else:
                self.set_list_cap(None)
        elif list_cap is not None:
            self.set_list_cap(int(list_cap))

    def set_list_cap(self, K):
        """Cap the tile lists at K entries per tile from the next step on
        (None or 0: whole lists)."""
        K = int(K or 0)
        if not 0 <= K < 1 << 32:
            raise ValueError("list cap must be in [0, 2^32)")
        if 0 < K <= 2048 and K * B.n_tiles(self.W, self.H) > self.capacity:
            raise ValueError("lists capped at K <= 2048 need n_tiles * K <= the pair capacity")
        self.list_cap = K
        self.fcfg_ready.list_cap = K
        self.fcfg_ready.list_overflow = self.overflow.data_ptr() if K else None
        self.overflow.zero_()

    def overflowed(self) -> bool:
        """Whether a pixel ran off a capped list in a step since the cap was
        set or clear_overflow() was called (reads the device; synchronizes).
        Always False with whole lists."""
        return bool(self.list_cap) and bool(self.overflow.item())

    def clear_overflow(self):
        """Clear the overflow report (on the current stream)."""
        self.overflow.zero_()

    def _alloc_lists(self, cap):
        dev = self.dL_dcolor.device
        self.point_list = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)[:cap]
        self.lws = torch.empty(B.bgs_tile_lists_workspace_bytes(self.W, self.H, self.P, cap), dtype=torch.uint8,
                               device=dev)

    def _project(self):
        p, pr = self.params, self.pr
        B.bgs_project(self.cam, p["means3D"], p["log_scales"], p["quats"], p["opacity"], p["colors"], self.sh_degree,
                      pr["means2D"], pr["conic_opacity"], pr["rgb"], pr["depth"], pr["radius"], pr["tiles_touched"])

    def _lists(self):
        pr = self.pr
        B.bgs_tile_lists(self.W, self.H, pr["means2D"], pr["radius"], pr["depth"], pr["tiles_touched"],
                         self.point_list if self.point_list.numel() else None, self.ranges, self.n_dev, self.lws,
                         conic_opacity=pr["conic_opacity"] if self.binning == "ellipse" else None,
                         max_per_tile=self.list_cap)

    def run(self, mark=None):
        """Issue one step; mark(i) (optional) is called at the stage
        boundaries 0..6: before project, after project, after the lists,
        after the forward queue, after the forward, after the backward queue
        (gradients zeroed), after the backward."""
        mark = mark or (lambda i: None)
        mark(0)
        self._project()
        mark(1)
        self._lists()
        mark(2)
        if self.fcfg.variant not in (B.STATIC, B.STATIC_WAVE):  # the static variants take no queue
            B.bgs_queue_build(self.frame, self.fcfg, None, self.rws)
        mark(3)
        f = self.fwd
        if self.poison_outputs:
            poison_fwd(f)
        B.bgs_render_fwd(self.frame, self.fcfg_ready, f["color"], f["alpha"], f["depth"], f["final_T"],
                         f["n_contrib"], self.rws)
        mark(4)
        if len(self._grad_list) == 1:  # the gradient records: one plain fill
            self._grad_list[0].zero_()
        else:
            torch._foreach_zero_(self._grad_list)
        if self.bcfg.variant not in (B.STATIC, B.STATIC_WAVE):
            B.bgs_queue_build(self.frame, self.bcfg, f["n_contrib"], self.rws)
        mark(5)
        if self.packed_grads:
            B.bgs_render_bwd(self.frame, self.bcfg_ready, f["final_T"], f["n_contrib"], self.dL_dcolor, None, None,
                             self.grad_records, None, None, None, self.rws)
        else:
            g = self.grads
            B.bgs_render_bwd(self.frame, self.bcfg_ready, f["final_T"], f["n_contrib"], self.dL_dcolor, None, None,
                             g["means2D"], g["conic_opacity"], g["rgb"], g["depth"], self.rws)
        mark(6)

    def n_pairs(self) -> int:
        """M of the last step (reads the device; synchronizes)."""
        return int(self.n_dev.item())

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Record one step as a hipGraph; graph.replay() then runs the whole
        step.  The step is run once first, outside the capture."""
        self.run()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.run()
        return graph


class AdaptiveSelector:
    """The training-time selection policy of Sec. 4.4: start from the given
    configuration and, every `interval` calls, re-measure the candidates on
    the current frame and switch to the fastest."""

    def __init__(self, rast: Rasterizer, base: B.RenderCfg, interval: int = 1000):
        self.rast, self.base, self.interval = rast, base, interval
        self.calls = 0
        self.fwd_cfg, self.bwd_cfg = base, base

    def select(self, prep: Prepared, dL_dcolor=None):
        if self.calls % self.interval == 0:
            self.fwd_cfg, self.bwd_cfg, _, _ = self.rast.autotune(prep, self.base, dL_dcolor)
        self.calls += 1
        return self.fwd_cfg, self.bwd_cfg


class RenderFn(torch.autograd.Function):
    """Differentiable render of prepared splats: inputs means2D [P,2],
    conic_opacity [P,4], rgb [P,3], depth [P] (the per-tile lists are taken
    from ``prep``); outputs color [3,H,W], alpha [H,W], depth [H,W].  The
    backward returns gradients for all four inputs."""

    @staticmethod
    def forward(ctx, means2D, conic_opacity, rgb, depth, prep: Prepared, cfg: B.RenderCfg, rast: Rasterizer):
        p2 = dataclasses.replace(prep, means2D=means2D.contiguous(), conic_opacity=conic_opacity.contiguous(),
                                 rgb=rgb.contiguous(), depth=depth.contiguous())
        out = rast.render_fwd(p2, cfg)
        ctx.prep, ctx.cfg, ctx.rast = p2, cfg, rast
        ctx.save_for_backward(out["final_T"], out["n_contrib"])
        ctx.mark_non_differentiable(out["final_T"], out["n_contrib"])
        # split walks read the forward's colour and depth (kept as plain copies)
        ctx.split_out = ((out["color"].detach().clone(), out["depth"].detach().clone())
                         if cfg.flags & B.FLAG_SPLIT_WALKS else None)
        return out["color"], out["alpha"], out["depth"]

    @staticmethod
    def backward(ctx, g_color, g_alpha, g_depth):
        final_T, n_contrib = ctx.saved_tensors
        prep, rast = ctx.prep, ctx.rast
        H, W = prep.height, prep.width
        dev = final_T.device
        g_color = torch.zeros(3, H, W, device=dev) if g_color is None else g_color.contiguous()
        g_alpha = None if g_alpha is None else g_alpha.contiguous()
        g_depth = None if g_depth is None else g_depth.contiguous()
        fwd = dict(final_T=final_T, n_contrib=n_contrib)
        if ctx.split_out is not None:
            fwd["color"], fwd["depth"] = ctx.split_out
        grads = rast.render_bwd(prep, ctx.cfg, fwd, g_color, g_alpha, g_depth)
        return grads["means2D"], grads["conic_opacity"], grads["rgb"], grads["depth"], None, None, None


def render(means2D, conic_opacity, rgb, depth, prep: Prepared, cfg: B.RenderCfg, rast: Rasterizer):
    return RenderFn.apply(means2D, conic_opacity, rgb, depth, prep, cfg, rast)


class Render3DFn(torch.autograd.Function):
    """Differentiable render from the 3D Gaussian parameters: projection, tile
    lists and the forward render, with the backward render followed by the
    projection's derivative (bgs_project_bwd).  Inputs means3D [P,3],
    log_scales [P,3], quats [P,4], opacity [P], colors (RGB [P,3] or SH
    [P,K,3]); outputs color [3,H,W], alpha [H,W], depth [H,W]."""

    @staticmethod
    def forward(ctx, means3D, log_scales, quats, opacity, colors, cam, sh_degree, fwd_cfg, bwd_cfg, rast,
                prep=None):
        args = [t.detach().contiguous() for t in (means3D, log_scales, quats, opacity, colors)]
        if prep is None:  # else: prepared by the caller from these same parameters
            prep = rast.prepare(cam, *args, sh_degree)
        out = rast.render_fwd(prep, fwd_cfg)
        ctx.save_for_backward(*args)
        ctx.prep, ctx.out, ctx.cam, ctx.sh_degree, ctx.bwd_cfg, ctx.rast = prep, out, cam, sh_degree, bwd_cfg, rast
        return out["color"], out["alpha"], out["depth"]

    @staticmethod
    def backward(ctx, g_color, g_alpha, g_depth):
        means3D, log_scales, quats, opacity, colors = ctx.saved_tensors
        rast = ctx.rast
        g2 = rast.render_bwd(ctx.prep, ctx.bwd_cfg, ctx.out, g_color.contiguous(),
                             None if g_alpha is None else g_alpha.contiguous(),
                             None if g_depth is None else g_depth.contiguous())
        g3 = rast.project_bwd(ctx.cam, means3D, log_scales, quats, colors, ctx.sh_degree, g2["means2D"],
                              g2["conic_opacity"], g2["rgb"], g2["depth"])
        return (g3["means3D"], g3["log_scales"], g3["quats"], g3["opacity"], g3["colors"].view_as(colors),
                None, None, None, None, None, None)


def render_gaussians(means3D, log_scales, quats, opacity, colors, cam, sh_degree: int, rast: Rasterizer,
                     fwd_cfg: Optional[B.RenderCfg] = None, bwd_cfg: Optional[B.RenderCfg] = None):
    """color, alpha, depth of the 3D Gaussians seen by `cam`, differentiable in
    all five parameter tensors."""
    fwd_cfg = fwd_cfg or B.make_cfg("pixel", 16, "cost")
    bwd_cfg = bwd_cfg or fwd_cfg
    return Render3DFn.apply(means3D, log_scales, quats, opacity, colors, cam, sh_degree, fwd_cfg, bwd_cfg, rast)


def fit(params: dict, cameras, targets, sh_degree: int, rast: Rasterizer, iters: int, lr: float = 1e-2,
        selector: Optional[AdaptiveSelector] = None, cfg: Optional[B.RenderCfg] = None):
    """A plain training loop over the 3D Gaussian parameters (the setting of
    the paper's self-adaptive kernel selection, Sec. 4.4): views are visited
    in turn, the image loss is the mean squared error against `targets`, Adam
    updates means3D / log_scales / quats / opacity / colors (opacity kept in
    (0, 1)).  When a selector is given, it chooses the forward and backward
    kernels from measurements every `selector.interval` iterations.  Returns
    the per-iteration losses."""
    keys = ("means3D", "log_scales", "quats", "opacity", "colors")
    opt = torch.optim.Adam([params[k] for k in keys], lr=lr)
    cfg = cfg or B.make_cfg("pixel", 16, "cost")
    losses = []
    for it in range(iters):
        v = it % len(cameras)
        cam = cameras[v]
        with torch.no_grad():
            prep = rast.prepare(cam, *[params[k].detach() for k in keys], sh_degree)
        fcfg, bcfg = selector.select(prep) if selector is not None else (cfg, cfg)
        color, _, _ = Render3DFn.apply(*[params[k] for k in keys], cam, sh_degree, fcfg, bcfg, rast, prep)
        loss = torch.mean((color - targets[v]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        with torch.no_grad():
            params["opacity"].clamp_(1e-3, 0.999)
        losses.append(float(loss.detach()))
    return losses
