/*
 * bgs.h - C ABI of the MI355X (gfx950) balanced 3DGS tile rasterizer.
 *
 * The library renders 3D Gaussian splats with the tile-based pipeline of
 * Balanced 3DGS (Gui et al., arXiv 2412.17378):
 *
 *   bgs_project  -> bgs_bin -> bgs_sort -> bgs_ranges -> bgs_render_fwd
 *                                                      -> bgs_render_bwd
 *
 * and its load-balanced forward renderer: a persistent work queue of
 * sub-tiles fed by a global atomic counter (Sec. 4.1, 4.3), pixel-wise and
 * Gaussian-wise wavefront modes (Sec. 4.2), a static one-workgroup-per-tile
 * baseline (Sec. 5.2.1, naive kernel) and a timing-based variant selector
 * (Sec. 4.4).
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller, unless a
 *     comment says "host".  The library allocates no device memory inside a
 *     call except where noted (bgs_plan_*); scratch comes from a caller
 *     workspace sized by the matching *_workspace_bytes function.
 *   - Every call enqueues work on `stream` and returns without waiting,
 *     except where a comment says it synchronizes.
 *   - Floating point is IEEE fp32; indices are 32-bit unsigned.
 *   - Errors: a non-zero bgs_status; no exception crosses the ABI;
 *     bgs_last_error() gives a thread-local message.  Invalid sizes or a
 *     missing required pointer -> BGS_EINVAL; a HIP runtime failure ->
 *     BGS_EHIP; an output too small for the data -> BGS_ECAPACITY.
 *   - Images are planar: colour [3][H][W], single channels [H][W], row-major.
 *   - Pixel (px, py) is sampled at integer coordinates (px, py).
 */
#ifndef BGS_H
#define BGS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bgs_status {
    BGS_OK = 0,
    BGS_EINVAL = -1,
    BGS_ECAPACITY = -2,
    BGS_EHIP = -3,
    BGS_EUNSUPPORTED = -4,
    BGS_EINTERNAL = -5
} bgs_status;

/* Pinhole camera, HOST memory.  camera = R * world + t, R row-major.
 * Pixel centre of the camera ray (x, y, z) is (fx x/z + cx - 1/2, fy y/z + cy - 1/2).
 * Gaussians with camera depth z <= znear are culled. */
typedef struct bgs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
} bgs_camera;

/* Render inputs of one view (Alg. 1-4 inputs XY, PL, CO, F, D), HOST struct
 * holding DEVICE pointers.  P Gaussians, n_tiles = ceil(W/tile)*ceil(H/tile). */
typedef struct bgs_frame {
    int32_t width, height;        /* image size in pixels, >= 1 */
    int32_t tile;                 /* binning tile edge in pixels: 16 */
    const uint32_t* ranges;       /* [n_tiles][2] start, end into point_list */
    const uint32_t* point_list;   /* [n_pairs] Gaussian ids, per tile front to back */
    const float* means2D;         /* [P][2] pixel-space centre (XY) */
    const float* conic_opacity;   /* [P][4] (a, b, c, o): inverse 2D covariance
                                     [[a, b], [b, c]] and opacity (CO) */
    const float* rgb;             /* [P][3] colour (F) */
    const float* depth;           /* [P] camera depth (D) */
} bgs_frame;

/* Forward / backward kernel variants. */
typedef enum bgs_variant {
    BGS_STATIC = 0,           /* one 256-lane workgroup per 16x16 tile, grid-static */
    BGS_BALANCED_PIXEL = 1,   /* balanced task distribution from the dealt queue, lane =
                                 pixel: subtile 8 persistent waves on the atomic sub-tile
                                 queue; subtile 16 / 32 the dealt items as a dispatched
                                 grid, or persistent waves with BGS_FLAG_PERSISTENT */
    BGS_BALANCED_GAUSS = 2,   /* persistent waves, atomic sub-tile queue, lane = Gaussian */
    BGS_BALANCED_HYBRID = 3,  /* lane = pixel, stragglers finished lane = Gaussian */
    BGS_STATIC_WAVE = 4       /* the wave-per-tile code of BGS_BALANCED_PIXEL with
                                 subtile 16, dispatched grid-statically: wave w of the
                                 grid renders tile w (raster order), no queue; the
                                 baseline that isolates the task pool's scheduling */
} bgs_variant;

/* Queue order of the balanced variants. */
typedef enum bgs_order {
    BGS_ORDER_RASTER = 0,     /* sub-tiles in raster order */
    BGS_ORDER_COST = 1        /* heaviest estimated sub-tile first */
} bgs_order;

/* Flags of bgs_render_cfg. */
enum {
    /* the workspace already holds a queue from bgs_queue_build for this frame
       and cfg (with the counter reset); render calls then skip building it */
    BGS_FLAG_QUEUE_READY = 1,
    /* backward of BGS_BALANCED_PIXEL, subtile 16, cost order: a tile whose walk
       reaches 128 list entries becomes two work items, the entries below a
       split point k (near half the walk, a multiple of 64) walked front to back
       from T = 1 and the entries from k on walked back to front from final_T.
       Needs the forward's outputs in split_color and split_depth (the sum over
       the whole walk that the lower part starts from is read off them).
       Halves the heaviest work items, so the queue balances better; the
       gradients equal the unsplit ones up to fp32 rounding. */
    BGS_FLAG_SPLIT_WALKS = 2,
    /* bgs_render_bwd / bgs_render_bwd_det: the gradients go, added (+=), into
       ONE array of 16-float records, passed as dL_dmeans2D (DEVICE [P][16],
       64-byte aligned; dL_dconic_opacity, dL_drgb and dL_ddepths must be
       null).  Record of Gaussian i: floats 0-3 d/d(a, b, c, o) of
       conic_opacity, 4-5 d/d(means2D), 6-8 d/d(rgb), 9 d/d(depth), 10-15
       unused (left as they are).  One list entry's ten gradient atomics then
       fall in one 64-byte segment instead of four arrays' cache lines.
       bgs_project_bwd_packed reads this layout.  Not for batched plans. */
    BGS_FLAG_PACKED_GRADS = 4,
    /* BGS_BALANCED_PIXEL with subtile 16 or 32: persistent waves take the
       dealt work items from the task pool's 64 fetch counters (Alg. 1's
       atomic task fetch).  Without the flag the dealt items go out as a plain
       grid in rank order -- four items per 256-lane workgroup -- and the
       hardware's workgroup dispatcher hands them to compute units as slots
       free up, heaviest first in cost order: the same dynamic distribution
       without atomics or a resident loop (and the register budget of the
       grid-static kernel).  Either way every dealt item is rendered once. */
    BGS_FLAG_PERSISTENT = 8
};

typedef struct bgs_render_cfg {
    int32_t variant;          /* bgs_variant */
    int32_t subtile;          /* balanced variants: work-item edge.  8: one wave per
                                 8x8 sub-tile (one pixel per lane).  16 (BGS_BALANCED_PIXEL
                                 and BGS_STATIC_WAVE): one wave per whole 16x16 tile,
                                 four pixels per lane, forward and backward.  32
                                 (BGS_BALANCED_PIXEL only): one wave per 32x32 block of
                                 2x2 tiles, rendered tile after tile */
    int32_t order;            /* bgs_order */
    int32_t flags;            /* BGS_FLAG_* */
    float bg[3];              /* background colour */
    /* Optional load-balance trace (DEVICE, nullable): render kernels write
       one record of three uint64 per wave, record w for wave
       (workgroup * 4 + wave in workgroup) while w < wg_trace_cap:
       [0] = 1 + (XCC id << 8 | HW_ID bits 15..8: shader engine, shader array,
       CU), [1] / [2] = the 100 MHz real-time counter at the wave's start / end.
       Records of waves not launched are left untouched (zero the buffer). */
    uint64_t* wg_trace;
    int64_t wg_trace_cap;
    /* Optional work count (DEVICE [H][W], nullable; bgs_render_fwd only):
       per pixel the number of list entries the sequential loop examines,
       skipped entries and the stopping entry included (the list length when
       the pixel never stops).  Written by BGS_BALANCED_PIXEL with subtile
       16; other variants return BGS_EUNSUPPORTED when it is set. */
    int32_t* n_examined;
    /* Lists capped at list_cap entries per tile (bgs_tile_lists with
       max_per_tile = list_cap; 0: whole lists).  bgs_render_fwd sets
       *list_overflow (DEVICE, nullable) to 1 when a pixel reaches the end of
       a list of list_cap or more entries without stopping: that pixel's
       result may differ from the whole list's.  The flag is only ever set;
       the caller clears it. */
    uint32_t list_cap;
    uint32_t* list_overflow;
    /* Optional queue audit (DEVICE, nullable, caller-zeroed): the balanced
       kernels of a one-view render add 1 to item_claims[i] each time a wave
       takes work item i from the task pool (Alg. 1), so after a render every
       dealt item shows exactly 1.  Items: subtile 8 -> tile * 4 + quadrant
       (4 n_tiles of them); subtile 32 -> block (ty / 2) * ceil(TX / 2) +
       tx / 2; subtile 16 -> tile + u * n_tiles with u the part of the tile's
       work the item covers: 0 the whole tile, 1 / 2 the lower / upper part of
       its backward walk (BGS_FLAG_SPLIT_WALKS), 3 + q the 16x4 pixel block q
       alone, 7 + 2 q + p part p of block q's walk -- cost-ordered queues deal
       a tile whose cost reaches a threshold as four blocks (and, with split
       walks, parts), so the array needs 15 n_tiles entries there.  Ignored by
       the static variants and by plans. */
    uint32_t* item_claims;
    /* With BGS_FLAG_SPLIT_WALKS: the forward's out_color [3][H][W] and
       out_depth [H][W] of this frame (DEVICE, read only by the backward). */
    const float* split_color;
    const float* split_depth;
} bgs_render_cfg;

/* Thread-local text for the last non-OK status of this thread. */
const char* bgs_last_error(void);

/* Library version string. */
const char* bgs_version(void);

/*
 * Projection, Eq. (1)-(3) (Sec. 2.1).  Per Gaussian i < P: camera transform,
 * 3D covariance R_q diag(exp(2 s)) R_q^T from log-scales s and the unit
 * quaternion (w, x, y, z), EWA covariance J W Sigma W^T J^T + 0.3 I (J
 * evaluated with x/z, y/z clamped to 1.3x the half field of view), its
 * inverse (conic), radius = ceil(3 sqrt(lambda_max)), colour, and the number
 * of tile x tile tiles its square [u-r, u+r] x [v-r, v+r] meets.
 *   means3D [P][3], log_scales [P][3], quats [P][4], opacity [P].
 *   colors: sh_degree < 0 -> RGB [P][3] used as is;
 *           0..3 -> SH coefficients [P][(d+1)^2][3], colour =
 *           max(0, sum_lm k_lm Y_lm(ray) + 1/2), Y_lm the real spherical
 *           harmonics without Condon-Shortley phase, index l*l + l + m.
 *   Outputs: means2D [P][2], conic_opacity [P][4], rgb [P][3], depth [P],
 *   radius [P] (0 = culled), tiles_touched [P].  Culled Gaussians get
 *   radius 0 and tiles_touched 0.
 */
bgs_status bgs_project(const bgs_camera* cam, int64_t P, const float* means3D, const float* log_scales,
                       const float* quats, const float* opacity, const float* colors, int32_t sh_degree,
                       int32_t tile, float* means2D, float* conic_opacity, float* rgb, float* depth,
                       int32_t* radius, uint32_t* tiles_touched, hipStream_t stream);

/*
 * Derivative of bgs_project (the preprocessing step before the render; it
 * closes a training step through the 3D parameters): from the gradients of
 * the projection outputs -- dL_dmeans2D [P][2], dL_dconic_opacity [P][4]
 * (a, b, c, opacity; 16-byte aligned, the layout bgs_render_bwd writes),
 * dL_drgb [P][3], dL_ddepth [P] (nullable) -- to those of its inputs, WRITTEN
 * (=), not accumulated: dL_dmeans3D [P][3], dL_dlog_scales [P][3],
 * dL_dquats [P][4] (16-byte aligned; through the quaternion's
 * normalization), dL_dopacity [P], dL_dcolors (the layout of `colors`: RGB
 * [P][3], or SH coefficients [P][(d+1)^2][3]).  Same camera, inputs and
 * sh_degree as the forward call.  The derivative through the 1.3x field-of-
 * view clamp of the Jacobian and through the colour's clamp at 0 is 0;
 * culled Gaussians get zeros.  Asynchronous on `stream`.
 */
bgs_status bgs_project_bwd(const bgs_camera* cam, int64_t P, const float* means3D, const float* log_scales,
                           const float* quats, const float* colors, int32_t sh_degree, const float* dL_dmeans2D,
                           const float* dL_dconic_opacity, const float* dL_drgb, const float* dL_ddepth,
                           float* dL_dmeans3D, float* dL_dlog_scales, float* dL_dquats, float* dL_dopacity,
                           float* dL_dcolors, hipStream_t stream);

/*
 * bgs_project_bwd with the screen-space gradients in the 16-float records of
 * BGS_FLAG_PACKED_GRADS (DEVICE [P][16], 64-byte aligned): the same
 * arithmetic on the same values, so the results equal bgs_project_bwd's on
 * the four arrays unpacked from the records bit for bit.
 */
bgs_status bgs_project_bwd_packed(const bgs_camera* cam, int64_t P, const float* means3D, const float* log_scales,
                                  const float* quats, const float* colors, int32_t sh_degree,
                                  const float* dL_drecords, float* dL_dmeans3D, float* dL_dlog_scales,
                                  float* dL_dquats, float* dL_dopacity, float* dL_dcolors, hipStream_t stream);

/* Workspace bytes for bgs_bin with P Gaussians. */
size_t bgs_bin_workspace_bytes(int64_t P);

/*
 * Tile binning (the pre-processing "patch" step of Sec. 4.3, producing the
 * sorted point list PL of Alg. 1-4).  Emits one (tile id, Gaussian id) pair
 * for every tile a Gaussian's square meets, Gaussians visited in increasing
 * depth (ties: increasing id), so a later stable sort by tile id yields, per
 * tile, the front-to-back order Eq. (4) needs.
 *   keys [capacity] tile ids, values [capacity] Gaussian ids.
 *   *n_pairs_host (HOST) receives the pair count M.  This call SYNCHRONIZES
 *   the stream to read M; if M > capacity nothing is written to keys/values
 *   and BGS_ECAPACITY is returned (M still reported).
 */
bgs_status bgs_bin(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                   const int32_t* radius, const float* depth, const uint32_t* tiles_touched, uint32_t* keys,
                   uint32_t* values, int64_t capacity, int64_t* n_pairs_host, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* Workspace bytes for bgs_sort of n pairs. */
size_t bgs_sort_workspace_bytes(int64_t n);

/*
 * Stable ascending sort of n (key, value) pairs by the low key_bits bits of
 * the key (1..32).  Input and output buffers must not alias.
 */
bgs_status bgs_sort(const uint32_t* keys_in, const uint32_t* values_in, uint32_t* keys_out,
                    uint32_t* values_out, int64_t n, int32_t key_bits, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/*
 * Per-tile [start, end) of a key array sorted by tile id (the range of PL a
 * tile's workgroup walks, Alg. 1 "Load XY, PL, CO").  ranges [n_tiles][2];
 * empty tiles get (0, 0).
 */
bgs_status bgs_ranges(const uint32_t* sorted_keys, int64_t n, int32_t n_tiles, uint32_t* ranges,
                      hipStream_t stream);

/* Workspace bytes for bgs_tile_lists with P Gaussians and a point list of
 * `capacity` entries (the workspace holds a coarse list of that size). */
size_t bgs_tile_lists_workspace_bytes(int32_t width, int32_t height, int64_t P, int64_t capacity);

/*
 * bgs_bin + bgs_sort + bgs_ranges fused: the same point list and ranges, bit
 * for bit, without materializing or sorting the (tile, Gaussian) keys.  The
 * Gaussians are put in depth order; a stable counting sort over groups of
 * 8x8 tiles (per-chunk group histograms from 2D difference arrays, a column
 * scan over chunks, in-order placement) builds coarse per-group lists, and
 * the coarse lists are split into the 64 tile lists of each group by ordered
 * ballot compaction, one workgroup per segment of 2048 coarse entries.
 *   point_list [capacity] Gaussian ids, ranges [n_tiles][2] (empty: (0, 0)),
 *   n_pairs_dev (DEVICE, uint64[1]) receives M.
 * Never synchronizes: every size the kernels need stays on the device and
 * the grids are fixed by P and the image size.  When M exceeds capacity,
 * point_list is not written, every range is written empty (0, 0), so a render
 * of the frame reads nothing from point_list, and n_pairs_dev receives M, or
 * a lower bound of M above capacity when the overflow shows already in the
 * coarse lists (sized by the same capacity); the caller reads n_pairs_dev when
 * convenient, grows point_list (and the workspace) and calls again.
 * capacity must be < 2^32.  Tile grids of more than 8192 groups return
 * BGS_EUNSUPPORTED (use the three separate calls).
 *   max_per_tile: 0 for whole lists.  K > 0 keeps only the first K entries of
 *   each tile's list (its front-most K Gaussians), where ranges say; M
 *   counts the kept entries.  K <= 2048: gathered per tile straight from the
 *   coarse lists into the fixed slot [t K, t K + n_t) of point_list (which
 *   then has gaps), needing capacity >= n_tiles K (else BGS_ECAPACITY before
 *   any work).  Larger K: compact, from the segment split.  Eq. (4) never
 *   reads past the entry at which a pixel's transmittance stops, so a render
 *   from the capped lists equals the render from whole lists unless some
 *   pixel reaches the end of a capped list without stopping;
 *   bgs_render_fwd reports that case through bgs_render_cfg.list_overflow,
 *   and the frame must then be built and rendered again with a larger K or
 *   whole lists.  The coarse lists are not capped, so capacity (which also
 *   sizes them) must hold the coarse entries too, e.g. capacity = the
 *   whole-list M.
 */
bgs_status bgs_tile_lists(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                          const int32_t* radius, const float* depth, const uint32_t* tiles_touched,
                          uint32_t* point_list, int64_t capacity, uint32_t max_per_tile, uint32_t* ranges,
                          uint64_t* n_pairs_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * bgs_tile_lists with exact ellipse-tile binning (the list-shrinking binning
 * refinement the paper names among related work, Sec. 2): a pair (tile, g)
 * of the square rule is kept only when the tile's rectangle of pixel centres,
 * widened by 2^-6 px, meets the ellipse q(d) <= 2 ln(255 o) (1 + 2^-10) +
 * 2^-10, q(d) = a dx^2 + 2 b dx dy + c dy^2 with (a, b, c, o) =
 * conic_opacity[g] -- outside it g's alpha stays below 1/255 and Eq. (4)
 * skips g.  So the forward and backward rendered from these lists equal
 * those from bgs_tile_lists (the removed entries are skipped at every pixel
 * of their tile); n_contrib counts positions in the shorter lists.  The GPU
 * evaluates the rule in fp32 on a slightly larger ellipse (2^-12 per axis,
 * row intervals padded by 2^-11 of the half extent), so rounding can add
 * pairs next to the boundary but never removes one.  A Gaussian whose conic
 * is not positive definite keeps the square rule; one with opacity below
 * 1/255 gets no pair.
 *   conic_opacity [P][4] (DEVICE, 16-byte aligned), everything else, the
 *   workspace size, max_per_tile and the overflow behaviour as for
 *   bgs_tile_lists.  Images over 16384 pixels high (1024 tile rows) return
 *   BGS_EUNSUPPORTED: the emit keeps a Gaussian's row intervals in LDS.
 */
bgs_status bgs_tile_lists_exact(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                                const float* conic_opacity, const int32_t* radius, const float* depth,
                                const uint32_t* tiles_touched, uint32_t* point_list, int64_t capacity,
                                uint32_t max_per_tile, uint32_t* ranges, uint64_t* n_pairs_dev, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for bgs_queue_build / bgs_render_fwd / bgs_render_bwd. */
size_t bgs_render_workspace_bytes(const bgs_frame* frame, const bgs_render_cfg* cfg);

/*
 * Task pool of the balanced renderer (Sec. 4.1 steps 1-4, Sec. 4.3): writes
 * the work items of `frame` (8x8 sub-tiles, 16x16 tiles or 32x32 blocks of
 * 2x2 tiles, by cfg->subtile) into the workspace in the order cfg->order asks
 * for and resets the fetch counters.  For BGS_ORDER_COST the forward cost
 * estimate of a tile is the list position by which its entries' opacities
 * alone could first take the transmittance below 1e-4 (the shortest walk any
 * of its pixels can have); when n_contrib (nullable, [H][W] from the forward
 * pass) is given the cost is the largest n_contrib in the tile (the
 * backward's exact walk); a block costs the sum of its tiles.
 * bgs_render_fwd / bgs_render_bwd call this themselves.  The workspace
 * begins with the queue's state: 64 uint32 fetch counters 128 bytes apart
 * (counter q at byte 128 q), then at byte 8192 the number of items.  The
 * static variants (BGS_STATIC, BGS_STATIC_WAVE) take no queue: for them the
 * call checks its arguments and returns BGS_OK without launching anything.
 */
bgs_status bgs_queue_build(const bgs_frame* frame, const bgs_render_cfg* cfg, const int32_t* n_contrib,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Forward render, Eq. (4) per pixel front to back with the rules of the
 * paper's naive per-pixel loop (Appendix): an entry is skipped when its
 * exponent is positive or alpha = min(0.99, o exp(power)) < 1/255; the pixel
 * stops, without blending the entry, once T (1 - alpha) < 1e-4.
 *   out_color [3][H][W] = sum rgb alpha T + T_final bg
 *   out_alpha [H][W]    = 1 - T_final   (= sum alpha T)
 *   out_depth [H][W]    = sum depth alpha T
 *   final_T   [H][W]    = T_final
 *   n_contrib [H][W]    = 1 + list position of the last blended entry (0 if none)
 * The variant in cfg only changes speed; all variants give the same result up
 * to fp32 rounding.
 */
bgs_status bgs_render_fwd(const bgs_frame* frame, const bgs_render_cfg* cfg, float* out_color, float* out_alpha,
                          float* out_depth, float* final_T, int32_t* n_contrib, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/*
 * bgs_render_fwd without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc): the same render, same arguments minus ws / ws_bytes,
 * with the balanced variants' work queue kept in a device array inside the
 * library (bgs_render_fwd_noalloc_max_bytes() = 2.5 MiB per device, held
 * until the process ends; queues of up to 65 536 tiles).  Allocates nothing and
 * builds the queue on every call (BGS_FLAG_QUEUE_READY is ignored).  A frame
 * whose queue does not fit returns BGS_ECAPACITY before any work is queued.
 * All calls on one device share that array: calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller.
 */
bgs_status bgs_render_fwd_noalloc(const bgs_frame* frame, const bgs_render_cfg* cfg, float* out_color,
                                  float* out_alpha, float* out_depth, float* final_T, int32_t* n_contrib,
                                  hipStream_t stream);
size_t bgs_render_fwd_noalloc_max_bytes(void);

/*
 * Backward render: the derivative of bgs_render_fwd for
 * L = <dL_dcolor, out_color> + <dL_dalpha, out_alpha> + <dL_ddepth, out_depth>
 * with every skip / stop decision of the forward held fixed.  Per pixel it
 * walks the list back to front from n_contrib, recovering T by division
 * T_{k-1} = T_k / (1 - alpha_k) from final_T.  Gradients are ADDED (+=) into
 * the caller's buffers (zero them first):
 *   dL_dmeans2D [P][2]; dL_dconic_opacity [P][4] laid out like
 *   conic_opacity: d/da, d/db, d/dc of power = -(a dx^2 + c dy^2)/2 - b dx dy,
 *   then d/do; dL_drgb [P][3]; dL_ddepths [P] (nullable);
 * or, with BGS_FLAG_PACKED_GRADS, one [P][16] record array in dL_dmeans2D
 * (the other three null; layout at the flag).  A long walk may be split
 * (BGS_FLAG_SPLIT_WALKS), the lower part walked front to back from T = 1.
 * dL_dalpha and dL_ddepth are nullable (zero).  final_T and n_contrib are the
 * forward's outputs for the same frame.  Errors: BGS_EINVAL for null or
 * misaligned required arrays, a workspace too small, or split walks without
 * split_color / split_depth; BGS_EUNSUPPORTED for split walks on another
 * variant.
 */
bgs_status bgs_render_bwd(const bgs_frame* frame, const bgs_render_cfg* cfg, const float* final_T,
                          const int32_t* n_contrib, const float* dL_dcolor, const float* dL_dalpha,
                          const float* dL_ddepth, float* dL_dmeans2D, float* dL_dconic_opacity, float* dL_drgb,
                          float* dL_ddepths, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of bgs_render_bwd_det for P Gaussians and up to max_occ
 * walked (tile, list entry) pairs. */
size_t bgs_render_bwd_det_workspace_bytes(const bgs_frame* frame, int64_t P, int64_t max_occ);

/*
 * Deterministic-order backward: the derivative bgs_render_bwd computes (same
 * arguments and += semantics; P = number of Gaussians, every id in the lists
 * below P), with gradients that are identical from run to run.  One wave per
 * 16x16 tile (cfg: BGS_BALANCED_PIXEL with subtile 16, else
 * BGS_EUNSUPPORTED) reduces each walked list entry's ten values over the
 * tile's pixels in a fixed order and stores them in the entry's own slot
 * instead of adding them with atomics (the wave-level pre-reduction of
 * backward atomics the paper cites, Sec. 3, kept, and the summation order
 * fixed); the (Gaussian, slot) pairs are sorted stably by Gaussian and one
 * wave per Gaussian sums its slots in (tile, list position) order.
 * SYNCHRONIZES the stream once, to read K = the number of walked (tile,
 * entry) pairs (sum over tiles of the largest n_contrib of the tile) into
 * *n_occ_host; K > max_occ returns BGS_ECAPACITY with nothing written.
 */
bgs_status bgs_render_bwd_det(const bgs_frame* frame, const bgs_render_cfg* cfg, int64_t P, const float* final_T,
                              const int32_t* n_contrib, const float* dL_dcolor, const float* dL_dalpha,
                              const float* dL_ddepth, float* dL_dmeans2D, float* dL_dconic_opacity, float* dL_drgb,
                              float* dL_ddepths, int64_t max_occ, int64_t* n_occ_host, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/*
 * Variant selection by measurement (the self-adaptive kernel selection of
 * Sec. 4.4, generalized): runs every forward candidate (static; one wave per
 * tile dispatched statically; pixel-wise 8x8 raster and cost-ordered; one wave
 * per 16x16 tile, raster and cost-ordered, the latter also through the
 * persistent pool; one wave per 32x32 block; hybrid; Gaussian-wise) on
 * `frame` with base's background, times each with HIP events (one warm-up,
 * two timed runs) and returns the fastest in *best_fwd; then renders once with
 * it and, if dL_dcolor and the gradient buffers are given, times the backward
 * candidates (static; wave per tile dispatched statically; balanced 8x8
 * raster and cost-ordered; wave per 16x16 tile, raster and cost-ordered, the
 * latter also through the persistent pool and with split walks; wave per
 * 32x32 block) into *best_bwd.  With BGS_FLAG_PACKED_GRADS in base the
 * backward candidates run on packed gradient records passed in dL_dmeans2D
 * (dL_dconic_opacity and dL_drgb null), and *best_bwd carries the flag.  The
 * output and gradient buffers are scratch (the gradients end up holding sums
 * of several runs).  When cache_path (HOST string, nullable) names a file,
 * the winners are appended to it under a workload signature (image size and
 * log2 buckets of the pair count and of the median / 99th percentile /
 * largest tile list), and a later call with a matching signature returns the
 * cached winners without timing.  fwd_ms / bwd_ms (HOST, nullable) receive the
 * winners' times (cached values on a hit; bwd -1 when not tuned).
 * SYNCHRONIZES the stream.
 */
bgs_status bgs_autotune(const bgs_frame* frame, const bgs_render_cfg* base, float* out_color, float* out_alpha,
                        float* out_depth, float* final_T, int32_t* n_contrib, const float* dL_dcolor,
                        float* dL_dmeans2D, float* dL_dconic_opacity, float* dL_drgb, void* ws, size_t ws_bytes,
                        const char* cache_path, bgs_render_cfg* best_fwd, bgs_render_cfg* best_bwd, float* fwd_ms,
                        float* bwd_ms, hipStream_t stream);

/* Per-view buffers of a batched plan (all DEVICE pointers, caller-owned). */
typedef struct bgs_view_io {
    int64_t P;                  /* Gaussians of this view's frame (size of the gradient arrays) */
    float* out_color;           /* [3][H][W] */
    float* out_alpha;           /* [H][W] */
    float* out_depth;           /* [H][W] */
    float* final_T;             /* [H][W] */
    int32_t* n_contrib;         /* [H][W] */
    const float* dL_dcolor;     /* [3][H][W] upstream gradient */
    const float* dL_dalpha;     /* [H][W] or NULL */
    const float* dL_ddepth;     /* [H][W] or NULL */
    float* dL_dmeans2D;         /* [P][2]   zeroed and accumulated by every launch */
    float* dL_dconic_opacity;   /* [P][4]   (16-byte aligned) */
    float* dL_drgb;             /* [P][3] */
    float* dL_ddepths;          /* [P] or NULL */
} bgs_view_io;

typedef struct bgs_plan bgs_plan;

/*
 * Batched multi-view render: records, into one hipGraph, the gradient
 * zero-fill, the cost pass and queue build of a cross-view work queue (every
 * work item of every view, heaviest first across views), one persistent
 * balanced forward over all views, the backward queue, and one persistent
 * backward over all views.  frames / io are HOST arrays of n_views (1..64)
 * entries; the device buffers they point to must stay valid (their contents
 * may change between launches, e.g. per-tile lists rebuilt in place).
 * cfg_fwd and cfg_bwd (nullable: same as cfg_fwd) must select
 * BGS_BALANCED_PIXEL with subtile 8 or 16; each gives its pass's queue order,
 * cfg_fwd the background.  Other variants return
 * BGS_EUNSUPPORTED.  The plan owns its queue memory and graph
 * (allocated here, freed by bgs_plan_destroy).  The graph is recorded on a
 * private stream; `stream` only receives the descriptor uploads and is
 * synchronized.
 */
bgs_status bgs_plan_create(bgs_plan** plan, int32_t n_views, const bgs_frame* frames, const bgs_view_io* io,
                           const bgs_render_cfg* cfg_fwd, const bgs_render_cfg* cfg_bwd, hipStream_t stream);

/* One forward + backward over all views of the plan: a single hipGraphLaunch
 * on `stream` (asynchronous). */
bgs_status bgs_plan_launch(bgs_plan* plan, hipStream_t stream);

/* Frees the plan (NULL is accepted). */
void bgs_plan_destroy(bgs_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* BGS_H */
