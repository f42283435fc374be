// Forward and backward alpha-compositing render of the 3DGS tile rasterizer,
// Eq. (4) of Balanced 3DGS (Sec. 2.1) with the skip / stop rules of the
// paper's naive per-pixel loop (Appendix), and its load-balanced scheduling
// (Sec. 4.1-4.3) re-designed for CDNA4 wave64:
//
//  * k_fwd_static   - the baseline: one 256-lane workgroup per 16x16 tile,
//                     grid-static dispatch, 256-Gaussian LDS batches, the
//                     workgroup leaves once every pixel has stopped.
//  * k_fwd_pixel    - persistent workgroups; every wave is an independent
//                     worker that takes one 8x8 sub-tile (64 pixels = one
//                     pixel per lane) at a time from a global atomic counter
//                     (the task pool of Sec. 4.1 at the finer grain of
//                     Sec. 4.3), stages its tile's Gaussians 64 at a time in
//                     its own LDS slice and leaves the item as soon as a
//                     ballot shows all 64 pixels stopped.
//  * k_bwd_pixel    - the backward over the same queue: per pixel back to
//                     front from n_contrib, T recovered by division, the
//                     per-Gaussian gradients of the 64 lanes summed in
//                     registers with DPP before one set of float atomics per
//                     (Gaussian, sub-tile).
//
// All kernels are FP32-VALU bound (no dense contraction).  Per examined
// (pixel, Gaussian) pair the forward spends ~22 VALU issues, the backward
// ~45 plus the wave reduction.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include <rocprim/block/block_scan.hpp>

#include "common.h"

namespace bgs {

constexpr int NBUCKET = 136;         // cost buckets: 0 and quarter-octaves of 1 .. 2^33
static_assert(NBUCKET <= 3 * 64, "k_queue_deal scans three buckets per lane");
constexpr int HYBRID_SWITCH = 16;    // hybrid: Gaussian-wise once <= 16 of 64 pixels are active
constexpr int WQ = 4;                // pixels per lane of the wave-per-tile kernels

struct FrameArgs {
    int W, H, TX, TY, n_tiles;
    const uint32_t* __restrict__ ranges;
    const uint32_t* __restrict__ point_list;
    const float2* __restrict__ means2D;
    const float4* __restrict__ conic_opacity;
    const float* __restrict__ rgb;
    const float* __restrict__ depth;
    float bg0, bg1, bg2;
    uint64_t* trace;  // per-wave timing records (nullable), trace_cap of them
    int64_t trace_cap;
    int* n_examined;  // optional per-pixel count of examined list entries (forward)
    uint32_t list_cap;        // lists capped at this many entries per tile (0: whole lists)
    uint32_t* list_overflow;  // set when a pixel runs off a capped list (nullable)
    uint32_t* item_claims;    // per-item claim counts of the task pool (nullable)
};

struct FwdOut {
    float* __restrict__ color;
    float* __restrict__ alpha;
    float* __restrict__ depth;
    float* __restrict__ final_T;
    int* __restrict__ n_contrib;
};

struct BwdIO {
    const float* __restrict__ final_T;
    const int* __restrict__ n_contrib;
    const float* __restrict__ dL_dcolor;
    const float* __restrict__ dL_dalpha;
    const float* __restrict__ dL_ddepth;
    float* __restrict__ g_means2D;
    float* __restrict__ g_conic_opacity;
    float* __restrict__ g_rgb;
    float* __restrict__ g_depth;
    // deterministic backward only: one 10-float partial per (tile, walked
    // entry), at slot det_base[tile] + entry
    float* __restrict__ det_partials;
    const uint32_t* __restrict__ det_base;
    // split walks only: the forward's out_color [3][H][W] and out_depth [H][W]
    const float* __restrict__ out_color;
    const float* __restrict__ out_depth;
    // 1: the gradients are 16-float records, g_means2D the record array
    // (GRAD_RECORD layout) and the other three pointers null
    int packed;
};


// One view of a batched plan: its frame, forward outputs and backward I/O.
struct ViewDesc {
    FrameArgs F;
    FwdOut O;
    BwdIO B;
    int64_t P;
};

// Items carry their view in the top bits: item = view << 26 | tile << 2 | sub.
constexpr int VIEW_SHIFT = 26;
constexpr uint32_t LOCAL_MASK = (1u << VIEW_SHIFT) - 1u;
constexpr int MAX_VIEWS = 64;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Optional per-wave timing records for load-balance measurements: record
// w = (3 words) hardware location + 1 (XCC id << 8 | HW_ID bits 15:8, i.e.
// shader engine, shader array and CU; 0 = no record), then the 100 MHz
// real-time counter at the wave's start and end.  Off (one uniform branch)
// when F.trace is null.
__device__ __forceinline__ uint64_t trace_begin(const FrameArgs& F) {
    return F.trace ? __builtin_amdgcn_s_memrealtime() : 0ull;
}

__device__ __forceinline__ void trace_end(const FrameArgs& F, uint64_t t0, int wave_index, int lane) {
    if (F.trace && lane == 0 && wave_index < F.trace_cap) {
        const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
        const uint32_t xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
        uint64_t* r = F.trace + 3 * (int64_t)wave_index;
        r[0] = ((uint64_t)(xcc & 0xFF) << 8 | ((hw >> 8) & 0xFF)) + 1;
        r[1] = t0;
        r[2] = __builtin_amdgcn_s_memrealtime();
    }
}

// Load one Gaussian of the list into registers in the staged form: co =
// (a2, r, q2, opacity) of splat_power2, cd = (rgb, depth).
__device__ __forceinline__ void load_splat(const FrameArgs& F, uint32_t g, float2& xy, float4& co, float4& cd) {
    xy = F.means2D[g];
    const float4 c = F.conic_opacity[g];
    const float3 s = stage_conic(c.x, c.y, c.z);
    co = make_float4(s.x, s.y, s.z, c.w);
    cd = make_float4(F.rgb[3 * g], F.rgb[3 * g + 1], F.rgb[3 * g + 2], F.depth[g]);
}

struct Pix {
    float T, C0, C1, C2, D;
    int last;
    bool done;
};

// One list entry at list position pos (0-based) for one pixel.  Branch-free:
// a skipped or stopping entry blends with weight 0 and leaves T unchanged.
// Callers stop calling once s.done is set.
__device__ __forceinline__ void blend(float fx, float fy, float2 xy, float4 co, float4 cd, int pos, Pix& s) {
    const float dx = fx - xy.x, dy = fy - xy.y;
    const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
    const float alpha = fminf(ALPHA_MAX, co.w * exp2_fast(p2));
    const bool skip = (p2 > 0.0f) | (alpha < ALPHA_MIN);
    const float w = alpha * s.T;
    const float Tn = s.T - w;
    const bool stop = !skip & (Tn < T_MIN);
    const bool take = !skip & !stop;
    const float we = take ? w : 0.0f;
    s.C0 = __builtin_fmaf(cd.x, we, s.C0);
    s.C1 = __builtin_fmaf(cd.y, we, s.C1);
    s.C2 = __builtin_fmaf(cd.z, we, s.C2);
    s.D = __builtin_fmaf(cd.w, we, s.D);
    s.T = take ? Tn : s.T;
    s.last = take ? pos + 1 : s.last;
    s.done = s.done | stop;
}

// blend() for an entry of an unrolled group: a pixel that stopped earlier in
// the group is left as it is.
__device__ __forceinline__ void blend_masked(float fx, float fy, float2 xy, float4 co, float4 cd, int pos, Pix& s) {
    const float dx = fx - xy.x, dy = fy - xy.y;
    const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
    const float alpha = fminf(ALPHA_MAX, co.w * exp2_fast(p2));
    const bool skip = (p2 > 0.0f) | (alpha < ALPHA_MIN) | s.done;
    const float w = alpha * s.T;
    const float Tn = s.T - w;
    const bool stop = !skip & (Tn < T_MIN);
    const bool take = !skip & !stop;
    const float we = take ? w : 0.0f;
    s.C0 = __builtin_fmaf(cd.x, we, s.C0);
    s.C1 = __builtin_fmaf(cd.y, we, s.C1);
    s.C2 = __builtin_fmaf(cd.z, we, s.C2);
    s.D = __builtin_fmaf(cd.w, we, s.D);
    s.T = take ? Tn : s.T;
    s.last = take ? pos + 1 : s.last;
    s.done = s.done | stop;
}

// One pixel over cnt LDS-staged entries (list positions pos0 ..), in groups of
// four so that the LDS reads of a group share one address register; the
// pixel leaves at the first group boundary after it stops.  Same arithmetic
// per entry as blend(), so the result is bit-identical.
__device__ __forceinline__ void blend_batch(float fx, float fy, const float2* __restrict__ xy,
                                            const float4* __restrict__ co, const float4* __restrict__ cd, int cnt,
                                            int pos0, Pix& s) {
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
        if (s.done) return;
#pragma unroll
        for (int u = 0; u < 4; ++u) blend_masked(fx, fy, xy[j + u], co[j + u], cd[j + u], pos0 + j + u, s);
    }
    for (; j < cnt; ++j) {
        if (s.done) return;
        blend(fx, fy, xy[j], co[j], cd[j], pos0 + j, s);
    }
}

__device__ __forceinline__ void write_pixel(const FrameArgs& F, const FwdOut& O, int px, int py, const Pix& s) {
    const int64_t HW = (int64_t)F.W * F.H;
    const int64_t p = (int64_t)py * F.W + px;
    O.color[p] = s.C0 + s.T * F.bg0;
    O.color[HW + p] = s.C1 + s.T * F.bg1;
    O.color[2 * HW + p] = s.C2 + s.T * F.bg2;
    O.alpha[p] = 1.0f - s.T;
    O.depth[p] = s.D;
    O.final_T[p] = s.T;
    O.n_contrib[p] = s.last;
    if (F.list_cap && F.list_overflow && !s.done) {  // ran to the end of its list without stopping
        const int64_t t = (int64_t)(py / TILE) * F.TX + px / TILE;
        if (F.ranges[2 * t + 1] - F.ranges[2 * t] >= F.list_cap) *F.list_overflow = 1u;
    }
}

// ------------------------------------------------------------------ static
__global__ __launch_bounds__(256) void k_fwd_static(FrameArgs F, FwdOut O) {
    const uint64_t t_begin = trace_begin(F);
    __shared__ float2 s_xy[256];
    __shared__ float4 s_co[256];
    __shared__ float4 s_cd[256];
    const int tile = blockIdx.x;
    const int tx = tile % F.TX, ty = tile / F.TX;
    const int px = tx * TILE + (threadIdx.x & 15), py = ty * TILE + (threadIdx.x >> 4);
    const bool inside = px < F.W && py < F.H;
    const uint32_t start = F.ranges[2 * tile], end = F.ranges[2 * tile + 1];
    Pix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
    const float fx = (float)px, fy = (float)py;
    for (uint32_t base = start; base < end; base += 256) {
        if (__syncthreads_count(s.done) == 256) break;
        const uint32_t k = base + threadIdx.x;
        if (k < end) {
            float2 xy; float4 co, cd;
            load_splat(F, F.point_list[k], xy, co, cd);
            s_xy[threadIdx.x] = xy;
            s_co[threadIdx.x] = co;
            s_cd[threadIdx.x] = cd;
        }
        __syncthreads();
        const int cnt = (int)min(256u, end - base);
        const int pos0 = (int)(base - start);
        blend_batch(fx, fy, s_xy, s_co, s_cd, cnt, pos0, s);
    }
    if (inside) write_pixel(F, O, px, py, s);
    trace_end(F, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// ------------------------------------------------------------- balanced fwd
// Item id = tile * 4 + quadrant (8x8 sub-tile of the 16x16 tile).
__device__ __forceinline__ void item_pixel(const FrameArgs& F, uint32_t item, int lane, int& tile, int& px, int& py,
                                           bool& any_inside) {
    tile = (int)(item >> 2);
    const int sub = (int)(item & 3);
    const int tx = tile % F.TX, ty = tile / F.TX;
    const int ox = tx * TILE + (sub & 1) * 8, oy = ty * TILE + (sub >> 1) * 8;
    px = ox + (lane & 7);
    py = oy + (lane >> 3);
    any_inside = ox < F.W && oy < F.H;
}

// Raw (unscaled) splat data of one list entry, held in registers while it is
// in flight.
struct SplatRegs {
    float2 xy;
    float4 co;
    float4 cd;
};

__device__ __forceinline__ void gather_splat(const FrameArgs& F, bool valid, uint32_t g, SplatRegs& r) {
    if (valid) load_splat(F, g, r.xy, r.co, r.cd);
}

// ---------------------------------------------------------------- work queue
// The task pool is NQ = 64 queues, each with its own fetch counter in its own
// 128-byte line.  Tiles are ranked by cost (heaviest first) and dealt
// round-robin to 16 groups of 4 queues; the 4 8x8 sub-tiles of a tile go to
// the 4 queues of its group.  A wave's home queue is (global wave id) mod 64;
// because workgroups are dispatched to the 8 XCDs round-robin, the 4 waves of
// a workgroup share one group, so a tile's sub-tiles stay on one XCD's L2.
// A wave whose queue is empty reads all 64 counters with one vector load
// (lane q reads counter q), picks the next non-empty queue and claims from it;
// it leaves when none is left.  One global counter serving every wave of all
// 8 XCDs was the bottleneck of the first design (same-address device atomics
// serialize), so the counters are spread over 64 lines.
constexpr int NQ = 64;
constexpr int QSTRIDE = 32;  // u32 words between two counters (128 bytes)
constexpr int QGROUPS = NQ / 4;

// First round without atomics: wave w of the persistent grid (nw waves) takes
// items[w] -- entry w / 64 of its home queue w mod 64 -- directly, so the
// first nw items cost no counter round trip.  A claim from queue q then draws
// t from the counter and takes entry t + first(q), first(q) = the number of
// waves whose home is q.  The offset comes from the launch itself (gridDim),
// so a queue is valid for any persistent grid; the counters start at 0.
struct WorkQueue {
    uint32_t* ctr;           // ctr[q * QSTRIDE], q < NQ; ctr[NQ * QSTRIDE] = number of items
    const uint32_t* items;   // items[i * NQ + q] = i-th item of queue q
    uint32_t* claims;        // claims[item] += 1 per claim (nullable; one-view launches only)
    uint32_t n;              // number of items
    uint32_t nw;             // waves of the persistent grid
    uint32_t nt;             // tiles of the frame (claim index of split walks' upper parts)
    int cur;
    __device__ __forceinline__ uint32_t size(int q) const { return n > (uint32_t)q ? (n - q - 1) / NQ + 1 : 0u; }
    __device__ __forceinline__ uint32_t first(int q) const { return nw > (uint32_t)q ? (nw - q - 1) / NQ + 1 : 0u; }
};

__device__ __forceinline__ WorkQueue make_queue(uint32_t* ctr, const uint32_t* items, int wave_global,
                                                uint32_t* claims = nullptr, uint32_t n_tiles = 0) {
    WorkQueue Q;
    Q.nt = n_tiles;
    Q.ctr = ctr;
    Q.items = items;
    Q.claims = claims;
    Q.n = ctr[NQ * QSTRIDE];
    Q.nw = gridDim.x * (blockDim.x / WAVE);
    Q.cur = wave_global & (NQ - 1);
    if (claims && wave_global == 0 && (threadIdx.x & (WAVE - 1)) == 0) ctr[NQ * QSTRIDE + 1] = Q.nw;  // for audits
    return Q;
}

__device__ __forceinline__ void note_claim(const WorkQueue& Q, int lane, uint32_t item) {
    if (Q.claims && lane == 0) {
        // one-view items: tile + unit * n_tiles (unit 0 for sub-tile and block items)
        atomicAdd(&Q.claims[(item & ((1u << 24) - 1u)) + (item >> 24) * Q.nt], 1u);
    }
}

// Item `rank` of the dealt list for a wave of a plain grid (the dealt items
// handed out by the hardware's workgroup dispatcher, lowest rank first):
// false past the item count.  With claims, lane 0 counts the claim as
// note_claim does.
__device__ __forceinline__ bool grid_item(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ items,
                                          uint32_t rank, uint32_t* claims, uint32_t n_tiles, int lane,
                                          uint32_t& item) {
    if (rank >= __builtin_amdgcn_readfirstlane(ctr[NQ * QSTRIDE])) return false;
    item = __builtin_amdgcn_readfirstlane(items[rank]);
    if (claims && lane == 0) atomicAdd(&claims[(item & ((1u << 24) - 1u)) + (item >> 24) * n_tiles], 1u);
    return true;
}

// Counter value t of queue q -> the item, if q still holds one.
__device__ __forceinline__ bool queue_slot(const WorkQueue& Q, int q, uint32_t t, int lane, uint32_t& item) {
    const uint32_t i = t + Q.first(q);
    if (i >= Q.size(q)) return false;
    item = __builtin_amdgcn_readfirstlane(Q.items[(size_t)i * NQ + q]);
    note_claim(Q, lane, item);
    return true;
}

// Every queue's home counter has run past its size: probe all 64 counters
// with one vector load (lane q reads counter q), move to the next non-empty
// queue and claim from it; false once every queue is drained.  Counters only
// grow, so the exit is final.
__device__ __forceinline__ bool queue_steal(WorkQueue& Q, int lane, uint32_t& item) {
    for (;;) {
        const uint32_t c = __hip_atomic_load(&Q.ctr[lane * QSTRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t m = ballot(c + Q.first(lane) < Q.size(lane));
        if (m == 0) return false;
        const uint64_t rot = Q.cur ? ((m >> Q.cur) | (m << (64 - Q.cur))) : m;
        Q.cur = (Q.cur + (int)__builtin_ctzll(rot)) & (NQ - 1);
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&Q.ctr[Q.cur * QSTRIDE], 1u);
        if (queue_slot(Q, Q.cur, __builtin_amdgcn_readfirstlane(t), lane, item)) return true;
    }
}

// Claim the next item for this wave (all 64 lanes active); false when every
// queue is drained.
__device__ __forceinline__ bool queue_next(WorkQueue& Q, int lane, uint32_t& item) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&Q.ctr[Q.cur * QSTRIDE], 1u);
    if (queue_slot(Q, Q.cur, __builtin_amdgcn_readfirstlane(t), lane, item)) return true;
    return queue_steal(Q, lane, item);
}

// The wave's first item: its own slot of the first round, else a claim.
__device__ __forceinline__ bool queue_first(WorkQueue& Q, int wave_global, int lane, uint32_t& item) {
    if ((uint32_t)wave_global < Q.n) {
        item = __builtin_amdgcn_readfirstlane(Q.items[wave_global]);
        note_claim(Q, lane, item);
        return true;
    }
    return queue_next(Q, lane, item);
}

template <bool PERSISTENT, bool MV = false>
__global__ __launch_bounds__(256) void k_fwd_pixel(FrameArgs F0, FwdOut O0, const ViewDesc* __restrict__ views,
                                                   const uint32_t* __restrict__ items, uint32_t* __restrict__ ctr) {
    const uint64_t t_begin = trace_begin(F0);
    __shared__ float2 s_xy[4][64];
    __shared__ float4 s_co[4][64];
    __shared__ float4 s_cd[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WorkQueue Q;
    if (PERSISTENT) Q = make_queue(ctr, items, blockIdx.x * 4 + wv, MV ? nullptr : F0.item_claims);
    bool first = true;
    for (;;) {
        uint32_t item;
        if (PERSISTENT) {
            if (!(first ? queue_first(Q, blockIdx.x * 4 + wv, lane, item) : queue_next(Q, lane, item))) break;
            first = false;
        } else {
            item = blockIdx.x * 4 + wv;
        }
        const FrameArgs F = MV ? views[item >> VIEW_SHIFT].F : F0;
        const FwdOut O = MV ? views[item >> VIEW_SHIFT].O : O0;
        item &= LOCAL_MASK;
        int tile, px, py;
        bool any_inside;
        item_pixel(F, item, lane, tile, px, py, any_inside);
        if (any_inside) {
            const bool inside = px < F.W && py < F.H;
            const uint32_t start = F.ranges[2 * tile], end = F.ranges[2 * tile + 1];
            Pix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
            const float fx = (float)px, fy = (float)py;
            // two-stage prefetch: ids two chunks ahead, splat data one chunk ahead
            SplatRegs cur{}, nxt{};
            {
                const uint32_t k0 = start + lane;
                gather_splat(F, k0 < end, k0 < end ? F.point_list[k0] : 0u, cur);
            }
            uint32_t k1 = start + 64 + lane;
            uint32_t id1 = k1 < end ? F.point_list[k1] : 0u;
            for (uint32_t base = start; base < end; base += 64) {
                if (ballot(!s.done) == 0) break;
                s_xy[wv][lane] = cur.xy;
                s_co[wv][lane] = cur.co;
                s_cd[wv][lane] = cur.cd;
                wave_sync();
                gather_splat(F, k1 < end, id1, nxt);
                k1 += 64;
                id1 = k1 < end ? F.point_list[k1] : 0u;
                const int cnt = (int)min(64u, end - base);
                const int pos0 = (int)(base - start);
                blend_batch(fx, fy, s_xy[wv], s_co[wv], s_cd[wv], cnt, pos0, s);
                wave_sync();
                cur = nxt;
            }
            if (inside) write_pixel(F, O, px, py, s);
        }
        if (!PERSISTENT) break;
    }
    trace_end(F0, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// --------------------------------------------------- Gaussian-wise / hybrid
// Gaussian-wise mode (Sec. 4.2, Alg. 2 and 6): the 64 lanes hold 64
// consecutive list entries and one pixel is blended at a time.  Each entry's
// transmittance factor (1 - alpha, or 1 for a skipped entry) goes through an
// inclusive product scan across the wave; the first non-skipped lane whose
// T_in * prefix drops below 1e-4 stops the pixel (that entry is not blended),
// entries before it blend with weight alpha * T_in * (exclusive prefix), and
// the weighted colour/depth are summed across the wave.  The pixel's state
// lives in lane p, which is exactly where the pixel-wise mode keeps it, so the
// hybrid switches a wave from pixel-wise to Gaussian-wise at a chunk boundary
// once few of its 64 pixels are still active (the stragglers then no longer
// hold 64 lanes hostage).

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_or(float v, float identity) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                                                 __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                                 false));
}

// inclusive product over lanes 0..lane (all 64 lanes active)
__device__ __forceinline__ float wave_incl_prod(float x) {
    x *= dpp_or<0x111>(x, 1.0f);        // row_shr:1
    x *= dpp_or<0x112>(x, 1.0f);        // row_shr:2
    x *= dpp_or<0x114>(x, 1.0f);        // row_shr:4
    x *= dpp_or<0x118>(x, 1.0f);        // row_shr:8   -> prefix within each row of 16
    x *= dpp_or<0x142, 0xA>(x, 1.0f);   // row_bcast:15 -> rows 1, 3 include the previous row
    x *= dpp_or<0x143, 0xC>(x, 1.0f);   // row_bcast:31 -> rows 2, 3 include rows 0-1
    return x;
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Pixel p (state in lane p of s) blends the 64 entries the lanes hold; pos0 is
// the list position of lane 0.  Clears bit p of act when the pixel stops.
__device__ __forceinline__ void gw_step(float fx, float fy, float2 xy, float4 co, float4 cd, bool valid, int lane,
                                        int p, int pos0, Pix& s, uint64_t& act) {
    const float dx = fx - xy.x, dy = fy - xy.y;
    const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
    const float alpha = fminf(ALPHA_MAX, co.w * exp2_fast(p2));
    const bool take = valid & !((p2 > 0.0f) | (alpha < ALPHA_MIN));
    const float incl = wave_incl_prod(take ? 1.0f - alpha : 1.0f);
    float excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 1.0f;
    const float Tin = readlane_f(s.T, p);
    const float Tafter = Tin * incl;
    const uint64_t stopm = ballot(take & (Tafter < T_MIN));
    const int f = stopm ? (int)__builtin_ctzll(stopm) : 64;
    const bool contrib = take & (lane < f);
    const float Tbefore = Tin * excl;
    const float w = contrib ? alpha * Tbefore : 0.0f;
    const float c0 = wave_sum(w * cd.x), c1 = wave_sum(w * cd.y), c2 = wave_sum(w * cd.z), dd = wave_sum(w * cd.w);
    const uint64_t cm = ballot(contrib);
    const float Tout = stopm ? readlane_f(Tbefore, f) : readlane_f(Tafter, 63);
    if (lane == p) {
        s.T = Tout;
        s.C0 += c0;
        s.C1 += c1;
        s.C2 += c2;
        s.D += dd;
        if (cm) s.last = pos0 + 64 - (int)__builtin_clzll(cm);
        if (stopm) s.done = true;
    }
    if (stopm) act &= ~(1ull << p);
}

// SWITCH_AT = 64: Gaussian-wise from the first chunk; otherwise pixel-wise
// while more than SWITCH_AT pixels of the wave are active.
template <int SWITCH_AT>
__global__ __launch_bounds__(256) void k_fwd_hybrid(FrameArgs F, FwdOut O, const uint32_t* __restrict__ items,
                                                    uint32_t* __restrict__ ctr) {
    const uint64_t t_begin = trace_begin(F);
    __shared__ float2 s_xy[4][64];
    __shared__ float4 s_co[4][64];
    __shared__ float4 s_cd[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WorkQueue Q = make_queue(ctr, items, blockIdx.x * 4 + wv, F.item_claims);
    for (bool first = true;; first = false) {
        uint32_t item;
        if (!(first ? queue_first(Q, blockIdx.x * 4 + wv, lane, item) : queue_next(Q, lane, item))) break;
        int tile, px, py;
        bool any_inside;
        item_pixel(F, item, lane, tile, px, py, any_inside);
        if (!any_inside) continue;
        const bool inside = px < F.W && py < F.H;
        const uint32_t start = F.ranges[2 * tile], end = F.ranges[2 * tile + 1];
        Pix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
        const float fx = (float)px, fy = (float)py;
        const int ox = px - (lane & 7), oy = py - (lane >> 3);
        uint32_t base = start;
        for (; base < end; base += 64) {  // pixel-wise phase
            const uint64_t act = ballot(!s.done);
            if (act == 0 || __builtin_popcountll(act) <= SWITCH_AT) break;
            const uint32_t k = base + lane;
            if (k < end) {
                float2 xy; float4 co, cd;
                load_splat(F, F.point_list[k], xy, co, cd);
                s_xy[wv][lane] = xy;
                s_co[wv][lane] = co;
                s_cd[wv][lane] = cd;
            }
            wave_sync();
            const int cnt = (int)min(64u, end - base);
            const int pos0 = (int)(base - start);
            blend_batch(fx, fy, s_xy[wv], s_co[wv], s_cd[wv], cnt, pos0, s);
            wave_sync();
        }
        uint64_t act = ballot(!s.done);
        for (; base < end && act; base += 64) {  // Gaussian-wise phase
            const uint32_t k = base + lane;
            const bool valid = k < end;
            float2 xy = make_float2(0.f, 0.f);
            float4 co = make_float4(0.f, 0.f, 0.f, 0.f), cd = co;
            if (valid) load_splat(F, F.point_list[k], xy, co, cd);
            const int pos0 = (int)(base - start);
            uint64_t todo = act;
            while (todo) {
                const int p = (int)__builtin_ctzll(todo);
                todo &= todo - 1;
                gw_step((float)(ox + (p & 7)), (float)(oy + (p >> 3)), xy, co, cd, valid, lane, p, pos0, s, act);
            }
        }
        if (inside) write_pixel(F, O, px, py, s);
    }
    trace_end(F, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// ------------------------------------------------- tile-granular persistent
// Persistent waves take whole 16x16 tiles from the queue (the inter-block
// dynamic distribution of Sec. 4.1, Alg. 1, with a wave as the worker):
// lane l owns the four pixels (l mod 16, l / 16 + 4q), q = 0..3, so pixel
// row q of the lanes forms the 16x4 block q.  One wave per tile loads the
// tile's list once (four 8x8 waves load it four times, a 256-lane workgroup
// synchronizes its four waves per batch), and each staged entry is read from
// LDS once for four pixels.
//
// Per list entry the wave works at the granularity of a block, on uniform
// (scalar) branches only:
//  * staging computes, per entry, the 4-bit mask of the blocks that the
//    entry's alpha >= 1/255 ellipse can reach (block_mask); a block outside
//    it skips the entry without evaluating it, since every one of its pixels
//    would skip it anyway;
//  * a block whose 64 pixels have all stopped leaves the walk, the wave
//    leaves once all four have;
//  * a block evaluates the entry's exponent and alpha and, only if one of its
//    pixels takes the entry, the blend (blend_u).
// Per pixel the arithmetic is that of blend(), so every variant gives the
// same image bit for bit.

// Global-memory form of one list entry, loaded without any arithmetic so that
// the loads of the next chunk stay in flight while the wave renders this one.
struct RawSplat {
    float2 xy;
    float4 con;  // a, b, c, opacity
    float r, g, b, d;
    uint32_t id;
};

__device__ __forceinline__ void load_raw(const FrameArgs& F, uint32_t id, RawSplat& s) {
    s.xy = F.means2D[id];
    s.con = F.conic_opacity[id];
    s.r = F.rgb[3 * (size_t)id];
    s.g = F.rgb[3 * (size_t)id + 1];
    s.b = F.rgb[3 * (size_t)id + 2];
    s.d = F.depth[id];
    s.id = id;
}

// Bit q (q = 0..3) is set when the 16x4 pixel block of rows y0 + 4q ..
// y0 + 4q + 3, columns x0 .. x0 + 15, meets the bounding box of the entry's
// ellipse {d : a dx^2 + 2 b dx dy + c dy^2 <= tau}, tau = 2 ln(255 o): outside
// it alpha = o exp(-q(d) / 2) < 1/255 and every pixel skips the entry.  The box
// half-extents sqrt(tau c / det), sqrt(tau a / det) are padded (tau by 2^-8
// relative and absolute, the extents by 2^-10 relative and 1/64 px) far beyond
// the few-ulp error of the fp32 exponent, so a clear bit never hides a pixel
// that blends.  A conic that is not positive definite (or NaN) gets all four
// bits; opacity below 1/255 with a positive-definite conic gets none
// (alpha <= o there).
__device__ __forceinline__ uint32_t block_mask(float u, float v, float a, float b, float c, float o, int x0,
                                               int y0) {
    const float bb = b * b;
    const float bb_err = __builtin_fmaf(b, b, -bb);
    const float det = __builtin_fmaf(a, c, -bb) - bb_err;
    if (!(a > 0.0f && det > 0.0f)) return 0xFu;
    if (!(o >= ALPHA_MIN)) return 0u;
    constexpr float TWO_LN2 = 1.3862943611198906f;
    constexpr float PAD = 1.0f / 256.0f;
    const float tau = __builtin_fmaf(TWO_LN2 * __builtin_amdgcn_logf(255.0f * o), 1.0f + PAD, PAD);
    const float inv_det = 1.0f / det;
    const float ex = __builtin_sqrtf(tau * c * inv_det) * (1.0f + 1.0f / 1024.0f) + 1.0f / 64.0f;
    const float ey = __builtin_sqrtf(tau * a * inv_det) * (1.0f + 1.0f / 1024.0f) + 1.0f / 64.0f;
    if (u + ex < (float)x0 || u - ex > (float)(x0 + TILE - 1)) return 0u;
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        const float r0 = (float)(y0 + 4 * q), r1 = r0 + 3.0f;
        if (!(v + ey < r0) && !(v - ey > r1)) m |= 1u << q;
    }
    return m;
}

// Work items of the wave-per-tile kernels.  A one-view item is a tile id
// (bits 0-23) and a unit u (bits 24-27) naming the part of the tile's work it
// covers: u = 0 the whole tile; u = 1 / 2 the lower / upper part of its
// backward walk (split walks, below); u = 3 + q block q alone, the 16x4
// pixels of pixel row q of the lanes; u = 7 + 2q + p part p of block q's walk.
// The queue builder deals a tile whose cost reaches BLOCK_MIN as four block
// items -- four waves instead of one on the tile's critical path (the finer
// tasks of Sec. 4.3, used only where a tile would otherwise dominate the
// kernel) -- and, with split walks, a backward walk of SPLIT_MIN entries or
// more as two parts.  The tile id space is 24 bits (at most 16.7 M tiles).
constexpr uint32_t ITEM_TILE = (1u << 24) - 1u;
constexpr int UNIT_SHIFT = 24;
constexpr int SPLIT_MIN = 128;       // backward walks of at least this many entries split in two
constexpr int BLOCK_MIN_FWD = 256;   // forward cost estimate at which a tile becomes four block items
constexpr int BLOCK_MIN_BWD = 512;   // backward walk at which a tile becomes four block items

// Blocks an item covers (4 bits) and the part of the walk (0 whole, 1 lower, 2 upper).
__host__ __device__ __forceinline__ uint32_t unit_blocks(uint32_t u) {
    return u >= 7 ? 1u << ((u - 7) >> 1) : (u >= 3 ? 1u << (u - 3) : 0xFu);
}
__host__ __device__ __forceinline__ int unit_part(uint32_t u) {
    return u >= 7 ? 1 + (int)((u - 7) & 1u) : (u == 1 ? 1 : (u == 2 ? 2 : 0));
}

// Split point of a walk of n entries (n >= SPLIT_MIN): near n / 2, a
// multiple of 64, at least 64, below n.
__host__ __device__ __forceinline__ int split_point(int n) {
    const int k = ((n / 2 + 32) / 64) * 64;
    return k < 64 ? 64 : k;
}

// LDS slice of one wave: 64 staged entries.  xym = (x, y, block mask bits,
// Gaussian id bits), co = (a2, r, q2, opacity) of splat_power2, cd = (rgb,
// depth), abc = the raw conic (backward only).
struct WaveStage {
    float4 xym[64];
    float4 co[64];
    float4 cd[64];
};

// Stages the lane's entry and returns its block mask (0 for an invalid lane).
__device__ __forceinline__ uint32_t stage_entry(WaveStage& st, int lane, const RawSplat& r, bool valid, int x0,
                                                int y0) {
    const float3 k = stage_conic(r.con.x, r.con.y, r.con.z);
    const uint32_t m = valid ? block_mask(r.xy.x, r.xy.y, r.con.x, r.con.y, r.con.z, r.con.w, x0, y0) : 0u;
    st.xym[lane] = make_float4(r.xy.x, r.xy.y, 0.0f, __uint_as_float(r.id));
    st.co[lane] = make_float4(k.x, k.y, k.z, r.con.w);
    st.cd[lane] = make_float4(r.r, r.g, r.b, r.d);
    return m;
}

// Entries of a staged chunk per block, as 64-bit masks in scalar registers:
// bit j of mq[q] is set when chunk entry j may reach block q.
__device__ __forceinline__ void chunk_masks(uint32_t m, uint64_t (&mq)[WQ]) {
#pragma unroll
    for (int q = 0; q < WQ; ++q) mq[q] = ballot((m >> q) & 1u);
}

// Entries still to visit: those that reach a block in `live`.
__device__ __forceinline__ uint64_t chunk_todo(const uint64_t (&mq)[WQ], uint32_t live) {
    uint64_t t = 0;
#pragma unroll
    for (int q = 0; q < WQ; ++q)
        if (live & (1u << q)) t |= mq[q];
    return t;
}

// Running state of the four pixels of a lane (one per block).  Which pixels
// of block q have stopped is one 64-bit mask per block, uniform across the
// wave (scalar registers); a lane reads its own bit with inverse_ballot.
struct PixQ {
    float T[WQ], C0[WQ], C1[WQ], C2[WQ], D[WQ];
    int last[WQ], stop_at[WQ];
    uint64_t done_m[WQ];
};

__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// blend() for block q (pixel q of every lane) and one entry, with the blend
// part behind a uniform branch: the block only pays for it when one of its
// pixels takes the entry.  Same arithmetic as blend().  Returns true
// (uniform) when a pixel of the block stopped at this entry.
// Offset of the first entry of list chunk base for this lane, clamped into
// the list (lanes past the end re-read its last entry; their slots are
// staged as empty).
__device__ __forceinline__ uint32_t chunk_id(const FrameArgs& F, uint32_t base, uint32_t end, int lane) {
    const uint32_t k = base + (uint32_t)lane;
    return F.point_list[k < end ? k : end - 1];
}

// One wave renders tile `tile` of F into O.  COUNT: also n_examined.
template <bool COUNT>
__device__ __forceinline__ void fwd_tile(const FrameArgs& F, const FwdOut& O, int tile, int lane, WaveStage& st) {
    const int tx = tile % F.TX, ty = tile / F.TX;
    const int x0 = tx * TILE, y0 = ty * TILE;
    const int px = x0 + (lane & 15);
    const float fx = (float)px;
    PixQ s;
    float fy[WQ];
    uint32_t live = 0;  // blocks with a pixel still walking (uniform)
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        const int py = y0 + (lane >> 4) + 4 * q;
        fy[q] = (float)py;
        s.T[q] = 1.0f;
        s.C0[q] = s.C1[q] = s.C2[q] = s.D[q] = 0.0f;
        s.last[q] = 0;
        s.stop_at[q] = -1;
        s.done_m[q] = ~ballot(px < F.W && py < F.H);  // pixels outside the image never walk
        if (~s.done_m[q]) live |= 1u << q;
    }
    const uint32_t start = __builtin_amdgcn_readfirstlane(F.ranges[2 * tile]);
    const uint32_t end = __builtin_amdgcn_readfirstlane(F.ranges[2 * tile + 1]);
    // two-stage prefetch: ids two chunks ahead, raw splat data one chunk ahead
    RawSplat cur{}, nxt{};
    uint32_t idn = 0;
    if (start < end) {
        load_raw(F, chunk_id(F, start, end, lane), cur);
        if (start + 64 < end) idn = chunk_id(F, start + 64, end, lane);
    }
    for (uint32_t base = start; base < end && live; base += 64) {
        // the chunk's entries that reach a live block; a block that stops
        // inside the chunk computes nothing more
        uint64_t todo = ballot((stage_entry(st, lane, cur, base + lane < end, x0, y0) & live) != 0u);
        wave_sync();
        if (base + 64 < end) load_raw(F, idn, nxt);
        if (base + 128 < end) idn = chunk_id(F, base + 128, end, lane);
        const int pos0 = (int)(base - start);
        // visit them front to back; per entry every block is evaluated
        // branch-free -- the four exponents as independent chains, then the
        // blends under lane masks combined on the scalar unit -- since a
        // uniform branch per block costs the scalar unit about what it saves
        // the vector unit
        while (todo && live) {
            const int j = (int)__builtin_ctzll(todo);
            todo &= todo - 1;
            const float4 xym = st.xym[j];
            const float4 co = st.co[j];
            const float4 cd = st.cd[j];
            const float dx = fx - xym.x;
            float al[WQ], pw[WQ];
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                pw[q] = splat_power2(dx, fy[q] - xym.y, co.x, co.y, co.z);
                al[q] = fminf(ALPHA_MAX, co.w * exp2_fast(pw[q]));
            }
            uint64_t stops = 0;
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                // pixels still walking that do not skip the entry (single
                // compares as lane masks, combined on the scalar unit)
                const uint64_t cand = ballot(!(pw[q] > 0.0f)) & ballot(!(al[q] < ALPHA_MIN)) & ~s.done_m[q];
                const float w = al[q] * s.T[q];
                const float Tn = s.T[q] - w;
                const uint64_t stop = cand & ballot(Tn < T_MIN);
                const bool take = lane_bit(cand & ~stop);
                const float we = take ? w : 0.0f;
                s.C0[q] = __builtin_fmaf(cd.x, we, s.C0[q]);
                s.C1[q] = __builtin_fmaf(cd.y, we, s.C1[q]);
                s.C2[q] = __builtin_fmaf(cd.z, we, s.C2[q]);
                s.D[q] = __builtin_fmaf(cd.w, we, s.D[q]);
                s.T[q] = take ? Tn : s.T[q];
                s.last[q] = take ? pos0 + j + 1 : s.last[q];
                if (COUNT) s.stop_at[q] = lane_bit(stop) ? pos0 + j + 1 : s.stop_at[q];
                s.done_m[q] |= stop;
                stops |= stop;
            }
            if (stops) {
#pragma unroll
                for (int q = 0; q < WQ; ++q)
                    if (s.done_m[q] == ~0ull) live &= ~(1u << q);
            }
        }
        wave_sync();
        cur = nxt;
    }
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        const int py = y0 + (lane >> 4) + 4 * q;
        if (px < F.W && py < F.H) {
            write_pixel(F, O, px, py, Pix{s.T[q], s.C0[q], s.C1[q], s.C2[q], s.D[q], s.last[q], lane_bit(s.done_m[q])});
            if (COUNT)
                F.n_examined[(int64_t)py * F.W + px] = s.stop_at[q] >= 0 ? s.stop_at[q] : (int)(end - start);
        }
    }
}

// One wave renders block q of tile `tile` alone (one pixel per lane): the
// block items of heavy tiles.  The walk is fwd_tile's restricted to the
// entries whose block mask has bit q.  When a heavy tile is all that is left
// its waves are alone on their SIMDs and the walk's latency is the cost, so
// entries go in groups of FB_GROUP: their LDS reads, exponents and alphas
// are independent and overlap, and only the transmittance update runs entry
// after entry, front to back.  A group short of entries repeats its first
// one with an empty lane mask, which takes nothing (its blend adds colour
// times zero, as for every entry a pixel skips).  Same per-pixel arithmetic
// as blend().
constexpr int FB_GROUP = 4;
template <bool COUNT>
__device__ __forceinline__ void fwd_block(const FrameArgs& F, const FwdOut& O, int tile, int q, int lane,
                                          WaveStage& st) {
    constexpr int G = FB_GROUP;
    const int tx = tile % F.TX, ty = tile / F.TX;
    const int x0 = tx * TILE, y0 = ty * TILE;
    const int px = x0 + (lane & 15), py = y0 + (lane >> 4) + 4 * q;
    const float fx = (float)px, fy = (float)py;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f;
    int last = 0, stop_at = -1;
    uint64_t done_m = ~ballot(px < F.W && py < F.H);
    const uint32_t start = __builtin_amdgcn_readfirstlane(F.ranges[2 * tile]);
    const uint32_t end = __builtin_amdgcn_readfirstlane(F.ranges[2 * tile + 1]);
    RawSplat cur{}, nxt{};
    uint32_t idn = 0;
    if (start < end) {
        load_raw(F, chunk_id(F, start, end, lane), cur);
        if (start + 64 < end) idn = chunk_id(F, start + 64, end, lane);
    }
    for (uint32_t base = start; base < end && ~done_m; base += 64) {
        uint64_t todo = ballot((stage_entry(st, lane, cur, base + lane < end, x0, y0) >> q) & 1u);
        wave_sync();
        if (base + 64 < end) load_raw(F, idn, nxt);
        if (base + 128 < end) idn = chunk_id(F, base + 128, end, lane);
        const int pos0 = (int)(base - start) + 1;
        while (todo && ~done_m) {
            int j[G];
            uint64_t use[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const bool has = todo != 0;
                j[k] = has ? (int)__builtin_ctzll(todo) : j[0];
                use[k] = has ? ~0ull : 0ull;
                todo &= todo - 1;
            }
            float4 xym[G], co[G], cd[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                xym[k] = st.xym[j[k]];
                co[k] = st.co[j[k]];
                cd[k] = st.cd[j[k]];
            }
            float pw[G], al[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                pw[k] = splat_power2(fx - xym[k].x, fy - xym[k].y, co[k].x, co[k].y, co[k].z);
                al[k] = fminf(ALPHA_MAX, co[k].w * exp2_fast(pw[k]));
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint64_t cand = ballot(!(pw[k] > 0.0f)) & ballot(!(al[k] < ALPHA_MIN)) & ~done_m & use[k];
                const float w = al[k] * T;
                const float Tn = T - w;
                const uint64_t stop = cand & ballot(Tn < T_MIN);
                const bool take = lane_bit(cand & ~stop);
                const float we = take ? w : 0.0f;
                C0 = __builtin_fmaf(cd[k].x, we, C0);
                C1 = __builtin_fmaf(cd[k].y, we, C1);
                C2 = __builtin_fmaf(cd[k].z, we, C2);
                D = __builtin_fmaf(cd[k].w, we, D);
                T = take ? Tn : T;
                last = take ? pos0 + j[k] : last;
                if (COUNT) stop_at = lane_bit(stop) ? pos0 + j[k] : stop_at;
                done_m |= stop;
            }
        }
        wave_sync();
        cur = nxt;
    }
    if (px < F.W && py < F.H) {
        write_pixel(F, O, px, py, Pix{T, C0, C1, C2, D, last, lane_bit(done_m)});
        if (COUNT) F.n_examined[(int64_t)py * F.W + px] = stop_at >= 0 ? stop_at : (int)(end - start);
    }
}

// Tiles of a work item: TPI = 1 -> the item is a tile; TPI = 4 -> the item
// is a 32x32 block of 2x2 tiles (those inside the grid), rendered in turn.
template <int TPI>
__device__ __forceinline__ int item_tiles(const FrameArgs& F, uint32_t item, int (&tiles)[TPI]) {
    if (TPI == 1) {
        tiles[0] = (int)item;
        return 1;
    }
    const int BX = (F.TX + 1) >> 1;
    const int bx = (int)item % BX, by = (int)item / BX;
    int n = 0;
#pragma unroll
    for (int k = 0; k < TPI; ++k) {
        const int tx = 2 * bx + (k & 1), ty = 2 * by + (k >> 1);
        if (tx < F.TX && ty < F.TY) tiles[n++] = ty * F.TX + tx;
    }
    return n;
}

// PERSISTENT: waves take items from the task pool; otherwise wave w of the
// grid renders item w (grid-static dispatch of the same code).  Five waves
// per SIMD: the register budget of 96 leaves one scalar-spill register
// to memory, outside the walk.
template <bool MV = false, bool COUNT = false, bool PERSISTENT = true, int TPI = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_fwd_wide(
    FrameArgs F0, FwdOut O0, const ViewDesc* __restrict__ views, const uint32_t* __restrict__ items,
    uint32_t* __restrict__ ctr, uint32_t n_static) {
    const uint64_t t_begin = trace_begin(F0);
    __shared__ WaveStage s_st[4];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    WorkQueue Q;
    if (PERSISTENT) Q = make_queue(ctr, items, blockIdx.x * 4 + wv, MV ? nullptr : F0.item_claims, (uint32_t)F0.n_tiles);
    for (bool first = true;; first = false) {
        uint32_t item;
        if (PERSISTENT) {
            if (!(first ? queue_first(Q, blockIdx.x * 4 + wv, lane, item) : queue_next(Q, lane, item))) break;
        } else {
            item = blockIdx.x * 4 + wv;
            if (item >= n_static) break;
            // the dealt items in rank order, handed out by the workgroup dispatcher
            if (items && !grid_item(ctr, items, item, F0.item_claims, (uint32_t)F0.n_tiles, lane, item)) break;
        }
        const FrameArgs F = MV ? views[item >> VIEW_SHIFT].F : F0;
        const FwdOut O = MV ? views[item >> VIEW_SHIFT].O : O0;
        const uint32_t code = MV ? (item & LOCAL_MASK) : item;
        if (TPI == 1) {
            const uint32_t u = code >> UNIT_SHIFT;  // 0: the whole tile, 3 + q: block q (forward units)
            if (u >= 3)
                fwd_block<COUNT>(F, O, (int)(code & ITEM_TILE), (int)(u - 3), lane, s_st[wv]);
            else
                fwd_tile<COUNT>(F, O, (int)(code & ITEM_TILE), lane, s_st[wv]);
        } else {
            int tiles[TPI];
            const int nt = item_tiles<TPI>(F, code, tiles);
            for (int k = 0; k < nt; ++k) fwd_tile<COUNT>(F, O, tiles[k], lane, s_st[wv]);
        }
        if (!PERSISTENT) break;
    }
    trace_end(F0, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// ------------------------------------------------------------------ backward
// The gradient slot a lane adds after wave_reduce_scatter10 depends only on
// the lane; its target array, stride and offset are resolved once per item.
struct GradLane {
    float* base;  // the lane's component of Gaussian 0; null: the lane adds nothing
    uint32_t stride;
};

__device__ __forceinline__ GradLane grad_lane(const BwdIO& B, int slot) {
    if (slot < 0) return GradLane{nullptr, 0u};
    if (B.packed) {  // slots 0-1 (means) at record floats 4-5, 2-5 (conic, opacity) at 0-3, 6-9 in place
        const int f = slot < 2 ? slot + 4 : (slot < 6 ? slot - 2 : slot);
        return GradLane{B.g_means2D + f, (uint32_t)GRAD_RECORD};
    }
    if (slot < 2) return GradLane{B.g_means2D + slot, 2u};
    if (slot < 6) return GradLane{B.g_conic_opacity + (slot - 2), 4u};
    if (slot < 9) return GradLane{B.g_rgb + (slot - 6), 3u};
    return GradLane{B.g_depth, 1u};
}


template <bool PERSISTENT, bool MV = false>
__global__ __launch_bounds__(256) void k_bwd_pixel(FrameArgs F0, BwdIO B0, const ViewDesc* __restrict__ views,
                                                   const uint32_t* __restrict__ items, uint32_t* __restrict__ ctr) {
    const uint64_t t_begin = trace_begin(F0);
    __shared__ float2 s_xy[4][64];
    __shared__ float4 s_co[4][64];
    __shared__ float4 s_cd[4][64];
    __shared__ float4 s_abc[4][64];  // raw conic a, b, c and the Gaussian id (bits)
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WorkQueue Q;
    if (PERSISTENT) Q = make_queue(ctr, items, blockIdx.x * 4 + wv, MV ? nullptr : F0.item_claims);
    bool first = true;
    for (;;) {
        uint32_t item;
        if (PERSISTENT) {
            if (!(first ? queue_first(Q, blockIdx.x * 4 + wv, lane, item) : queue_next(Q, lane, item))) break;
            first = false;
        } else {
            item = blockIdx.x * 4 + wv;
        }
        const FrameArgs F = MV ? views[item >> VIEW_SHIFT].F : F0;
        const BwdIO B = MV ? views[item >> VIEW_SHIFT].B : B0;
        item &= LOCAL_MASK;
        const int64_t HW = (int64_t)F.W * F.H;
        int tile, px, py;
        bool any_inside;
        item_pixel(F, item, lane, tile, px, py, any_inside);
        if (any_inside) {
            const GradLane GL = grad_lane(B, scatter10_slot(lane));
            const bool inside = px < F.W && py < F.H;
            const int64_t p = inside ? (int64_t)py * F.W + px : 0;
            const float TN = inside ? B.final_T[p] : 1.0f;
            const uint32_t start = F.ranges[2 * tile];
            const int len = (int)(F.ranges[2 * tile + 1] - start);
            int nc = inside ? B.n_contrib[p] : 0;
            nc = nc < 0 ? 0 : (nc > len ? len : nc);  // stay inside the tile's list
            const float gC0 = inside ? B.dL_dcolor[p] : 0.f;
            const float gC1 = inside ? B.dL_dcolor[HW + p] : 0.f;
            const float gC2 = inside ? B.dL_dcolor[2 * HW + p] : 0.f;
            const float gA = (inside && B.dL_dalpha) ? B.dL_dalpha[p] : 0.f;
            const float gD = (inside && B.dL_ddepth) ? B.dL_ddepth[p] : 0.f;
            // part of dL/dalpha that does not depend on the entry: the
            // background seen through T_N and the alpha output
            const float kconst = TN * (gC0 * F.bg0 + gC1 * F.bg1 + gC2 * F.bg2) - gA * TN;
            const int max_n = __builtin_amdgcn_readfirstlane(wave_max(nc));  // uniform: the loop runs on scalars
            // S = dL/dC . (colour, depth accumulated behind the entry) + kconst:
            // the only use of those sums, so one scalar carries them
            float T = TN, S = kconst;
            const float fx = (float)px, fy = (float)py;
            for (int hi = max_n; hi > 0; hi -= 64) {
                const int lo = hi > 64 ? hi - 64 : 0;
                if (lo + lane < hi) {
                    const uint32_t g = F.point_list[start + lo + lane];
                    float2 xy; float4 co, cd;
                    load_splat(F, g, xy, co, cd);
                    const float4 raw = F.conic_opacity[g];
                    s_xy[wv][lane] = xy;
                    s_co[wv][lane] = co;
                    s_cd[wv][lane] = cd;
                    s_abc[wv][lane] = make_float4(raw.x, raw.y, raw.z, __uint_as_float(g));
                }
                wave_sync();
                for (int j = hi - 1; j >= lo; --j) {
                    const int jj = j - lo;
                    const float2 xy = s_xy[wv][jj];
                    const float4 co = s_co[wv][jj];
                    const float dx = fx - xy.x, dy = fy - xy.y;
                    const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
                    const float G = exp2_fast(p2);
                    const float ga = co.w * G;
                    const float alpha = fminf(ALPHA_MAX, ga);
                    const bool contrib = (j < nc) && !(p2 > 0.0f || alpha < ALPHA_MIN);
                    if (ballot(contrib) == 0) continue;
                    const float4 cd = s_cd[wv][jj];
                    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f, v6 = 0.f, v7 = 0.f, v8 = 0.f,
                          v9 = 0.f;
                    if (contrib) {
                        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                        const float Tb = T * inv;
                        const float w = alpha * Tb;
                        v6 = w * gC0;
                        v7 = w * gC1;
                        v8 = w * gC2;
                        v9 = w * gD;
                        const float gc = gC0 * cd.x + gC1 * cd.y + gC2 * cd.z + gD * cd.w;
                        const float dA = Tb * gc - inv * S;
                        S = __builtin_fmaf(gc, w, S);
                        T = Tb;
                        if (ga <= ALPHA_MAX) {
                            const float4 abc = s_abc[wv][jj];
                            const float dP = ga * dA;  // dL/dpower
                            v5 = G * dA;               // dL/dopacity
                            v2 = -0.5f * dx * dx * dP;
                            v3 = -dx * dy * dP;
                            v4 = -0.5f * dy * dy * dP;
                            v0 = (abc.x * dx + abc.y * dy) * dP;
                            v1 = (abc.y * dx + abc.z * dy) * dP;
                        }
                    }
                    const float vals[10] = {v0, v1, v2, v3, v4, v5, v6, v7, v8, v9};
                    float tot;
                    wave_reduce_scatter10(vals, lane, tot);
                    if (GL.base) {
                        const uint32_t g = __float_as_uint(s_abc[wv][jj].w);
                        unsafeAtomicAdd(GL.base + (size_t)g * GL.stride, tot);
                    }
                }
                wave_sync();
            }
        }
        if (!PERSISTENT) break;
    }
    trace_end(F0, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// Backward with one wave per 16x16 tile: lane l owns the four pixels
// (l mod 16, l / 16 + 4q), q = 0..3, of the tile (block q = pixel row q of
// the lanes).  The per-entry work that does not scale with pixels -- the LDS
// reads, the 10-value wave reduction and the one multi-lane gradient atomic --
// is paid once per 256 pixels instead of once per 64, and dx (shared by a
// lane's four pixels) once per entry.  Each pixel's arithmetic is the same as
// in k_bwd_pixel.  Per entry a block is visited on uniform branches only: not
// at all when the entry lies beyond every n_contrib of the block or outside
// the block's ellipse mask (staged as in the forward), and its gradient terms
// only when one of its pixels blended the entry.  The chunks of 64 entries are
// walked with the forward's two-stage prefetch (ids two chunks ahead, raw
// splat data one chunk ahead).
//
// Split walks.  A long walk can be cut at list position k into two work
// items that run in parallel, because every quantity an entry's derivative
// needs is known at both ends of the walk.  Writing w_m = alpha_m T_m for the
// weight of entry m and g_m for the upstream gradient dotted with its colour
// and depth, the derivative at entry j needs T_j and the sum S_j of g_m w_m
// over the entries behind it (plus the background and alpha-output terms).
//  * Upper part [k, N): back to front from T_N = final_T and S = those terms,
//    T_j recovered by division -- the unsplit walk, stopped at k.
//  * Lower part [0, k): front to back from T_0 = 1, T advanced exactly as the
//    forward advances it, and S_j = S_total - (prefix of g_m w_m up to and
//    including j), where S_total is the same sum over the whole walk, which
//    the forward's outputs give directly: S_total = dL/dC . out_color +
//    dL/dD . out_depth - dL/dA . T_N (the background terms cancel).
// The split point of a tile with deepest n_contrib N is split_point(N); the
// queue builder and the kernel compute it from the same N.


// Gradient terms of one (pixel, entry) pair added into the lane's ten sums,
// in factored form.  With h = G dL/dalpha where alpha is not clamped (else
// 0), the entry's terms at a pixel are dL/dopacity = h and, since dL/dpower =
// o h, dL/dmean = o h (a dx + b dy, b dx + c dy) and dL/d(a, b, c) =
// -o h (dx^2 / 2, dx dy, dy^2 / 2): all of them are o, a, b, c (the entry's)
// times h, dx h, dy h, dx^2 h, dx dy h, dy^2 h, and dx is the same for the
// four pixels of a lane.  So per pixel only h, dy h and dy^2 h are summed
// (v[5], v[1], v[4]); finish_terms forms the dx moments once per entry
// (v[0] = dx h, v[2] = dx^2 h, v[3] = dx dy h, summed over the lane's
// pixels), and after the wave reduction slot_value applies the entry's
// o, a, b, c to the totals.  v[6..9] are the colour and depth terms.
__device__ __forceinline__ void add_terms(float (&v)[10], float w, float dA, float G, bool unclamped, float gC0,
                                          float gC1, float gC2, float gD, float dy) {
    v[6] = __builtin_fmaf(w, gC0, v[6]);
    v[7] = __builtin_fmaf(w, gC1, v[7]);
    v[8] = __builtin_fmaf(w, gC2, v[8]);
    v[9] = __builtin_fmaf(w, gD, v[9]);
    const float h = unclamped ? G * dA : 0.0f;
    v[5] += h;
    const float u = dy * h;
    v[1] += u;
    v[4] = __builtin_fmaf(u, dy, v[4]);
}

__device__ __forceinline__ void finish_terms(float (&v)[10], float dx) {
    v[0] = dx * v[5];
    v[2] = dx * v[0];
    v[3] = dx * v[1];
}

// Per-lane coefficients of slot_value for the gradient slot the lane holds
// after wave_reduce_scatter10 (slot 0 / 1 also need the total of the other,
// which sits in the lane xor 4).
struct SlotCoef {
    float fa, fc, fo, f1, fb;
};

__device__ __forceinline__ SlotCoef slot_coef(int slot) {
    switch (slot) {
        case 0: return SlotCoef{1.0f, 0.0f, 0.0f, 0.0f, 1.0f};   // dL/du = o (a X + b Y)
        case 1: return SlotCoef{0.0f, 1.0f, 0.0f, 0.0f, 1.0f};   // dL/dv = o (c Y + b X)
        case 2: return SlotCoef{0.0f, 0.0f, -0.5f, 0.0f, 0.0f};  // dL/da = -o XX / 2
        case 3: return SlotCoef{0.0f, 0.0f, -1.0f, 0.0f, 0.0f};  // dL/db = -o XY
        case 4: return SlotCoef{0.0f, 0.0f, -0.5f, 0.0f, 0.0f};  // dL/dc = -o YY / 2
        default: return SlotCoef{0.0f, 0.0f, 0.0f, 1.0f, 0.0f};  // opacity, colour, depth as summed
    }
}

// The lane's gradient component from its reduced total e (all lanes active).
__device__ __forceinline__ float slot_value(const SlotCoef& k, float e, float4 abc, float o) {
    const float other = xor4(e);
    const float ka = __builtin_fmaf(o, __builtin_fmaf(k.fa, abc.x, __builtin_fmaf(k.fc, abc.z, k.fo)), k.f1);
    return __builtin_fmaf(ka, e, o * abc.y * k.fb * other);
}

// DET: instead of adding its per-entry totals to the gradients, the wave
// stores them (zeros for an entry no pixel blends) at the entry's slot of
// B.det_partials, for an ordered reduction afterwards.
// part: 0 the whole walk, 1 the lower part of a split walk, 2 the upper part.
template <bool DET>
__device__ __forceinline__ void bwd_tile(const FrameArgs& F, const BwdIO& B, int tile, int lane, WaveStage& st,
                                         float4* __restrict__ s_abc, int part, uint32_t bmask = 0xFu) {
    const int64_t HW = (int64_t)F.W * F.H;
    const int tx = tile % F.TX, ty = tile / F.TX;
    const int x0 = tx * TILE, y0 = ty * TILE;
    const int px = x0 + (lane & 15);
    const uint32_t start = __builtin_amdgcn_readfirstlane(F.ranges[2 * tile]);
    const int len = (int)(__builtin_amdgcn_readfirstlane(F.ranges[2 * tile + 1]) - start);
    const GradLane GL = grad_lane(B, scatter10_slot(lane));
    const int dslot = scatter10_slot(lane);
    const SlotCoef kc = slot_coef(dslot);
    float* const dpart = DET ? B.det_partials + (size_t)B.det_base[tile] * 10 + dslot : nullptr;
    // S[q]: dL/dC . (colour, depth accumulated behind the entry) + the
    // entry-independent part of dL/dalpha, as in k_bwd_pixel (lower part:
    // S_total, the same sum over the whole walk)
    float T[WQ], S[WQ], gC0[WQ], gC1[WQ], gC2[WQ], gD[WQ], fy[WQ];
    int nc[WQ], bmax[WQ];
    int max_n = 0;
    int tile_max = 0;  // the deepest walk of the whole tile: the split point comes from it
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        const int py = y0 + (lane >> 4) + 4 * q;
        const bool in_image = px < F.W && py < F.H;
        const int64_t p = in_image ? (int64_t)py * F.W + px : 0;
        int n = in_image ? B.n_contrib[p] : 0;
        n = n < 0 ? 0 : (n > len ? len : n);  // stay inside the tile's list
        tile_max = n > tile_max ? n : tile_max;
        const bool inside = in_image && ((bmask >> q) & 1u);  // pixels of a block this item covers
        const float TN = inside ? B.final_T[p] : 1.0f;
        nc[q] = inside ? n : 0;
        gC0[q] = inside ? B.dL_dcolor[p] : 0.f;
        gC1[q] = inside ? B.dL_dcolor[HW + p] : 0.f;
        gC2[q] = inside ? B.dL_dcolor[2 * HW + p] : 0.f;
        const float ga = (inside && B.dL_dalpha) ? B.dL_dalpha[p] : 0.f;
        gD[q] = (inside && B.dL_ddepth) ? B.dL_ddepth[p] : 0.f;
        if (part == 1) {
            const float c0 = inside ? B.out_color[p] : 0.f, c1 = inside ? B.out_color[HW + p] : 0.f;
            const float c2 = inside ? B.out_color[2 * HW + p] : 0.f, d = inside ? B.out_depth[p] : 0.f;
            S[q] = gC0[q] * c0 + gC1[q] * c1 + gC2[q] * c2 + gD[q] * d - ga * TN;
            T[q] = 1.0f;
        } else {
            S[q] = TN * (gC0[q] * F.bg0 + gC1[q] * F.bg1 + gC2[q] * F.bg2) - ga * TN;
            T[q] = TN;
        }
        fy[q] = (float)py;
    }
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        bmax[q] = __builtin_amdgcn_readfirstlane(wave_max(nc[q]));  // uniform: block q walks entries < bmax[q]
        max_n = bmax[q] > max_n ? bmax[q] : max_n;
    }
    const int k = part ? split_point(__builtin_amdgcn_readfirstlane(wave_max(tile_max))) : 0;
    // the entries this item walks: [lo_end, hi_end)
    const int lo_end = part == 2 ? k : 0;
    const int hi_end = part == 1 ? (k < max_n ? k : max_n) : max_n;
    const float fx = (float)px;
    float* const dchunk = DET ? B.det_partials + (size_t)B.det_base[tile] * 10 : nullptr;
    RawSplat cur{}, nxt{};
    uint32_t idn = 0;
    if (part == 1) {
        // ---- lower part, front to back over [0, hi_end)
        float Pf[WQ];  // prefix of g_m w_m over the entries before the current one
#pragma unroll
        for (int q = 0; q < WQ; ++q) Pf[q] = 0.0f;
        const uint32_t end = start + (uint32_t)hi_end;
        if (hi_end > 0) {
            load_raw(F, chunk_id(F, start, end, lane), cur);
            idn = chunk_id(F, start + (uint32_t)(64 < hi_end ? 64 : hi_end - 1), end, lane);
        }
        for (int base = 0; base < hi_end; base += 64) {
            const int cnt = hi_end - base < 64 ? hi_end - base : 64;
            uint64_t mq[WQ];
            chunk_masks(stage_entry(st, lane, cur, lane < cnt, x0, y0), mq);
            s_abc[lane] = make_float4(cur.con.x, cur.con.y, cur.con.z, 0.0f);
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                const int n = bmax[q] - base;
                mq[q] &= n >= 64 ? ~0ull : (n > 0 ? (1ull << n) - 1ull : 0ull);
            }
            wave_sync();
            // branch-free prefetch (past the end: re-reads of the last entry)
            load_raw(F, idn, nxt);
            idn = chunk_id(F, start + (uint32_t)(base + 128 < hi_end ? base + 128 : hi_end - 1), end, lane);
            uint64_t todo = chunk_todo(mq, 0xFu);
            while (todo) {
                const int jj = (int)__builtin_ctzll(todo);
                todo &= todo - 1;
                const int j = base + jj;
                const float4 xym = st.xym[jj];
                const float4 co = st.co[jj];
                const float4 cd = st.cd[jj];
                const float4 abc = s_abc[jj];
                const float dx = fx - xym.x;
                float v[10];
#pragma unroll
                for (int i = 0; i < 10; ++i) v[i] = 0.f;
                bool any = false;  // a block had a pixel that blended the entry (uniform)
#pragma unroll
                for (int q = 0; q < WQ; ++q) {
                    if (!((mq[q] >> jj) & 1u)) continue;
                    const float dy = fy[q] - xym.y;
                    const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
                    const float G = exp2_fast(p2);
                    const float ga = co.w * G;
                    const float alpha = fminf(ALPHA_MAX, ga);
                    const uint64_t cm = ballot(j < nc[q]) & ballot(!(p2 > 0.0f)) & ballot(!(alpha < ALPHA_MIN));
                    if (cm == 0) continue;
                    const bool contrib = lane_bit(cm);
                    any = true;
                    const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                    const float Tb = T[q];
                    const float w = contrib ? alpha * Tb : 0.0f;
                    const float gc = gC0[q] * cd.x + gC1[q] * cd.y + gC2[q] * cd.z + gD[q] * cd.w;
                    const float Pn = __builtin_fmaf(gc, w, Pf[q]);
                    const float dA = Tb * gc - inv * (S[q] - Pn);  // S[q] - Pn: the sum behind the entry
                    Pf[q] = Pn;
                    T[q] = contrib ? Tb - w : T[q];  // as the forward advances T
                    add_terms(v, w, dA, G, lane_bit(cm & ballot(ga <= ALPHA_MAX)), gC0[q], gC1[q], gC2[q], gD[q],
                              dy);
                }
                if (!any) continue;
                finish_terms(v, dx);
                float tot;
                wave_reduce_scatter10(v, lane, tot);
                tot = slot_value(kc, tot, abc, co.w);
                if (GL.base) unsafeAtomicAdd(GL.base + (size_t)__float_as_uint(xym.w) * GL.stride, tot);
            }
            wave_sync();
            cur = nxt;
        }
        return;
    }
    // ---- whole walk or upper part, back to front over [lo_end, hi_end)
    if (hi_end > lo_end) {
        const int lo0 = hi_end - 64 > lo_end ? hi_end - 64 : lo_end;
        load_raw(F, chunk_id(F, start + (uint32_t)lo0, start + (uint32_t)hi_end, lane), cur);
        const int nlo = lo0 - 64 > lo_end ? lo0 - 64 : lo_end;
        idn = chunk_id(F, start + (uint32_t)nlo, start + (uint32_t)(lo0 > nlo ? lo0 : nlo + 1), lane);
    }
    for (int hi = hi_end; hi > lo_end; hi -= 64) {
        const int lo = hi - 64 > lo_end ? hi - 64 : lo_end;
        uint64_t mq[WQ];
        chunk_masks(stage_entry(st, lane, cur, lo + lane < hi, x0, y0), mq);
        s_abc[lane] = make_float4(cur.con.x, cur.con.y, cur.con.z, 0.0f);
        // block q walks only the entries below its deepest n_contrib
#pragma unroll
        for (int q = 0; q < WQ; ++q) {
            const int n = bmax[q] - lo;
            mq[q] &= n >= 64 ? ~0ull : (n > 0 ? (1ull << n) - 1ull : 0ull);
        }
        wave_sync();
        {
            // prefetch without a branch, so that nothing waits for the loads
            // before the chunk is done: the chunk [max(lo - 64, lo_end), lo)
            // and the ids of the one below it; past the walk's last chunk the
            // loads re-read entry lo_end of the list (a valid id) and go unused
            load_raw(F, idn, nxt);
            const int nlo = lo - 64 > lo_end ? lo - 64 : lo_end;
            const int nnlo = nlo - 64 > lo_end ? nlo - 64 : lo_end;
            idn = chunk_id(F, start + (uint32_t)nnlo, start + (uint32_t)(nlo > nnlo ? nlo : nnlo + 1), lane);
        }
        uint64_t todo = chunk_todo(mq, 0xFu);
        uint64_t wrote = 0;  // DET: entries whose partial slot holds a total
        // visit back to front only the entries that reach a block
        while (todo) {
            const int jj = 63 - (int)__builtin_clzll(todo);
            todo &= ~(1ull << jj);
            const int j = lo + jj;
            const float4 xym = st.xym[jj];
            const float4 co = st.co[jj];
            const float4 cd = st.cd[jj];
            const float4 abc = s_abc[jj];
            const float dx = fx - xym.x;
            float v[10];
#pragma unroll
            for (int i = 0; i < 10; ++i) v[i] = 0.f;
            bool any = false;  // a block had a pixel that blended the entry (uniform)
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                if (!((mq[q] >> jj) & 1u)) continue;
                const float dy = fy[q] - xym.y;
                const float p2 = splat_power2(dx, dy, co.x, co.y, co.z);
                const float G = exp2_fast(p2);
                const float ga = co.w * G;
                const float alpha = fminf(ALPHA_MAX, ga);
                const uint64_t cm = ballot(j < nc[q]) & ballot(!(p2 > 0.0f)) & ballot(!(alpha < ALPHA_MIN));
                if (cm == 0) continue;
                const bool contrib = lane_bit(cm);
                any = true;
                const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                const float Tb = T[q] * inv;
                const float w = contrib ? alpha * Tb : 0.0f;
                const float gc = gC0[q] * cd.x + gC1[q] * cd.y + gC2[q] * cd.z + gD[q] * cd.w;
                const float dA = Tb * gc - inv * S[q];
                S[q] = __builtin_fmaf(gc, w, S[q]);
                T[q] = contrib ? Tb : T[q];
                add_terms(v, w, dA, G, lane_bit(cm & ballot(ga <= ALPHA_MAX)), gC0[q], gC1[q], gC2[q], gD[q], dy);
            }
            if (!any) continue;
            finish_terms(v, dx);
            float tot;
            wave_reduce_scatter10(v, lane, tot);
            tot = slot_value(kc, tot, abc, co.w);
            if (DET) {
                if (dslot >= 0) dpart[(size_t)j * 10] = tot;
                wrote |= 1ull << jj;
            } else if (GL.base) {
                unsafeAtomicAdd(GL.base + (size_t)__float_as_uint(xym.w) * GL.stride, tot);
            }
        }
        if (DET && lo + lane < hi && !((wrote >> lane) & 1ull)) {  // zeros for the entries no pixel blended
            float* z = dchunk + (size_t)(lo + lane) * 10;
#pragma unroll
            for (int k2 = 0; k2 < 10; ++k2) z[k2] = 0.0f;
        }
        wave_sync();
        cur = nxt;
    }
}

// The one-view grid dispatch of whole-tile items (the cost-ordered and
// grid-static backward) is held to five waves per SIMD (96 VGPRs, no
// spills): measured faster on the cost-ordered queue, where the heavy items
// start together.  The other instances keep the compiler's allocation (the
// limit spills their queue or split state).
template <bool MV = false, bool DET = false, bool PERSISTENT = true, int TPI = 1, bool SPLIT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    (!MV && !DET && !PERSISTENT && TPI == 1 && !SPLIT) ? 5 : 1))) void k_bwd_wide(FrameArgs F0, BwdIO B0,
                                                                                 const ViewDesc* __restrict__ views,
                                                  const uint32_t* __restrict__ items, uint32_t* __restrict__ ctr,
                                                  uint32_t n_static) {
    const uint64_t t_begin = trace_begin(F0);
    __shared__ WaveStage s_st[4];
    __shared__ float4 s_abc[4][64];  // raw conic a, b, c
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    WorkQueue Q;
    if (PERSISTENT) Q = make_queue(ctr, items, blockIdx.x * 4 + wv, MV ? nullptr : F0.item_claims, (uint32_t)F0.n_tiles);
    for (bool first = true;; first = false) {
        uint32_t item;
        if (PERSISTENT) {
            if (!(first ? queue_first(Q, blockIdx.x * 4 + wv, lane, item) : queue_next(Q, lane, item))) break;
        } else {
            item = blockIdx.x * 4 + wv;
            if (item >= n_static) break;
            // the dealt items in rank order, handed out by the workgroup dispatcher
            if (items && !grid_item(ctr, items, item, F0.item_claims, (uint32_t)F0.n_tiles, lane, item)) break;
        }
        const FrameArgs F = MV ? views[item >> VIEW_SHIFT].F : F0;
        const BwdIO B = MV ? views[item >> VIEW_SHIFT].B : B0;
        const uint32_t code = MV ? (item & LOCAL_MASK) : item;
        if (TPI == 1) {
            const uint32_t u = code >> UNIT_SHIFT;
            bwd_tile<DET>(F, B, (int)(code & ITEM_TILE), lane, s_st[wv], s_abc[wv], SPLIT ? unit_part(u) : 0,
                          unit_blocks(u));
        } else {
            int tiles[TPI];
            const int nt = item_tiles<TPI>(F, code, tiles);
            for (int k = 0; k < nt; ++k) bwd_tile<DET>(F, B, tiles[k], lane, s_st[wv], s_abc[wv], 0);
        }
        if (!PERSISTENT) break;
    }
    trace_end(F0, t_begin, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// ---------------------------------------------------------------- task pool
__device__ __forceinline__ int cost_bucket(uint32_t c) {
    if (c == 0) return 0;
    const int b = 1 + (int)(__log2f((float)c) * 4.0f);
    return b < NBUCKET - 1 ? b : NBUCKET - 1;
}

// Backward cost of every work item (one wave per item): a tile costs
// the largest n_contrib among its 256 pixels (clamped into its list, as the
// backward clamps it) -- the length of the walk; with block2 the item is a
// 32x32 block and costs the sum over its tiles.
__global__ __launch_bounds__(256) void k_tile_costs(FrameArgs F, const int* __restrict__ n_contrib, int block2,
                                                    int n_items, uint32_t* __restrict__ cost) {
    // one wave per item; lane l reads the tile's pixels (l mod 16, l / 16 + 4q), q = 0..3
    const int item = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (item >= n_items) return;  // whole waves
    int tiles[4];
    int nt = 1;
    if (block2) {
        nt = item_tiles<4>(F, (uint32_t)item, tiles);
    } else {
        tiles[0] = item;
    }
    uint32_t c = 0;
    for (int k = 0; k < nt; ++k) {
        const int tile = tiles[k];
        const int tx = tile % F.TX, ty = tile / F.TX;
        const int px = tx * TILE + (lane & 15);
        const int len = (int)(F.ranges[2 * tile + 1] - F.ranges[2 * tile]);
        int m = 0;
#pragma unroll
        for (int q = 0; q < WQ; ++q) {
            const int py = ty * TILE + (lane >> 4) + 4 * q;
            int nc = (px < F.W && py < F.H) ? n_contrib[(int64_t)py * F.W + px] : 0;
            nc = nc < 0 ? 0 : (nc > len ? len : nc);
            m = nc > m ? nc : m;
        }
        c += (uint32_t)wave_max(m);
    }
    if (lane == 0) cost[item] = c;
}

// Forward cost estimate of a work item, one wave per item: the list position
// by which the entries' opacities alone could first take T below 1e-4,
// i.e. the first position where sum_i -log2(1 - min(0.99, o_i)) reaches
// log2(1e4) -- the shortest walk any pixel of the tile can have, met when every
// entry covers the pixel at its peak (the list length if never).  It ranks a
// tile behind many faint entries (a long walk) above one whose first entries
// are opaque, where the list length, the same K for every capped list, cannot.
// A block item costs the sum over its tiles.
__global__ __launch_bounds__(256) void k_fwd_costs(FrameArgs F, int block2, int n_items, uint32_t* __restrict__ cost) {
    const int item = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (item >= n_items) return;  // uniform per wave
    int tiles[4];
    int nt = 1;
    if (block2) {
        nt = item_tiles<4>(F, (uint32_t)item, tiles);
    } else {
        tiles[0] = item;
    }
    constexpr float BUDGET = 13.287712379549449f;  // log2(1 / 1e-4)
    uint32_t c = 0;
    for (int k = 0; k < nt; ++k) {
        const uint32_t start = __builtin_amdgcn_readfirstlane(F.ranges[2 * tiles[k]]);
        const uint32_t end = __builtin_amdgcn_readfirstlane(F.ranges[2 * tiles[k] + 1]);
        float acc = 0.0f;
        uint32_t walk = end - start;
        for (uint32_t base = start; base < end; base += 64) {
            const uint32_t i = base + (uint32_t)lane;
            const float o = i < end ? F.conic_opacity[F.point_list[i]].w : 0.0f;
            const float w = -__builtin_amdgcn_logf(1.0f - fminf(ALPHA_MAX, fmaxf(o, 0.0f)));
            // inclusive prefix sum over the wave (identity 0 for the shifted-in lanes)
            float x = w;
            x += dpp_or<0x111>(x, 0.0f);       // row_shr:1
            x += dpp_or<0x112>(x, 0.0f);       // row_shr:2
            x += dpp_or<0x114>(x, 0.0f);       // row_shr:4
            x += dpp_or<0x118>(x, 0.0f);       // row_shr:8
            x += dpp_or<0x142, 0xA>(x, 0.0f);  // row_bcast:15
            x += dpp_or<0x143, 0xC>(x, 0.0f);  // row_bcast:31
            const uint64_t hit = ballot(i < end && acc + x >= BUDGET);
            if (hit) {
                walk = base + (uint32_t)__builtin_ctzll(hit) + 1u - start;
                break;
            }
            acc += readlane_f(x, 63);
        }
        c += walk;
    }
    if (lane == 0) cost[item] = c;
}

// Batched views: global tile g (over all views, tile_off = per-view prefix of
// tile counts) -> cost, as k_tile_costs for its view.
__global__ __launch_bounds__(256) void k_tile_costs_mv(const ViewDesc* __restrict__ views,
                                                       const uint32_t* __restrict__ tile_off, int n_views, int backward,
                                                       uint32_t* __restrict__ cost) {
    __shared__ int wmax[4];
    const uint32_t g = blockIdx.x;
    int v = 0;
    while (v + 1 < n_views && tile_off[v + 1] <= g) ++v;
    const FrameArgs F = views[v].F;
    const int tile = (int)(g - tile_off[v]);
    uint32_t c = 0;
    if (backward) {
        const int* nc_arr = views[v].B.n_contrib;
        const int tx = tile % F.TX, ty = tile / F.TX;
        const int px = tx * TILE + (threadIdx.x & 15), py = ty * TILE + (threadIdx.x >> 4);
        const int nc = (px < F.W && py < F.H) ? nc_arr[(int64_t)py * F.W + px] : 0;
        const int m = wave_max(nc);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
        __syncthreads();
        c = (uint32_t)max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    } else {
        c = F.ranges[2 * tile + 1] - F.ranges[2 * tile];
    }
    if (threadIdx.x == 0) cost[g] = c;
}

// Single workgroup: rank tiles (raster order, or by descending cost bucket)
// and deal them.  Sub-tile items: tile of rank r goes to queue group r mod 16,
// its sub-tile s to queue 4 (r mod 16) + s, at queue position r / 16.  Tile
// items (per_tile): queue r mod 64, position r / 64.  Also resets the 64 fetch
// counters and stores the item count.
// Units a tile of cost c is dealt as (per-tile items, cost order, one view):
// the whole tile; the two parts of its backward walk (c >= split_min); its
// four blocks (c >= block_min); or both.  Returns the count; unit i has
// unit code u[i] and cost w[i].
__device__ __forceinline__ int tile_units(uint32_t c, int split_min, int block_min, uint32_t (&u)[8],
                                          uint32_t (&w)[8]) {
    const bool blk = block_min > 0 && c >= (uint32_t)block_min;
    const bool prt = split_min > 0 && c >= (uint32_t)split_min;
    const uint32_t k = prt ? (uint32_t)split_point((int)c) : 0u;
    if (!blk && !prt) {
        u[0] = 0; w[0] = c;
        return 1;
    }
    if (!blk) {
        u[0] = 1; w[0] = k;
        u[1] = 2; w[1] = c - k;
        return 2;
    }
    if (!prt) {
        for (int q = 0; q < 4; ++q) {
            u[q] = 3 + q; w[q] = c;
        }
        return 4;
    }
    for (int q = 0; q < 4; ++q) {
        u[2 * q] = 7 + 2 * q; w[2 * q] = k;
        u[2 * q + 1] = 8 + 2 * q; w[2 * q + 1] = c - k;
    }
    return 8;
}

// The cost-order queue is a counting sort of the work units by descending
// cost bucket, spread over workgroups of QB tiles: k_queue_count takes each
// workgroup's bucket histogram, k_queue_deal gives every unit its rank --
// the units of all higher buckets, of its own bucket in earlier workgroups,
// and an LDS atomic within its workgroup -- and deals it.  (One workgroup
// for the whole frame spends its time on same-address LDS atomics: tiles of
// a frame fall into a few buckets.)
constexpr int QB = 1024;

__host__ __device__ __forceinline__ int queue_groups(int n_tiles) { return n_tiles > 0 ? (n_tiles + QB - 1) / QB : 1; }

// Units of tile t (0 past the end), with codes u and costs w.
__device__ __forceinline__ int queue_units(uint32_t t, int n_tiles, const uint32_t* __restrict__ cost, bool units,
                                           int split_min, int block_min, uint32_t (&u)[8], uint32_t (&w)[8]) {
    if (t >= (uint32_t)n_tiles) return 0;
    const uint32_t c = cost[t];
    if (units) return tile_units(c, split_min, block_min, u, w);
    u[0] = 0;
    w[0] = c;
    return 1;
}

// Finer units for heavy tiles: one-view per-tile items in cost order only.
__device__ __forceinline__ bool queue_has_units(int by_cost, int per_tile, const uint32_t* tile_off, int split_min,
                                                int block_min) {
    return by_cost && per_tile && !tile_off && (split_min > 0 || block_min > 0);
}

__global__ __launch_bounds__(QB) void k_queue_count(int n_tiles, const uint32_t* __restrict__ cost, int per_tile,
                                                    const uint32_t* __restrict__ tile_off, int split_min,
                                                    int block_min, uint32_t* __restrict__ qhist) {
    __shared__ uint32_t hist[NBUCKET];
    for (int b = threadIdx.x; b < NBUCKET; b += QB) hist[b] = 0;
    __syncthreads();
    const bool units = queue_has_units(1, per_tile, tile_off, split_min, block_min);
    uint32_t u[8], w[8];
    const int n = queue_units(blockIdx.x * QB + threadIdx.x, n_tiles, cost, units, split_min, block_min, u, w);
    for (int i = 0; i < n; ++i) atomicAdd(&hist[NBUCKET - 1 - cost_bucket(w[i])], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < NBUCKET; b += QB) qhist[(size_t)blockIdx.x * NBUCKET + b] = hist[b];
}

// Ranks tiles (raster order, or by descending cost bucket from the
// histograms of k_queue_count) and deals them.  Sub-tile items: tile of rank
// r goes to queue group r mod 16, its sub-tile s to queue 4 (r mod 16) + s,
// at queue position r / 16.  Tile items (per_tile): queue r mod 64, position
// r / 64.  Workgroup 0 also resets the 64 fetch counters and stores the
// item count.
__global__ __launch_bounds__(QB) void k_queue_deal(int n_tiles, const uint32_t* __restrict__ cost, int by_cost,
                                                   int per_tile, const uint32_t* __restrict__ tile_off, int n_views,
                                                   int split_min, int block_min, const uint32_t* __restrict__ qhist,
                                                   uint32_t* __restrict__ items, uint32_t* __restrict__ ctr) {
    __shared__ uint32_t tot[NBUCKET], pre[NBUCKET];
    __shared__ uint32_t n_units;
    const int lane = threadIdx.x & 63;
    auto deal = [&](uint32_t r, uint32_t tile, uint32_t unit) {
        uint32_t vbits = 0;
        if (tile_off) {  // batched views: global tile -> (view, tile of the view)
            int v = 0;
            while (v + 1 < n_views && tile_off[v + 1] <= tile) ++v;
            tile -= tile_off[v];
            vbits = (uint32_t)v << VIEW_SHIFT;
        }
        if (per_tile) {  // tile of rank r: queue r mod 64, position r / 64, i.e. items[r]
            items[r] = vbits | (unit << UNIT_SHIFT) | tile;
            return;
        }
        const uint32_t grp = r % QGROUPS, pos = r / QGROUPS;
        for (uint32_t sub = 0; sub < 4; ++sub) items[(size_t)pos * NQ + grp * 4 + sub] = vbits | (tile * 4 + sub);
    };
    const bool units = queue_has_units(by_cost, per_tile, tile_off, split_min, block_min);
    const uint32_t t = blockIdx.x * QB + threadIdx.x;
    if (!by_cost) {
        if (t < (uint32_t)n_tiles) deal(t, t, 0u);
    } else {
        for (int b = threadIdx.x; b < NBUCKET; b += QB) tot[b] = pre[b] = 0;
        __syncthreads();
        // bucket totals over all workgroups, and this workgroup's predecessors' share
        const int ng = (int)gridDim.x;
        for (int k = threadIdx.x; k < ng * NBUCKET; k += QB) {
            const uint32_t h = qhist[k];
            const int g = k / NBUCKET, b = k - g * NBUCKET;
            if (h) {
                atomicAdd(&tot[b], h);
                if (g < (int)blockIdx.x) atomicAdd(&pre[b], h);
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {  // exclusive scan of the totals, three buckets per lane
            uint32_t h[3], sum = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int b = 3 * lane + k;
                h[k] = b < NBUCKET ? tot[b] : 0u;
                sum += h[k];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t o = (uint32_t)__shfl_up((int)incl, off, 64);
                if (lane >= off) incl += o;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int b = 3 * lane + k;
                if (b < NBUCKET) pre[b] += run;  // first rank of the bucket in this workgroup
                run += h[k];
            }
            if (lane == 63) n_units = incl;
        }
        __syncthreads();
        uint32_t u[8], w[8];
        const int n = queue_units(t, n_tiles, cost, units, split_min, block_min, u, w);
        for (int i = 0; i < n; ++i) deal(atomicAdd(&pre[NBUCKET - 1 - cost_bucket(w[i])], 1u), t, u[i]);
    }
    if (blockIdx.x == 0) {
        for (int q = threadIdx.x; q < NQ; q += QB) ctr[q * QSTRIDE] = 0;
        if (threadIdx.x == 0) ctr[NQ * QSTRIDE] = units ? n_units : (uint32_t)n_tiles * (per_tile ? 1u : 4u);
    }
}

// Queue of n_tiles tiles (see k_queue_deal); qhist: queue_groups(n_tiles) *
// NBUCKET words, used in cost order.
static void launch_queue(hipStream_t stream, int n_tiles, const uint32_t* cost, int by_cost, int per_tile,
                         const uint32_t* tile_off, int n_views, int split_min, int block_min, uint32_t* qhist,
                         uint32_t* items, uint32_t* ctr) {
    const int ng = queue_groups(n_tiles);
    if (by_cost)
        hipLaunchKernelGGL(k_queue_count, dim3(ng), dim3(QB), 0, stream, n_tiles, cost, per_tile, tile_off, split_min,
                           block_min, qhist);
    hipLaunchKernelGGL(k_queue_deal, dim3(ng), dim3(QB), 0, stream, n_tiles, cost, by_cost, per_tile, tile_off,
                       n_views, split_min, block_min, (const uint32_t*)qhist, items, ctr);
}

// ---------------------------------------------------------------- host side
struct RenderLayout {
    size_t ctr, items, cost, qhist, bytes;
    uint32_t n_items;
};

static RenderLayout render_layout(int n_tiles) {
    RenderLayout L{};
    L.n_items = (uint32_t)n_tiles * 4u;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b, 256);
        return o;
    };
    L.ctr = take(4 * (size_t)(NQ * QSTRIDE + QSTRIDE));
    // the item array: room for four sub-tiles or up to eight units per tile
    // (blocks, walk parts), padded to whole rounds of NQ
    const size_t rounds = (8 * (size_t)n_tiles + NQ - 1) / NQ;
    L.items = take(4 * (rounds * NQ > 0 ? rounds * NQ : 1));
    L.cost = take(4 * (size_t)(n_tiles ? n_tiles : 1));
    L.qhist = take(4 * (size_t)queue_groups(n_tiles) * NBUCKET);
    L.bytes = off;
    return L;
}

static bgs_status check_frame(const bgs_frame* f, const bgs_render_cfg* cfg, FrameArgs& A, const char* who) {
    if (!f || !cfg) return fail(BGS_EINVAL, std::string(who) + ": null frame or cfg");
    if (f->width <= 0 || f->height <= 0) return fail(BGS_EINVAL, std::string(who) + ": image size must be positive");
    if (f->tile != TILE) return fail(BGS_EUNSUPPORTED, std::string(who) + ": only 16x16 tiles are supported");
    if (!f->ranges || !f->point_list || !f->means2D || !f->conic_opacity || !f->rgb || !f->depth)
        return fail(BGS_EINVAL, std::string(who) + ": null frame array");
    if ((reinterpret_cast<uintptr_t>(f->conic_opacity) & 15) || (reinterpret_cast<uintptr_t>(f->means2D) & 7))
        return fail(BGS_EINVAL, std::string(who) + ": means2D must be 8-byte and conic_opacity 16-byte aligned");
    if (cfg->variant < BGS_STATIC || cfg->variant > BGS_STATIC_WAVE)
        return fail(BGS_EINVAL, std::string(who) + ": unknown variant");
    if (cfg->variant == BGS_STATIC_WAVE && cfg->subtile != 16)
        return fail(BGS_EUNSUPPORTED, std::string(who) + ": the static wave-per-tile variant needs sub-tile 16");
    if (cfg->variant != BGS_STATIC && cfg->variant != BGS_STATIC_WAVE && cfg->subtile != 8 &&
        !(cfg->variant == BGS_BALANCED_PIXEL && (cfg->subtile == 16 || cfg->subtile == 32)))
        return fail(BGS_EUNSUPPORTED,
                    std::string(who) + ": sub-tile must be 8, or 16 or 32 with the pixel-wise variant");
    if (cfg->order != BGS_ORDER_RASTER && cfg->order != BGS_ORDER_COST)
        return fail(BGS_EINVAL, std::string(who) + ": unknown order");
    A.W = f->width;
    A.H = f->height;
    A.TX = (f->width + TILE - 1) / TILE;
    A.TY = (f->height + TILE - 1) / TILE;
    A.n_tiles = A.TX * A.TY;
    A.ranges = f->ranges;
    A.point_list = f->point_list;
    A.means2D = reinterpret_cast<const float2*>(f->means2D);
    A.conic_opacity = reinterpret_cast<const float4*>(f->conic_opacity);
    A.rgb = f->rgb;
    A.depth = f->depth;
    A.bg0 = cfg->bg[0];
    A.bg1 = cfg->bg[1];
    A.bg2 = cfg->bg[2];
    A.trace = cfg->wg_trace;
    A.trace_cap = cfg->wg_trace ? cfg->wg_trace_cap : 0;
    A.n_examined = cfg->n_examined;
    A.list_cap = cfg->list_cap;
    A.list_overflow = cfg->list_overflow;
    A.item_claims = cfg->item_claims;
    return BGS_OK;
}

template <typename K>
static int persistent_blocks(K kernel, uint32_t n_items) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, 0) != hipSuccess || occ < 1) occ = 1;
    const int64_t want = (int64_t)cu_count() * occ;
    const int64_t cap = ((int64_t)n_items + 3) / 4;
    return (int)(want < cap ? want : (cap > 0 ? cap : 1));
}

// Whole 16x16 tiles (or 32x32 blocks of them) as work items: the forward's
// and the backward's wave-per-tile kernels.
static bool tile_items(const bgs_render_cfg* cfg) {
    return cfg->variant == BGS_BALANCED_PIXEL && (cfg->subtile == 16 || cfg->subtile == 32);
}

static bool block_items(const bgs_render_cfg* cfg) {
    return cfg->variant == BGS_BALANCED_PIXEL && cfg->subtile == 32;
}

// The wave-per-tile variants take their dealt items through the persistent
// task pool with BGS_FLAG_PERSISTENT, else as a plain grid in rank order.
static bool pool_waves(const bgs_render_cfg* cfg) { return (cfg->flags & BGS_FLAG_PERSISTENT) != 0; }

// Split backward walks: the wave-per-tile backward with cost order and the flag.
static bool split_walks(const bgs_render_cfg* cfg) {
    return (cfg->flags & BGS_FLAG_SPLIT_WALKS) && cfg->variant == BGS_BALANCED_PIXEL && cfg->subtile == 16 &&
           cfg->order == BGS_ORDER_COST;
}

// Number of queue entries: blocks, tiles, or 8x8 sub-tiles.
static uint32_t queue_items(const FrameArgs& A, const bgs_render_cfg* cfg) {
    if (block_items(cfg)) return (uint32_t)(((A.TX + 1) / 2) * ((A.TY + 1) / 2));
    return (uint32_t)A.n_tiles * (tile_items(cfg) ? 1u : 4u);
}

// units: deal heavy tiles as finer units (blocks, walk parts) where the
// configuration allows it (not for the deterministic backward, which keeps
// one item per tile).
static bgs_status build_queue(const FrameArgs& A, const bgs_render_cfg* cfg, const int* n_contrib, char* ws,
                              const RenderLayout& L, hipStream_t stream, bool units = true) {
    auto* ctr = reinterpret_cast<uint32_t*>(ws + L.ctr);
    auto* items = reinterpret_cast<uint32_t*>(ws + L.items);
    auto* cost = reinterpret_cast<uint32_t*>(ws + L.cost);
    const int by_cost = cfg->order == BGS_ORDER_COST;
    const bool blocks = block_items(cfg);
    const int n_cost = blocks ? (int)queue_items(A, cfg) : A.n_tiles;
    if (by_cost && n_cost > 0) {
        if (n_contrib)  // backward: the exact walk
            hipLaunchKernelGGL(k_tile_costs, dim3((n_cost + 3) / 4), dim3(256), 0, stream, A, n_contrib, blocks ? 1 : 0,
                               n_cost, cost);
        else  // forward: the opacity-budget estimate
            hipLaunchKernelGGL(k_fwd_costs, dim3((n_cost + 3) / 4), dim3(256), 0, stream, A, blocks ? 1 : 0, n_cost,
                               cost);
        BGS_HIP(hipGetLastError());
    }
    const int per_tile = tile_items(cfg) ? 1 : 0;
    // finer units for heavy tiles of the one-wave-per-tile kernels: four blocks
    // in either direction, and split walks for backward queues (n_contrib given)
    const bool wave_tile = units && cfg->variant == BGS_BALANCED_PIXEL && cfg->subtile == 16;
    const int split_min = (wave_tile && split_walks(cfg) && n_contrib) ? SPLIT_MIN : 0;
    const int block_min = wave_tile ? (n_contrib ? BLOCK_MIN_BWD : BLOCK_MIN_FWD) : 0;
    launch_queue(stream, n_cost, cost, by_cost, per_tile, nullptr, 1, split_min, block_min,
                 reinterpret_cast<uint32_t*>(ws + L.qhist), items, ctr);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

}  // namespace bgs

using namespace bgs;

extern "C" size_t bgs_render_workspace_bytes(const bgs_frame* frame, const bgs_render_cfg* cfg) {
    (void)cfg;
    if (!frame || frame->width <= 0 || frame->height <= 0) return 0;
    const int n_tiles = ((frame->width + TILE - 1) / TILE) * ((frame->height + TILE - 1) / TILE);
    return render_layout(n_tiles).bytes;
}

extern "C" bgs_status bgs_queue_build(const bgs_frame* frame, const bgs_render_cfg* cfg, const int32_t* n_contrib,
                                      void* ws, size_t ws_bytes, hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_queue_build");
    if (st != BGS_OK) return st;
    // the static variants take no queue
    if (cfg->variant == BGS_STATIC || cfg->variant == BGS_STATIC_WAVE) return BGS_OK;
    const RenderLayout L = render_layout(A.n_tiles);
    BGS_REQUIRE(ws && ws_bytes >= L.bytes, "bgs_queue_build: workspace too small");
    return build_queue(A, cfg, n_contrib, static_cast<char*>(ws), L, stream);
}

extern "C" bgs_status bgs_render_fwd(const bgs_frame* frame, const bgs_render_cfg* cfg, float* out_color,
                                     float* out_alpha, float* out_depth, float* final_T, int32_t* n_contrib, void* ws,
                                     size_t ws_bytes, hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_render_fwd");
    if (st != BGS_OK) return st;
    BGS_REQUIRE(out_color && out_alpha && out_depth && final_T && n_contrib, "bgs_render_fwd: null output");
    if (cfg->n_examined && !(tile_items(cfg) && cfg->subtile == 16))
        return fail(BGS_EUNSUPPORTED, "bgs_render_fwd: n_examined is written by the pixel-wise subtile-16 variant");
    FwdOut O{out_color, out_alpha, out_depth, final_T, n_contrib};
    if (cfg->variant == BGS_STATIC) {
        hipLaunchKernelGGL(k_fwd_static, dim3(A.n_tiles), dim3(256), 0, stream, A, O);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    if (cfg->variant == BGS_STATIC_WAVE) {
        if (A.n_tiles > 0)
            hipLaunchKernelGGL((k_fwd_wide<false, false, false>), dim3((A.n_tiles + 3) / 4), dim3(256), 0, stream,
                               A, O, (const ViewDesc*)nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                               (uint32_t)A.n_tiles);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    const RenderLayout L = render_layout(A.n_tiles);
    BGS_REQUIRE(ws && ws_bytes >= L.bytes, "bgs_render_fwd: workspace too small");
    char* w = static_cast<char*>(ws);
    if (!(cfg->flags & BGS_FLAG_QUEUE_READY)) {
        st = build_queue(A, cfg, nullptr, w, L, stream);
        if (st != BGS_OK) return st;
    }
    auto* ctr = reinterpret_cast<uint32_t*>(w + L.ctr);
    auto* items = reinterpret_cast<const uint32_t*>(w + L.items);
    const uint32_t n_items = queue_items(A, cfg);
    // wave-per-tile kernels: n_max = the most items the queue can hold (up
    // to four block units per tile); a plain grid of n_max / 4 workgroups in
    // rank order, or the persistent pool
    const bool pool = pool_waves(cfg);
    if (block_items(cfg)) {
        if (pool)
            hipLaunchKernelGGL((k_fwd_wide<false, false, true, 4>), dim3(persistent_blocks(k_fwd_wide<false, false,
                               true, 4>, n_items)), dim3(256), 0, stream, A, O, (const ViewDesc*)nullptr, items, ctr,
                               0u);
        else
            hipLaunchKernelGGL((k_fwd_wide<false, false, false, 4>), dim3((n_items + 3) / 4), dim3(256), 0, stream,
                               A, O, (const ViewDesc*)nullptr, items, ctr, n_items);
    } else if (tile_items(cfg) && A.n_examined) {
        if (pool)
            hipLaunchKernelGGL((k_fwd_wide<false, true>), dim3(persistent_blocks(k_fwd_wide<false, true>,
                               4 * n_items)), dim3(256), 0, stream, A, O, (const ViewDesc*)nullptr, items, ctr, 0u);
        else
            hipLaunchKernelGGL((k_fwd_wide<false, true, false>), dim3(n_items), dim3(256), 0, stream, A, O,
                               (const ViewDesc*)nullptr, items, ctr, 4 * n_items);
    } else if (tile_items(cfg)) {
        if (pool)
            hipLaunchKernelGGL(k_fwd_wide<false>, dim3(persistent_blocks(k_fwd_wide<false>, 4 * n_items)),
                               dim3(256), 0, stream, A, O, (const ViewDesc*)nullptr, items, ctr, 0u);
        else
            hipLaunchKernelGGL((k_fwd_wide<false, false, false>), dim3(n_items), dim3(256), 0, stream, A, O,
                               (const ViewDesc*)nullptr, items, ctr, 4 * n_items);
    } else if (cfg->variant == BGS_BALANCED_GAUSS) {
        const int blocks = persistent_blocks(k_fwd_hybrid<64>, L.n_items);
        hipLaunchKernelGGL(k_fwd_hybrid<64>, dim3(blocks), dim3(256), 0, stream, A, O, items, ctr);
    } else if (cfg->variant == BGS_BALANCED_HYBRID) {
        const int blocks = persistent_blocks(k_fwd_hybrid<HYBRID_SWITCH>, L.n_items);
        hipLaunchKernelGGL(k_fwd_hybrid<HYBRID_SWITCH>, dim3(blocks), dim3(256), 0, stream, A, O, items, ctr);
    } else {
        const int blocks = persistent_blocks(k_fwd_pixel<true>, L.n_items);
        hipLaunchKernelGGL(k_fwd_pixel<true>, dim3(blocks), dim3(256), 0, stream, A, O, (const ViewDesc*)nullptr,
                           items, ctr);
    }
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

// ---------------------------------------------------------- no-alloc forward
// bgs_render_fwd for callers that cannot allocate device memory: the work
// queue (fetch counters, dealt items, tile costs) lives in this file-scope
// device array instead of a caller workspace.  Each device holds its own copy
// until the process ends; its address is looked up once per device.
namespace bgs {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)5 << 19;  // 2.5 MiB: queues of up to 65 536 tiles
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device.  In host code the
// array's name is only a stand-in; kernels must get this address.
static bgs_status scratch_address(void** out) {
    int dev = 0;
    BGS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(BGS_EUNSUPPORTED, "bgs_render_fwd_noalloc: device index >= 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        BGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(BGS_EINTERNAL, "bgs_render_fwd_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BGS_OK;
}

}  // namespace bgs

extern "C" size_t bgs_render_fwd_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" bgs_status bgs_render_fwd_noalloc(const bgs_frame* frame, const bgs_render_cfg* cfg, float* out_color,
                                             float* out_alpha, float* out_depth, float* final_T,
                                             int32_t* n_contrib, hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_render_fwd_noalloc");
    if (st != BGS_OK) return st;
    const RenderLayout L = render_layout(A.n_tiles);
    if (L.bytes > NOALLOC_SCRATCH_BYTES)
        return fail(BGS_ECAPACITY, "bgs_render_fwd_noalloc: " + std::to_string(A.n_tiles) + " tiles need " +
                                       std::to_string(L.bytes) + " bytes of queue state, more than the " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES) + " the library holds");
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != BGS_OK) return st;
    // the array keeps the previous call's queue: always build this call's
    bgs_render_cfg c = *cfg;
    c.flags &= ~BGS_FLAG_QUEUE_READY;
    return bgs_render_fwd(frame, &c, out_color, out_alpha, out_depth, final_T, n_contrib, ws, L.bytes, stream);
}

namespace bgs {
// Gradient outputs of a backward entry point: the four arrays, or with
// BGS_FLAG_PACKED_GRADS one array of 16-float records in dL_dmeans2D.
static bgs_status grad_outputs(const bgs_render_cfg* cfg, float* m2, float* co, float* rgb, float* d, BwdIO& B,
                               const char* who) {
    const std::string w(who);
    if (cfg->flags & BGS_FLAG_PACKED_GRADS) {
        BGS_REQUIRE(m2 && !co && !rgb && !d, w + ": packed gradients go in dL_dmeans2D alone ([P][16] records); "
                                                 "the other gradient outputs must be null");
        BGS_REQUIRE((reinterpret_cast<uintptr_t>(m2) & 63) == 0, w + ": gradient records must be 64-byte aligned");
        B.g_means2D = m2;
        B.g_conic_opacity = B.g_rgb = B.g_depth = nullptr;
        B.packed = 1;
        return BGS_OK;
    }
    BGS_REQUIRE(m2 && co && rgb, w + ": null gradient output");
    B.g_means2D = m2;
    B.g_conic_opacity = co;
    B.g_rgb = rgb;
    B.g_depth = d;
    B.packed = 0;
    return BGS_OK;
}
}  // namespace bgs

extern "C" bgs_status bgs_render_bwd(const bgs_frame* frame, const bgs_render_cfg* cfg, const float* final_T,
                                     const int32_t* n_contrib, const float* dL_dcolor, const float* dL_dalpha,
                                     const float* dL_ddepth, float* dL_dmeans2D, float* dL_dconic_opacity,
                                     float* dL_drgb, float* dL_ddepths, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_render_bwd");
    if (st != BGS_OK) return st;
    BGS_REQUIRE(final_T && n_contrib && dL_dcolor, "bgs_render_bwd: null forward state or dL_dcolor");
    BwdIO B{final_T, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, nullptr, nullptr, nullptr,
            nullptr, nullptr, nullptr, cfg->split_color, cfg->split_depth, 0};
    st = grad_outputs(cfg, dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepths, B, "bgs_render_bwd");
    if (st != BGS_OK) return st;
    if ((cfg->flags & BGS_FLAG_SPLIT_WALKS) && !split_walks(cfg))
        return fail(BGS_EUNSUPPORTED, "bgs_render_bwd: split walks need BGS_BALANCED_PIXEL, subtile 16, cost order");
    if (split_walks(cfg) && !(cfg->split_color && cfg->split_depth))
        return fail(BGS_EINVAL, "bgs_render_bwd: split walks need the forward's out_color and out_depth "
                                "(cfg.split_color, cfg.split_depth)");
    if (cfg->variant == BGS_STATIC) {
        hipLaunchKernelGGL(k_bwd_pixel<false>, dim3(A.n_tiles), dim3(256), 0, stream, A, B, (const ViewDesc*)nullptr,
                           (const uint32_t*)nullptr, (uint32_t*)nullptr);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    if (cfg->variant == BGS_STATIC_WAVE) {
        if (A.n_tiles > 0)
            hipLaunchKernelGGL((k_bwd_wide<false, false, false>), dim3((A.n_tiles + 3) / 4), dim3(256), 0, stream,
                               A, B, (const ViewDesc*)nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                               (uint32_t)A.n_tiles);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    const RenderLayout L = render_layout(A.n_tiles);
    BGS_REQUIRE(ws && ws_bytes >= L.bytes, "bgs_render_bwd: workspace too small");
    char* w = static_cast<char*>(ws);
    if (!(cfg->flags & BGS_FLAG_QUEUE_READY)) {
        st = build_queue(A, cfg, n_contrib, w, L, stream);
        if (st != BGS_OK) return st;
    }
    auto* ctr = reinterpret_cast<uint32_t*>(w + L.ctr);
    auto* items = reinterpret_cast<const uint32_t*>(w + L.items);
    const uint32_t n_items = queue_items(A, cfg);
    // wave-per-tile kernels as in bgs_render_fwd: up to four block units per
    // tile, eight with split walks
    const bool pool = pool_waves(cfg);
    if (block_items(cfg)) {
        if (pool)
            hipLaunchKernelGGL((k_bwd_wide<false, false, true, 4>), dim3(persistent_blocks(k_bwd_wide<false, false,
                               true, 4>, n_items)), dim3(256), 0, stream, A, B, (const ViewDesc*)nullptr, items, ctr,
                               0u);
        else
            hipLaunchKernelGGL((k_bwd_wide<false, false, false, 4>), dim3((n_items + 3) / 4), dim3(256), 0, stream,
                               A, B, (const ViewDesc*)nullptr, items, ctr, n_items);
    } else if (split_walks(cfg)) {
        if (pool)
            hipLaunchKernelGGL((k_bwd_wide<false, false, true, 1, true>), dim3(persistent_blocks(k_bwd_wide<false,
                               false, true, 1, true>, 8 * n_items)), dim3(256), 0, stream, A, B,
                               (const ViewDesc*)nullptr, items, ctr, 0u);
        else
            hipLaunchKernelGGL((k_bwd_wide<false, false, false, 1, true>), dim3(2 * n_items), dim3(256), 0, stream,
                               A, B, (const ViewDesc*)nullptr, items, ctr, 8 * n_items);
    } else if (tile_items(cfg)) {
        if (pool)
            hipLaunchKernelGGL(k_bwd_wide<false>, dim3(persistent_blocks(k_bwd_wide<false>, 4 * n_items)),
                               dim3(256), 0, stream, A, B, (const ViewDesc*)nullptr, items, ctr, 0u);
        else
            hipLaunchKernelGGL((k_bwd_wide<false, false, false>), dim3(n_items), dim3(256), 0, stream, A, B,
                               (const ViewDesc*)nullptr, items, ctr, 4 * n_items);
    } else {
        const int blocks = persistent_blocks(k_bwd_pixel<true>, L.n_items);
        hipLaunchKernelGGL(k_bwd_pixel<true>, dim3(blocks), dim3(256), 0, stream, A, B, (const ViewDesc*)nullptr,
                           items, ctr);
    }
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

// ======================================================================
// Deterministic-order backward.  The wide backward (one wave per 16x16
// tile) produces, for every list entry a tile walks, one 10-value partial
// from a fixed-order wave reduction; instead of adding it to the Gaussian's
// gradient with float atomics (whose order varies from run to run), it is
// stored at its own slot.  The (Gaussian, slot) pairs are then sorted stably
// by Gaussian, so each Gaussian's partials come in (tile, list position)
// order, and one wave per Gaussian sums them in a fixed order and adds the
// sums to the gradients.  The result is the same sum up to fp32 rounding and
// identical from run to run.
// ======================================================================
namespace bgs {

// base = exclusive scan of cnt over the tiles; total[0] = the sum (one workgroup)
__global__ __launch_bounds__(1024) void k_det_scan(int nt, const uint32_t* __restrict__ cnt,
                                                   uint32_t* __restrict__ base, uint64_t* __restrict__ total) {
    using Scan = rocprim::block_scan<uint64_t, 1024>;
    __shared__ typename Scan::storage_type s_scan;
    const int per = (nt + 1023) / 1024;
    const int t0 = min(nt, (int)threadIdx.x * per), t1 = min(nt, t0 + per);
    uint64_t sum = 0;
    for (int t = t0; t < t1; ++t) sum += cnt[t];
    uint64_t run = 0, grand = 0;
    Scan().exclusive_scan(sum, run, (uint64_t)0, grand, s_scan);
    for (int t = t0; t < t1; ++t) {
        base[t] = (uint32_t)run;
        run += cnt[t];
    }
    if (threadIdx.x == 0) total[0] = grand;
}

// (Gaussian id, slot) of every walked entry, in slot order; one wave per tile
__global__ __launch_bounds__(64) void k_det_keys(FrameArgs F, const uint32_t* __restrict__ cnt,
                                                 const uint32_t* __restrict__ base, uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals) {
    const int t = blockIdx.x;
    const uint32_t b = base[t], c = cnt[t], start = F.ranges[2 * t];
    for (uint32_t j = threadIdx.x; j < c; j += 64) {
        keys[b + j] = F.point_list[start + j];
        vals[b + j] = b + j;
    }
}

__global__ __launch_bounds__(256) void k_det_clear(int64_t P, uint32_t* __restrict__ seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * P) seg[i] = 0u;
}

// seg[2g], seg[2g + 1] = the first and one past the last position of
// Gaussian g among the sorted keys (0, 0 when it has none)
__global__ __launch_bounds__(256) void k_det_bounds(int64_t K, int64_t P, const uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const uint32_t g = keys[i];
    if ((int64_t)g >= P) return;
    if (i == 0 || keys[i - 1] != g) seg[2 * (size_t)g] = (uint32_t)i;
    if (i == K - 1 || keys[i + 1] != g) seg[2 * (size_t)g + 1] = (uint32_t)(i + 1);
}

// One wave per Gaussian: lane l sums partials l, l + 64, ... of the
// Gaussian's run in order, a fixed butterfly combines the lanes, and the
// sums are added to the gradients (one writer per element).
__global__ __launch_bounds__(256) void k_det_reduce(int64_t P, const uint32_t* __restrict__ seg,
                                                    const uint32_t* __restrict__ vals,
                                                    const float* __restrict__ partials, BwdIO B) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= P) return;  // uniform per wave
    const uint32_t s = seg[2 * g], e = seg[2 * g + 1];
    float v[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = 0.0f;
    for (uint32_t i = s + lane; i < e; i += 64) {
        const float* pp = partials + (size_t)vals[i] * 10;
#pragma unroll
        for (int k = 0; k < 10; ++k) v[k] += pp[k];
    }
    float tot;
    const int slot = wave_reduce_scatter10(v, lane, tot);
    const GradLane GL = grad_lane(B, slot);
    if (GL.base) GL.base[(size_t)g * GL.stride] += tot;
}

struct DetLayout {
    RenderLayout R;
    size_t cnt, base, total, partials, keys, vals, keys2, vals2, sscr, scr_bytes, seg, bytes;
};

static DetLayout det_layout(int n_tiles, int64_t P, int64_t max_occ) {
    DetLayout D{};
    D.R = render_layout(n_tiles);
    size_t off = D.R.bytes;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b, 256);
        return o;
    };
    const size_t m = (size_t)(max_occ > 0 ? max_occ : 1), nt = (size_t)(n_tiles > 0 ? n_tiles : 1);
    D.cnt = take(4 * nt);
    D.base = take(4 * nt);
    D.total = take(8);
    D.partials = take(40 * m);
    D.keys = take(4 * m);
    D.vals = take(4 * m);
    D.keys2 = take(4 * m);
    D.vals2 = take(4 * m);
    D.scr_bytes = radix_sort_pairs_u32_scratch((int64_t)m);  // digit counts, then 256 digit totals
    D.sscr = take(D.scr_bytes);
    D.seg = take(8 * (size_t)(P > 0 ? P : 1));
    D.bytes = off;
    return D;
}

}  // namespace bgs

extern "C" size_t bgs_render_bwd_det_workspace_bytes(const bgs_frame* frame, int64_t P, int64_t max_occ) {
    if (!frame || frame->width <= 0 || frame->height <= 0 || P < 0 || max_occ < 0) return 0;
    const int n_tiles = ((frame->width + TILE - 1) / TILE) * ((frame->height + TILE - 1) / TILE);
    return det_layout(n_tiles, P, max_occ).bytes;
}

extern "C" bgs_status bgs_render_bwd_det(const bgs_frame* frame, const bgs_render_cfg* cfg, int64_t P,
                                         const float* final_T, const int32_t* n_contrib, const float* dL_dcolor,
                                         const float* dL_dalpha, const float* dL_ddepth, float* dL_dmeans2D,
                                         float* dL_dconic_opacity, float* dL_drgb, float* dL_ddepths,
                                         int64_t max_occ, int64_t* n_occ_host, void* ws, size_t ws_bytes,
                                         hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_render_bwd_det");
    if (st != BGS_OK) return st;
    if (!(tile_items(cfg) && cfg->subtile == 16))
        return fail(BGS_EUNSUPPORTED, "bgs_render_bwd_det: needs BGS_BALANCED_PIXEL with subtile 16 "
                                      "(one wave per tile)");
    BGS_REQUIRE(P >= 0 && max_occ >= 0 && n_occ_host, "bgs_render_bwd_det: bad P, max_occ or n_occ_host");
    BGS_REQUIRE(P < ((int64_t)1 << 32) && max_occ < ((int64_t)1 << 32), "bgs_render_bwd_det: sizes must be < 2^32");
    BGS_REQUIRE(final_T && n_contrib && dL_dcolor, "bgs_render_bwd_det: null forward state or dL_dcolor");
    BwdIO B{final_T, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
            nullptr, nullptr, 0};
    st = grad_outputs(cfg, dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepths, B, "bgs_render_bwd_det");
    if (st != BGS_OK) return st;
    const DetLayout D = det_layout(A.n_tiles, P, max_occ);
    BGS_REQUIRE(ws && ws_bytes >= D.bytes, "bgs_render_bwd_det: workspace too small");
    char* w = static_cast<char*>(ws);
    *n_occ_host = 0;
    if (!(cfg->flags & BGS_FLAG_QUEUE_READY)) {
        st = build_queue(A, cfg, n_contrib, w, D.R, stream, false);  // one item per tile: one writer per slot
        if (st != BGS_OK) return st;
    }
    auto* cnt = reinterpret_cast<uint32_t*>(w + D.cnt);
    auto* base = reinterpret_cast<uint32_t*>(w + D.base);
    auto* total = reinterpret_cast<uint64_t*>(w + D.total);
    if (A.n_tiles == 0) return BGS_OK;
    // cnt[t] = the entries the wide backward walks in tile t (its walk cost)
    hipLaunchKernelGGL(k_tile_costs, dim3((A.n_tiles + 3) / 4), dim3(256), 0, stream, A, n_contrib, 0, A.n_tiles,
                       cnt);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_det_scan, dim3(1), dim3(1024), 0, stream, A.n_tiles, cnt, base, total);
    BGS_HIP(hipGetLastError());
    uint64_t K = 0;
    BGS_HIP(hipMemcpyAsync(&K, total, sizeof(K), hipMemcpyDeviceToHost, stream));
    BGS_HIP(hipStreamSynchronize(stream));
    *n_occ_host = (int64_t)K;
    if ((int64_t)K > max_occ)
        return fail(BGS_ECAPACITY, "bgs_render_bwd_det: " + std::to_string(K) + " walked entries exceed max_occ " +
                                       std::to_string(max_occ));
    if (K == 0 || P == 0) return BGS_OK;
    auto* partials = reinterpret_cast<float*>(w + D.partials);
    B.det_partials = partials;
    B.det_base = base;
    auto* ctr = reinterpret_cast<uint32_t*>(w + D.R.ctr);
    auto* items = reinterpret_cast<const uint32_t*>(w + D.R.items);
    const int blocks = persistent_blocks(k_bwd_wide<false, true>, (uint32_t)A.n_tiles);
    hipLaunchKernelGGL((k_bwd_wide<false, true>), dim3(blocks), dim3(256), 0, stream, A, B, (const ViewDesc*)nullptr,
                       items, ctr, 0u);
    BGS_HIP(hipGetLastError());
    auto* keys = reinterpret_cast<uint32_t*>(w + D.keys);
    auto* vals = reinterpret_cast<uint32_t*>(w + D.vals);
    auto* keys2 = reinterpret_cast<uint32_t*>(w + D.keys2);
    auto* vals2 = reinterpret_cast<uint32_t*>(w + D.vals2);
    hipLaunchKernelGGL(k_det_keys, dim3(A.n_tiles), dim3(64), 0, stream, A, (const uint32_t*)cnt,
                       (const uint32_t*)base, keys, vals);
    BGS_HIP(hipGetLastError());
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < P) ++bits;
    bool second = false;
    st = radix_sort_pairs_u32((int64_t)K, bits, keys, vals, keys2, vals2, reinterpret_cast<uint32_t*>(w + D.sscr),
                              reinterpret_cast<uint32_t*>(w + D.sscr + D.scr_bytes - 4 * 256), &second, stream);
    if (st != BGS_OK) return st;
    const uint32_t* skeys = second ? keys2 : keys;
    const uint32_t* svals = second ? vals2 : vals;
    auto* seg = reinterpret_cast<uint32_t*>(w + D.seg);
    hipLaunchKernelGGL(k_det_clear, dim3((unsigned)((2 * P + 255) / 256)), dim3(256), 0, stream, P, seg);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_det_bounds, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, stream, (int64_t)K, P, skeys,
                       seg);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_det_reduce, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, stream, P, (const uint32_t*)seg,
                       svals, (const float*)partials, B);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

// ======================================================================
// Batched views in one graph: a cross-view queue (every sub-tile of every
// view, ranked by cost across views) feeds one persistent forward and one
// persistent backward launch; the gradient zero-fill, both cost passes and
// both queue builds (which reset the fetch counters with a kernel, not a
// memset) are captured with them into one hipGraph, so a training step over
// all views is a single hipGraphLaunch.
// ======================================================================
namespace bgs {

// zero the gradient outputs of every view (blockIdx.y = view)
__global__ __launch_bounds__(256) void k_zero_grads(const ViewDesc* __restrict__ views) {
    const ViewDesc& V = views[blockIdx.y];
    const int64_t P = V.P;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += stride) {
        reinterpret_cast<float2*>(V.B.g_means2D)[i] = make_float2(0.f, 0.f);
        reinterpret_cast<float4*>(V.B.g_conic_opacity)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        V.B.g_rgb[3 * i] = 0.f;
        V.B.g_rgb[3 * i + 1] = 0.f;
        V.B.g_rgb[3 * i + 2] = 0.f;
        if (V.B.g_depth) V.B.g_depth[i] = 0.f;
    }
}

}  // namespace bgs

struct bgs_plan {
    int n_views = 0;
    uint32_t total_tiles = 0;
    bgs::ViewDesc* d_views = nullptr;
    uint32_t* d_tile_off = nullptr;
    uint32_t* d_items = nullptr;
    uint32_t* d_cost = nullptr;
    uint32_t* d_ctr = nullptr;
    uint32_t* d_qhist = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" void bgs_plan_destroy(bgs_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    (void)hipFree(plan->d_views);
    (void)hipFree(plan->d_tile_off);
    (void)hipFree(plan->d_items);
    (void)hipFree(plan->d_cost);
    (void)hipFree(plan->d_ctr);
    (void)hipFree(plan->d_qhist);
    delete plan;
}

extern "C" bgs_status bgs_plan_create(bgs_plan** out, int32_t n_views, const bgs_frame* frames,
                                      const bgs_view_io* io, const bgs_render_cfg* cfg,
                                      const bgs_render_cfg* cfg_bwd, hipStream_t stream) {
    BGS_REQUIRE(out && frames && io && cfg, "bgs_plan_create: null argument");
    *out = nullptr;
    BGS_REQUIRE(n_views >= 1 && n_views <= MAX_VIEWS, "bgs_plan_create: 1..64 views");
    if (!cfg_bwd) cfg_bwd = cfg;
    if (cfg->variant != BGS_BALANCED_PIXEL || (cfg->subtile != 8 && cfg->subtile != 16))
        return fail(BGS_EUNSUPPORTED, "bgs_plan_create: the batched forward uses the balanced pixel-wise variant");
    if (cfg_bwd->variant != BGS_BALANCED_PIXEL || (cfg_bwd->subtile != 8 && cfg_bwd->subtile != 16))
        return fail(BGS_EUNSUPPORTED, "bgs_plan_create: the batched backward uses the balanced pixel-wise variant");
    if (cfg_bwd->order != BGS_ORDER_RASTER && cfg_bwd->order != BGS_ORDER_COST)
        return fail(BGS_EINVAL, "bgs_plan_create: unknown backward order");
    if ((cfg->flags | cfg_bwd->flags) & BGS_FLAG_PACKED_GRADS)
        return fail(BGS_EUNSUPPORTED, "bgs_plan_create: plans write the four gradient arrays (no packed records)");
    std::vector<ViewDesc> vd(n_views);
    std::vector<uint32_t> off(n_views + 1, 0);
    for (int v = 0; v < n_views; ++v) {
        FrameArgs A;
        bgs_status st = check_frame(&frames[v], cfg, A, "bgs_plan_create");
        if (st != BGS_OK) return st;
        const bgs_view_io& q = io[v];
        BGS_REQUIRE(q.P >= 0, "bgs_plan_create: view P < 0");
        BGS_REQUIRE(q.out_color && q.out_alpha && q.out_depth && q.final_T && q.n_contrib,
                    "bgs_plan_create: null forward output");
        BGS_REQUIRE(q.dL_dcolor && q.dL_dmeans2D && q.dL_dconic_opacity && q.dL_drgb,
                    "bgs_plan_create: null upstream or gradient buffer");
        BGS_REQUIRE((reinterpret_cast<uintptr_t>(q.dL_dconic_opacity) & 15) == 0 &&
                        (reinterpret_cast<uintptr_t>(q.dL_dmeans2D) & 7) == 0,
                    "bgs_plan_create: gradient buffers must be aligned like their inputs");
        BGS_REQUIRE((uint64_t)A.n_tiles < (1u << (VIEW_SHIFT - 2)), "bgs_plan_create: too many tiles in a view");
        vd[v].F = A;
        vd[v].O = FwdOut{q.out_color, q.out_alpha, q.out_depth, q.final_T, q.n_contrib};
        vd[v].B = BwdIO{q.final_T,     q.n_contrib,     q.dL_dcolor,       q.dL_dalpha, q.dL_ddepth,
                        q.dL_dmeans2D, q.dL_dconic_opacity, q.dL_drgb,     q.dL_ddepths, nullptr, nullptr};
        vd[v].P = q.P;
        off[v + 1] = off[v] + (uint32_t)A.n_tiles;
    }
    bgs_plan* plan = new bgs_plan();
    plan->n_views = n_views;
    plan->total_tiles = off[n_views];
    const size_t rounds = ((size_t)plan->total_tiles + QGROUPS - 1) / QGROUPS;
    auto cleanup_fail = [&](const std::string& what, hipError_t e) {
        bgs_plan_destroy(plan);
        return fail(BGS_EHIP, what + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMalloc(&plan->d_views, sizeof(ViewDesc) * n_views)) != hipSuccess) return cleanup_fail("hipMalloc", e);
    if ((e = hipMalloc(&plan->d_tile_off, sizeof(uint32_t) * (n_views + 1))) != hipSuccess)
        return cleanup_fail("hipMalloc", e);
    if ((e = hipMalloc(&plan->d_items, sizeof(uint32_t) * (rounds * NQ > 0 ? rounds * NQ : 1))) != hipSuccess)
        return cleanup_fail("hipMalloc", e);
    if ((e = hipMalloc(&plan->d_cost, sizeof(uint32_t) * (plan->total_tiles ? plan->total_tiles : 1))) != hipSuccess)
        return cleanup_fail("hipMalloc", e);
    if ((e = hipMalloc(&plan->d_ctr, sizeof(uint32_t) * (NQ * QSTRIDE + QSTRIDE))) != hipSuccess)
        return cleanup_fail("hipMalloc", e);
    if ((e = hipMalloc(&plan->d_qhist, sizeof(uint32_t) * NBUCKET * queue_groups((int)plan->total_tiles))) !=
        hipSuccess)
        return cleanup_fail("hipMalloc", e);
    if ((e = hipMemcpyAsync(plan->d_views, vd.data(), sizeof(ViewDesc) * n_views, hipMemcpyHostToDevice, stream)) !=
        hipSuccess)
        return cleanup_fail("hipMemcpyAsync", e);
    if ((e = hipMemcpyAsync(plan->d_tile_off, off.data(), sizeof(uint32_t) * (n_views + 1), hipMemcpyHostToDevice,
                            stream)) != hipSuccess)
        return cleanup_fail("hipMemcpyAsync", e);
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return cleanup_fail("hipStreamSynchronize", e);

    int64_t maxP = 1;
    for (int v = 0; v < n_views; ++v) maxP = std::max<int64_t>(maxP, io[v].P);
    const unsigned zero_blocks = (unsigned)std::min<int64_t>((maxP + 255) / 256, 1024);
    const uint32_t n_items = plan->total_tiles * 4u;
    const bool fwd_wide = tile_items(cfg);
    const int fblocks = fwd_wide ? persistent_blocks(k_fwd_wide<true>, plan->total_tiles)
                                 : persistent_blocks(k_fwd_pixel<true, true>, n_items);
    const bool bwd_wide = tile_items(cfg_bwd);
    const int bblocks = bwd_wide ? persistent_blocks(k_bwd_wide<true>, plan->total_tiles)
                                 : persistent_blocks(k_bwd_pixel<true, true>, n_items);
    const int by_cost = cfg->order == BGS_ORDER_COST;
    const int bwd_by_cost = cfg_bwd->order == BGS_ORDER_COST;
    const FrameArgs F0{};
    const FwdOut O0{};
    const BwdIO B0{};

    // record on a private stream (the legacy default stream cannot capture);
    // the graph is launched later on the caller's stream
    hipStream_t cap = nullptr;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
        return cleanup_fail("hipStreamCreateWithFlags", e);
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed)) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return cleanup_fail("hipStreamBeginCapture", e);
    }
    stream = cap;
    hipLaunchKernelGGL(k_zero_grads, dim3(zero_blocks, n_views), dim3(256), 0, stream, plan->d_views);
    if (by_cost)
        hipLaunchKernelGGL(k_tile_costs_mv, dim3(plan->total_tiles), dim3(256), 0, stream, plan->d_views,
                           plan->d_tile_off, n_views, 0, plan->d_cost);
    launch_queue(stream, (int)plan->total_tiles, plan->d_cost, by_cost, fwd_wide ? 1 : 0, plan->d_tile_off, n_views,
                 0, 0, plan->d_qhist, plan->d_items, plan->d_ctr);
    if (fwd_wide)
        hipLaunchKernelGGL((k_fwd_wide<true>), dim3(fblocks), dim3(256), 0, stream, F0, O0, plan->d_views,
                           plan->d_items, plan->d_ctr, 0u);
    else
        hipLaunchKernelGGL((k_fwd_pixel<true, true>), dim3(fblocks), dim3(256), 0, stream, F0, O0, plan->d_views,
                           plan->d_items, plan->d_ctr);
    if (bwd_by_cost)
        hipLaunchKernelGGL(k_tile_costs_mv, dim3(plan->total_tiles), dim3(256), 0, stream, plan->d_views,
                           plan->d_tile_off, n_views, 1, plan->d_cost);
    launch_queue(stream, (int)plan->total_tiles, plan->d_cost, bwd_by_cost, bwd_wide ? 1 : 0, plan->d_tile_off,
                 n_views, 0, 0, plan->d_qhist, plan->d_items, plan->d_ctr);
    if (bwd_wide)
        hipLaunchKernelGGL((k_bwd_wide<true>), dim3(bblocks), dim3(256), 0, stream, F0, B0, plan->d_views,
                           plan->d_items, plan->d_ctr, 0u);
    else
        hipLaunchKernelGGL((k_bwd_pixel<true, true>), dim3(bblocks), dim3(256), 0, stream, F0, B0, plan->d_views,
                           plan->d_items, plan->d_ctr);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return cleanup_fail("hipStreamEndCapture", e);
    plan->graph = graph;
    if ((e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0)) != hipSuccess)
        return cleanup_fail("hipGraphInstantiate", e);
    *out = plan;
    return BGS_OK;
}

extern "C" bgs_status bgs_plan_launch(bgs_plan* plan, hipStream_t stream) {
    BGS_REQUIRE(plan && plan->exec, "bgs_plan_launch: null plan");
    BGS_HIP(hipGraphLaunch(plan->exec, stream));
    return BGS_OK;
}
