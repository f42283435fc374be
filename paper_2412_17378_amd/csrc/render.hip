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
#include "common.h"

namespace bgs {

constexpr float KA = -0.5f * LOG2E;  // a -> a2
constexpr float KB = -LOG2E;         // b -> b2
constexpr int NBUCKET = 136;         // cost buckets: 0 and quarter-octaves of 1 .. 2^33

struct FrameArgs {
    int W, H, TX, TY, n_tiles;
    const uint32_t* __restrict__ ranges;
    const uint32_t* __restrict__ point_list;
    const float2* __restrict__ means2D;
    const float4* __restrict__ conic_opacity;
    const float* __restrict__ rgb;
    const float* __restrict__ depth;
    float bg0, bg1, bg2;
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
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Load one Gaussian of the list into registers in the staged (pre-scaled) form.
__device__ __forceinline__ void load_splat(const FrameArgs& F, uint32_t g, float2& xy, float4& co, float4& cd) {
    xy = F.means2D[g];
    const float4 c = F.conic_opacity[g];
    co = make_float4(c.x * KA, c.y * KB, c.z * KA, c.w);
    cd = make_float4(F.rgb[3 * g], F.rgb[3 * g + 1], F.rgb[3 * g + 2], F.depth[g]);
}

struct Pix {
    float T, C0, C1, C2, D;
    int last;
    bool done;
};

// One list entry at list position pos (0-based) for one pixel.  Branch-free:
// a skipped or stopping entry blends with weight 0 and leaves T unchanged.
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
}

// ------------------------------------------------------------------ static
__global__ __launch_bounds__(256) void k_fwd_static(FrameArgs F, FwdOut O) {
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
        for (int j = 0; j < cnt; ++j) {
            if (s.done) break;
            blend(fx, fy, s_xy[j], s_co[j], s_cd[j], pos0 + j, s);
        }
    }
    if (inside) write_pixel(F, O, px, py, s);
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

template <bool PERSISTENT>
__global__ __launch_bounds__(256) void k_fwd_pixel(FrameArgs F, FwdOut O, const uint32_t* __restrict__ items,
                                                   uint32_t* __restrict__ ctr) {
    __shared__ float2 s_xy[4][64];
    __shared__ float4 s_co[4][64];
    __shared__ float4 s_cd[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t n_items = PERSISTENT ? ctr[1] : 0u;
    for (;;) {
        uint32_t item;
        if (PERSISTENT) {
            uint32_t q = 0;
            if (lane == 0) q = atomicAdd(&ctr[0], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (q >= n_items) break;
            item = items[q];
        } else {
            item = blockIdx.x * 4 + wv;
        }
        int tile, px, py;
        bool any_inside;
        item_pixel(F, item, lane, tile, px, py, any_inside);
        if (any_inside) {
            const bool inside = px < F.W && py < F.H;
            const uint32_t start = F.ranges[2 * tile], end = F.ranges[2 * tile + 1];
            Pix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
            const float fx = (float)px, fy = (float)py;
            for (uint32_t base = start; base < end; base += 64) {
                if (ballot(!s.done) == 0) break;
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
                for (int j = 0; j < cnt; ++j) {
                    if (s.done) break;
                    blend(fx, fy, s_xy[wv][j], s_co[wv][j], s_cd[wv][j], pos0 + j, s);
                }
                wave_sync();
            }
            if (inside) write_pixel(F, O, px, py, s);
        }
        if (!PERSISTENT) break;
    }
}

// ------------------------------------------------------------------ backward
template <bool PERSISTENT>
__global__ __launch_bounds__(256) void k_bwd_pixel(FrameArgs F, BwdIO B, const uint32_t* __restrict__ items,
                                                   uint32_t* __restrict__ ctr) {
    __shared__ float2 s_xy[4][64];
    __shared__ float4 s_co[4][64];
    __shared__ float4 s_cd[4][64];
    __shared__ float4 s_abc[4][64];  // raw conic a, b, c and the Gaussian id (bits)
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t n_items = PERSISTENT ? ctr[1] : 0u;
    const int64_t HW = (int64_t)F.W * F.H;
    for (;;) {
        uint32_t item;
        if (PERSISTENT) {
            uint32_t q = 0;
            if (lane == 0) q = atomicAdd(&ctr[0], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (q >= n_items) break;
            item = items[q];
        } else {
            item = blockIdx.x * 4 + wv;
        }
        int tile, px, py;
        bool any_inside;
        item_pixel(F, item, lane, tile, px, py, any_inside);
        if (any_inside) {
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
            const int max_n = wave_max(nc);
            float T = TN, R0 = 0.f, R1 = 0.f, R2 = 0.f, Rd = 0.f;
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
                        const float dA = Tb * (gC0 * cd.x + gC1 * cd.y + gC2 * cd.z + gD * cd.w) -
                                         inv * (gC0 * R0 + gC1 * R1 + gC2 * R2 + gD * Rd + kconst);
                        R0 = __builtin_fmaf(cd.x, w, R0);
                        R1 = __builtin_fmaf(cd.y, w, R1);
                        R2 = __builtin_fmaf(cd.z, w, R2);
                        Rd = __builtin_fmaf(cd.w, w, Rd);
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
                    v0 = wave_sum(v0); v1 = wave_sum(v1); v2 = wave_sum(v2); v3 = wave_sum(v3);
                    v4 = wave_sum(v4); v5 = wave_sum(v5); v6 = wave_sum(v6); v7 = wave_sum(v7);
                    v8 = wave_sum(v8); v9 = wave_sum(v9);
                    if (lane == 0) {
                        const uint32_t g = __float_as_uint(s_abc[wv][jj].w);
                        unsafeAtomicAdd(&B.g_means2D[2 * g], v0);
                        unsafeAtomicAdd(&B.g_means2D[2 * g + 1], v1);
                        unsafeAtomicAdd(&B.g_conic_opacity[4 * g], v2);
                        unsafeAtomicAdd(&B.g_conic_opacity[4 * g + 1], v3);
                        unsafeAtomicAdd(&B.g_conic_opacity[4 * g + 2], v4);
                        unsafeAtomicAdd(&B.g_conic_opacity[4 * g + 3], v5);
                        unsafeAtomicAdd(&B.g_rgb[3 * g], v6);
                        unsafeAtomicAdd(&B.g_rgb[3 * g + 1], v7);
                        unsafeAtomicAdd(&B.g_rgb[3 * g + 2], v8);
                        if (B.g_depth) unsafeAtomicAdd(&B.g_depth[g], v9);
                    }
                }
                wave_sync();
            }
        }
        if (!PERSISTENT) break;
    }
}

// ---------------------------------------------------------------- task pool
__device__ __forceinline__ int cost_bucket(uint32_t c) {
    if (c == 0) return 0;
    const int b = 1 + (int)(__log2f((float)c) * 4.0f);
    return b < NBUCKET - 1 ? b : NBUCKET - 1;
}

// Cost of every item: forward = list length of its tile; backward = the
// largest n_contrib among its 64 pixels (one wave per item).
__global__ __launch_bounds__(256) void k_item_costs(FrameArgs F, const int* __restrict__ n_contrib, uint32_t n_items,
                                                    uint32_t* __restrict__ cost) {
    const int lane = threadIdx.x & 63;
    const uint32_t item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= n_items) return;
    int tile, px, py;
    bool any_inside;
    item_pixel(F, item, lane, tile, px, py, any_inside);
    uint32_t c = 0;
    if (any_inside) {
        if (n_contrib) {
            const bool inside = px < F.W && py < F.H;
            const int nc = inside ? n_contrib[(int64_t)py * F.W + px] : 0;
            c = (uint32_t)wave_max(nc);
        } else {
            c = F.ranges[2 * tile + 1] - F.ranges[2 * tile];
        }
    }
    if (lane == 0) cost[item] = c;
}

// Single workgroup: raster order, or a counting sort by descending cost
// bucket (largest first).  Also resets the fetch counter: ctr[0] = 0,
// ctr[1] = number of items.
__global__ __launch_bounds__(1024) void k_queue(uint32_t n_items, const uint32_t* __restrict__ cost, int by_cost,
                                                uint32_t* __restrict__ items, uint32_t* __restrict__ ctr) {
    __shared__ uint32_t hist[NBUCKET];
    if (!by_cost) {
        for (uint32_t i = threadIdx.x; i < n_items; i += blockDim.x) items[i] = i;
    } else {
        for (int b = threadIdx.x; b < NBUCKET; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n_items; i += blockDim.x)
            atomicAdd(&hist[NBUCKET - 1 - cost_bucket(cost[i])], 1u);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int b = 0; b < NBUCKET; ++b) {
                const uint32_t h = hist[b];
                hist[b] = run;
                run += h;
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n_items; i += blockDim.x) {
            const uint32_t pos = atomicAdd(&hist[NBUCKET - 1 - cost_bucket(cost[i])], 1u);
            items[pos] = i;
        }
    }
    if (threadIdx.x == 0) {
        ctr[0] = 0;
        ctr[1] = n_items;
    }
}

// ---------------------------------------------------------------- host side
struct RenderLayout {
    size_t ctr, items, cost, bytes;
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
    L.ctr = take(256);
    L.items = take(4 * (size_t)(L.n_items ? L.n_items : 1));
    L.cost = take(4 * (size_t)(L.n_items ? L.n_items : 1));
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
    if (cfg->variant < BGS_STATIC || cfg->variant > BGS_BALANCED_HYBRID)
        return fail(BGS_EINVAL, std::string(who) + ": unknown variant");
    if (cfg->variant != BGS_STATIC && cfg->variant != BGS_BALANCED_PIXEL)
        return fail(BGS_EUNSUPPORTED, std::string(who) + ": variant not built yet");
    if (cfg->variant != BGS_STATIC && cfg->subtile != 8)
        return fail(BGS_EUNSUPPORTED, std::string(who) + ": balanced variants take 8x8 sub-tiles");
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

static bgs_status build_queue(const FrameArgs& A, const bgs_render_cfg* cfg, const int* n_contrib, char* ws,
                              const RenderLayout& L, hipStream_t stream) {
    auto* ctr = reinterpret_cast<uint32_t*>(ws + L.ctr);
    auto* items = reinterpret_cast<uint32_t*>(ws + L.items);
    auto* cost = reinterpret_cast<uint32_t*>(ws + L.cost);
    const int by_cost = cfg->order == BGS_ORDER_COST;
    if (by_cost) {
        hipLaunchKernelGGL(k_item_costs, dim3((L.n_items + 3) / 4), dim3(256), 0, stream, A, n_contrib, L.n_items,
                           cost);
        BGS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_queue, dim3(1), dim3(1024), 0, stream, L.n_items, cost, by_cost, items, ctr);
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
    FwdOut O{out_color, out_alpha, out_depth, final_T, n_contrib};
    if (cfg->variant == BGS_STATIC) {
        hipLaunchKernelGGL(k_fwd_static, dim3(A.n_tiles), dim3(256), 0, stream, A, O);
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
    const int blocks = persistent_blocks(k_fwd_pixel<true>, L.n_items);
    hipLaunchKernelGGL(k_fwd_pixel<true>, dim3(blocks), dim3(256), 0, stream, A, O, items, ctr);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

extern "C" bgs_status bgs_render_bwd(const bgs_frame* frame, const bgs_render_cfg* cfg, const float* final_T,
                                     const int32_t* n_contrib, const float* dL_dcolor, const float* dL_dalpha,
                                     const float* dL_ddepth, float* dL_dmeans2D, float* dL_dconic_opacity,
                                     float* dL_drgb, float* dL_ddepths, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
    FrameArgs A;
    bgs_status st = check_frame(frame, cfg, A, "bgs_render_bwd");
    if (st != BGS_OK) return st;
    BGS_REQUIRE(final_T && n_contrib && dL_dcolor, "bgs_render_bwd: null forward state or dL_dcolor");
    BGS_REQUIRE(dL_dmeans2D && dL_dconic_opacity && dL_drgb, "bgs_render_bwd: null gradient output");
    BwdIO B{final_T, n_contrib, dL_dcolor, dL_dalpha, dL_ddepth, dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepths};
    if (cfg->variant == BGS_STATIC) {
        hipLaunchKernelGGL(k_bwd_pixel<false>, dim3(A.n_tiles), dim3(256), 0, stream, A, B, nullptr, nullptr);
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
    const int blocks = persistent_blocks(k_bwd_pixel<true>, L.n_items);
    hipLaunchKernelGGL(k_bwd_pixel<true>, dim3(blocks), dim3(256), 0, stream, A, B, items, ctr);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}
