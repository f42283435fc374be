// Tile binning, per-tile sort and ranges: the pre-processing that produces the
// sorted point list PL and the per-tile ranges the render kernels walk
// (Balanced 3DGS Sec. 4.3 "patch"; Eq. (4) needs each tile's Gaussians
// front to back).
//
// Instead of one 64-bit (tile | depth) sort over all M pairs, the pairs are
// emitted with the Gaussians already in depth order (a 32-bit sort over P
// Gaussians, P << M), so the M pairs only need a stable sort by tile id:
// ceil(log2(n_tiles)) key bits (13 at 1080p) instead of 45.  The result is
// the same list a (tile, depth, id) sort gives.
#include <algorithm>
#include <cstring>

#include <rocprim/block/block_reduce.hpp>
#include <rocprim/block/block_scan.hpp>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"

namespace bgs {

// ----------------------------------------------------------------------
// Depth order of the Gaussians: a stable sort of 32-bit keys (positive fp32
// depths order like their bit patterns; Gaussians with no pairs get the
// largest key and go last), so equal depths keep id order.  LSD radix sort,
// four passes of 8 bits, over blocks of DS_TILE = 2048 consecutive items
// (512 threads; wave w of the block owns items [256 w, 256 w + 256), 64 at a
// time: 245 blocks at P = 500 k, so every pass spreads over the CUs).  Per pass: every block's digit histogram (the first one fused into
// the key generation), an exclusive scan of each digit's counts over the
// blocks, and a scatter in which each block ranks its items stably in LDS
// (ballots over the 8 digit bits find the lanes with the same digit) and
// writes them out as per-digit runs.  Grids depend on P alone and nothing is
// cleared with a memset, so the sort can be captured into a graph.
// ----------------------------------------------------------------------
constexpr int DS_THREADS = 512;
constexpr int DS_WAVES = DS_THREADS / 64;
constexpr int DS_TILE = DS_THREADS * 4;
constexpr int DS_RADIX = 256;

static inline int ds_blocks(int64_t P) { return (int)((P + DS_TILE - 1) / DS_TILE); }

__device__ __forceinline__ int64_t ds_item(int j) {  // item j (0..3) of this lane, block-relative
    return (int64_t)(threadIdx.x >> 6) * 256 + j * 64 + (threadIdx.x & 63);
}

// cnt[d * nb + b] = number of block b's items with digit d
__device__ __forceinline__ void ds_hist_store(uint32_t* s_hist, uint32_t* __restrict__ cnt, int nb) {
    __syncthreads();
    if (threadIdx.x < DS_RADIX) cnt[(size_t)threadIdx.x * nb + blockIdx.x] = s_hist[threadIdx.x];
}

// Tile rectangles of the fused list builder, computed with the depth keys
// (both are one pass over the projected Gaussians): rect[g] for every g, or
// nothing when rect is null.  conic_opacity non-null: the exact ellipse-tile
// rule.  gaussian_rect is defined with the binning rules below.
struct RectArgs {
    int TX, TY;
    const float* means2D;
    const int* radius;
    const float4* conic_opacity;
    uint2* rect;
};

template <bool EXACT>
__device__ uint2 gaussian_rect(int64_t g, const RectArgs& R, bool listed);

// Also stores the AND and the OR of the block's keys of listed Gaussians at
// andor[2 b], [2 b + 1] (k_ds_colscan of the first pass folds them into the
// mask of key bits that vary: a later pass whose byte does not vary keeps
// the listed Gaussians' order; the others, which emit no pairs, may end up
// anywhere).
// RECT: 0 no rectangles, 1 the square rule's, 2 the exact rule's (R).
template <int RECT>
__global__ __launch_bounds__(DS_THREADS) void k_ds_keys(int64_t P, const float* __restrict__ depth,
                                                        const uint32_t* __restrict__ tiles_touched,
                                                        uint32_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                        uint32_t* __restrict__ cnt, int nb,
                                                        uint32_t* __restrict__ andor, RectArgs R) {
    __shared__ uint32_t s_hist[DS_RADIX];
    __shared__ uint32_t s_and, s_or;
    if (threadIdx.x < DS_RADIX) s_hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        s_and = ~0u;
        s_or = 0u;
    }
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * DS_TILE;
    uint32_t a = ~0u, o = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + ds_item(j);
        if (i < P) {
            const bool listed = tiles_touched[i] != 0u;
            const uint32_t k = listed ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
            keys[i] = k;
            ids[i] = (uint32_t)i;
            if (RECT) R.rect[i] = gaussian_rect<RECT == 2>(i, R, listed);
            atomicAdd(&s_hist[k & 0xFFu], 1u);
            if (listed) {  // a Gaussian with no pairs may sit anywhere in the order
                a &= k;
                o |= k;
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {  // over the wave first: one LDS atomic per wave
        a &= (uint32_t)__shfl_xor((int)a, off, 64);
        o |= (uint32_t)__shfl_xor((int)o, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAnd(&s_and, a);
        atomicOr(&s_or, o);
    }
    ds_hist_store(s_hist, cnt, nb);  // (synchronizes)
    if (threadIdx.x == 0) {
        andor[2 * blockIdx.x] = s_and;
        andor[2 * blockIdx.x + 1] = s_or;
    }
}

// Whether the byte of the keys at `shift` varies (vary: the mask of key bits
// that differ between keys; null: sort every pass).
__device__ __forceinline__ bool ds_byte_varies(const uint32_t* vary, int shift) {
    return !vary || ((*vary >> shift) & 0xFFu) != 0u;
}

__global__ __launch_bounds__(DS_THREADS) void k_ds_hist(int64_t P, const uint32_t* __restrict__ keys, int shift,
                                                        uint32_t* __restrict__ cnt, int nb,
                                                        const uint32_t* __restrict__ vary) {
    if (!ds_byte_varies(vary, shift)) return;  // an identity pass
    __shared__ uint32_t s_hist[DS_RADIX];
    if (threadIdx.x < DS_RADIX) s_hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * DS_TILE;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + ds_item(j);
        if (i < P) atomicAdd(&s_hist[(keys[i] >> shift) & 0xFFu], 1u);
    }
    ds_hist_store(s_hist, cnt, nb);
}

// One workgroup per digit d: exclusive scan of cnt[d][0..nb) in place,
// tot[d] = the digit's total.
// First pass (andor given): workgroup 0 also folds the blocks' key ANDs and
// ORs into tot[DS_RADIX] = the mask of key bits that vary.  Later passes
// (vary given) leave an identity pass alone.
__global__ __launch_bounds__(256) void k_ds_colscan(int nb, uint32_t* __restrict__ cnt, uint32_t* __restrict__ tot,
                                                    const uint32_t* __restrict__ andor, int shift,
                                                    const uint32_t* __restrict__ vary) {
    using Scan = rocprim::block_scan<uint32_t, 256>;
    __shared__ typename Scan::storage_type s_scan;
    if (!ds_byte_varies(vary, shift)) return;
    if (andor && blockIdx.x == 0) {
        __shared__ uint32_t s_and, s_or;
        if (threadIdx.x == 0) {
            s_and = ~0u;
            s_or = 0u;
        }
        __syncthreads();
        uint32_t a = ~0u, o = 0u;
        for (int b = threadIdx.x; b < nb; b += 256) {
            a &= andor[2 * b];
            o |= andor[2 * b + 1];
        }
        atomicAnd(&s_and, a);
        atomicOr(&s_or, o);
        __syncthreads();
        if (threadIdx.x == 0) tot[DS_RADIX] = s_and ^ s_or;
    }
    uint32_t* c = cnt + (size_t)blockIdx.x * nb;
    const int per = (nb + 255) / 256;
    const int t0 = min(nb, (int)threadIdx.x * per), t1 = min(nb, t0 + per);
    uint32_t sum = 0;
    for (int t = t0; t < t1; ++t) sum += c[t];
    uint32_t run = 0, total = 0;
    Scan().exclusive_scan(sum, run, 0u, total, s_scan);
    for (int t = t0; t < t1; ++t) {
        const uint32_t v = c[t];
        c[t] = run;
        run += v;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Block b's items go to keys_out / vals_out at base[d] + (rank among the
// block's items of digit d), base[d] = (items with a smaller digit) + (items
// of digit d in earlier blocks).  KEYS = false skips the key output (the last
// pass only needs the values).
template <bool KEYS>
__global__ __launch_bounds__(DS_THREADS) void k_ds_scatter(int64_t P, const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out, int shift,
                                                           const uint32_t* __restrict__ cnt,
                                                           const uint32_t* __restrict__ tot, int nb,
                                                           const uint32_t* __restrict__ vary) {
    if (!ds_byte_varies(vary, shift)) {  // every key has this byte: the pass keeps the order
        const int64_t b0 = (int64_t)blockIdx.x * DS_TILE;
        for (int j = 0; j < 4; ++j) {
            const int64_t i = b0 + ds_item(j);
            if (i < P) {
                if (KEYS) keys_out[i] = keys_in[i];
                vals_out[i] = vals_in[i];
            }
        }
        return;
    }
    using Scan = rocprim::block_scan<uint32_t, DS_THREADS>;
    __shared__ typename Scan::storage_type s_scan;
    __shared__ uint32_t s_wcnt[DS_WAVES][DS_RADIX];  // per-wave digit counts, then their offsets
    __shared__ uint32_t s_keys[DS_TILE], s_vals[DS_TILE];
    __shared__ uint32_t s_lstart[DS_RADIX], s_base[DS_RADIX];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < DS_WAVES * DS_RADIX; i += DS_THREADS) (&s_wcnt[0][0])[i] = 0u;
    const int64_t b0 = (int64_t)blockIdx.x * DS_TILE;
    const int n_valid = (int)min((int64_t)DS_TILE, P - b0);
    uint32_t k[4], v[4], d[4], r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + ds_item(j);
        k[j] = i < P ? keys_in[i] : 0u;
        v[j] = i < P ? vals_in[i] : 0u;
        d[j] = (k[j] >> shift) & 0xFFu;
    }
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool valid = ds_item(j) < n_valid;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d[j] >> bit) & 1u;
            const uint64_t bal = ballot(set);
            peers &= set ? bal : ~bal;
        }
        // the wave's items so far with this digit, then this batch's earlier lanes
        const uint32_t prior = valid ? s_wcnt[w][d[j]] : 0u;
        r[j] = prior + (uint32_t)__builtin_popcountll(peers & lt);
        if (valid && (peers & lt) == 0ull) s_wcnt[w][d[j]] = prior + (uint32_t)__builtin_popcountll(peers);
    }
    __syncthreads();
    uint32_t nd = 0;  // the block's count of digit tid (tid < 256)
    if (tid < DS_RADIX) {
#pragma unroll
        for (int ww = 0; ww < DS_WAVES; ++ww) {
            const uint32_t c = s_wcnt[ww][tid];
            s_wcnt[ww][tid] = nd;
            nd += c;
        }
    }
    uint32_t lstart = 0, dbase = 0, agg = 0;
    Scan().exclusive_scan(nd, lstart, 0u, agg, s_scan);
    __syncthreads();
    Scan().exclusive_scan(tid < DS_RADIX ? tot[tid] : 0u, dbase, 0u, agg, s_scan);
    if (tid < DS_RADIX) {
        s_lstart[tid] = lstart;
        s_base[tid] = dbase + cnt[(size_t)tid * nb + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (ds_item(j) < n_valid) {
            const uint32_t pos = s_lstart[d[j]] + s_wcnt[w][d[j]] + r[j];
            s_keys[pos] = k[j];
            s_vals[pos] = v[j];
        }
    }
    __syncthreads();
    for (int i = tid; i < n_valid; i += DS_THREADS) {
        const uint32_t kk = s_keys[i];
        const uint32_t dd = (kk >> shift) & 0xFFu;
        const uint32_t dest = s_base[dd] + (uint32_t)i - s_lstart[dd];
        if (KEYS) keys_out[dest] = kk;
        vals_out[dest] = s_vals[i];
    }
}

// Stable sort of n (key, value) pairs by the low `bits` bits of the key with
// the same passes (ceil(bits / 8) of them, first histogram included).  The
// pairs start in (k0, v0); the sorted pairs end in (k0, v0) or (k1, v1):
// *in_second tells which.  cnt [256 ds_blocks(n)] and tot [256] are scratch.
bgs_status radix_sort_pairs_u32(int64_t n, int bits, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                                uint32_t* cnt, uint32_t* tot, bool* in_second, hipStream_t stream) {
    *in_second = false;
    if (n <= 0) return BGS_OK;
    const int nb = ds_blocks(n);
    const int passes = bits <= 0 ? 0 : (bits + 7) / 8;
    uint32_t *kin = k0, *vin = v0, *kout = k1, *vout = v1;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        const uint32_t* no_skip = nullptr;
        hipLaunchKernelGGL(k_ds_hist, dim3(nb), dim3(DS_THREADS), 0, stream, n, (const uint32_t*)kin, shift, cnt, nb,
                           no_skip);
        BGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_ds_colscan, dim3(DS_RADIX), dim3(256), 0, stream, nb, cnt, tot, no_skip, shift, no_skip);
        BGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_ds_scatter<true>, dim3(nb), dim3(DS_THREADS), 0, stream, n, (const uint32_t*)kin,
                           (const uint32_t*)vin, kout, vout, shift, (const uint32_t*)cnt, (const uint32_t*)tot, nb,
                           no_skip);
        BGS_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
        *in_second = !*in_second;
    }
    return BGS_OK;
}

size_t radix_sort_pairs_u32_scratch(int64_t n) { return 4 * ((size_t)DS_RADIX * ds_blocks(n > 0 ? n : 1) + DS_RADIX); }

// Words of tot for depth_order: the digit totals, the mask of varying key
// bits, and two words per block.
static size_t depth_order_tot_words(int64_t P) { return DS_RADIX + 1 + 2 * (size_t)ds_blocks(P > 0 ? P : 1); }

// Sorted Gaussian ids into order[P]; keys / keys2 / ids2 [P] are scratch,
// cnt [256 ds_blocks(P)] and tot [depth_order_tot_words(P)] the histograms.
// A pass whose byte is the same in every key (typically the top one: depths
// within one or two binades share it) is an identity pass and runs as a copy.
static bgs_status depth_order(int64_t P, const float* depth, const uint32_t* tiles_touched, uint32_t* keys,
                              uint32_t* order, uint32_t* keys2, uint32_t* ids2, uint32_t* cnt, uint32_t* tot,
                              const RectArgs& R, hipStream_t stream) {
    if (P == 0) return BGS_OK;
    const int nb = ds_blocks(P);
    uint32_t* andor = tot + DS_RADIX + 1;
    const uint32_t* vary = tot + DS_RADIX;
    if (!R.rect)
        hipLaunchKernelGGL(k_ds_keys<0>, dim3(nb), dim3(DS_THREADS), 0, stream, P, depth, tiles_touched, keys, order,
                           cnt, nb, andor, R);
    else if (R.conic_opacity)
        hipLaunchKernelGGL(k_ds_keys<2>, dim3(nb), dim3(DS_THREADS), 0, stream, P, depth, tiles_touched, keys, order,
                           cnt, nb, andor, R);
    else
        hipLaunchKernelGGL(k_ds_keys<1>, dim3(nb), dim3(DS_THREADS), 0, stream, P, depth, tiles_touched, keys, order,
                           cnt, nb, andor, R);
    BGS_HIP(hipGetLastError());
    // (keys, order) -> (keys2, ids2) -> (keys, order) -> ... : four passes end in order
    uint32_t* kin = keys;
    uint32_t* vin = order;
    uint32_t* kout = keys2;
    uint32_t* vout = ids2;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        // the first pass sorts always (its histogram came with the keys) and finds the varying bits
        const uint32_t* skip = pass > 0 ? vary : nullptr;
        if (pass > 0) {
            hipLaunchKernelGGL(k_ds_hist, dim3(nb), dim3(DS_THREADS), 0, stream, P, (const uint32_t*)kin, shift, cnt,
                               nb, skip);
            BGS_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_ds_colscan, dim3(DS_RADIX), dim3(256), 0, stream, nb, cnt, tot,
                           pass == 0 ? (const uint32_t*)andor : nullptr, shift, skip);
        BGS_HIP(hipGetLastError());
        if (pass < 3)
            hipLaunchKernelGGL(k_ds_scatter<true>, dim3(nb), dim3(DS_THREADS), 0, stream, P, (const uint32_t*)kin,
                               (const uint32_t*)vin, kout, vout, shift, (const uint32_t*)cnt, (const uint32_t*)tot, nb,
                               skip);
        else
            hipLaunchKernelGGL(k_ds_scatter<false>, dim3(nb), dim3(DS_THREADS), 0, stream, P, (const uint32_t*)kin,
                               (const uint32_t*)vin, kout, vout, shift, (const uint32_t*)cnt, (const uint32_t*)tot, nb,
                               skip);
        BGS_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return BGS_OK;
}

__global__ __launch_bounds__(256) void k_gather_counts(int64_t P, const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ tiles_touched,
                                                       uint64_t* __restrict__ counts) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    counts[k] = tiles_touched[order[k]];
}

// offsets[k] = exclusive prefix of counts; the total lands in total[0]
__global__ void k_total(int64_t P, const uint64_t* __restrict__ offsets, const uint32_t* __restrict__ order,
                        const uint32_t* __restrict__ tiles_touched, uint64_t* __restrict__ total) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        total[0] = P > 0 ? offsets[P - 1] + tiles_touched[order[P - 1]] : 0;
}

// Pair emission, wave-cooperative so that stores are coalesced: each wave
// owns 64 consecutive Gaussians of the depth order and walks them one at a
// time; the 64 lanes write consecutive pairs of the current Gaussian's run
// (pair j of a w x h rectangle is tile (x0 + j % w, y0 + j / w)).
__global__ __launch_bounds__(256) void k_emit(int64_t P, int TX, int TY, const uint32_t* __restrict__ order,
                                              const uint64_t* __restrict__ offsets, const float* __restrict__ means2D,
                                              const int* __restrict__ radius,
                                              const uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ values) {
    const int lane = threadIdx.x & 63;
    const int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;  // first Gaussian of this wave
    if (base >= P) return;
    const int64_t k = base + lane;
    uint32_t g = 0, n = 0;
    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    uint64_t o = 0;
    if (k < P) {
        g = order[k];
        if (tiles_touched[g] != 0 &&
            tile_rect(means2D[2 * g], means2D[2 * g + 1], radius[g], TX, TY, x0, y0, x1, y1)) {
            // never more than this Gaussian's own run, whatever tiles_touched says
            const uint32_t area = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
            n = area < tiles_touched[g] ? area : tiles_touched[g];
            o = offsets[k];
        }
    }
    const int cnt = (int)((P - base) < 64 ? (P - base) : 64);
    for (int i = 0; i < cnt; ++i) {
        const uint32_t ni = __builtin_amdgcn_readlane(n, i);
        if (ni == 0) continue;
        const uint32_t gi = __builtin_amdgcn_readlane(g, i);
        const int xi = __builtin_amdgcn_readlane(x0, i), yi = __builtin_amdgcn_readlane(y0, i);
        const int wi = __builtin_amdgcn_readlane(x1, i) - xi + 1;
        const uint64_t oi = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(o >> 32), i) << 32) |
                            (uint64_t)__builtin_amdgcn_readlane((uint32_t)o, i);
        const float inv_w = 1.0f / (float)wi;
        for (uint32_t j = lane; j < ni; j += 64) {
            // j / wi via a float estimate and one correction step (j < 2^24)
            int q = (int)((float)j * inv_w);
            int r = (int)j - q * wi;
            if (r >= wi) { ++q; r -= wi; }
            if (r < 0) { --q; r += wi; }
            keys[oi + j] = (uint32_t)((yi + q) * TX + xi + r);
            values[oi + j] = gi;
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ranges from sorted tile keys: a new tile starts where the key changes
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, int64_t n, int n_tiles,
                                                uint32_t* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = keys[i];
    if (t >= (uint32_t)n_tiles) return;
    if (i == 0 || keys[i - 1] != t) ranges[2 * t] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
}

static unsigned blocks_for(int64_t n, int threads = 256) { return (unsigned)((n + threads - 1) / threads); }

struct BinLayout {
    size_t keys, ids, keys2, order, dcnt, dtot, counts, offsets, total, temp, temp_bytes, bytes;
};

static BinLayout bin_layout(int64_t P) {
    BinLayout L{};
    const size_t n = (size_t)(P > 0 ? P : 1);
    size_t scan_bytes = 0;
    (void)rocprim::exclusive_scan((void*)nullptr, scan_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (uint64_t)0, n,
                            rocprim::plus<uint64_t>());
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.keys = take(4 * n);
    L.ids = take(4 * n);
    L.keys2 = take(4 * n);
    L.order = take(4 * n);
    L.counts = take(8 * n);
    L.offsets = take(8 * n);
    L.total = take(8);
    L.dcnt = take(4 * (size_t)DS_RADIX * ds_blocks((int64_t)n));
    L.dtot = take(4 * depth_order_tot_words((int64_t)n));
    L.temp_bytes = scan_bytes;
    L.temp = take(L.temp_bytes);
    L.bytes = off;
    return L;
}

}  // namespace bgs

using namespace bgs;

extern "C" size_t bgs_bin_workspace_bytes(int64_t P) { return bin_layout(P).bytes; }

extern "C" bgs_status bgs_bin(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                              const int32_t* radius, const float* depth, const uint32_t* tiles_touched, uint32_t* keys,
                              uint32_t* values, int64_t capacity, int64_t* n_pairs_host, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    BGS_REQUIRE(width > 0 && height > 0, "bgs_bin: image size must be positive");
    BGS_REQUIRE(P >= 0 && capacity >= 0, "bgs_bin: negative size");
    BGS_REQUIRE(n_pairs_host != nullptr, "bgs_bin: n_pairs_host is null");
    if (tile != TILE) return fail(BGS_EUNSUPPORTED, "bgs_bin: only 16x16 tiles are supported");
    *n_pairs_host = 0;
    if (P == 0) return BGS_OK;
    BGS_REQUIRE(means2D && radius && depth && tiles_touched && ws, "bgs_bin: null array");
    BGS_REQUIRE(P < ((int64_t)1 << 31), "bgs_bin: P must be < 2^31");
    const BinLayout L = bin_layout(P);
    BGS_REQUIRE(ws_bytes >= L.bytes, "bgs_bin: workspace too small");
    char* w = static_cast<char*>(ws);
    auto* dkeys = reinterpret_cast<uint32_t*>(w + L.keys);
    auto* ids = reinterpret_cast<uint32_t*>(w + L.ids);
    auto* dkeys2 = reinterpret_cast<uint32_t*>(w + L.keys2);
    auto* order = reinterpret_cast<uint32_t*>(w + L.order);
    auto* counts = reinterpret_cast<uint64_t*>(w + L.counts);
    auto* offsets = reinterpret_cast<uint64_t*>(w + L.offsets);
    auto* total = reinterpret_cast<uint64_t*>(w + L.total);
    void* temp = w + L.temp;
    size_t temp_bytes = L.temp_bytes;

    const int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    {
        const bgs_status st = depth_order(P, depth, tiles_touched, dkeys, order, dkeys2, ids,
                                          reinterpret_cast<uint32_t*>(w + L.dcnt),
                                          reinterpret_cast<uint32_t*>(w + L.dtot), RectArgs{}, stream);
        if (st != BGS_OK) return st;
    }
    hipLaunchKernelGGL(k_gather_counts, dim3(blocks_for(P)), dim3(256), 0, stream, P, order, tiles_touched, counts);
    BGS_HIP(hipGetLastError());
    BGS_HIP(rocprim::exclusive_scan(temp, temp_bytes, counts, offsets, (uint64_t)0, (size_t)P,
                                    rocprim::plus<uint64_t>(), stream));
    hipLaunchKernelGGL(k_total, dim3(1), dim3(64), 0, stream, P, offsets, order, tiles_touched, total);
    BGS_HIP(hipGetLastError());
    uint64_t M = 0;
    BGS_HIP(hipMemcpyAsync(&M, total, sizeof(M), hipMemcpyDeviceToHost, stream));
    BGS_HIP(hipStreamSynchronize(stream));
    *n_pairs_host = (int64_t)M;
    if ((int64_t)M > capacity)
        return fail(BGS_ECAPACITY, "bgs_bin: " + std::to_string(M) + " pairs exceed capacity " +
                                       std::to_string(capacity));
    if (M == 0) return BGS_OK;
    BGS_REQUIRE(keys && values, "bgs_bin: null output");
    BGS_REQUIRE(M < ((uint64_t)1 << 32), "bgs_bin: more than 2^32 pairs");
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(P)), dim3(256), 0, stream, P, TX, TY, order, offsets, means2D, radius,
                       tiles_touched, keys, values);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

extern "C" size_t bgs_sort_workspace_bytes(int64_t n) {
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                              (uint32_t*)nullptr, (size_t)(n > 0 ? n : 1), 0, 32);
    return align_up(bytes, 256);
}

extern "C" bgs_status bgs_sort(const uint32_t* keys_in, const uint32_t* values_in, uint32_t* keys_out,
                               uint32_t* values_out, int64_t n, int32_t key_bits, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
    BGS_REQUIRE(n >= 0, "bgs_sort: n < 0");
    BGS_REQUIRE(key_bits >= 1 && key_bits <= 32, "bgs_sort: key_bits must be in 1..32");
    if (n == 0) return BGS_OK;
    BGS_REQUIRE(keys_in && values_in && keys_out && values_out && ws, "bgs_sort: null array");
    BGS_REQUIRE(keys_in != keys_out && values_in != values_out, "bgs_sort: in and out buffers alias");
    size_t need = bgs_sort_workspace_bytes(n);
    BGS_REQUIRE(ws_bytes >= need, "bgs_sort: workspace too small");
    BGS_HIP(rocprim::radix_sort_pairs(ws, need, keys_in, keys_out, values_in, values_out, (size_t)n, 0, key_bits,
                                      stream));
    return BGS_OK;
}

extern "C" bgs_status bgs_ranges(const uint32_t* sorted_keys, int64_t n, int32_t n_tiles, uint32_t* ranges,
                                 hipStream_t stream) {
    BGS_REQUIRE(n >= 0 && n_tiles >= 0, "bgs_ranges: negative size");
    if (n_tiles == 0) return BGS_OK;
    BGS_REQUIRE(ranges != nullptr, "bgs_ranges: ranges is null");
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * (int64_t)n_tiles)), dim3(256), 0, stream, ranges,
                       2 * (int64_t)n_tiles, 0u);
    BGS_HIP(hipGetLastError());
    if (n == 0) return BGS_OK;
    BGS_REQUIRE(sorted_keys != nullptr, "bgs_ranges: keys is null");
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(n)), dim3(256), 0, stream, sorted_keys, n, (int)n_tiles, ranges);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

// ======================================================================
// Fused tile lists: bin + stable sort by tile + ranges, without ever
// materializing or sorting the M (tile, Gaussian) keys.
//
// 1. The Gaussians are put in depth order (a P-element sort) and each one's
//    tile rectangle is computed once.
// 2. Coarse lists per group of 8x8 tiles (128x128 px): a stable counting sort of
//    the (group, Gaussian) pairs.  The depth order is cut into chunks of
//    CHUNK Gaussians; per chunk a group histogram (2D difference array in LDS,
//    four updates per Gaussian, then a 2D prefix sum), a column scan over
//    chunks and a scan over groups give every (chunk, group) its base slot,
//    and one wave per chunk drops the chunk's pairs, in depth order, at base +
//    running count.  Each coarse entry is one aligned 16-byte store: the
//    scattered coarse writes cost one memory sector each, and 8x8 groups
//    keep their number low (135 groups at 1080p).
// 3. Fine lists: one workgroup per segment of a group's coarse list (in
//    depth order) splits it into the group's 64 tile lists; wave w owns tiles
//    16 w .. 16 w + 15 and appends, with a ballot and a prefix count, the
//    Gaussians whose tile mask holds the tile -- coalesced sequential
//    appends, first counting (to size the tiles), then writing.
// The result is exactly the list a stable sort of the depth-ordered
// (tile, Gaussian) pairs by tile gives.
// ======================================================================
namespace bgs {

constexpr int CHUNK = 64;        // Gaussians per chunk of the coarse sort (one wave emits a chunk)
constexpr int PART = 32;         // chunks per column-scan block
constexpr int GSHIFT = 3;        // group = 8x8 tiles
constexpr int GTILES = 1 << GSHIFT;
constexpr int MAX_GROUPS = 8192;

// ----------------------------------------------------------------------
// Exact ellipse-tile binning (optional).  Eq. (4) blends Gaussian g at pixel
// offset d only when o exp(-q(d)/2) reaches 1/255, q(d) = a dx^2 + 2 b dx dy
// + c dy^2 with (a, b, c) the conic: inside the ellipse q <= 2 ln(255 o).  A
// tile of the square rule is kept only when its rectangle of pixel centres
// meets that ellipse, so every removed pair is one the forward would skip at
// each pixel of its tile.  The bound is widened by 2^-10 (relative and
// absolute) and the tile rectangles by 2^-6 px, as in the rule's fp64
// definition; on top, the fp32 evaluation below uses an ellipse 2^-12 larger
// per axis and widens each row interval by 2^-11 of the half extent, so
// rounding only ever adds tiles.
// Per tile row, the tiles met form one run of columns: the x-range of the
// ellipse within the row's slab of pixel centres, whose ends lie at the
// ellipse's right- and leftmost points clamped into the slab.
// ----------------------------------------------------------------------
constexpr float BIN_PX_SLACK = 1.0f / 64.0f;

struct Ellipse {
    float b, inv_a, det;  // conic b, 1/a, a c - b^2
    float xe, ye;         // half extents of the (enlarged) ellipse
    float yr;             // y of its rightmost point (the leftmost is at -yr)
    float mx, my;
    bool blends;          // false: alpha never reaches 1/255, no tile
    bool proper;          // false: not an ellipse, the square rule stands
};

__device__ __forceinline__ Ellipse make_ellipse(float4 co, float mx, float my) {
    Ellipse e;
    e.mx = mx;
    e.my = my;
    const float a = co.x, b = co.y, c = co.z, o = co.w;
    const float bb = b * b;
    e.det = __builtin_fmaf(a, c, -bb) - __builtin_fmaf(b, b, -bb);
    e.b = b;
    e.inv_a = 1.0f / a;
    const float t255 = 1.0f / 255.0f;
    e.blends = o > 0.0f;
    float lim = e.blends ? 2.0f * logf(o / t255) : -1.0f;
    lim = lim * (1.0f + 1.0f / 1024.0f) + 1.0f / 1024.0f;
    e.blends = e.blends && lim >= 0.0f;
    e.proper = a > 0.0f && c > 0.0f && e.det > 0.0f;
    const float grow = 1.0f + 1.0f / 4096.0f;
    e.xe = grow * sqrtf(lim * c / e.det);
    e.ye = grow * sqrtf(lim * a / e.det);
    e.yr = -b * e.xe / c;
    e.proper = e.proper && e.blends && e.xe < 1.0e7f && e.ye < 1.0e7f;
    return e;
}

// x of the ellipse boundary at height y (right or left end of its chord).
// The hardware square root (within 1 ulp, denormals may flush to zero) is
// far inside the padding that row_interval adds, 2^-6 px + 2^-11 of the
// half extent, so the interval stays conservative.
__device__ __forceinline__ float chord_end(const Ellipse& e, float y, float sign) {
    const float ay = fabsf(y);
    const float D = fmaxf(0.0f, e.det * (e.ye - ay) * (e.ye + ay));  // = a lim' - det y^2
    return (-e.b * y + sign * __builtin_amdgcn_sqrtf(D)) * e.inv_a;
}

// The run of tile columns of tile row ty that the ellipse meets, clamped to
// [tx0, tx1]: packed lo | (hi + 1) << 16 (empty: lo >= hi + 1).
__device__ __forceinline__ uint32_t row_interval(const Ellipse& e, int ty, int tx0, int tx1) {
    const float y0 = (float)(TILE * ty) - BIN_PX_SLACK - e.my, y1 = (float)(TILE * ty + TILE - 1) + BIN_PX_SLACK - e.my;
    const float lo = fmaxf(y0, -e.ye), hi = fminf(y1, e.ye);
    if (!(lo <= hi)) return (uint32_t)(tx1 + 1) | ((uint32_t)tx0 << 16);
    const float pad = BIN_PX_SLACK + e.xe * (1.0f / 2048.0f);
    const float xr = chord_end(e, fminf(fmaxf(e.yr, lo), hi), 1.0f) + pad;
    const float xl = chord_end(e, fminf(fmaxf(-e.yr, lo), hi), -1.0f) - pad;
    // tile tx (pixel centres 16 tx .. 16 tx + 15, widened) meets [xl, xr]
    const float flo = ceilf((xl + e.mx - BIN_PX_SLACK - (float)(TILE - 1)) * (1.0f / TILE));
    const float fhi = floorf((xr + e.mx + BIN_PX_SLACK) * (1.0f / TILE));
    const int c0 = (int)fminf(fmaxf(flo, (float)tx0), (float)(tx1 + 1));
    const int c1 = (int)fmaxf(fminf(fhi, (float)tx1), (float)(tx0 - 1));
    return (uint32_t)c0 | ((uint32_t)(c1 + 1) << 16);
}

// (x0 | y0 << 16, x1 | y1 << 16) of Gaussian g's tile rectangle; an empty
// one has x0 > x1.  EXACT: cut to the tiles that the ellipse's bounding box
// meets.
template <bool EXACT>
__device__ uint2 gaussian_rect(int64_t g, const RectArgs& R, bool listed) {
    int x0 = 1, y0 = 0, x1 = 0, y1 = 0;
    const float mx = R.means2D[2 * g], my = R.means2D[2 * g + 1];
    if (!listed || !tile_rect(mx, my, R.radius[g], R.TX, R.TY, x0, y0, x1, y1)) {
        x0 = 1; y0 = 0; x1 = 0; y1 = 0;
    } else if (EXACT) {
        const Ellipse e = make_ellipse(R.conic_opacity[g], mx, my);
        if (!e.blends) {
            x0 = 1; y0 = 0; x1 = 0; y1 = 0;
        } else if (e.proper) {
            // tiles whose widened pixel-centre range meets [m - extent, m + extent];
            // the float bounds are clamped into the rectangle before conversion
            const float ph = BIN_PX_SLACK + (float)(TILE - 1);
            const float fx0 = ceilf((mx - e.xe - ph) / TILE), fx1 = floorf((mx + e.xe + BIN_PX_SLACK) / TILE);
            const float fy0 = ceilf((my - e.ye - ph) / TILE), fy1 = floorf((my + e.ye + BIN_PX_SLACK) / TILE);
            x0 = max(x0, (int)fminf(fmaxf(fx0, (float)x0), (float)x1 + 1.0f));
            x1 = min(x1, (int)fmaxf(fminf(fx1, (float)x1), (float)x0 - 1.0f));
            y0 = max(y0, (int)fminf(fmaxf(fy0, (float)y0), (float)y1 + 1.0f));
            y1 = min(y1, (int)fmaxf(fminf(fy1, (float)y1), (float)y0 - 1.0f));
            if (x0 > x1 || y0 > y1) {
                x0 = 1; y0 = 0; x1 = 0; y1 = 0;
            }
        }
    }
    return make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
}

__device__ __forceinline__ bool group_rect(uint2 r, int& x0, int& y0, int& x1, int& y1) {
    x0 = (int)(r.x & 0xFFFF); y0 = (int)(r.x >> 16); x1 = (int)(r.y & 0xFFFF); y1 = (int)(r.y >> 16);
    if (x0 > x1) return false;
    x0 >>= GSHIFT; y0 >>= GSHIFT; x1 >>= GSHIFT; y1 >>= GSHIFT;
    return true;
}

// h[c][grp] = number of chunk c's Gaussians whose rectangle meets group grp
__global__ __launch_bounds__(256) void k_chunk_hist(int64_t P, int GX, int GY, const uint32_t* __restrict__ order,
                                                    const uint2* __restrict__ rect, uint32_t* __restrict__ h) {
    extern __shared__ int d[];  // (GY+1) x (GX+1) difference grid
    const int W1 = GX + 1, H1 = GY + 1, ng = GX * GY;
    const int c = blockIdx.x;
    for (int i = threadIdx.x; i < W1 * H1; i += blockDim.x) d[i] = 0;
    __syncthreads();
    const int64_t k = (int64_t)c * CHUNK + threadIdx.x;
    if (k < P) {
        int x0, y0, x1, y1;
        if (group_rect(rect[order[k]], x0, y0, x1, y1)) {
            atomicAdd(&d[y0 * W1 + x0], 1);
            atomicAdd(&d[y0 * W1 + x1 + 1], -1);
            atomicAdd(&d[(y1 + 1) * W1 + x0], -1);
            atomicAdd(&d[(y1 + 1) * W1 + x1 + 1], 1);
        }
    }
    __syncthreads();
    for (int y = threadIdx.x; y < H1; y += blockDim.x) {
        int run = 0;
        for (int x = 0; x < W1; ++x) {
            run += d[y * W1 + x];
            d[y * W1 + x] = run;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < W1; x += blockDim.x) {
        int run = 0;
        for (int y = 0; y < H1; ++y) {
            run += d[y * W1 + x];
            d[y * W1 + x] = run;
        }
    }
    __syncthreads();
    uint32_t* hc = h + (int64_t)c * ng;
    for (int t = threadIdx.x; t < ng; t += blockDim.x) hc[t] = (uint32_t)d[(t / GX) * W1 + (t % GX)];
}

// part[b][t] = sum of h[c][t] over the chunks c of block b.  Workgroup
// (b, 64-column slice): wave w sums chunks c0 + 8 w .. c0 + 8 w + 7 of the
// slice's 64 columns (coalesced rows), and the four partial sums meet in LDS.
constexpr int PS_COLS = 64;

__global__ __launch_bounds__(256) void k_part_sums(int C, int nt, const uint32_t* __restrict__ h,
                                                   uint32_t* __restrict__ part) {
    static_assert(PART == 4 * 8, "four waves of eight chunks");
    __shared__ uint32_t s_sum[4][PS_COLS];
    const int slices = (nt + PS_COLS - 1) / PS_COLS;
    const int b = blockIdx.x / slices, t = (blockIdx.x % slices) * PS_COLS + (threadIdx.x & 63);
    const int w = threadIdx.x >> 6;
    const int c0 = b * PART + 8 * w, n = max(0, min(C - c0, 8));
    uint32_t sum = 0;
    if (t < nt) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < n) sum += h[(int64_t)(c0 + c) * nt + t];
    }
    s_sum[w][threadIdx.x & 63] = sum;
    __syncthreads();
    if (w == 0 && t < nt)
        part[(int64_t)b * nt + t] = sum + s_sum[1][threadIdx.x] + s_sum[2][threadIdx.x] + s_sum[3][threadIdx.x];
}

// exclusive scan of part[.][t] over the nb blocks, one wave per column t;
// total[t] = column sum
__global__ __launch_bounds__(256) void k_part_scan(int nb, int nt, uint32_t* __restrict__ part,
                                                   uint32_t* __restrict__ total) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= nt) return;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 64) {
        const int b = b0 + lane;
        const uint32_t v = b < nb ? part[(int64_t)b * nt + t] : 0u;
        uint32_t x = v;  // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (b < nb) part[(int64_t)b * nt + t] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) total[t] = carry;
}

// Single workgroup: exclusive scan of n_t = min(total[t], keep_max) -> start;
// ranges (empty: (0, 0)); the grand total in n_pairs[0].  Thread i owns the
// contiguous run [i per, (i+1) per); the per-thread sums are scanned with a
// block scan.  Overflow: when coarse_n (nullable) exceeds coarse_cap,
// n_pairs[0] receives coarse_n (a lower bound of the pair count); then, or
// when the total exceeds cap, every range is written empty, so that nothing
// reads the unwritten point list.
__global__ __launch_bounds__(1024) void k_tile_scan(int nt, const uint32_t* __restrict__ total,
                                                    uint32_t* __restrict__ start, uint32_t* __restrict__ ranges,
                                                    uint64_t* __restrict__ n_pairs, const uint64_t* __restrict__ coarse_n,
                                                    uint64_t coarse_cap, uint64_t cap, uint32_t keep_max) {
    using Scan = rocprim::block_scan<uint64_t, 1024>;
    __shared__ typename Scan::storage_type s_scan;
    const int per = (nt + 1023) / 1024;
    const int t0 = min(nt, (int)threadIdx.x * per), t1 = min(nt, t0 + per);
    uint64_t s = 0;
    for (int t = t0; t < t1; ++t) s += min(total[t], keep_max);
    uint64_t run = 0, grand = 0;
    Scan().exclusive_scan(s, run, (uint64_t)0, grand, s_scan);
    const bool coarse_over = coarse_n != nullptr && coarse_n[0] > coarse_cap;
    if (threadIdx.x == 0) n_pairs[0] = coarse_over ? coarse_n[0] : grand;
    const bool keep = !coarse_over && grand <= cap;
    for (int t = t0; t < t1; ++t) {
        const uint32_t n = min(total[t], keep_max);
        start[t] = (uint32_t)run;
        if (ranges) {
            ranges[2 * t] = n && keep ? (uint32_t)run : 0u;
            ranges[2 * t + 1] = n && keep ? (uint32_t)(run + n) : 0u;
        }
        run += n;
    }
}

// h[c][t] <- start[t] + (number of pairs of t in chunks before c)
__global__ __launch_bounds__(256) void k_chunk_base(int C, int nt, const uint32_t* __restrict__ start,
                                                    const uint32_t* __restrict__ part, uint32_t* __restrict__ h) {
    const int nb = (C + PART - 1) / PART;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * nt) return;
    const int b = (int)(i / nt), t = (int)(i % nt);
    const int c0 = b * PART, n = min(C - c0, PART);
    uint32_t v[PART];
#pragma unroll
    for (int c = 0; c < PART; ++c) v[c] = c < n ? h[(int64_t)(c0 + c) * nt + t] : 0u;  // all loads first
    uint32_t run = start[t] + part[i];
#pragma unroll
    for (int c = 0; c < PART; ++c) {
        if (c < n) h[(int64_t)(c0 + c) * nt + t] = run;
        run += v[c];
    }
}

// One wave per chunk: drop the chunk's (group, Gaussian) pairs, Gaussians in
// depth order, at the chunk's base slot of each group plus a running count
// kept in LDS.  An entry is (Gaussian id, 64-bit mask of the group's tiles
// the Gaussian covers, bit (x mod 8) + 8 (y mod 8), 0), so the split into
// tile lists streams the coarse lists without a gather.
// The 64-bit mask of a group's tiles with columns cols (8 bits) in the rows
// rl .. rh - 1 (0 <= rl < rh <= 8): cols copied into every row by one
// multiply (no carries, cols < 256), then the rows outside cut away.
__device__ __forceinline__ uint64_t rect_mask(uint32_t cols, int rl, int rh) {
    const uint64_t every_row = (uint64_t)cols * 0x0101010101010101ull;
    const uint64_t below_hi = rh >= GTILES ? ~0ull : (1ull << (GTILES * rh)) - 1ull;
    const uint64_t below_lo = (1ull << (GTILES * rl)) - 1ull;
    return every_row & below_hi & ~below_lo;
}

// The chunk's (Gaussian, group) pairs are flattened over the lanes, 64 at a
// time in (Gaussian, group) order.  A pair's slot is its group's running
// position plus the number of lower lanes of the batch with the same group
// id (found with one ballot per bit of the id), and the last such lane
// advances the running position, so a group receives the chunk's Gaussians in
// depth order.  EXACT: the run of tile columns that a proper ellipse meets on
// each tile row of its rectangle (row_interval) is evaluated once, one
// (Gaussian, row) per lane, into an LDS buffer of EMIT_ROWS rows; the pairs
// OR their group's rows from it.  The chunk is taken in windows of
// consecutive Gaussians whose rows fit the buffer; the host admits at most
// EMIT_ROWS tile rows, so every Gaussian's rows fit one window.
constexpr int EMIT_ROWS = 1024;

template <bool EXACT>
__global__ __launch_bounds__(64) void k_chunk_emit(int64_t P, int GX, int GY, int gbits,
                                                   const uint32_t* __restrict__ order, const uint2* __restrict__ rect,
                                                   const uint32_t* __restrict__ base, uint4* __restrict__ coarse,
                                                   const uint64_t* __restrict__ coarse_n, uint64_t coarse_cap,
                                                   const float* __restrict__ means2D,
                                                   const float4* __restrict__ conic_opacity) {
    extern __shared__ uint32_t nextpos[];  // ng running slots
    __shared__ uint32_t s_off[65];         // first pair of each Gaussian of the chunk; s_off[64] = pairs
    __shared__ uint32_t s_g[64];
    __shared__ uint2 s_rr[64];
    __shared__ int4 s_grp[64];  // group rectangle: x0, y0, width, -
    __shared__ float s_invw[64];
    __shared__ uint32_t s_roff[EXACT ? 65 : 1];  // first row of each Gaussian (0 rows: not proper)
    __shared__ uint32_t s_rows[EXACT ? EMIT_ROWS : 1];
    if (coarse_n[0] > coarse_cap) return;  // the coarse lists do not fit: nothing is written
    static_assert(CHUNK == 64, "one Gaussian per lane");
    const int ng = GX * GY;
    const int lane = threadIdx.x;
    const int c = blockIdx.x;
    const uint32_t* bc = base + (int64_t)c * ng;
    for (int t = lane; t < ng; t += 64) nextpos[t] = bc[t];
    const int64_t k = (int64_t)c * CHUNK + lane;
    uint32_t g = 0, n = 0;
    uint2 rr = make_uint2(1u, 0u);
    int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    if (k < P) {
        g = order[k];
        rr = rect[g];
        if (group_rect(rr, x0, y0, x1, y1)) n = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    }
    uint32_t incl = n;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    s_off[lane] = incl - n;
    if (lane == 63) s_off[64] = total;
    s_g[lane] = g;
    s_rr[lane] = rr;
    s_grp[lane] = make_int4(x0, y0, x1 - x0 + 1, 0);
    s_invw[lane] = 1.0f / (float)(x1 - x0 + 1 > 0 ? x1 - x0 + 1 : 1);
    Ellipse el{};  // EXACT: this lane's Gaussian; proper stays false for the square rule's mask
    if (EXACT) {
        if (n) el = make_ellipse(conic_opacity[g], means2D[2 * g], means2D[2 * g + 1]);
        const uint32_t nr = el.proper ? (rr.y >> 16) - (rr.x >> 16) + 1u : 0u;
        uint32_t ri = nr;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(ri, off, 64);
            if (lane >= off) ri += y;
        }
        s_roff[lane] = ri - nr;
        if (lane == 63) s_roff[64] = ri;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int ga = 0;  // first Gaussian of the window
    while (ga < 64) {
        int gb = 64;
        uint32_t rbase = 0, nw = 0;  // the window's first row and the rows held in s_rows
        if (EXACT) {
            rbase = __builtin_amdgcn_readfirstlane(s_roff[ga]);
            // s_roff is nondecreasing: the Gaussians from ga whose rows end within the buffer are a run
            const uint64_t fits = ballot(lane >= ga && s_roff[lane + 1] - rbase <= (uint32_t)EMIT_ROWS);
            gb = max(ga + 1, ga + __builtin_popcountll(fits));
            nw = min(__builtin_amdgcn_readfirstlane(s_roff[gb]) - rbase, (uint32_t)EMIT_ROWS);
            for (uint32_t pr0 = 0; pr0 < nw; pr0 += 64) {  // every lane takes part in the shuffles
                const uint32_t pr = pr0 + lane, rg = rbase + pr;
                int kk = 0;  // the row's Gaussian: the last whose rows start at or before it
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_roff[kk + step] <= rg) kk += step;  // kk + step <= 63
                Ellipse ek{};  // lane kk's ellipse
                ek.b = __shfl(el.b, kk, 64);
                ek.inv_a = __shfl(el.inv_a, kk, 64);
                ek.det = __shfl(el.det, kk, 64);
                ek.xe = __shfl(el.xe, kk, 64);
                ek.ye = __shfl(el.ye, kk, 64);
                ek.yr = __shfl(el.yr, kk, 64);
                ek.mx = __shfl(el.mx, kk, 64);
                ek.my = __shfl(el.my, kk, 64);
                const uint2 rk = s_rr[kk];
                const int row = (int)(rk.x >> 16) + (int)(rg - s_roff[kk]);
                if (pr < nw) s_rows[pr] = row_interval(ek, row, (int)(rk.x & 0xFFFFu), (int)(rk.y & 0xFFFFu));
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const uint32_t pa = __builtin_amdgcn_readfirstlane(s_off[ga]), pb = __builtin_amdgcn_readfirstlane(s_off[gb]);
        for (uint32_t p0 = pa; p0 < pb; p0 += 64) {
            const uint32_t p = p0 + lane;
            const bool valid = p < pb;
            int i = 0;  // the pair's Gaussian: the last lane whose first pair is at or before p
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (s_off[i + step] <= p) i += step;  // i + step <= 63
            int t = 0;
            uint64_t mask = 0;
            if (valid) {
                const int4 gr = s_grp[i];
                const int wi = gr.z;
                const int j = (int)(p - s_off[i]);
                int q = (int)((float)j * s_invw[i]);
                int r = j - q * wi;
                if (r >= wi) { ++q; r -= wi; }
                if (r < 0) { --q; r += wi; }
                const int gx = gr.x + r, gy = gr.y + q;
                t = gy * GX + gx;
                const uint2 rk = s_rr[i];
                const int tx0 = (int)(rk.x & 0xFFFF), ty0 = (int)(rk.x >> 16), tx1 = (int)(rk.y & 0xFFFF),
                          ty1 = (int)(rk.y >> 16);
                // the tile rectangle is clamped to the image, so the mask only
                // holds tiles inside it
                const int bx = gx * GTILES, by = gy * GTILES;
                const int cl = max(tx0 - bx, 0), ch = min(tx1 - bx + 1, GTILES);
                const int rl = max(ty0 - by, 0), rh = min(ty1 - by + 1, GTILES);
                const uint32_t cols = ((1u << ch) - 1u) & ~((1u << cl) - 1u);
                mask = rect_mask(cols, rl, rh);
                if (EXACT && s_roff[i + 1] > s_roff[i]) {  // a proper ellipse: its rows
                    // s_rows index of group row rw (wraps below for rw < rl; clamped, then unused)
                    const uint32_t r0 = s_roff[i] - rbase + (uint32_t)(by - ty0);
                    uint32_t iv[GTILES];
#pragma unroll
                    for (int rw = 0; rw < GTILES; ++rw) iv[rw] = s_rows[min(r0 + (uint32_t)rw, EMIT_ROWS - 1u)];
                    mask = 0u;
#pragma unroll
                    for (int rw = 0; rw < GTILES; ++rw) {
                        const int c0 = max((int)(iv[rw] & 0xFFFFu) - bx, 0), c1 = min((int)(iv[rw] >> 16) - bx, GTILES);
                        if (rw >= rl && rw < rh && c0 < c1)
                            mask |= (uint64_t)(((1u << c1) - 1u) & ~((1u << c0) - 1u)) << (GTILES * rw);
                    }
                }
            }
            uint64_t eq = ballot(valid);  // lanes of the batch with this lane's group id
            for (int b = 0; b < gbits; ++b) {
                const bool bit = ((t >> b) & 1) != 0;
                const uint64_t m = ballot(bit);
                eq &= bit ? m : ~m;
            }
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(eq >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)eq, 0u));
            const uint32_t pos = valid ? nextpos[t] + rank : 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid && rank + 1 == (uint32_t)__builtin_popcountll(eq)) nextpos[t] = pos + 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid) coarse[pos] = make_uint4(s_g[i], (uint32_t)mask, (uint32_t)(mask >> 32), 0u);
        }
        if (EXACT) {  // the next window overwrites s_rows
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        ga = gb;
    }
}

// The fine split runs on segments of SEG consecutive coarse entries of one
// group, so that a heavily covered group does not serialize on one
// workgroup.  nseg[g] = ceil(gtotal[g] / SEG).
constexpr int SEG = 2048;

__global__ __launch_bounds__(256) void k_seg_count(int ng, const uint32_t* __restrict__ gtotal,
                                                   uint32_t* __restrict__ nseg) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) nseg[g] = (gtotal[g] + SEG - 1) / SEG;
}

// segmap[segstart[g] + s] = (g, s), one wave per group; nothing when the
// coarse lists overflowed (the segment table is sized for lists that fit)
__global__ __launch_bounds__(256) void k_seg_map(int ng, const uint32_t* __restrict__ nseg,
                                                 const uint32_t* __restrict__ segstart, uint2* __restrict__ segmap,
                                                 const uint64_t* __restrict__ coarse_n, uint64_t coarse_cap,
                                                 uint32_t max_segs) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (g >= ng || coarse_n[0] > coarse_cap) return;
    const uint32_t n = nseg[g], b = segstart[g];
    for (uint32_t q = lane; q < n && b + q < max_segs; q += 64) segmap[b + q] = make_uint2((uint32_t)g, q);
}

// A fixed grid of workgroups strides over the segments (the segment count
// stays on the device); per segment, wave w takes its 16 tiles (local index
// i = (x mod 8) + 8 (y mod 8) in [16 w, 16 w + 16)) in turn and, 64 entries
// at a time, the ballot of the entries whose mask holds the tile.
// COUNT: segcnt[seg][i] = the segment's entries whose mask holds tile i.
// WRITE: the k-th such entry goes to segcnt[seg][i] (by then the slot where
// the segment's run of tile i starts) + k, if that slot is below the end of
// the tile's range (which stops short of the tile's count when lists are
// capped).  Each lane keeps its 32 entries of the segment in registers and
// the wave takes its tiles one after another, so a (tile, 64 entries) step
// is a bit test, a ballot, the lane's rank (mbcnt) and one store of the
// compacted run at a wave-uniform base.  A wave none of whose 16 tiles has
// room left in this segment reads nothing.
constexpr size_t SPLIT_GRID = 2048;  // workgroups of the split passes: 8 per CU

struct TileGrid {
    int TX, TY, GX;
    const uint32_t* ranges;  // WRITE: [n_tiles][2] of the final lists
};

template <bool WRITE>
__device__ __forceinline__ void split_segment(uint32_t sidx, const uint2* __restrict__ segmap,
                                              const uint4* __restrict__ coarse, const uint32_t* __restrict__ gstart,
                                              const uint32_t* __restrict__ gtotal, uint32_t* __restrict__ segcnt,
                                              uint32_t* __restrict__ point_list, const TileGrid& tg) {
    const uint2 gs = segmap[sidx];
    const int grp = (int)gs.x;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // WRITE: lane i < 16 holds the run start and the range end of the wave's tile i
    uint32_t my_run = 0u, my_end = 0u;
    if (WRITE) {
        if (lane < 16) {
            const int li = wv * 16 + lane;
            const int tx = (grp % tg.GX) * GTILES + (li % GTILES), ty = (grp / tg.GX) * GTILES + (li / GTILES);
            my_run = segcnt[(size_t)sidx * 64 + li];
            my_end = (tx < tg.TX && ty < tg.TY) ? tg.ranges[2 * ((size_t)ty * tg.TX + tx) + 1] : 0u;
        }
        if (ballot(lane < 16 && my_run < my_end) == 0) return;  // this wave's tiles are full
    }
    const uint32_t gt = gtotal[grp];
    const uint32_t e0 = min(gt, gs.y * SEG), e1 = min(gt, (gs.y + 1) * SEG);
    const uint32_t b0 = gstart[grp];
    // the segment's entries in registers: entry e0 + 64 b + lane in slot b
    constexpr int NB = SEG / 64;
    uint32_t ids[NB], bits[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const uint32_t k = e0 + 64 * b + lane;
        ids[b] = 0u;
        bits[b] = 0u;
        if (k < e1) {
            const uint4 e = coarse[b0 + k];
            ids[b] = e.x;
            bits[b] = ((wv < 2 ? e.y : e.z) >> (16 * (wv & 1))) & 0xFFFFu;
        }
    }
    for (int i = 0; i < 16; ++i) {
        uint32_t run = WRITE ? (uint32_t)__builtin_amdgcn_readlane((int)my_run, i) : 0u;
        const uint32_t end = WRITE ? (uint32_t)__builtin_amdgcn_readlane((int)my_end, i) : 0u;
        if (WRITE && run >= end) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bool in = (bits[b] >> i) & 1u;
            const uint64_t m = ballot(in);
            if (WRITE) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                uint32_t* dst = point_list + run;
                if (in && run + rank < end) dst[rank] = ids[b];
            }
            run = __builtin_amdgcn_readfirstlane(run + (uint32_t)__builtin_popcountll(m));
        }
        if (!WRITE && lane == 0) segcnt[(size_t)sidx * 64 + wv * 16 + i] = run;
    }
}

template <bool WRITE>
__global__ __launch_bounds__(256) void k_seg_split(const uint64_t* __restrict__ n_segs, const uint2* __restrict__ segmap,
                                                   const uint4* __restrict__ coarse,
                                                   const uint32_t* __restrict__ gstart,
                                                   const uint32_t* __restrict__ gtotal, uint32_t* __restrict__ segcnt,
                                                   uint32_t* __restrict__ point_list, const uint64_t* __restrict__ n_pairs,
                                                   uint64_t capacity, const uint64_t* __restrict__ coarse_n,
                                                   uint64_t coarse_cap, uint32_t max_segs, TileGrid tg) {
    if (coarse_n[0] > coarse_cap) return;  // no coarse lists to split
    // the pair count is final here; a list that does not fit is not written
    // at all (the caller grows the buffer and builds again)
    if (WRITE && n_pairs[0] > capacity) return;
    const uint32_t nsg = (uint32_t)min(n_segs[0], (uint64_t)max_segs);
    for (uint32_t sidx = blockIdx.x; sidx < nsg; sidx += gridDim.x)
        split_segment<WRITE>(sidx, segmap, coarse, gstart, gtotal, segcnt, point_list, tg);
}

// One workgroup per group, thread (part p, local tile i): p takes a
// contiguous sixteenth of the group's segments.  OFFSETS = false: ttotal[tile]
// = sum of the tile's segment counts.  OFFSETS = true: the counts become the
// tile's slot at the start of each segment's run (from tstart).  After a
// coarse overflow there are no segments: every tile total is zero.
constexpr int SCAN_PARTS = 16;

template <bool OFFSETS>
__global__ __launch_bounds__(SCAN_PARTS * 64) void k_seg_scan(int TX, int TY, int GX,
                                                               const uint32_t* __restrict__ nseg,
                                                               const uint32_t* __restrict__ segstart,
                                                               uint32_t* __restrict__ segcnt,
                                                               const uint32_t* __restrict__ tstart,
                                                               uint32_t* __restrict__ ttotal,
                                                               const uint64_t* __restrict__ coarse_n,
                                                               uint64_t coarse_cap) {
    __shared__ uint32_t s_part[SCAN_PARTS][64];
    const int grp = blockIdx.x, li = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int tx = (grp % GX) * GTILES + (li % GTILES), ty = (grp / GX) * GTILES + (li / GTILES);
    const bool valid = tx < TX && ty < TY;
    const int tile = ty * TX + tx;
    if (coarse_n[0] > coarse_cap) {
        if (!OFFSETS && valid && p == 0) ttotal[tile] = 0u;
        return;
    }
    const uint32_t n = nseg[grp], b = segstart[grp];
    const uint32_t q0 = (uint32_t)(((uint64_t)n * p) / SCAN_PARTS), q1 = (uint32_t)(((uint64_t)n * (p + 1)) / SCAN_PARTS);
    uint32_t sum = 0;
    for (uint32_t q = q0; q < q1; ++q) sum += segcnt[(size_t)(b + q) * 64 + li];
    s_part[p][li] = sum;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int pp = 0; pp < SCAN_PARTS; ++pp) {
        const uint32_t v = s_part[pp][li];
        before += pp < p ? v : 0u;
        total += v;
    }
    if (!valid) return;
    if (!OFFSETS) {
        if (p == 0) ttotal[tile] = total;
        return;
    }
    uint32_t run = tstart[tile] + before;
    for (uint32_t q = q0; q < q1; ++q) {
        uint32_t& c = segcnt[(size_t)(b + q) * 64 + li];
        const uint32_t v = c;
        c = run;
        run += v;
    }
}

// Lists capped at a small K (<= GATHER_MAX_K): one wave per tile walks its
// group's coarse list in order, 64 entries at a time, keeps the entries
// whose mask holds the tile (bit test, ballot, mbcnt rank) and stops once it
// has K.  Tile t's list is written at the fixed slot [t K, t K + n_t), so no
// count pass or scan is needed; k_sum_ranges then puts the sum of the n_t in
// n_pairs (one reduction: 8160 same-address atomics would serialize for
// ~0.1 ms).  After a coarse overflow every range is empty and n_pairs
// receives the coarse count, as for whole lists.  A larger K makes the walk
// of a sparse tile long and serial; such caps go through the segment split.
constexpr uint32_t GATHER_MAX_K = 2048;
constexpr int GATHER_BATCHES = 8;
__global__ __launch_bounds__(256) void k_tile_gather(int TX, int TY, int GX, uint32_t K,
                                                     const uint4* __restrict__ coarse,
                                                     const uint32_t* __restrict__ gstart,
                                                     const uint32_t* __restrict__ gtotal,
                                                     uint32_t* __restrict__ point_list, uint32_t* __restrict__ ranges,
                                                     const uint64_t* __restrict__ coarse_n, uint64_t coarse_cap) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= TX * TY) return;
    const bool over = coarse_n[0] > coarse_cap;
    uint32_t cnt = 0;
    if (!over) {
        const int tx = t % TX, ty = t / TX;
        const int grp = (ty / GTILES) * GX + tx / GTILES;
        const int li = (tx % GTILES) + GTILES * (ty % GTILES);
        const uint32_t b0 = gstart[grp], n = gtotal[grp];
        uint32_t* dst = point_list + (size_t)t * K;
        // GATHER_BATCHES batches of 64 entries are loaded at once, so the walk
        // pays one memory round trip per 512 entries
        for (uint32_t k0 = 0; k0 < n && cnt < K; k0 += 64 * GATHER_BATCHES) {
            uint32_t ids[GATHER_BATCHES];
            bool in[GATHER_BATCHES];
#pragma unroll
            for (int u = 0; u < GATHER_BATCHES; ++u) {
                const uint32_t k = k0 + 64 * u + lane;
                in[u] = false;
                ids[u] = 0u;
                if (k < n) {
                    const uint4 e = coarse[b0 + k];
                    in[u] = (((li < 32 ? e.y : e.z) >> (li & 31)) & 1u) != 0u;
                    ids[u] = e.x;
                }
            }
#pragma unroll
            for (int u = 0; u < GATHER_BATCHES; ++u) {
                const uint64_t m = ballot(in[u]);
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (in[u] && cnt + rank < K) dst[cnt + rank] = ids[u];
                cnt = __builtin_amdgcn_readfirstlane(cnt + (uint32_t)__builtin_popcountll(m));
            }
        }
        cnt = min(cnt, K);
    }
    if (lane == 0) {
        ranges[2 * t] = cnt ? (uint32_t)t * K : 0u;
        ranges[2 * t + 1] = cnt ? (uint32_t)t * K + cnt : 0u;
    }
}

// Single workgroup: n_pairs[0] = the sum of the range lengths, or the coarse
// count after a coarse overflow.
__global__ __launch_bounds__(1024) void k_sum_ranges(int nt, const uint32_t* __restrict__ ranges,
                                                     uint64_t* __restrict__ n_pairs,
                                                     const uint64_t* __restrict__ coarse_n, uint64_t coarse_cap) {
    using Reduce = rocprim::block_reduce<uint64_t, 1024>;
    __shared__ typename Reduce::storage_type s_red;
    uint64_t sum = 0;
    for (int t = threadIdx.x; t < nt; t += 1024) sum += ranges[2 * t + 1] - ranges[2 * t];
    uint64_t total = 0;
    Reduce().reduce(sum, total, s_red);
    if (threadIdx.x == 0) n_pairs[0] = coarse_n[0] > coarse_cap ? coarse_n[0] : total;
}

struct ListsLayout {
    size_t dkeys, ids, dkeys2, order, rect, h, part, gtotal, gstart, nseg, segstart, nsegs, mg, coarse_cap, coarse, ttotal,
        tstart, dcnt, dtot, bytes;
    size_t max_segs, segmap, segcnt;
    int C, nb, GX, GY, ng, nt;
};

// the coarse list is at most a fraction of M; its capacity is sized from the
// pairs of the previous call through coarse_cap (grown on demand by the host)
static ListsLayout lists_layout(int32_t width, int32_t height, int64_t P, size_t coarse_cap) {
    ListsLayout L{};
    const size_t n = (size_t)(P > 0 ? P : 1);
    const int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    L.nt = TX * TY;
    L.GX = (TX + GTILES - 1) / GTILES;
    L.GY = (TY + GTILES - 1) / GTILES;
    L.ng = L.GX * L.GY;
    L.C = (int)((n + CHUNK - 1) / CHUNK);
    L.nb = (L.C + PART - 1) / PART;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.dkeys = take(4 * n);
    L.ids = take(4 * n);
    L.dkeys2 = take(4 * n);
    L.order = take(4 * n);
    L.rect = take(8 * n);
    L.h = take(4 * (size_t)L.C * L.ng);
    L.part = take(4 * (size_t)L.nb * L.ng);
    L.gtotal = take(4 * (size_t)L.ng);
    L.gstart = take(4 * (size_t)L.ng);
    L.nseg = take(4 * (size_t)L.ng);
    L.segstart = take(4 * (size_t)L.ng);
    L.nsegs = take(8);
    L.mg = take(8);
    L.ttotal = take(4 * (size_t)L.nt);
    L.tstart = take(4 * (size_t)L.nt);
    L.coarse_cap = coarse_cap;
    L.coarse = take(16 * (coarse_cap > 0 ? coarse_cap : 1));  // (id, 64-bit tile mask, 0) entries
    // segments: at most coarse_cap / SEG + ng of them
    L.max_segs = coarse_cap / SEG + (size_t)L.ng + 1;
    L.segmap = take(8 * L.max_segs);
    L.segcnt = take(4 * 64 * L.max_segs);  // one count per (segment, tile of the group)
    L.dcnt = take(4 * (size_t)DS_RADIX * ds_blocks((int64_t)n));
    L.dtot = take(4 * depth_order_tot_words((int64_t)n));
    L.bytes = off;
    return L;
}

}  // namespace bgs

// Every (group, Gaussian) pair stands for at least one (tile, Gaussian) pair,
// so a coarse list of the point list's capacity always suffices.
extern "C" size_t bgs_tile_lists_workspace_bytes(int32_t width, int32_t height, int64_t P, int64_t capacity) {
    if (width <= 0 || height <= 0 || P < 0 || capacity < 0) return 0;
    return lists_layout(width, height, P, (size_t)capacity).bytes;
}

// conic_opacity == nullptr: the square tile rule; else exact ellipse-tile
// binning
static bgs_status tile_lists(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                             const float* conic_opacity, const int32_t* radius, const float* depth,
                             const uint32_t* tiles_touched, uint32_t* point_list, int64_t capacity,
                             uint32_t max_per_tile, uint32_t* ranges, uint64_t* n_pairs_dev, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
    BGS_REQUIRE(width > 0 && height > 0, "bgs_tile_lists: image size must be positive");
    BGS_REQUIRE(P >= 0 && capacity >= 0, "bgs_tile_lists: negative size");
    if (tile != TILE) return fail(BGS_EUNSUPPORTED, "bgs_tile_lists: only 16x16 tiles are supported");
    BGS_REQUIRE(ranges && n_pairs_dev, "bgs_tile_lists: null ranges or n_pairs");
    BGS_REQUIRE(P < ((int64_t)1 << 31), "bgs_tile_lists: P must be < 2^31");
    BGS_REQUIRE(capacity < ((int64_t)1 << 32), "bgs_tile_lists: capacity must be < 2^32 (32-bit list offsets)");
    const int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    const ListsLayout L = lists_layout(width, height, P, (size_t)capacity);
    if (L.ng > MAX_GROUPS || (size_t)(L.GX + 1) * (L.GY + 1) * sizeof(int) > 65536 || TX > 65535 || TY > 65535)
        return fail(BGS_EUNSUPPORTED, "bgs_tile_lists: tile grid too large (over 8192 groups of 8x8 tiles); use "
                                      "bgs_bin + bgs_sort + bgs_ranges");
    if (conic_opacity && TY > EMIT_ROWS)
        return fail(BGS_EUNSUPPORTED, "bgs_tile_lists_exact: images over 16384 pixels high are not supported");
    BGS_REQUIRE(ws && ws_bytes >= L.bytes, "bgs_tile_lists: workspace too small");
    const bool gather = max_per_tile && max_per_tile <= GATHER_MAX_K;
    if (gather && (int64_t)L.nt * max_per_tile > capacity)
        return fail(BGS_ECAPACITY, "bgs_tile_lists: lists capped at K <= 2048 need capacity >= n_tiles * K");
    BGS_REQUIRE(capacity == 0 || point_list != nullptr, "bgs_tile_lists: null point_list");
    char* w = static_cast<char*>(ws);
    auto* dkeys = reinterpret_cast<uint32_t*>(w + L.dkeys);
    auto* ids = reinterpret_cast<uint32_t*>(w + L.ids);
    auto* dkeys2 = reinterpret_cast<uint32_t*>(w + L.dkeys2);
    auto* order = reinterpret_cast<uint32_t*>(w + L.order);
    auto* rect = reinterpret_cast<uint2*>(w + L.rect);
    auto* h = reinterpret_cast<uint32_t*>(w + L.h);
    auto* part = reinterpret_cast<uint32_t*>(w + L.part);
    auto* gtotal = reinterpret_cast<uint32_t*>(w + L.gtotal);
    auto* gstart = reinterpret_cast<uint32_t*>(w + L.gstart);
    auto* ttotal = reinterpret_cast<uint32_t*>(w + L.ttotal);
    auto* tstart = reinterpret_cast<uint32_t*>(w + L.tstart);
    auto* coarse = reinterpret_cast<uint4*>(w + L.coarse);
    if (P == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * (int64_t)L.nt)), dim3(256), 0, stream, ranges,
                           2 * (int64_t)L.nt, 0u);
        BGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint32_t*>(n_pairs_dev),
                           (int64_t)2, 0u);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    const auto* co4 = reinterpret_cast<const float4*>(conic_opacity);
    {
        // the depth keys and every Gaussian's tile rectangle in one pass
        const RectArgs R{TX, TY, means2D, radius, co4, rect};
        const bgs_status st = depth_order(P, depth, tiles_touched, dkeys, order, dkeys2, ids,
                                          reinterpret_cast<uint32_t*>(w + L.dcnt),
                                          reinterpret_cast<uint32_t*>(w + L.dtot), R, stream);
        if (st != BGS_OK) return st;
    }
    // coarse (group) lists
    hipLaunchKernelGGL(k_chunk_hist, dim3(L.C), dim3(CHUNK), sizeof(int) * (size_t)(L.GX + 1) * (L.GY + 1), stream, P,
                       L.GX, L.GY, order, rect, h);
    BGS_HIP(hipGetLastError());
    const int64_t nbg = (int64_t)L.nb * L.ng;
    hipLaunchKernelGGL(k_part_sums, dim3((unsigned)(L.nb * ((L.ng + PS_COLS - 1) / PS_COLS))), dim3(256), 0, stream,
                       L.C, L.ng, h, part);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_part_scan, dim3((unsigned)((L.ng + 3) / 4)), dim3(256), 0, stream, L.nb, L.ng, part, gtotal);
    BGS_HIP(hipGetLastError());
    // the coarse total Mg stays on the device; every later kernel checks it
    // against the coarse capacity, so the call never waits for the GPU
    auto* mg = reinterpret_cast<uint64_t*>(w + L.mg);
    const uint64_t ccap = (uint64_t)L.coarse_cap, pcap = (uint64_t)capacity;
    const uint64_t no_cap = ~(uint64_t)0;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, stream, L.ng, gtotal, gstart, (uint32_t*)nullptr, mg,
                       (const uint64_t*)nullptr, no_cap, no_cap, ~0u);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_chunk_base, dim3(blocks_for(nbg)), dim3(256), 0, stream, L.C, L.ng, gstart, part, h);
    BGS_HIP(hipGetLastError());
    {
        const int gbits = L.ng > 1 ? 32 - __builtin_clz((unsigned)(L.ng - 1)) : 0;
        if (conic_opacity)
            hipLaunchKernelGGL(k_chunk_emit<true>, dim3(L.C), dim3(64), sizeof(uint32_t) * (size_t)L.ng, stream, P,
                               L.GX, L.GY, gbits, order, rect, h, coarse, (const uint64_t*)mg, ccap, means2D, co4);
        else
            hipLaunchKernelGGL(k_chunk_emit<false>, dim3(L.C), dim3(64), sizeof(uint32_t) * (size_t)L.ng, stream, P,
                               L.GX, L.GY, gbits, order, rect, h, coarse, (const uint64_t*)mg, ccap,
                               (const float*)nullptr, (const float4*)nullptr);
    }
    BGS_HIP(hipGetLastError());
    if (gather) {  // lists capped at a small K: gathered per tile at fixed slots
        hipLaunchKernelGGL(k_tile_gather, dim3((unsigned)((L.nt + 3) / 4)), dim3(256), 0, stream, TX, TY, L.GX,
                           max_per_tile, coarse, gstart, gtotal, point_list, ranges, (const uint64_t*)mg, ccap);
        BGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sum_ranges, dim3(1), dim3(1024), 0, stream, L.nt, ranges, n_pairs_dev,
                           (const uint64_t*)mg, ccap);
        BGS_HIP(hipGetLastError());
        return BGS_OK;
    }
    // fine (tile) lists, on segments of the coarse lists
    auto* nseg = reinterpret_cast<uint32_t*>(w + L.nseg);
    auto* segstart = reinterpret_cast<uint32_t*>(w + L.segstart);
    auto* nsegs = reinterpret_cast<uint64_t*>(w + L.nsegs);
    auto* segmap = reinterpret_cast<uint2*>(w + L.segmap);
    auto* segcnt = reinterpret_cast<uint32_t*>(w + L.segcnt);
    const uint32_t max_segs = (uint32_t)L.max_segs;
    const unsigned grid_split = (unsigned)std::min<size_t>(L.max_segs, SPLIT_GRID);
    hipLaunchKernelGGL(k_seg_count, dim3(blocks_for(L.ng)), dim3(256), 0, stream, L.ng, gtotal, nseg);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, stream, L.ng, nseg, segstart, (uint32_t*)nullptr, nsegs,
                       (const uint64_t*)nullptr, no_cap, no_cap, ~0u);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_map, dim3((unsigned)((L.ng + 3) / 4)), dim3(256), 0, stream, L.ng, nseg, segstart, segmap,
                       (const uint64_t*)mg, ccap, max_segs);
    BGS_HIP(hipGetLastError());
    const TileGrid tg{TX, TY, L.GX, ranges};
    hipLaunchKernelGGL(k_seg_split<false>, dim3(grid_split), dim3(256), 0, stream, nsegs, segmap, coarse, gstart,
                       gtotal, segcnt, (uint32_t*)nullptr, (const uint64_t*)nullptr, (uint64_t)0, (const uint64_t*)mg,
                       ccap, max_segs, tg);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_scan<false>, dim3(L.ng), dim3(SCAN_PARTS * 64), 0, stream, TX, TY, L.GX, nseg,
                       segstart, segcnt, (const uint32_t*)nullptr, ttotal, (const uint64_t*)mg, ccap);
    BGS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, stream, L.nt, ttotal, tstart, ranges, n_pairs_dev,
                       (const uint64_t*)mg, ccap, pcap, max_per_tile ? max_per_tile : ~0u);
    BGS_HIP(hipGetLastError());
    if (capacity > 0) {
        hipLaunchKernelGGL(k_seg_scan<true>, dim3(L.ng), dim3(SCAN_PARTS * 64), 0, stream, TX, TY, L.GX, nseg,
                           segstart, segcnt, tstart, (uint32_t*)nullptr, (const uint64_t*)mg, ccap);
        BGS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_seg_split<true>, dim3(grid_split), dim3(256), 0, stream, nsegs, segmap, coarse, gstart,
                           gtotal, segcnt, point_list, (const uint64_t*)n_pairs_dev, pcap, (const uint64_t*)mg, ccap,
                           max_segs, tg);
        BGS_HIP(hipGetLastError());
    }
    return BGS_OK;
}

extern "C" bgs_status bgs_tile_lists(int32_t width, int32_t height, int32_t tile, int64_t P, const float* means2D,
                                     const int32_t* radius, const float* depth, const uint32_t* tiles_touched,
                                     uint32_t* point_list, int64_t capacity, uint32_t max_per_tile, uint32_t* ranges,
                                     uint64_t* n_pairs_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
    return tile_lists(width, height, tile, P, means2D, nullptr, radius, depth, tiles_touched, point_list, capacity,
                      max_per_tile, ranges, n_pairs_dev, ws, ws_bytes, stream);
}

extern "C" bgs_status bgs_tile_lists_exact(int32_t width, int32_t height, int32_t tile, int64_t P,
                                           const float* means2D, const float* conic_opacity, const int32_t* radius,
                                           const float* depth, const uint32_t* tiles_touched, uint32_t* point_list,
                                           int64_t capacity, uint32_t max_per_tile, uint32_t* ranges,
                                           uint64_t* n_pairs_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
    BGS_REQUIRE(P == 0 || conic_opacity != nullptr, "bgs_tile_lists_exact: conic_opacity is null");
    BGS_REQUIRE(((uintptr_t)conic_opacity & 15u) == 0, "bgs_tile_lists_exact: conic_opacity must be 16-byte aligned");
    return tile_lists(width, height, tile, P, means2D, P ? conic_opacity : nullptr, radius, depth, tiles_touched,
                      point_list, capacity, max_per_tile, ranges, n_pairs_dev, ws, ws_bytes, stream);
}
