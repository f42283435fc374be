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
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"

namespace bgs {

// depth keys of the Gaussians: positive fp32 depths order like their bit
// patterns; Gaussians with no pairs go last.
__global__ __launch_bounds__(256) void k_depth_keys(int64_t P, const float* __restrict__ depth,
                                                    const uint32_t* __restrict__ tiles_touched,
                                                    uint32_t* __restrict__ keys, uint32_t* __restrict__ ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    keys[i] = tiles_touched[i] ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
    ids[i] = (uint32_t)i;
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

// One thread per Gaussian (in depth order) writes its run of pairs.
__global__ __launch_bounds__(256) void k_emit(int64_t P, int TX, int TY, const uint32_t* __restrict__ order,
                                              const uint64_t* __restrict__ offsets, const float* __restrict__ means2D,
                                              const int* __restrict__ radius,
                                              const uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ values) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const uint32_t g = order[k];
    if (tiles_touched[g] == 0) return;
    int x0, y0, x1, y1;
    if (!tile_rect(means2D[2 * g], means2D[2 * g + 1], radius[g], TX, TY, x0, y0, x1, y1)) return;
    uint64_t o = offsets[k];
    // never write past this Gaussian's own run, whatever tiles_touched says
    const uint64_t o_end = o + tiles_touched[g];
    for (int ty = y0; ty <= y1; ++ty)
        for (int tx = x0; tx <= x1; ++tx) {
            if (o >= o_end) return;
            keys[o] = (uint32_t)(ty * TX + tx);
            values[o] = g;
            ++o;
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
    size_t keys, ids, keys2, order, counts, offsets, total, temp, temp_bytes, bytes;
};

static BinLayout bin_layout(int64_t P) {
    BinLayout L{};
    const size_t n = (size_t)(P > 0 ? P : 1);
    size_t sort_bytes = 0, scan_bytes = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, sort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                              (uint32_t*)nullptr, n, 0, 32);
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
    L.temp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
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
    hipLaunchKernelGGL(k_depth_keys, dim3(blocks_for(P)), dim3(256), 0, stream, P, depth, tiles_touched, dkeys, ids);
    BGS_HIP(hipGetLastError());
    BGS_HIP(rocprim::radix_sort_pairs(temp, temp_bytes, dkeys, dkeys2, ids, order, (size_t)P, 0, 32, stream));
    hipLaunchKernelGGL(k_gather_counts, dim3(blocks_for(P)), dim3(256), 0, stream, P, order, tiles_touched, counts);
    BGS_HIP(hipGetLastError());
    temp_bytes = L.temp_bytes;
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
