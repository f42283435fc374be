// Internal helpers of the bgs HIP library (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "bgs.h"

namespace bgs {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
bgs_status fail(bgs_status code, const std::string& msg);

#define BGS_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::bgs::fail(BGS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BGS_REQUIRE(cond, msg)                                   \
    do {                                                         \
        if (!(cond)) return ::bgs::fail(BGS_EINVAL, (msg));      \
    } while (0)

// Number of compute units of the current device (cached per device).
int cu_count();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- device math
constexpr int WAVE = 64;
constexpr int TILE = 16;             // binning tile edge
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_MIN = 1e-4f;
constexpr float LOG2E = 1.4426950408889634f;

// Gradient record of one Gaussian (packed gradients): d/d(a, b, c, o) at
// floats 0-3 (16-byte aligned), d/d(u, v) at 4-5, d/d(r, g, b) at 6-8,
// d/d(depth) at 9, floats 10-15 unused.  A record is one 64-byte segment, so
// the ten atomic adds of one list entry's gradient land in one cache line
// instead of four arrays' lines.
constexpr int GRAD_RECORD = 16;

// floor(a / b) for b > 0
__host__ __device__ inline int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    return (q * b > a) ? q - 1 : q;
}

// Inclusive tile rectangle of a screen square [u-r, u+r] x [v-r, v+r]: tiles
// k with [k*TILE, (k+1)*TILE) meeting [u-r, u+r].  Because r is an integer,
// floor((u +- r)/TILE) = floor((floor(u) +- r)/TILE), so the rectangle is
// exact integer arithmetic on floor(u).  Returns false when empty.
__device__ inline bool tile_rect(float u, float v, int r, int TX, int TY, int& x0, int& y0, int& x1,
                                 int& y1) {
    if (r <= 0) return false;
    // clamp far off-screen centres so that the integer conversion is defined;
    // any clamped value lies far outside every tile either way
    const float lim = 1.0e9f;
    float uc = fminf(fmaxf(u, -lim), lim), vc = fminf(fmaxf(v, -lim), lim);
    int64_t fu = (int64_t)floorf(uc), fv = (int64_t)floorf(vc);
    int64_t a0 = floor_div(fu - r, TILE), a1 = floor_div(fu + r, TILE);
    int64_t b0 = floor_div(fv - r, TILE), b1 = floor_div(fv + r, TILE);
    if (a0 < 0) a0 = 0;
    if (b0 < 0) b0 = 0;
    if (a1 > TX - 1) a1 = TX - 1;
    if (b1 > TY - 1) b1 = TY - 1;
    if (a0 > a1 || b0 > b1) return false;
    x0 = (int)a0; y0 = (int)b0; x1 = (int)a1; y1 = (int)b1;
    return true;
}

// Exponent of one (pixel, Gaussian) pair, base 2, from the conic staged in
// pivoted form.  With r = b / a, q = (a c - b^2) / a and t = dx + r dy,
//     a dx^2 + 2 b dx dy + c dy^2 = a t^2 + q dy^2,
// two non-negative terms for a positive-definite conic, so the fp32 value has
// no cancellation; the expanded form loses up to cond(conic) ulps at pixels
// far along a needle-shaped Gaussian (measured: 2e-3 absolute in the
// exponent at condition ~1e4, against 1e-5 here).  The staged numbers are
// a2 = -log2(e) a / 2, r, q2 = -log2(e) q / 2, so the result is
// log2(e) * power.  Written with explicit fma so that forward and backward
// kernels evaluate bit-identical values (the backward re-takes the forward's
// skip decisions).
__device__ __forceinline__ float splat_power2(float dx, float dy, float a2, float r, float q2) {
    const float t = __builtin_fmaf(r, dy, dx);
    const float qdd = (q2 * dy) * dy;
    return __builtin_fmaf(a2 * t, t, qdd);
}

// (a2, r, q2) of splat_power2 from the conic (a, b, c).  a c - b^2 is formed
// with an fma-compensated product, so its relative error stays a few ulps
// when b^2 is close to a c.  A conic with a = 0 (not positive definite,
// outside the render contract) is staged as (0, 0, c-term): its b dx dy term
// is dropped.
__device__ __forceinline__ float3 stage_conic(float a, float b, float c) {
    constexpr float K = -0.5f * LOG2E;
    if (!(a != 0.0f)) return make_float3(0.0f, 0.0f, K * c);
    const float bb = b * b;
    const float bb_err = __builtin_fmaf(b, b, -bb);  // b*b - bb, exact
    const float det = __builtin_fmaf(a, c, -bb) - bb_err;
    const float inv_a = 1.0f / a;
    return make_float3(K * a, b * inv_a, (K * det) * inv_a);
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                                 false));
}

// Sum over the 64 lanes of a wave (all lanes must be active); the total is
// returned in every lane (through lane 63).
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);       // row_half_mirror
    v += dpp<0x140>(v);       // row_mirror        -> every lane holds its row's sum
    v += dpp<0x142, 0xA>(v);  // row_bcast:15      -> rows 1, 3 hold pair sums
    v += dpp<0x143, 0xC>(v);  // row_bcast:31      -> row 3 holds the total
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Lane exchanges of gfx950 that stay in the VALU (no LDS round trip):
// permlane32_swap exchanges lanes 32..63 of x with lanes 0..31 of y, and
// permlane16_swap exchanges the odd 16-lane rows of x with the even rows of
// y.  For a butterfly stage that keeps x in the lower partner and y in the
// upper one, (x' + y') is then the partner sum in every lane.
__device__ __forceinline__ float swap_sum32(float x, float y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                    false, false);
    return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}

__device__ __forceinline__ float swap_sum16(float x, float y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                    false, false);
    return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}

// v from lane (lane xor 8) / (lane xor 4), as two DPP moves each:
// row_mirror then row_half_mirror reads lane 8 - (i & 8) + (i & 7) of the row;
// row_half_mirror then quad_perm [3,2,1,0] reads lane i xor 4.
__device__ __forceinline__ float xor8(float v) { return dpp<0x141>(dpp<0x140>(v)); }
__device__ __forceinline__ float xor4(float v) { return dpp<0x1B>(dpp<0x141>(v)); }

// Transposed reduction of 10 per-lane values over the 64 lanes of a wave
// (all lanes active).  Each butterfly stage halves the values a lane keeps
// while it adds its partner's copy (xor 32: 10 -> 5, xor 16: 5 -> 3 (padded),
// xor 8: 3 -> 2, xor 4: 2 -> 1), then xor 2 and xor 1 finish the sum, so 13
// exchanges replace 10 full 64-lane reductions; all of them are VALU lane
// swaps or DPP moves.  Value k's total ends in the lanes whose bits
// (5,4,3,2) = (b5,b4,b3,b2) satisfy k = 5 b5 + 3 b4 + 2 b3 + b2 (with
// 2 b3 + b2 < 3 and 3 b4 + 2 b3 + b2 < 5).  Returns k in the first lane of
// that quad (others: -1) and the total in out.
__device__ __forceinline__ int scatter10_slot(int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
    const int p3 = 2 * (int)b3 + (int)b2;
    const int p5 = 3 * (int)b4 + p3;
    const bool valid = p3 < 3 && p5 < 5 && (lane & 3) == 0;
    return valid ? 5 * (int)b5 + p5 : -1;
}

__device__ __forceinline__ int wave_reduce_scatter10(const float (&v)[10], int lane, float& out) {
    const bool b3 = lane & 8, b2 = lane & 4;
    float a[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) a[i] = swap_sum32(v[i], v[5 + i]);  // b5 ? v[5+i] : v[i]
    float c[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = swap_sum16(a[i], i < 2 ? a[3 + i] : 0.0f);  // b4 ? a[3+i] : a[i]
    float d[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float hi = i == 0 ? c[2] : 0.0f;
        const float keep = b3 ? hi : c[i];
        const float send = b3 ? c[i] : hi;
        d[i] = keep + xor8(send);
    }
    float e = (b2 ? d[1] : d[0]) + xor4(b2 ? d[0] : d[1]);
    e += dpp<0x4E>(e);  // quad_perm [2,3,0,1]: lane xor 2
    e += dpp<0xB1>(e);  // quad_perm [1,0,3,2]: lane xor 1
    out = e;
    return scatter10_slot(lane);
}

// Stable LSD radix sort of n (key, value) pairs by the low `bits` key bits
// (binning.hip): the result is in (k0, v0), or in (k1, v1) when *in_second.
// cnt and tot: radix_sort_pairs_u32_scratch(n) bytes.
bgs_status radix_sort_pairs_u32(int64_t n, int bits, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                                uint32_t* cnt, uint32_t* tot, bool* in_second, hipStream_t stream);
size_t radix_sort_pairs_u32_scratch(int64_t n);

__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off >= 1; off >>= 1) {
        int o = __shfl_xor(v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}

}  // namespace bgs
