// Projection of 3D Gaussians to screen-space splats, Eq. (1)-(3) of Balanced
// 3DGS (Sec. 2.1): camera transform, 3D covariance from scale and rotation,
// EWA covariance Sigma' = J W Sigma W^T J^T (+0.3 px^2 low-pass), its inverse
// (conic), 3-sigma radius, colour from RGB or real spherical harmonics, and
// the number of 16x16 tiles the splat's square meets.
//
// One thread per Gaussian; fp32 throughout.  O(P) work, a few hundred flops
// per Gaussian: bandwidth-bound on the input arrays (52 B, or 240 B with
// degree-3 SH, per Gaussian).  The kernels are instantiated per SH degree, so
// the SH loops unroll and their tables stay in registers; with degree >= 1 a
// workgroup's colour coefficients (and, in the backward, their gradients)
// pass through LDS so that global memory sees one contiguous, coalesced run
// per workgroup instead of one 4-byte access per Gaussian and coefficient.
#include "common.h"

namespace bgs {

struct ProjParams {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float campos[3];
    float znear, limx, limy;
    int TX, TY;
};

constexpr int PROJ_THREADS = 256;

// Colour layout per SH degree D (-1: plain RGB): NC floats per Gaussian; in
// LDS a Gaussian's row has the odd stride NC | 1, so the 64 lanes of a wave
// reading word j of their own rows hit 64 distinct banks.
template <int D>
struct ShDim {
    static constexpr int NSH = D < 0 ? 1 : (D + 1) * (D + 1);
    static constexpr int NC = 3 * NSH;
    static constexpr int STRIDE = NC | 1;
    static constexpr bool STAGED = D >= 1;
    static constexpr int LDS_FLOATS = STAGED ? PROJ_THREADS * STRIDE : 1;
};

// Element e of the workgroup's contiguous run <-> its LDS slot.
template <int NC, int STRIDE>
__device__ __forceinline__ int lds_slot(int e) {
    const int t = e / NC;
    return t * STRIDE + (e - t * NC);
}

// LDS rows <- src[first * NC .. (first + n) * NC): coalesced, 16-byte
// vectors when the run is 16-byte aligned.
template <int NC, int STRIDE>
__device__ inline void stage_in(const float* src, int64_t first, int n, float* s) {
    const float* g = src + first * NC;
    const int total = n * NC;
    int e0 = 0;
    if ((reinterpret_cast<uintptr_t>(g) & 15) == 0) {
        const int n4 = total >> 2;
        for (int v = threadIdx.x; v < n4; v += PROJ_THREADS) {
            const float4 x = reinterpret_cast<const float4*>(g)[v];
            s[lds_slot<NC, STRIDE>(4 * v)] = x.x;
            s[lds_slot<NC, STRIDE>(4 * v + 1)] = x.y;
            s[lds_slot<NC, STRIDE>(4 * v + 2)] = x.z;
            s[lds_slot<NC, STRIDE>(4 * v + 3)] = x.w;
        }
        e0 = 4 * n4;
    }
    for (int e = e0 + threadIdx.x; e < total; e += PROJ_THREADS) s[lds_slot<NC, STRIDE>(e)] = g[e];
}

// dst[first * NC .. (first + n) * NC) <- LDS rows, the reverse of stage_in.
template <int NC, int STRIDE>
__device__ inline void stage_out(float* dst, int64_t first, int n, const float* s) {
    float* g = dst + first * NC;
    const int total = n * NC;
    int e0 = 0;
    if ((reinterpret_cast<uintptr_t>(g) & 15) == 0) {
        const int n4 = total >> 2;
        for (int v = threadIdx.x; v < n4; v += PROJ_THREADS)
            reinterpret_cast<float4*>(g)[v] =
                make_float4(s[lds_slot<NC, STRIDE>(4 * v)], s[lds_slot<NC, STRIDE>(4 * v + 1)],
                            s[lds_slot<NC, STRIDE>(4 * v + 2)], s[lds_slot<NC, STRIDE>(4 * v + 3)]);
        e0 = 4 * n4;
    }
    for (int e = e0 + threadIdx.x; e < total; e += PROJ_THREADS) g[e] = s[lds_slot<NC, STRIDE>(e)];
}

// Real spherical harmonics (no Condon-Shortley phase), index l*l + l + m,
// at the unit vector (x, y, z), for l <= degree.  Amplitudes: C0 = 1/(2
// sqrt(pi)), C1 = sqrt(3/(4 pi)), and for l = 2, 3 the closed forms written
// beside each constant.
__device__ inline void sh_basis(int degree, float x, float y, float z, float Y[16]) {
    const float C0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
    const float C1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
    const float C2a = 1.0925484305920792f;   // sqrt(15/pi)/2
    const float C2b = 0.31539156525252005f;  // sqrt(5/pi)/4
    const float C2c = 0.5462742152960396f;   // sqrt(15/pi)/4
    const float C3a = 0.5900435899266435f;   // sqrt(35/(2 pi))/4
    const float C3b = 2.890611442640554f;    // sqrt(105/pi)/2
    const float C3c = 0.4570457994644658f;   // sqrt(21/(2 pi))/4
    const float C3d = 0.3731763325901154f;   // sqrt(7/pi)/4
    const float C3e = 1.445305721320277f;    // sqrt(105/pi)/4
    Y[0] = C0;
    if (degree >= 1) {
        Y[1] = C1 * y;
        Y[2] = C1 * z;
        Y[3] = C1 * x;
    }
    if (degree >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = C2a * x * y;
        Y[5] = C2a * y * z;
        Y[6] = C2b * (3.0f * zz - 1.0f);
        Y[7] = C2a * x * z;
        Y[8] = C2c * (xx - yy);
        if (degree >= 3) {
            Y[9] = C3a * y * (3.0f * xx - yy);
            Y[10] = C3b * x * y * z;
            Y[11] = C3c * y * (5.0f * zz - 1.0f);
            Y[12] = C3d * z * (5.0f * zz - 3.0f);
            Y[13] = C3c * x * (5.0f * zz - 1.0f);
            Y[14] = C3e * z * (xx - yy);
            Y[15] = C3a * x * (xx - 3.0f * yy);
        }
    }
}

// colour = max(0, 1/2 + sum_i k_i Y_i) per channel; coefficients k[i][3].
template <int D>
__device__ inline void sh_colour(const float* k, float x, float y, float z, float out[3]) {
    float Y[16];
    sh_basis(D, x, y, z, Y);
    constexpr int n = (D + 1) * (D + 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float s = 0.5f;
#pragma unroll
        for (int i = 0; i < n; ++i) s += k[3 * i + c] * Y[i];
        out[c] = fmaxf(s, 0.0f);
    }
}

template <int D>
__global__ __launch_bounds__(PROJ_THREADS) void k_project(ProjParams pp, int64_t P, const float* __restrict__ means3D,
                                                          const float* __restrict__ log_scales,
                                                          const float* __restrict__ quats,
                                                          const float* __restrict__ opacity,
                                                          const float* __restrict__ colors, float* __restrict__ means2D,
                                                          float* __restrict__ conic_opacity, float* __restrict__ rgb,
                                                          float* __restrict__ depth, int* __restrict__ radius,
                                                          uint32_t* __restrict__ tiles_touched) {
    using S = ShDim<D>;
    __shared__ float s_sh[S::LDS_FLOATS];
    const int64_t first = (int64_t)blockIdx.x * PROJ_THREADS;
    const int64_t i = first + threadIdx.x;
    if (S::STAGED) {
        stage_in<S::NC, S::STRIDE>(colors, first, (int)(P - first < PROJ_THREADS ? P - first : PROJ_THREADS), s_sh);
        __syncthreads();
    }
    if (i >= P) return;
    const float mx = means3D[3 * i], my = means3D[3 * i + 1], mz = means3D[3 * i + 2];
    const float* R = pp.R;
    const float px = R[0] * mx + R[1] * my + R[2] * mz + pp.t[0];
    const float py = R[3] * mx + R[4] * my + R[5] * mz + pp.t[1];
    const float pz = R[6] * mx + R[7] * my + R[8] * mz + pp.t[2];

    bool keep = pz > pp.znear;
    float s00 = 0, s01 = 0, s11 = 0, det = 0;
    if (keep) {
        // 3D covariance  Sigma = Rq diag(e^{2s}) Rq^T, symmetric (6 values)
        float qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
        const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= qn; qx *= qn; qy *= qn; qz *= qn;
        const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                             2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                             2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
        // Jacobian of the pinhole map at the (clamped) ray, times the view rotation
        const float iz = 1.0f / pz;
        const float xz = fminf(fmaxf(px * iz, -pp.limx), pp.limx);
        const float yz = fminf(fmaxf(py * iz, -pp.limy), pp.limy);
        const float j00 = pp.fx * iz, j02 = -pp.fx * xz * iz;
        const float j11 = pp.fy * iz, j12 = -pp.fy * yz * iz;
        float T0[3], T1[3];
        for (int c = 0; c < 3; ++c) {
            T0[c] = j00 * R[c] + j02 * R[6 + c];
            T1[c] = j11 * R[3 + c] + j12 * R[6 + c];
        }
        // Sigma = sum_b e_b^2 r_b r_b^T (r_b the columns of Rq, e_b^2 = exp(2 s_b)),
        // so Sigma' = sum_b e_b^2 u_b u_b^T + 0.3 I with u_b = T r_b the screen
        // images of the axes.  Its determinant (Cauchy-Binet)
        //   det = sum_{b<c} e_b^2 e_c^2 (u_b x u_c)^2 + 0.3 sum_b e_b^2 |u_b|^2 + 0.09
        // is a sum of non-negative terms: no cancellation, where the expanded
        // s00 s11 - s01^2 of a needle-shaped Gaussian loses ~cond ulps.
        float u[3][2], e2[3];
        for (int b = 0; b < 3; ++b) {
            e2[b] = __expf(2.f * log_scales[3 * i + b]);
            u[b][0] = T0[0] * Rq[b] + T0[1] * Rq[3 + b] + T0[2] * Rq[6 + b];
            u[b][1] = T1[0] * Rq[b] + T1[1] * Rq[3 + b] + T1[2] * Rq[6 + b];
        }
        s00 = 0.3f;
        s01 = 0.f;
        s11 = 0.3f;
        float tr = 0.f;
        for (int b = 0; b < 3; ++b) {
            s00 += e2[b] * u[b][0] * u[b][0];
            s01 += e2[b] * u[b][0] * u[b][1];
            s11 += e2[b] * u[b][1] * u[b][1];
            tr += e2[b] * (u[b][0] * u[b][0] + u[b][1] * u[b][1]);
        }
        det = 0.3f * tr + 0.09f;
        for (int b = 0; b < 3; ++b)
            for (int c = b + 1; c < 3; ++c) {
                const float x = u[b][0] * u[c][1] - u[b][1] * u[c][0];
                det += e2[b] * e2[c] * x * x;
            }
        keep = det > 0.0f;
    }
    int r = 0;
    float u = 0, v = 0;
    if (keep) {
        const float mid = 0.5f * (s00 + s11);
        const float lmax = mid + sqrtf(fmaxf(mid * mid - det, 0.0f));
        const float rf = ceilf(3.0f * sqrtf(lmax));
        r = rf < 1.0e9f ? (int)rf : 1000000000;  // bounded so the integer tile maths cannot overflow
        u = pp.fx * px / pz + pp.cx - 0.5f;
        v = pp.fy * py / pz + pp.cy - 0.5f;
    }
    if (!keep) {
        // culled: no pairs, all outputs zero
        means2D[2 * i] = 0.f; means2D[2 * i + 1] = 0.f;
        reinterpret_cast<float4*>(conic_opacity)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        rgb[3 * i] = 0.f; rgb[3 * i + 1] = 0.f; rgb[3 * i + 2] = 0.f;
        depth[i] = 0.f;
        radius[i] = 0;
        tiles_touched[i] = 0;
        return;
    }
    int x0, y0, x1, y1;
    const bool on_screen = tile_rect(u, v, r, pp.TX, pp.TY, x0, y0, x1, y1);
    const float idet = 1.0f / det;
    means2D[2 * i] = u;
    means2D[2 * i + 1] = v;
    reinterpret_cast<float4*>(conic_opacity)[i] = make_float4(s11 * idet, -s01 * idet, s00 * idet, opacity[i]);
    depth[i] = pz;
    radius[i] = r;
    tiles_touched[i] = on_screen ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;

    if (D < 0) {
        rgb[3 * i] = colors[3 * i];
        rgb[3 * i + 1] = colors[3 * i + 1];
        rgb[3 * i + 2] = colors[3 * i + 2];
    } else {
        float dx = mx - pp.campos[0], dy = my - pp.campos[1], dz = mz - pp.campos[2];
        const float n = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= n; dy *= n; dz *= n;
        float c[3];
        sh_colour<D < 0 ? 0 : D>(S::STAGED ? s_sh + threadIdx.x * S::STRIDE : colors + (int64_t)S::NC * i, dx, dy,
                                 dz, c);
        rgb[3 * i] = c[0];
        rgb[3 * i + 1] = c[1];
        rgb[3 * i + 2] = c[2];
    }
}

// ---------------------------------------------------------------- backward
// Gradients of the real spherical harmonics above with respect to the
// (unnormalized) direction components, the derivatives of the same
// polynomials.
__device__ inline void sh_grad(int degree, float x, float y, float z, float g[16][3]) {
    const float C1 = 0.4886025119029199f;
    const float C2a = 1.0925484305920792f, C2b = 0.31539156525252005f, C2c = 0.5462742152960396f;
    const float C3a = 0.5900435899266435f, C3b = 2.890611442640554f, C3c = 0.4570457994644658f;
    const float C3d = 0.3731763325901154f, C3e = 1.445305721320277f;
    for (int i = 0; i < 16; ++i) g[i][0] = g[i][1] = g[i][2] = 0.f;
    if (degree >= 1) {
        g[1][1] = C1;
        g[2][2] = C1;
        g[3][0] = C1;
    }
    if (degree >= 2) {
        g[4][0] = C2a * y; g[4][1] = C2a * x;
        g[5][1] = C2a * z; g[5][2] = C2a * y;
        g[6][2] = 6.0f * C2b * z;
        g[7][0] = C2a * z; g[7][2] = C2a * x;
        g[8][0] = 2.0f * C2c * x; g[8][1] = -2.0f * C2c * y;
    }
    if (degree >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        g[9][0] = 6.0f * C3a * x * y; g[9][1] = 3.0f * C3a * (xx - yy);
        g[10][0] = C3b * y * z; g[10][1] = C3b * x * z; g[10][2] = C3b * x * y;
        g[11][1] = C3c * (5.0f * zz - 1.0f); g[11][2] = 10.0f * C3c * y * z;
        g[12][2] = C3d * (15.0f * zz - 3.0f);
        g[13][0] = C3c * (5.0f * zz - 1.0f); g[13][2] = 10.0f * C3c * x * z;
        g[14][0] = 2.0f * C3e * x * z; g[14][1] = -2.0f * C3e * y * z; g[14][2] = C3e * (xx - yy);
        g[15][0] = 3.0f * C3a * (xx - yy); g[15][1] = -6.0f * C3a * x * y;
    }
}

// One thread per Gaussian: the forward is recomputed and every step is
// differentiated in reverse order (conic inverse; Sigma' = T Sigma T^T with
// T = J R; J of the clamped ray, whose derivative through the clamp is 0;
// the pinhole map and depth; Sigma = M M^T, M = Rq diag(e^s); the rotation
// of the normalized quaternion; the SH colour along the view ray and its 0
// clamp).  Gradients are written (=); culled Gaussians get zeros.
// Gaussian i.  coef: its colour row (RGB or SH coefficients [j][3]); dc:
// where its colour gradient goes, in the same layout.  In the LDS-staged
// kernels coef and dc are the same row: each coefficient is read before its
// slot is overwritten.
// REC = 0: the screen-space gradients in their four arrays; REC = GRAD_RECORD:
// in gradient records (g_conic_opacity the record array, g_means2D, g_rgb and
// g_depth its floats 4, 6 and 9).
template <int D, int REC = 0>
__device__ inline void project_bwd_one(const ProjParams& pp, int64_t i, const float* __restrict__ means3D,
                                       const float* __restrict__ log_scales, const float* __restrict__ quats,
                                       const float* coef, const float* __restrict__ g_means2D,
                                       const float* __restrict__ g_conic_opacity, const float* __restrict__ g_rgb,
                                       const float* __restrict__ g_depth, float* __restrict__ d_means3D,
                                       float* __restrict__ d_log_scales, float* __restrict__ d_quats,
                                       float* __restrict__ d_opacity, float* dc) {
    constexpr int nsh = ShDim<D>::NSH;
    const float mx = means3D[3 * i], my = means3D[3 * i + 1], mz = means3D[3 * i + 2];
    const float* R = pp.R;
    const float p[3] = {R[0] * mx + R[1] * my + R[2] * mz + pp.t[0], R[3] * mx + R[4] * my + R[5] * mz + pp.t[1],
                        R[6] * mx + R[7] * my + R[8] * mz + pp.t[2]};
    auto zero = [&]() {
        for (int k = 0; k < 3; ++k) d_means3D[3 * i + k] = d_log_scales[3 * i + k] = 0.f;
        reinterpret_cast<float4*>(d_quats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        d_opacity[i] = 0.f;
        for (int k = 0; k < 3 * nsh; ++k) dc[k] = 0.f;
    };
    if (!(p[2] > pp.znear)) {
        zero();
        return;
    }
    // ---- forward recomputation
    const float q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3), iqn = 1.0f / qn;
    const float w = q0 * iqn, x = q1 * iqn, y = q2 * iqn, z = q3 * iqn;
    const float Rq[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                         2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                         2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    const float e[3] = {__expf(log_scales[3 * i]), __expf(log_scales[3 * i + 1]), __expf(log_scales[3 * i + 2])};
    const float iz = 1.0f / p[2];
    const float rx = p[0] * iz, ry = p[1] * iz;
    const bool clx = rx < -pp.limx || rx > pp.limx, cly = ry < -pp.limy || ry > pp.limy;
    const float xz = fminf(fmaxf(rx, -pp.limx), pp.limx), yz = fminf(fmaxf(ry, -pp.limy), pp.limy);
    const float J[6] = {pp.fx * iz, 0.f, -pp.fx * xz * iz, 0.f, pp.fy * iz, -pp.fy * yz * iz};
    float T[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) T[3 * a + b] = J[3 * a] * R[b] + J[3 * a + 1] * R[3 + b] + J[3 * a + 2] * R[6 + b];
    // Sigma' = S = sum_b e_b^2 u_b u_b^T + 0.3 I with u_b = T r_b (r_b the
    // columns of Rq), as in the forward.  With C = S^-1 (the conic) and
    // Gamma = dL/dC (symmetric; b enters C twice), dL/dS = -C Gamma C, so
    //   dL/ds_b  = 2 e_b^2 u_b^T (dL/dS) u_b = -2 e_b^2 v_b^T Gamma v_b,  v_b = C u_b
    //   dL/dr_b  = 2 e_b^2 T^T (dL/dS) u_b   = -2 e_b^2 T^T z_b,         z_b = C Gamma v_b
    //   dL/dT    = -2 sum_b e_b^2 z_b r_b^T.
    // C w = adj(S) w / det with adj(S) w = sum_c e_c^2 (u_c x w) u_c_perp + 0.3 w
    // (u_perp = (-u_y, u_x)) and det by Cauchy-Binet: for w = u_b the c = b
    // term vanishes exactly, so v_b of a needle's long axis -- tiny, and
    // formed by cancellation in the expanded adj(S) u_b -- keeps its relative
    // accuracy.
    float u[3][2], e2[3];
    for (int b = 0; b < 3; ++b) {
        e2[b] = e[b] * e[b];
        for (int a = 0; a < 2; ++a) u[b][a] = T[3 * a] * Rq[b] + T[3 * a + 1] * Rq[3 + b] + T[3 * a + 2] * Rq[6 + b];
    }
    float tr = 0.f, det = 0.09f;
    for (int b = 0; b < 3; ++b) {
        tr += e2[b] * (u[b][0] * u[b][0] + u[b][1] * u[b][1]);
        for (int c = b + 1; c < 3; ++c) {
            const float x = u[b][0] * u[c][1] - u[b][1] * u[c][0];
            det += e2[b] * e2[c] * x * x;
        }
    }
    det += 0.3f * tr;
    const float idet = 1.0f / det;
    // C w for a 2-vector w; `skip` names an axis whose term is known to be 0
    auto conic_apply = [&](float w0, float w1, int skip, float& o0, float& o1) {
        o0 = 0.3f * w0;
        o1 = 0.3f * w1;
        for (int c = 0; c < 3; ++c) {
            if (c == skip) continue;
            const float k = e2[c] * (u[c][0] * w1 - u[c][1] * w0);
            o0 -= k * u[c][1];
            o1 += k * u[c][0];
        }
        o0 *= idet;
        o1 *= idet;
    };
    const float4 gco = REC ? *reinterpret_cast<const float4*>(g_conic_opacity + (int64_t)REC * i)
                           : reinterpret_cast<const float4*>(g_conic_opacity)[i];
    const float G00 = gco.x, G01 = 0.5f * gco.y, G11 = gco.z;  // Gamma
    float gR[9], dT[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < 3; ++b) {
        float v0, v1, z0, z1;
        conic_apply(u[b][0], u[b][1], b, v0, v1);
        const float h0 = G00 * v0 + G01 * v1, h1 = G01 * v0 + G11 * v1;  // Gamma v_b
        conic_apply(h0, h1, -1, z0, z1);
        const float k2 = -2.0f * e2[b];
        d_log_scales[3 * i + b] = k2 * (v0 * h0 + v1 * h1);
        for (int k = 0; k < 3; ++k) {
            gR[3 * k + b] = k2 * (T[k] * z0 + T[3 + k] * z1);
            dT[k] += k2 * z0 * Rq[3 * k + b];
            dT[3 + k] += k2 * z1 * Rq[3 * k + b];
        }
    }
    float dJ[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            dJ[3 * a + b] = dT[3 * a] * R[3 * b] + dT[3 * a + 1] * R[3 * b + 1] + dT[3 * a + 2] * R[3 * b + 2];
    // ---- J(p), pinhole map, depth
    const float iz2 = iz * iz;
    float dp[3] = {0.f, 0.f, 0.f};
    dp[2] -= (dJ[0] * pp.fx + dJ[4] * pp.fy) * iz2;
    if (clx) {
        dp[2] += dJ[2] * pp.fx * xz * iz2;
    } else {
        dp[0] -= dJ[2] * pp.fx * iz2;
        dp[2] += dJ[2] * 2.0f * pp.fx * p[0] * iz2 * iz;
    }
    if (cly) {
        dp[2] += dJ[5] * pp.fy * yz * iz2;
    } else {
        dp[1] -= dJ[5] * pp.fy * iz2;
        dp[2] += dJ[5] * 2.0f * pp.fy * p[1] * iz2 * iz;
    }
    const int64_t im = REC ? (int64_t)REC * i : 2 * i;
    const float gu = g_means2D[im], gv = g_means2D[im + 1];
    dp[0] += gu * pp.fx * iz;
    dp[1] += gv * pp.fy * iz;
    dp[2] -= (gu * pp.fx * p[0] + gv * pp.fy * p[1]) * iz2;
    if (g_depth) dp[2] += g_depth[REC ? (int64_t)REC * i : i];
    float dmu[3];
    for (int k = 0; k < 3; ++k) dmu[k] = R[k] * dp[0] + R[3 + k] * dp[1] + R[6 + k] * dp[2];
    // rotation: a world-frame turn by dtheta moves each axis r_b by dtheta x r_b,
    // so the torque is omega = sum_b r_b x dL/dr_b, and the unit quaternion
    // moves by (0, dtheta) (x) q_hat / 2; the gradient in the tangent space of
    // the unit sphere is 2 (0, omega) (x) q_hat, divided by |q| for the
    // normalization.  (Forming the 4-vector gradient of the rotation formula
    // and then removing its radial part cancels when that part dominates.)
    float om[3] = {0.f, 0.f, 0.f};
    for (int b = 0; b < 3; ++b) {
        const float r0 = Rq[b], r1 = Rq[3 + b], r2 = Rq[6 + b];
        const float g0 = gR[b], g1 = gR[3 + b], g2 = gR[6 + b];
        om[0] += r1 * g2 - r2 * g1;
        om[1] += r2 * g0 - r0 * g2;
        om[2] += r0 * g1 - r1 * g0;
    }
    const float k2q = 2.0f * iqn;
    reinterpret_cast<float4*>(d_quats)[i] =
        make_float4(-k2q * (om[0] * x + om[1] * y + om[2] * z), k2q * (w * om[0] + om[1] * z - om[2] * y),
                    k2q * (w * om[1] + om[2] * x - om[0] * z), k2q * (w * om[2] + om[0] * y - om[1] * x));
    d_opacity[i] = gco.w;
    // ---- colour
    const float* gr = g_rgb + (REC ? (int64_t)REC * i : 3 * i);
    if (D < 0) {
        dc[0] = gr[0];
        dc[1] = gr[1];
        dc[2] = gr[2];
    } else {
        float v[3] = {mx - pp.campos[0], my - pp.campos[1], mz - pp.campos[2]};
        const float vn = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), ivn = 1.0f / vn;
        const float d[3] = {v[0] * ivn, v[1] * ivn, v[2] * ivn};
        float Y[16], G[16][3];
        sh_basis(D, d[0], d[1], d[2], Y);
        sh_grad(D, d[0], d[1], d[2], G);
        float c[3];  // the colour before its clamp at 0
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            c[ch] = 0.5f;
#pragma unroll
            for (int j = 0; j < nsh; ++j) c[ch] += coef[3 * j + ch] * Y[j];
        }
        float gd[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const bool live = c[ch] > 0.0f;
#pragma unroll
            for (int j = 0; j < nsh; ++j) {
                const float kv = coef[3 * j + ch];
                dc[3 * j + ch] = live ? gr[ch] * Y[j] : 0.0f;
                if (live)
#pragma unroll
                    for (int a = 0; a < 3; ++a) gd[a] += gr[ch] * kv * G[j][a];
            }
        }
        const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
        for (int a = 0; a < 3; ++a) dmu[a] += (gd[a] - d[a] * dd) * ivn;
    }
    for (int a = 0; a < 3; ++a) d_means3D[3 * i + a] = dmu[a];
}

template <int D, int REC = 0>
__global__ __launch_bounds__(PROJ_THREADS) void k_project_bwd(ProjParams pp, int64_t P, const float* __restrict__ means3D,
                                                              const float* __restrict__ log_scales,
                                                              const float* __restrict__ quats,
                                                              const float* __restrict__ colors,
                                                              const float* __restrict__ g_means2D,
                                                              const float* __restrict__ g_conic_opacity,
                                                              const float* __restrict__ g_rgb,
                                                              const float* __restrict__ g_depth,
                                                              float* __restrict__ d_means3D,
                                                              float* __restrict__ d_log_scales,
                                                              float* __restrict__ d_quats, float* __restrict__ d_opacity,
                                                              float* __restrict__ d_colors) {
    using S = ShDim<D>;
    __shared__ float s_sh[S::LDS_FLOATS];
    const int64_t first = (int64_t)blockIdx.x * PROJ_THREADS;
    const int64_t i = first + threadIdx.x;
    const int n = (int)(P - first < PROJ_THREADS ? P - first : PROJ_THREADS);
    if (S::STAGED) {
        stage_in<S::NC, S::STRIDE>(colors, first, n, s_sh);
        __syncthreads();
    }
    if (i < P) {
        float* row = S::STAGED ? s_sh + threadIdx.x * S::STRIDE : d_colors + (int64_t)S::NC * i;
        const float* coef = S::STAGED ? row : colors + (int64_t)S::NC * i;
        project_bwd_one<D, REC>(pp, i, means3D, log_scales, quats, coef, g_means2D, g_conic_opacity, g_rgb, g_depth,
                                d_means3D, d_log_scales, d_quats, d_opacity, row);
    }
    if (S::STAGED) {
        __syncthreads();
        stage_out<S::NC, S::STRIDE>(d_colors, first, n, s_sh);
    }
}

}  // namespace bgs

using namespace bgs;

static ProjParams proj_params(const bgs_camera* cam) {
    ProjParams pp;
    pp.fx = cam->fx; pp.fy = cam->fy; pp.cx = cam->cx; pp.cy = cam->cy;
    for (int k = 0; k < 9; ++k) pp.R[k] = cam->R[k];
    for (int k = 0; k < 3; ++k) pp.t[k] = cam->t[k];
    // camera centre -R^T t, in double on the host
    for (int c = 0; c < 3; ++c)
        pp.campos[c] = (float)(-((double)cam->R[c] * cam->t[0] + (double)cam->R[3 + c] * cam->t[1] +
                                 (double)cam->R[6 + c] * cam->t[2]));
    pp.znear = cam->znear;
    pp.limx = (float)(1.3 * (0.5 * cam->width) / cam->fx);
    pp.limy = (float)(1.3 * (0.5 * cam->height) / cam->fy);
    pp.TX = (cam->width + TILE - 1) / TILE;
    pp.TY = (cam->height + TILE - 1) / TILE;
    return pp;
}

extern "C" bgs_status bgs_project(const bgs_camera* cam, int64_t P, const float* means3D, const float* log_scales,
                                  const float* quats, const float* opacity, const float* colors, int32_t sh_degree,
                                  int32_t tile, float* means2D, float* conic_opacity, float* rgb, float* depth,
                                  int32_t* radius, uint32_t* tiles_touched, hipStream_t stream) {
    BGS_REQUIRE(cam != nullptr, "bgs_project: camera is null");
    BGS_REQUIRE(P >= 0, "bgs_project: P < 0");
    BGS_REQUIRE(cam->width > 0 && cam->height > 0, "bgs_project: image size must be positive");
    BGS_REQUIRE(sh_degree >= -1 && sh_degree <= 3, "bgs_project: sh_degree must be in -1..3");
    if (tile != TILE) return fail(BGS_EUNSUPPORTED, "bgs_project: only 16x16 tiles are supported");
    if (P == 0) return BGS_OK;
    BGS_REQUIRE(means3D && log_scales && quats && opacity && colors && means2D && conic_opacity && rgb && depth &&
                    radius && tiles_touched,
                "bgs_project: null array");
    BGS_REQUIRE((reinterpret_cast<uintptr_t>(conic_opacity) & 15) == 0, "bgs_project: conic_opacity must be 16-byte aligned");
    const ProjParams pp = proj_params(cam);
    const int threads = PROJ_THREADS;
    const int64_t blocks = (P + threads - 1) / threads;
    BGS_REQUIRE(blocks < (int64_t)1 << 31, "bgs_project: P too large");
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, pp, P, means3D, log_scales, quats,
                           opacity, colors, means2D, conic_opacity, rgb, depth, radius, tiles_touched);
    };
    switch (sh_degree) {
        case -1: launch(k_project<-1>); break;
        case 0: launch(k_project<0>); break;
        case 1: launch(k_project<1>); break;
        case 2: launch(k_project<2>); break;
        default: launch(k_project<3>); break;
    }
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

extern "C" bgs_status bgs_project_bwd(const bgs_camera* cam, int64_t P, const float* means3D, const float* log_scales,
                                      const float* quats, const float* colors, int32_t sh_degree,
                                      const float* dL_dmeans2D, const float* dL_dconic_opacity, const float* dL_drgb,
                                      const float* dL_ddepth, float* dL_dmeans3D, float* dL_dlog_scales,
                                      float* dL_dquats, float* dL_dopacity, float* dL_dcolors, hipStream_t stream) {
    BGS_REQUIRE(cam != nullptr, "bgs_project_bwd: camera is null");
    BGS_REQUIRE(P >= 0, "bgs_project_bwd: P < 0");
    BGS_REQUIRE(cam->width > 0 && cam->height > 0, "bgs_project_bwd: image size must be positive");
    BGS_REQUIRE(sh_degree >= -1 && sh_degree <= 3, "bgs_project_bwd: sh_degree must be in -1..3");
    if (P == 0) return BGS_OK;
    BGS_REQUIRE(means3D && log_scales && quats && colors && dL_dmeans2D && dL_dconic_opacity && dL_drgb &&
                    dL_dmeans3D && dL_dlog_scales && dL_dquats && dL_dopacity && dL_dcolors,
                "bgs_project_bwd: null array");
    BGS_REQUIRE((reinterpret_cast<uintptr_t>(dL_dconic_opacity) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(dL_dquats) & 15) == 0,
                "bgs_project_bwd: dL_dconic_opacity and dL_dquats must be 16-byte aligned");
    const ProjParams pp = proj_params(cam);
    const int threads = PROJ_THREADS;
    const int64_t blocks = (P + threads - 1) / threads;
    BGS_REQUIRE(blocks < (int64_t)1 << 31, "bgs_project_bwd: P too large");
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, pp, P, means3D, log_scales, quats,
                           colors, dL_dmeans2D, dL_dconic_opacity, dL_drgb, dL_ddepth, dL_dmeans3D, dL_dlog_scales,
                           dL_dquats, dL_dopacity, dL_dcolors);
    };
    switch (sh_degree) {
        case -1: launch(k_project_bwd<-1>); break;
        case 0: launch(k_project_bwd<0>); break;
        case 1: launch(k_project_bwd<1>); break;
        case 2: launch(k_project_bwd<2>); break;
        default: launch(k_project_bwd<3>); break;
    }
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}

extern "C" bgs_status bgs_project_bwd_packed(const bgs_camera* cam, int64_t P, const float* means3D,
                                             const float* log_scales, const float* quats, const float* colors,
                                             int32_t sh_degree, const float* dL_drecords, float* dL_dmeans3D,
                                             float* dL_dlog_scales, float* dL_dquats, float* dL_dopacity,
                                             float* dL_dcolors, hipStream_t stream) {
    BGS_REQUIRE(cam != nullptr, "bgs_project_bwd_packed: camera is null");
    BGS_REQUIRE(P >= 0, "bgs_project_bwd_packed: P < 0");
    BGS_REQUIRE(cam->width > 0 && cam->height > 0, "bgs_project_bwd_packed: image size must be positive");
    BGS_REQUIRE(sh_degree >= -1 && sh_degree <= 3, "bgs_project_bwd_packed: sh_degree must be in -1..3");
    if (P == 0) return BGS_OK;
    BGS_REQUIRE(means3D && log_scales && quats && colors && dL_drecords && dL_dmeans3D && dL_dlog_scales &&
                    dL_dquats && dL_dopacity && dL_dcolors,
                "bgs_project_bwd_packed: null array");
    BGS_REQUIRE((reinterpret_cast<uintptr_t>(dL_drecords) & 63) == 0 &&
                    (reinterpret_cast<uintptr_t>(dL_dquats) & 15) == 0,
                "bgs_project_bwd_packed: dL_drecords must be 64-byte and dL_dquats 16-byte aligned");
    const ProjParams pp = proj_params(cam);
    const int threads = PROJ_THREADS;
    const int64_t blocks = (P + threads - 1) / threads;
    BGS_REQUIRE(blocks < (int64_t)1 << 31, "bgs_project_bwd_packed: P too large");
    // record floats 0-3 conic and opacity, 4-5 means2D, 6-8 rgb, 9 depth
    const float* rec = dL_drecords;
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, pp, P, means3D, log_scales, quats,
                           colors, rec + 4, rec, rec + 6, rec + 9, dL_dmeans3D, dL_dlog_scales, dL_dquats,
                           dL_dopacity, dL_dcolors);
    };
    switch (sh_degree) {
        case -1: launch(k_project_bwd<-1, GRAD_RECORD>); break;
        case 0: launch(k_project_bwd<0, GRAD_RECORD>); break;
        case 1: launch(k_project_bwd<1, GRAD_RECORD>); break;
        case 2: launch(k_project_bwd<2, GRAD_RECORD>); break;
        default: launch(k_project_bwd<3, GRAD_RECORD>); break;
    }
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}
