// Projection of 3D Gaussians to screen-space splats, Eq. (1)-(3) of Balanced
// 3DGS (Sec. 2.1): camera transform, 3D covariance from scale and rotation,
// EWA covariance Sigma' = J W Sigma W^T J^T (+0.3 px^2 low-pass), its inverse
// (conic), 3-sigma radius, colour from RGB or real spherical harmonics, and
// the number of 16x16 tiles the splat's square meets.
//
// One thread per Gaussian; fp32 throughout.  O(P) work, a few hundred flops
// per Gaussian: bandwidth-bound on the input arrays (52 B, or 220 B with
// degree-3 SH, per Gaussian).
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

// Real spherical harmonics (no Condon-Shortley phase), index l*l + l + m.
// Amplitudes: C0 = 1/(2 sqrt(pi)), C1 = sqrt(3/(4 pi)), and for l = 2, 3 the
// closed forms written beside each constant.
__device__ inline void sh_colour(const float* __restrict__ k, int degree, float x, float y, float z, float out[3]) {
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
    float Y[16];
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
    const int n = (degree + 1) * (degree + 1);
    for (int c = 0; c < 3; ++c) {
        float s = 0.5f;
        for (int i = 0; i < n; ++i) s += k[3 * i + c] * Y[i];
        out[c] = fmaxf(s, 0.0f);
    }
}

__global__ __launch_bounds__(256) void k_project(ProjParams pp, int64_t P, const float* __restrict__ means3D,
                                                 const float* __restrict__ log_scales, const float* __restrict__ quats,
                                                 const float* __restrict__ opacity, const float* __restrict__ colors,
                                                 int sh_degree, float* __restrict__ means2D,
                                                 float* __restrict__ conic_opacity, float* __restrict__ rgb,
                                                 float* __restrict__ depth, int* __restrict__ radius,
                                                 uint32_t* __restrict__ tiles_touched) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
        const float e0 = __expf(2.f * log_scales[3 * i]), e1 = __expf(2.f * log_scales[3 * i + 1]),
                    e2 = __expf(2.f * log_scales[3 * i + 2]);
        float S[6];  // 00 01 02 11 12 22
        {
            int idx = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b)
                    S[idx++] = Rq[3 * a] * e0 * Rq[3 * b] + Rq[3 * a + 1] * e1 * Rq[3 * b + 1] +
                               Rq[3 * a + 2] * e2 * Rq[3 * b + 2];
        }
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
        // Sigma' = T Sigma T^T
        const float SigT0[3] = {S[0] * T0[0] + S[1] * T0[1] + S[2] * T0[2], S[1] * T0[0] + S[3] * T0[1] + S[4] * T0[2],
                                S[2] * T0[0] + S[4] * T0[1] + S[5] * T0[2]};
        const float SigT1[3] = {S[0] * T1[0] + S[1] * T1[1] + S[2] * T1[2], S[1] * T1[0] + S[3] * T1[1] + S[4] * T1[2],
                                S[2] * T1[0] + S[4] * T1[1] + S[5] * T1[2]};
        s00 = T0[0] * SigT0[0] + T0[1] * SigT0[1] + T0[2] * SigT0[2] + 0.3f;
        s01 = T0[0] * SigT1[0] + T0[1] * SigT1[1] + T0[2] * SigT1[2];
        s11 = T1[0] * SigT1[0] + T1[1] * SigT1[1] + T1[2] * SigT1[2] + 0.3f;
        det = s00 * s11 - s01 * s01;
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

    if (sh_degree < 0) {
        rgb[3 * i] = colors[3 * i];
        rgb[3 * i + 1] = colors[3 * i + 1];
        rgb[3 * i + 2] = colors[3 * i + 2];
    } else {
        float dx = mx - pp.campos[0], dy = my - pp.campos[1], dz = mz - pp.campos[2];
        const float n = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= n; dy *= n; dz *= n;
        const int nsh = (sh_degree + 1) * (sh_degree + 1);
        float c[3];
        sh_colour(colors + (int64_t)3 * nsh * i, sh_degree, dx, dy, dz, c);
        rgb[3 * i] = c[0];
        rgb[3 * i + 1] = c[1];
        rgb[3 * i + 2] = c[2];
    }
}

}  // namespace bgs

using namespace bgs;

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
    const int threads = 256;
    const int64_t blocks = (P + threads - 1) / threads;
    BGS_REQUIRE(blocks < (int64_t)1 << 31, "bgs_project: P too large");
    hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(threads), 0, stream, pp, P, means3D, log_scales, quats,
                       opacity, colors, (int)sh_degree, means2D, conic_opacity, rgb, depth, radius, tiles_touched);
    BGS_HIP(hipGetLastError());
    return BGS_OK;
}
