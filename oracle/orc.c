/*
 * FP64 CPU oracle of the 3DGS tile-rasterizer render path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the HIP
 * library: every constant below is computed here from its closed form.
 *
 * What it computes (Balanced 3DGS, arXiv 2412.17378, Sec. 2.1):
 *   orc_project      Eq. (1)-(3): world->camera transform, 3D covariance from
 *                    scale and rotation, EWA covariance J W Sigma W^T J^T plus
 *                    a 0.3 px^2 low-pass, its inverse (the "conic"), the 3-sigma
 *                    screen radius, and the colour (given RGB, or real spherical
 *                    harmonics of degree <= 3 evaluated along the view ray).
 *   orc_bin          the (tile, Gaussian) pairs: a Gaussian is listed in every
 *                    16x16 tile that its screen square [u-r, u+r] x [v-r, v+r]
 *                    meets.
 *   orc_bin_exact    the same pairs, keeping a tile only when its pixel-centre
 *                    rectangle meets the ellipse inside which the Gaussian's
 *                    alpha can reach 1/255 (exact ellipse-tile binning, the
 *                    list-shrinking refinement of the tile rule that the paper
 *                    lists among related work); all other pairs are skipped by
 *                    Eq. (4)'s rules at every pixel of their tile.
 *   orc_sort         order the pairs by (tile, view depth); equal depths keep
 *                    the input order (Eq. (4) blends "N-sorted" Gaussians).
 *   orc_ranges       per-tile [start, end) into the sorted list.
 *   orc_render_fwd   Eq. (4) evaluated per pixel front to back, with the skip
 *                    and stop rules of the paper's naive per-pixel loop
 *                    (Appendix, detailed naive render): skip when the exponent
 *                    is positive or alpha < 1/255, stop (without blending) once
 *                    the transmittance would drop below 1e-4; alpha is clamped
 *                    to 0.99.
 *   orc_render_bwd   the exact derivative of orc_render_fwd with every skip /
 *                    stop decision held fixed, summed over pixels.
 *   orc_project_bwd  the derivative of orc_project (3D means, log-scales,
 *                    quaternions, opacity, colour coefficients).
 *
 * All arithmetic is double precision.  The three thresholds are the FP32
 * constants (1/255, 1e-4, 0.99 as floats) promoted to double.
 *
 * Pinned by tests: closed forms (on-axis isotropic projection, single
 * Gaussian, identical-alpha stack), finite-difference Jacobian of the pinhole
 * map, orthonormality of the SH basis, brute-force tile membership and
 * per-pixel blending, permutation invariance, central finite differences of
 * the forward for the backward.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9]; /* row-major world -> camera rotation */
    double t[3];
    double znear;
} orc_camera;

static const double ORC_PI = 3.14159265358979323846;

/* thresholds: the FP32 literals of the paper's per-pixel loop, widened */
static double thr_alpha_min(void) { return (double)(1.0f / 255.0f); }
static double thr_T_min(void) { return (double)(1e-4f); }
static double thr_alpha_max(void) { return (double)(0.99f); }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- project */

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* m-th derivative of the Legendre polynomial P_l at z, l <= 3 */
static double legendre_deriv(int l, int m, double z)
{
    /* P0 = 1, P1 = z, P2 = (3z^2-1)/2, P3 = (5z^3-3z)/2 */
    switch (l * 4 + m) {
    case 0: return 1.0;
    case 4: return z;
    case 5: return 1.0;
    case 8: return 0.5 * (3.0 * z * z - 1.0);
    case 9: return 3.0 * z;
    case 10: return 3.0;
    case 12: return 0.5 * (5.0 * z * z * z - 3.0 * z);
    case 13: return 0.5 * (15.0 * z * z - 3.0);
    case 14: return 15.0 * z;
    case 15: return 15.0;
    default: return 0.0;
    }
}

/*
 * Real spherical harmonic Y_lm at the unit vector (x, y, z), textbook
 * definition without the Condon-Shortley phase:
 *   Y_l0  = K_l0 P_l(z)
 *   Y_lm  = sqrt(2) K_lm Re[(x+iy)^m] P_l^(m)(z)      m > 0
 *   Y_l-m = sqrt(2) K_lm Im[(x+iy)^m] P_l^(m)(z)      m > 0
 * with K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^(m) the m-th
 * derivative of P_l (so sin^m(theta) P_l^(m)(cos theta) is the associated
 * Legendre function).  Index order: l*l + l + m.
 */
double orc_sh_basis(int l, int m, double x, double y, double z)
{
    int am = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * factorial(l - am) / factorial(l + am));
    double re = 1.0, im = 0.0; /* (x + iy)^am */
    for (int k = 0; k < am; ++k) {
        double r2 = re * x - im * y;
        double i2 = re * y + im * x;
        re = r2;
        im = i2;
    }
    double d = legendre_deriv(l, am, z);
    if (m == 0) return K * d;
    if (m > 0) return sqrt(2.0) * K * re * d;
    return sqrt(2.0) * K * im * d;
}

static void quat_to_rot(const float *q, double Rq[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
    Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
    Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
}

/* C = A B for 3x3 row-major */
static void mat3_mul(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}

/*
 * Per Gaussian:
 *   p = R mu + t; culled (radius 0) when p.z <= znear.
 *   Sigma  = Rq diag(exp(2 s)) Rq^T.
 *   J      = [[fx/z, 0, -fx x'/z^2], [0, fy/z, -fy y'/z^2]], with x'/z, y'/z
 *            clamped to +-1.3 (W/2)/fx and +-1.3 (H/2)/fy.
 *   Sigma' = J R Sigma R^T J^T + 0.3 I; culled when det(Sigma') <= 0.
 *   conic  = Sigma'^-1 = (Sigma'11, -Sigma'01, Sigma'00) / det.
 *   extent = 3 sqrt(lambda_max(Sigma')), radius = ceil(extent).
 *   (u, v) = (fx x/z + cx - 1/2, fy y/z + cy - 1/2); depth = z.
 *   colour = given RGB, or max(0, sum_lm k_lm Y_lm(d) + 1/2) with d the unit
 *            ray from the camera centre -R^T t to mu.
 * Outputs for culled Gaussians are zero (radius 0).
 * cov2d (nullable) receives (Sigma'00, Sigma'01, Sigma'11) including the 0.3.
 */
int orc_project(const orc_camera *cam, int64_t P, const float *means3D, const float *log_scales,
                const float *quats, const float *opacity, const float *colors, int32_t sh_degree,
                double *means2D, double *conic_opacity, double *rgb, double *depth, int32_t *radius,
                double *extent, double *cov2d)
{
    if (sh_degree > 3) return -1;
    const double *R = cam->R;
    double campos[3];
    for (int i = 0; i < 3; ++i)
        campos[i] = -(R[0 * 3 + i] * cam->t[0] + R[1 * 3 + i] * cam->t[1] + R[2 * 3 + i] * cam->t[2]);
    const double limx = 1.3 * (0.5 * cam->width) / cam->fx;
    const double limy = 1.3 * (0.5 * cam->height) / cam->fy;
    const int nsh = sh_degree < 0 ? 1 : (sh_degree + 1) * (sh_degree + 1);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i) {
        const float *mu = means3D + 3 * i;
        means2D[2 * i] = means2D[2 * i + 1] = 0;
        for (int k = 0; k < 4; ++k) conic_opacity[4 * i + k] = 0;
        for (int k = 0; k < 3; ++k) rgb[3 * i + k] = 0;
        depth[i] = 0;
        radius[i] = 0;
        if (extent) extent[i] = 0;
        if (cov2d) cov2d[3 * i] = cov2d[3 * i + 1] = cov2d[3 * i + 2] = 0;

        double p[3];
        for (int r = 0; r < 3; ++r)
            p[r] = R[r * 3 + 0] * mu[0] + R[r * 3 + 1] * mu[1] + R[r * 3 + 2] * mu[2] + cam->t[r];
        if (p[2] <= cam->znear) continue;

        double Rq[9], S[9] = {0}, M[9], Sig[9], RqT[9];
        quat_to_rot(quats + 4 * i, Rq);
        for (int k = 0; k < 3; ++k) S[k * 4] = exp(2.0 * (double)log_scales[3 * i + k]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) RqT[a * 3 + b] = Rq[b * 3 + a];
        mat3_mul(Rq, S, M);
        mat3_mul(M, RqT, Sig);

        double z = p[2];
        double xz = p[0] / z, yz = p[1] / z;
        if (xz < -limx) xz = -limx;
        if (xz > limx) xz = limx;
        if (yz < -limy) yz = -limy;
        if (yz > limy) yz = limy;
        /* J as a 3x3 with a zero last row, so that everything stays 3x3 */
        double J[9] = {cam->fx / z, 0, -cam->fx * xz / z, 0, cam->fy / z, -cam->fy * yz / z, 0, 0, 0};
        double T[9], TS[9], TT[9], C2[9];
        mat3_mul(J, R, T);
        mat3_mul(T, Sig, TS);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) TT[a * 3 + b] = T[b * 3 + a];
        mat3_mul(TS, TT, C2);
        double s00 = C2[0] + 0.3, s01 = C2[1], s11 = C2[4] + 0.3;
        double det = s00 * s11 - s01 * s01;
        if (!(det > 0)) continue;

        double mid = 0.5 * (s00 + s11);
        double disc = mid * mid - det;
        if (disc < 0) disc = 0;
        double lmax = mid + sqrt(disc);
        double ext = 3.0 * sqrt(lmax);
        int32_t r = (int32_t)ceil(ext);
        if (r <= 0) continue;

        means2D[2 * i] = cam->fx * p[0] / z + cam->cx - 0.5;
        means2D[2 * i + 1] = cam->fy * p[1] / z + cam->cy - 0.5;
        conic_opacity[4 * i + 0] = s11 / det;
        conic_opacity[4 * i + 1] = -s01 / det;
        conic_opacity[4 * i + 2] = s00 / det;
        conic_opacity[4 * i + 3] = opacity[i];
        depth[i] = z;
        radius[i] = r;
        if (extent) extent[i] = ext;
        if (cov2d) { cov2d[3 * i] = s00; cov2d[3 * i + 1] = s01; cov2d[3 * i + 2] = s11; }

        const float *col = colors + (int64_t)3 * nsh * i;
        if (sh_degree < 0) {
            for (int c = 0; c < 3; ++c) rgb[3 * i + c] = col[c];
        } else {
            double d[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
            double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int k = 0; k < 3; ++k) d[k] /= n;
            for (int c = 0; c < 3; ++c) {
                double s = 0.5;
                for (int l = 0; l <= sh_degree; ++l)
                    for (int m = -l; m <= l; ++m)
                        s += (double)col[3 * (l * l + l + m) + c] * orc_sh_basis(l, m, d[0], d[1], d[2]);
                rgb[3 * i + c] = s > 0 ? s : 0;
            }
        }
    }
    return 0;
}

/*
 * Gradient of a real spherical harmonic (as orc_sh_basis defines it, a
 * polynomial in x, y, z) at (x, y, z):  with A = (x + iy)^m, dA/dx =
 * m (x + iy)^(m-1), dA/dy = i m (x + iy)^(m-1), and d/dz P_l^(m) = P_l^(m+1).
 */
static void sh_basis_grad(int l, int m, double x, double y, double z, double g[3])
{
    int am = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * factorial(l - am) / factorial(l + am));
    double re = 1.0, im = 0.0, re1 = 0.0, im1 = 0.0; /* (x+iy)^am and (x+iy)^(am-1) */
    for (int k = 0; k < am; ++k) {
        re1 = re;
        im1 = im;
        double r2 = re * x - im * y;
        double i2 = re * y + im * x;
        re = r2;
        im = i2;
    }
    double d = legendre_deriv(l, am, z), dz = legendre_deriv(l, am + 1, z);
    if (m == 0) {
        g[0] = 0.0;
        g[1] = 0.0;
        g[2] = K * dz;
        return;
    }
    const double c = sqrt(2.0) * K;
    /* dA/dx = am (re1 + i im1), dA/dy = i am (re1 + i im1) = am (-im1 + i re1) */
    if (m > 0) {
        g[0] = c * am * re1 * d;
        g[1] = c * am * (-im1) * d;
        g[2] = c * re * dz;
    } else {
        g[0] = c * am * im1 * d;
        g[1] = c * am * re1 * d;
        g[2] = c * im * dz;
    }
}

/*
 * Derivative of orc_project for a loss L of its outputs: given dL/dmeans2D
 * [P][2], dL/dconic_opacity [P][4] (a, b, c, opacity), dL/drgb [P][3] and
 * dL/ddepth [P] (nullable), writes (=) dL/dmeans3D [P][3], dL/dlog_scales
 * [P][3], dL/dquats [P][4] (w, x, y, z, through the normalization),
 * dL/dopacity [P] and dL/dcolors [P][K][3] (K SH coefficients, or the RGB).
 * Culled Gaussians get zeros.  Every step is the derivative of the forward's
 * step, taken in reverse order:
 *   conic (a, b, c) = (s11, -s01, s00) / det,  det = s00 s11 - s01^2;
 *   Sigma'_2x2 = T Sigma T^T (+0.3 I),  T = J R;  Sigma = M M^T, M = Rq S;
 *   J depends on p through z and the clamped x/z, y/z (derivative 0 where
 *   clamped);  (u, v) = (fx x / z, fy y / z) + const;  depth = z;
 *   p = R mu + t;  colour = max(0, 1/2 + sum_lm k_lm Y_lm(d)), d the unit ray
 *   (derivative 0 where clamped at 0).
 */
int orc_project_bwd(const orc_camera *cam, int64_t P, const float *means3D, const float *log_scales,
                    const float *quats, const float *opacity, const float *colors, int32_t sh_degree,
                    const double *g_means2D, const double *g_conic_opacity, const double *g_rgb,
                    const double *g_depth, double *d_means3D, double *d_log_scales, double *d_quats,
                    double *d_opacity, double *d_colors)
{
    (void)opacity;
    if (sh_degree > 3) return -1;
    const double *R = cam->R;
    double campos[3];
    for (int i = 0; i < 3; ++i)
        campos[i] = -(R[0 * 3 + i] * cam->t[0] + R[1 * 3 + i] * cam->t[1] + R[2 * 3 + i] * cam->t[2]);
    const double limx = 1.3 * (0.5 * cam->width) / cam->fx;
    const double limy = 1.3 * (0.5 * cam->height) / cam->fy;
    const int nsh = sh_degree < 0 ? 1 : (sh_degree + 1) * (sh_degree + 1);
    const double fx = cam->fx, fy = cam->fy;

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i) {
        const float *mu = means3D + 3 * i;
        double *dmu = d_means3D + 3 * i, *ds = d_log_scales + 3 * i, *dq = d_quats + 4 * i;
        double *dc = d_colors + (int64_t)3 * nsh * i;
        for (int k = 0; k < 3; ++k) dmu[k] = ds[k] = 0;
        for (int k = 0; k < 4; ++k) dq[k] = 0;
        for (int k = 0; k < 3 * nsh; ++k) dc[k] = 0;
        d_opacity[i] = 0;

        /* ---- recompute the forward */
        double p[3];
        for (int r = 0; r < 3; ++r)
            p[r] = R[r * 3 + 0] * mu[0] + R[r * 3 + 1] * mu[1] + R[r * 3 + 2] * mu[2] + cam->t[r];
        if (p[2] <= cam->znear) continue;
        const float *qf = quats + 4 * i;
        double qn = sqrt((double)qf[0] * qf[0] + (double)qf[1] * qf[1] + (double)qf[2] * qf[2] + (double)qf[3] * qf[3]);
        double qh[4] = {qf[0] / qn, qf[1] / qn, qf[2] / qn, qf[3] / qn};
        double Rq[9], Sd[3], M[9], Sig[9];
        quat_to_rot(qf, Rq);
        for (int k = 0; k < 3; ++k) Sd[k] = exp((double)log_scales[3 * i + k]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a * 3 + b] = Rq[a * 3 + b] * Sd[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += M[a * 3 + k] * M[b * 3 + k];
                Sig[a * 3 + b] = acc;
            }
        const double z = p[2];
        double xz = p[0] / z, yz = p[1] / z;
        const int cx_ = xz < -limx || xz > limx, cy_ = yz < -limy || yz > limy;
        if (xz < -limx) xz = -limx;
        if (xz > limx) xz = limx;
        if (yz < -limy) yz = -limy;
        if (yz > limy) yz = limy;
        double J[6] = {fx / z, 0, -fx * xz / z, 0, fy / z, -fy * yz / z}; /* 2x3 */
        double T[6];                                                      /* J R */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) T[a * 3 + b] = J[a * 3 + 0] * R[0 * 3 + b] + J[a * 3 + 1] * R[1 * 3 + b] + J[a * 3 + 2] * R[2 * 3 + b];
        double TS[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) TS[a * 3 + b] = T[a * 3 + 0] * Sig[0 * 3 + b] + T[a * 3 + 1] * Sig[1 * 3 + b] + T[a * 3 + 2] * Sig[2 * 3 + b];
        double C2[4];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) C2[a * 2 + b] = TS[a * 3 + 0] * T[b * 3 + 0] + TS[a * 3 + 1] * T[b * 3 + 1] + TS[a * 3 + 2] * T[b * 3 + 2];
        const double s00 = C2[0] + 0.3, s01 = C2[1], s11 = C2[3] + 0.3;
        const double det = s00 * s11 - s01 * s01;
        if (!(det > 0)) continue;
        double mid = 0.5 * (s00 + s11), disc = mid * mid - det;
        if (disc < 0) disc = 0;
        if ((int32_t)ceil(3.0 * sqrt(mid + sqrt(disc))) <= 0) continue;

        /* ---- conic -> Sigma'  */
        const double ga = g_conic_opacity[4 * i + 0], gb = g_conic_opacity[4 * i + 1], gc = g_conic_opacity[4 * i + 2];
        d_opacity[i] = g_conic_opacity[4 * i + 3];
        const double Kd = -(ga * s11 - gb * s01 + gc * s00) / (det * det);
        const double g00 = gc / det + Kd * s11;
        const double g11 = ga / det + Kd * s00;
        const double g01 = -gb / det + Kd * (-2.0 * s01);
        const double Gm[4] = {g00, 0.5 * g01, 0.5 * g01, g11}; /* symmetric dL/dC2 */

        /* ---- C2 = T Sig T^T:  dL/dSig = T^T Gm T,  dL/dT = 2 Gm T Sig */
        double GT[6]; /* Gm T (2x3) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) GT[a * 3 + b] = Gm[a * 2 + 0] * T[0 * 3 + b] + Gm[a * 2 + 1] * T[1 * 3 + b];
        double dSig[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) dSig[a * 3 + b] = T[0 * 3 + a] * GT[0 * 3 + b] + T[1 * 3 + a] * GT[1 * 3 + b];
        double dT[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b)
                dT[a * 3 + b] = 2.0 * (GT[a * 3 + 0] * Sig[0 * 3 + b] + GT[a * 3 + 1] * Sig[1 * 3 + b] + GT[a * 3 + 2] * Sig[2 * 3 + b]);
        /* T = J R:  dL/dJ = dL/dT R^T */
        double dJ[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b)
                dJ[a * 3 + b] = dT[a * 3 + 0] * R[b * 3 + 0] + dT[a * 3 + 1] * R[b * 3 + 1] + dT[a * 3 + 2] * R[b * 3 + 2];

        /* ---- J(p) and the screen position, depth */
        double dp[3] = {0, 0, 0};
        const double z2 = z * z;
        dp[2] += dJ[0] * (-fx / z2) + dJ[4] * (-fy / z2);
        if (cx_) {
            dp[2] += dJ[2] * (fx * xz / z2);
        } else {
            dp[0] += dJ[2] * (-fx / z2);
            dp[2] += dJ[2] * (2.0 * fx * p[0] / (z2 * z));
        }
        if (cy_) {
            dp[2] += dJ[5] * (fy * yz / z2);
        } else {
            dp[1] += dJ[5] * (-fy / z2);
            dp[2] += dJ[5] * (2.0 * fy * p[1] / (z2 * z));
        }
        const double gu = g_means2D[2 * i], gv = g_means2D[2 * i + 1];
        dp[0] += gu * fx / z;
        dp[1] += gv * fy / z;
        dp[2] += -gu * fx * p[0] / z2 - gv * fy * p[1] / z2;
        if (g_depth) dp[2] += g_depth[i];
        /* p = R mu + t */
        for (int k = 0; k < 3; ++k) dmu[k] = R[0 * 3 + k] * dp[0] + R[1 * 3 + k] * dp[1] + R[2 * 3 + k] * dp[2];

        /* ---- Sigma = M M^T, M = Rq diag(e^s):  dL/dM = 2 dSig M */
        double dM[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                dM[a * 3 + b] = 2.0 * (dSig[a * 3 + 0] * M[0 * 3 + b] + dSig[a * 3 + 1] * M[1 * 3 + b] + dSig[a * 3 + 2] * M[2 * 3 + b]);
        double gR[9];
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int a = 0; a < 3; ++a) {
                acc += dM[a * 3 + b] * Rq[a * 3 + b];
                gR[a * 3 + b] = dM[a * 3 + b] * Sd[b];
            }
            ds[b] = acc * Sd[b]; /* d e^s / ds = e^s */
        }
        /* rotation of the unit quaternion (w, x, y, z) */
        const double w = qh[0], x = qh[1], y = qh[2], zq = qh[3];
        double gq[4];
        gq[0] = 2.0 * (-zq * gR[1] + y * gR[2] + zq * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
        gq[1] = 2.0 * (y * gR[1] + zq * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + zq * gR[6] + w * gR[7] -
                       2.0 * x * gR[8]);
        gq[2] = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + zq * gR[5] - w * gR[6] + zq * gR[7] -
                       2.0 * y * gR[8]);
        gq[3] = 2.0 * (-2.0 * zq * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * zq * gR[4] + y * gR[5] +
                       x * gR[6] + y * gR[7]);
        /* q_hat = q / |q|:  dL/dq = (g - q_hat (q_hat . g)) / |q| */
        const double dot = qh[0] * gq[0] + qh[1] * gq[1] + qh[2] * gq[2] + qh[3] * gq[3];
        for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - qh[k] * dot) / qn;

        /* ---- colour */
        const float *col = colors + (int64_t)3 * nsh * i;
        const double *gr = g_rgb + 3 * i;
        if (sh_degree < 0) {
            for (int c = 0; c < 3; ++c) dc[c] = gr[c];
        } else {
            double dv[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
            const double n = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            for (int k = 0; k < 3; ++k) dv[k] /= n;
            double gd[3] = {0, 0, 0}; /* dL/d(unit ray) */
            for (int c = 0; c < 3; ++c) {
                double s = 0.5;
                for (int l = 0; l <= sh_degree; ++l)
                    for (int m = -l; m <= l; ++m)
                        s += (double)col[3 * (l * l + l + m) + c] * orc_sh_basis(l, m, dv[0], dv[1], dv[2]);
                if (!(s > 0)) continue; /* clamped at 0 */
                for (int l = 0; l <= sh_degree; ++l)
                    for (int m = -l; m <= l; ++m) {
                        const int idx = l * l + l + m;
                        dc[3 * idx + c] = gr[c] * orc_sh_basis(l, m, dv[0], dv[1], dv[2]);
                        double gy[3];
                        sh_basis_grad(l, m, dv[0], dv[1], dv[2], gy);
                        for (int k = 0; k < 3; ++k) gd[k] += gr[c] * (double)col[3 * idx + c] * gy[k];
                    }
            }
            /* d = v / |v|:  dL/dv = (gd - d (d . gd)) / |v| */
            const double dd = dv[0] * gd[0] + dv[1] * gd[1] + dv[2] * gd[2];
            for (int k = 0; k < 3; ++k) dmu[k] += (gd[k] - dv[k] * dd) / n;
        }
    }
    return 0;
}

/* ------------------------------------------------------- bin / sort / ranges */

static int tiles_x(int32_t width, int32_t tile) { return (width + tile - 1) / tile; }
static int tiles_y(int32_t height, int32_t tile) { return (height + tile - 1) / tile; }

/*
 * Tile rectangle of one Gaussian, inclusive: the tiles whose pixel range
 * [k*tile, (k+1)*tile) meets [u - r, u + r], clipped to the grid.  Returns 0
 * when there is none (culled or off-screen).
 */
static int tile_rect(double u, double v, int32_t r, int TX, int TY, int32_t tile, int rect[4])
{
    if (r <= 0) return 0;
    int x0 = (int)floor((u - r) / tile), x1 = (int)floor((u + r) / tile);
    int y0 = (int)floor((v - r) / tile), y1 = (int)floor((v + r) / tile);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > TX - 1) x1 = TX - 1;
    if (y1 > TY - 1) y1 = TY - 1;
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = x0; rect[1] = y0; rect[2] = x1; rect[3] = y1;
    return 1;
}

/*
 * Emit every (tile, Gaussian) pair, Gaussians in input order, tiles row-major
 * within a Gaussian.  window (nullable) = tile rectangle [tx0, ty0, tx1, ty1)
 * to which pairs are restricted.  With tile_ids == NULL only counts.  Returns
 * the number of pairs.
 */
int64_t orc_bin(int32_t width, int32_t height, int32_t tile, int64_t P, const double *means2D,
                const int32_t *radius, const int32_t *window, int32_t *tile_ids, int32_t *gauss_ids)
{
    int TX = tiles_x(width, tile), TY = tiles_y(height, tile);
    int64_t m = 0;
    for (int64_t i = 0; i < P; ++i) {
        int rc[4];
        if (!tile_rect(means2D[2 * i], means2D[2 * i + 1], radius[i], TX, TY, tile, rc)) continue;
        for (int ty = rc[1]; ty <= rc[3]; ++ty)
            for (int tx = rc[0]; tx <= rc[2]; ++tx) {
                if (window && (tx < window[0] || ty < window[1] || tx >= window[2] || ty >= window[3]))
                    continue;
                if (tile_ids) {
                    tile_ids[m] = ty * TX + tx;
                    gauss_ids[m] = (int32_t)i;
                }
                ++m;
            }
    }
    return m;
}

/*
 * Minimum of q(x, y) = a x^2 + 2 b x y + c y^2 (a > 0, a c - b^2 > 0) over the
 * rectangle [lx, hx] x [ly, hy].  q is convex with its minimum 0 at the
 * origin, so the value is 0 when the rectangle holds the origin and
 * otherwise the least of the four edge minima; along an edge q is a convex
 * quadratic in one variable, minimised at its stationary point clamped to the
 * edge.
 */
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

double orc_rect_min_q(double a, double b, double c, double lx, double hx, double ly, double hy)
{
    if (lx <= 0.0 && hx >= 0.0 && ly <= 0.0 && hy >= 0.0) return 0.0;
    double best = INFINITY;
    const double xs[2] = {lx, hx}, ys[2] = {ly, hy};
    for (int k = 0; k < 2; ++k) {
        const double x = xs[k], y = clampd(-b * x / c, ly, hy);      /* edge x = const */
        const double qx = a * x * x + 2.0 * b * x * y + c * y * y;
        const double y2 = ys[k], x2 = clampd(-b * y2 / a, lx, hx);  /* edge y = const */
        const double qy = a * x2 * x2 + 2.0 * b * x2 * y2 + c * y2 * y2;
        if (qx < best) best = qx;
        if (qy < best) best = qy;
    }
    return best;
}

/*
 * The exact binning rule.  A pixel at offset d from the mean is blended only
 * when o exp(-q(d)/2) >= 1/255 (alpha below 1/255 is skipped), i.e. when
 * q(d) <= 2 ln(255 o).  The rule keeps a tile when q <= that bound plus
 * 2^-10 (relative and absolute) somewhere on the tile's rectangle of pixel
 * centres widened by 2^-6 px on every side; the widenings only add tiles.
 */
static const double BIN_Q_SLACK = 1.0 / 1024.0;
static const double BIN_PX_SLACK = 1.0 / 64.0;

double orc_bin_q_limit(double opacity)
{
    if (!(opacity > 0.0)) return -1.0;
    const double tau = 2.0 * log(opacity / thr_alpha_min());
    return tau * (1.0 + BIN_Q_SLACK) + BIN_Q_SLACK;
}

static int exact_keep(double u, double v, const double *co, int tx, int ty, int32_t tile)
{
    const double a = co[0], b = co[1], c = co[2];
    const double lim = orc_bin_q_limit(co[3]);
    if (lim < 0.0) return 0;
    if (!(a > 0.0 && c > 0.0 && a * c - b * b > 0.0)) return 1; /* not an ellipse: keep the square rule */
    const double lx = (double)tx * tile - BIN_PX_SLACK - u, hx = (double)tx * tile + (tile - 1) + BIN_PX_SLACK - u;
    const double ly = (double)ty * tile - BIN_PX_SLACK - v, hy = (double)ty * tile + (tile - 1) + BIN_PX_SLACK - v;
    return orc_rect_min_q(a, b, c, lx, hx, ly, hy) <= lim;
}

/* orc_bin restricted by the exact rule; conic_opacity [P][4] = (a, b, c, o). */
int64_t orc_bin_exact(int32_t width, int32_t height, int32_t tile, int64_t P, const double *means2D,
                      const int32_t *radius, const double *conic_opacity, const int32_t *window,
                      int32_t *tile_ids, int32_t *gauss_ids)
{
    int TX = tiles_x(width, tile), TY = tiles_y(height, tile);
    int64_t m = 0;
    for (int64_t i = 0; i < P; ++i) {
        int rc[4];
        const double u = means2D[2 * i], v = means2D[2 * i + 1];
        if (!tile_rect(u, v, radius[i], TX, TY, tile, rc)) continue;
        for (int ty = rc[1]; ty <= rc[3]; ++ty)
            for (int tx = rc[0]; tx <= rc[2]; ++tx) {
                if (window && (tx < window[0] || ty < window[1] || tx >= window[2] || ty >= window[3]))
                    continue;
                if (!exact_keep(u, v, conic_opacity + 4 * i, tx, ty, tile)) continue;
                if (tile_ids) {
                    tile_ids[m] = ty * TX + tx;
                    gauss_ids[m] = (int32_t)i;
                }
                ++m;
            }
    }
    return m;
}

typedef struct {
    int32_t tile;
    int32_t gid;
    double depth;
} orc_pair;

static int pair_cmp(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
    if (x->gid != y->gid) return x->gid < y->gid ? -1 : 1;
    return 0;
}

/*
 * Sort the pairs by (tile, depth of the Gaussian), ties in Gaussian-id order
 * (= input order, i.e. a stable sort by the (tile, depth) key).  In place.
 */
int orc_sort(int64_t M, int32_t *tile_ids, int32_t *gauss_ids, const double *depth)
{
    orc_pair *v = (orc_pair *)malloc(sizeof(orc_pair) * (M > 0 ? M : 1));
    if (!v) return -1;
    for (int64_t k = 0; k < M; ++k) {
        v[k].tile = tile_ids[k];
        v[k].gid = gauss_ids[k];
        v[k].depth = depth[gauss_ids[k]];
    }
    qsort(v, (size_t)M, sizeof(orc_pair), pair_cmp);
    for (int64_t k = 0; k < M; ++k) {
        tile_ids[k] = v[k].tile;
        gauss_ids[k] = v[k].gid;
    }
    free(v);
    return 0;
}

/* ranges[2*t] = first index of tile t, ranges[2*t+1] = one past the last (0,0 if empty) */
int orc_ranges(int64_t M, const int32_t *sorted_tile_ids, int32_t n_tiles, int32_t *ranges)
{
    for (int32_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
    for (int64_t k = 0; k < M; ++k) {
        int32_t t = sorted_tile_ids[k];
        if (t < 0 || t >= n_tiles) return -1;
        if (k == 0 || sorted_tile_ids[k - 1] != t) ranges[2 * t] = (int32_t)k;
        ranges[2 * t + 1] = (int32_t)k + 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ render */

typedef struct {
    int32_t width, height, tile;
    const int32_t *ranges, *point_list;
    const double *means2D, *conic_opacity, *rgb, *depth, *bg;
} orc_frame;

/*
 * One pixel, Eq. (4) in list order:
 *   d = (px - u, py - v); power = -1/2 (a dx^2 + c dy^2) - b dx dy
 *   skip when power > 0;  alpha = min(0.99, o e^power);  skip when alpha < 1/255
 *   T' = T (1 - alpha);   stop (this entry not blended) when T' < 1e-4
 *   C += rgb alpha T;  D += depth alpha T;  A += alpha T;  T = T';  n = k + 1
 * Returns the number of list entries examined (skipped and stopping entries
 * included); *blended receives the number of entries blended (the pixel's
 * contributors, at most *n_out); *margin receives the smallest relative
 * distance of any skip / clamp / stop decision to its threshold.
 */
static int64_t pixel_forward(const orc_frame *f, int px, int py, double C[3], double *D, double *A,
                             double *T_out, int32_t *n_out, int32_t *blended, double *margin)
{
    const int TX = tiles_x(f->width, f->tile);
    const int t = (py / f->tile) * TX + (px / f->tile);
    const int32_t s = f->ranges[2 * t], e = f->ranges[2 * t + 1];
    const double amin = thr_alpha_min(), amax = thr_alpha_max(), tmin = thr_T_min();
    double T = 1.0, mg = INFINITY;
    int32_t n = 0, nb = 0;
    int64_t examined = 0;
    C[0] = C[1] = C[2] = 0;
    *D = 0;
    *A = 0;
    for (int32_t k = s; k < e; ++k) {
        const int32_t g = f->point_list[k];
        ++examined;
        const double dx = px - f->means2D[2 * g], dy = py - f->means2D[2 * g + 1];
        const double *co = f->conic_opacity + 4 * g;
        const double power = -0.5 * (co[0] * dx * dx + co[2] * dy * dy) - co[1] * dx * dy;
        if (power > 0) continue;
        const double ga = co[3] * exp(power);
        const double alpha = ga < amax ? ga : amax;
        double m1 = fabs(ga - amin) / amin, m2 = fabs(ga - amax) / amax;
        if (m1 < mg) mg = m1;
        if (m2 < mg) mg = m2;
        if (alpha < amin) continue;
        const double Tn = T * (1.0 - alpha);
        double m3 = fabs(Tn - tmin) / tmin;
        if (m3 < mg) mg = m3;
        if (Tn < tmin) break;
        const double w = alpha * T;
        for (int c = 0; c < 3; ++c) C[c] += f->rgb[3 * g + c] * w;
        *D += f->depth[g] * w;
        *A += w;
        T = Tn;
        n = k - s + 1;
        ++nb;
    }
    *T_out = T;
    *n_out = n;
    *blended = nb;
    if (margin) *margin = mg;
    return examined;
}

static void window_or_full(const int32_t *window, int32_t w, int32_t h, int32_t out[4])
{
    if (window) {
        out[0] = window[0] < 0 ? 0 : window[0];
        out[1] = window[1] < 0 ? 0 : window[1];
        out[2] = window[2] > w ? w : window[2];
        out[3] = window[3] > h ? h : window[3];
    } else {
        out[0] = 0; out[1] = 0; out[2] = w; out[3] = h;
    }
}

/*
 * Forward render of the pixels in window = [x0, y0, x1, y1) (nullable: whole
 * image).  Image outputs are planar [3,H,W] / [H,W]; pixels outside the
 * window are left untouched.  out_color = C + T bg.  n_examined, n_blended
 * (entries blended per pixel) and margin are nullable.  Returns the total
 * number of examined entries (the forward "blend" count).
 */
int64_t orc_render_fwd(int32_t width, int32_t height, int32_t tile, const int32_t *ranges,
                       const int32_t *point_list, const double *means2D, const double *conic_opacity,
                       const double *rgb, const double *depth, const double *bg, const int32_t *window,
                       double *out_color, double *out_alpha, double *out_depth, double *final_T,
                       int32_t *n_contrib, int64_t *n_examined, int32_t *n_blended, double *margin)
{
    orc_frame f = {width, height, tile, ranges, point_list, means2D, conic_opacity, rgb, depth, bg};
    int32_t win[4];
    window_or_full(window, width, height, win);
    const int64_t HW = (int64_t)width * height;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int py = win[1]; py < win[3]; ++py) {
        for (int px = win[0]; px < win[2]; ++px) {
            double C[3], D, A, T, mg;
            int32_t n, nb;
            int64_t ex = pixel_forward(&f, px, py, C, &D, &A, &T, &n, &nb, &mg);
            const int64_t o = (int64_t)py * width + px;
            for (int c = 0; c < 3; ++c) out_color[c * HW + o] = C[c] + T * bg[c];
            out_alpha[o] = A;
            out_depth[o] = D;
            final_T[o] = T;
            n_contrib[o] = n;
            if (n_examined) n_examined[o] = ex;
            if (n_blended) n_blended[o] = nb;
            if (margin) margin[o] = mg;
            total += ex;
        }
    }
    return total;
}

static void atomic_add(double *p, double v)
{
#pragma omp atomic
    *p += v;
}

/* p[i] += v and, when the magnitude array m is given, m[i] += |v|: the sum
 * of absolute per-pixel contributions, the natural scale of a gradient that
 * is a sum of terms of both signs. */
static void grad_add(double *p, double *m, int64_t i, double v)
{
    atomic_add(&p[i], v);
    if (m) atomic_add(&m[i], fabs(v));
}

/*
 * Backward of orc_render_fwd for the loss L = sum g_C . out_color
 * + g_A . out_alpha + g_D . out_depth (g_A, g_D nullable).  Per pixel the
 * contributors k = 1..N (alpha_k, T_{k-1} = prod_{j<k} (1 - alpha_j)) are
 * recomputed exactly, then walked back to front with the accumulated sums
 * behind k:  R_k = sum_{j>k} rgb_j alpha_j T_{j-1},  Rd_k likewise for depth:
 *   dL/d rgb_k   += alpha_k T_{k-1} g_C
 *   dL/d depth_k += alpha_k T_{k-1} g_D
 *   dL/d alpha_k  = g_C . (rgb_k T_{k-1} - (R_k + T_N bg) / (1 - alpha_k))
 *                 + g_A T_N / (1 - alpha_k)
 *                 + g_D (depth_k T_{k-1} - Rd_k / (1 - alpha_k))
 * and, where alpha_k = o G (not clamped at 0.99; the clamp has derivative 0):
 *   dL/d o += G dL/dalpha;  dL/dpower = o G dL/dalpha
 *   dL/d (a, b, c) += (-dx^2 / 2, -dx dy, -dy^2 / 2) dL/dpower
 *   dL/d (u, v)    += (a dx + b dy, b dx + c dy) dL/dpower
 * Gradients are added (+=) into the caller's buffers; the mag_* arrays
 * (nullable, same layouts) receive the sums of the absolute per-pixel terms.
 * Returns the number of contributors walked (the backward "blend" count).
 */
int64_t orc_render_bwd(int32_t width, int32_t height, int32_t tile, const int32_t *ranges,
                       const int32_t *point_list, const double *means2D, const double *conic_opacity,
                       const double *rgb, const double *depth, const double *bg, const int32_t *window,
                       const double *dL_dcolor, const double *dL_dalpha, const double *dL_ddepth,
                       double *dL_dmeans2D, double *dL_dconic, double *dL_dopacity, double *dL_drgb,
                       double *dL_ddepths, double *mag_means2D, double *mag_conic, double *mag_opacity,
                       double *mag_rgb, double *mag_depths)
{
    int32_t win[4];
    window_or_full(window, width, height, win);
    const int TX = tiles_x(width, tile);
    const int64_t HW = (int64_t)width * height;
    const double amin = thr_alpha_min(), amax = thr_alpha_max(), tmin = thr_T_min();
    int32_t maxlen = 0;
    for (int t = 0; t < TX * tiles_y(height, tile); ++t) {
        int32_t l = ranges[2 * t + 1] - ranges[2 * t];
        if (l > maxlen) maxlen = l;
    }
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        /* contributors of one pixel: list position, alpha, o*G, T before */
        int32_t *ck = (int32_t *)malloc(sizeof(int32_t) * (maxlen + 1));
        double *ca = (double *)malloc(sizeof(double) * (maxlen + 1));
        double *cg = (double *)malloc(sizeof(double) * (maxlen + 1));
        double *cT = (double *)malloc(sizeof(double) * (maxlen + 1));
#pragma omp for schedule(dynamic, 1)
        for (int py = win[1]; py < win[3]; ++py) {
            for (int px = win[0]; px < win[2]; ++px) {
                const int t = (py / tile) * TX + (px / tile);
                const int32_t s = ranges[2 * t], e = ranges[2 * t + 1];
                const int64_t o = (int64_t)py * width + px;
                double T = 1.0;
                int N = 0;
                for (int32_t k = s; k < e; ++k) {
                    const int32_t g = point_list[k];
                    const double dx = px - means2D[2 * g], dy = py - means2D[2 * g + 1];
                    const double *co = conic_opacity + 4 * g;
                    const double power = -0.5 * (co[0] * dx * dx + co[2] * dy * dy) - co[1] * dx * dy;
                    if (power > 0) continue;
                    const double ga = co[3] * exp(power);
                    const double alpha = ga < amax ? ga : amax;
                    if (alpha < amin) continue;
                    const double Tn = T * (1.0 - alpha);
                    if (Tn < tmin) break;
                    ck[N] = k;
                    ca[N] = alpha;
                    cg[N] = ga;
                    cT[N] = T;
                    ++N;
                    T = Tn;
                }
                const double TN = T;
                const double gC[3] = {dL_dcolor[o], dL_dcolor[HW + o], dL_dcolor[2 * HW + o]};
                const double gA = dL_dalpha ? dL_dalpha[o] : 0.0;
                const double gD = dL_ddepth ? dL_ddepth[o] : 0.0;
                double R[3] = {0, 0, 0}, Rd = 0;
                for (int q = N - 1; q >= 0; --q) {
                    const int32_t g = point_list[ck[q]];
                    const double a = ca[q], Tb = cT[q], w = a * Tb;
                    const double *col = rgb + 3 * g;
                    const double dk = depth[g];
                    double dA = 0;
                    for (int c = 0; c < 3; ++c) {
                        grad_add(dL_drgb, mag_rgb, 3 * g + c, w * gC[c]);
                        dA += gC[c] * (col[c] * Tb - (R[c] + TN * bg[c]) / (1.0 - a));
                    }
                    dA += gA * TN / (1.0 - a);
                    dA += gD * (dk * Tb - Rd / (1.0 - a));
                    if (dL_ddepths) grad_add(dL_ddepths, mag_depths, g, w * gD);
                    for (int c = 0; c < 3; ++c) R[c] += col[c] * w;
                    Rd += dk * w;
                    if (cg[q] <= amax) {
                        const double *co = conic_opacity + 4 * g;
                        const double G = cg[q] / co[3];
                        const double dx = px - means2D[2 * g], dy = py - means2D[2 * g + 1];
                        const double dP = cg[q] * dA;
                        grad_add(dL_dopacity, mag_opacity, g, G * dA);
                        grad_add(dL_dconic, mag_conic, 3 * g + 0, -0.5 * dx * dx * dP);
                        grad_add(dL_dconic, mag_conic, 3 * g + 1, -dx * dy * dP);
                        grad_add(dL_dconic, mag_conic, 3 * g + 2, -0.5 * dy * dy * dP);
                        grad_add(dL_dmeans2D, mag_means2D, 2 * g + 0, (co[0] * dx + co[1] * dy) * dP);
                        grad_add(dL_dmeans2D, mag_means2D, 2 * g + 1, (co[1] * dx + co[2] * dy) * dP);
                    }
                }
                total += N > 0 ? (ck[N - 1] - s + 1) : 0;
            }
        }
        free(ck);
        free(ca);
        free(cg);
        free(cT);
    }
    return total;
}
