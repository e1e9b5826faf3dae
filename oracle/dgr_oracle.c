/*
 * dgr_oracle.c -- plain, slow CPU oracle for the DGR hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library in paper_2411_04844_amd/;
 * neither side includes or links the other.
 *
 * Paper: Wu et al., "Discretized Gaussian Representation for Tomographic
 * Reconstruction" (arXiv 2411.04844).  Every function names the passage it
 * follows.  Floating point is IEEE binary64 except the bounding-box
 * computation, which the box definition fixes to binary32 (see orc_bbox).
 * Build with -ffp-contract=off -fno-fast-math so that no FMA contraction or
 * reassociation changes any rounding.
 *
 * Coordinates.  World points are (x, y, z).  A grid of dims (nx, ny, nz)
 * has its lower faces at glo[3] and voxel size 1/inv_h[a] on axis a; voxel
 * i's centre is glo + (i + 1/2)/inv_h.  The continuous voxel coordinate of
 * a world point is u = (p - glo)*inv_h - 1/2, so voxel centres sit at the
 * integers.  Volumes are stored [nz][ny][nx] with x fastest.
 *
 * Parity status of each function (what pins it) is listed in the header of
 * oracle/__init__.py.
 */
#include <math.h>
#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* O1. Per-Gaussian truncation box (binary32, bit-exact by definition).      */
/*                                                                          */
/* The paper confines each Gaussian to an odd cuboid anchored at the floor  */
/* of its mean and drops indices outside the volume (sec. 4.1, Gaussian     */
/* Effect Confinement; Alg. 1, position and validity steps).  The per-      */
/* Gaussian variant used here keeps every voxel centre i with               */
/* |i_k - u_k| <= k_sigma * sqrt(Sigma_kk) * inv_h_k on each axis k, i.e.   */
/* the axis-aligned box around the k_sigma ellipsoid.  Ties are included;   */
/* the clamp to the grid is the validity mask.  With k_sigma <= 0 the box   */
/* is the paper's fixed cuboid floor(u) +- box_half.                        */
/* The float sequence below is the definition of record: every operation is */
/* one correctly rounded binary32 operation, evaluated in the order written.*/
/* box[g] = {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z}; empty iff lo > hi on an   */
/* axis.                                                                    */
/* ------------------------------------------------------------------------ */
static void rot_f32(const float q[4], float R[3][3])
{
    float w = q[0], x = q[1], y = q[2], z = q[3];
    float n2 = ((w * w + x * x) + y * y) + z * z;
    if (n2 == 0.0f) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = (i == j) ? 1.0f : 0.0f;
        return;
    }
    float m = sqrtf(n2);
    float a = w / m, b = x / m, c = y / m, d = z / m;
    R[0][0] = 1.0f - 2.0f * (c * c + d * d);
    R[0][1] = 2.0f * (b * c - a * d);
    R[0][2] = 2.0f * (b * d + a * c);
    R[1][0] = 2.0f * (b * c + a * d);
    R[1][1] = 1.0f - 2.0f * (b * b + d * d);
    R[1][2] = 2.0f * (c * d - a * b);
    R[2][0] = 2.0f * (b * d - a * c);
    R[2][1] = 2.0f * (c * d + a * b);
    R[2][2] = 1.0f - 2.0f * (b * b + c * c);
}

void orc_bbox(const float *mu, const float *scale, const float *quat, int64_t n,
              const int32_t dims[3], const float glo[3], const float inv_h[3],
              float k_sigma, int32_t box_half, int32_t *box)
{
    for (int64_t g = 0; g < n; ++g) {
        float R[3][3];
        rot_f32(quat + 4 * g, R);
        const float *s = scale + 3 * g;
        for (int k = 0; k < 3; ++k) {
            float u = (mu[3 * g + k] - glo[k]) * inv_h[k] - 0.5f;
            float flo, fhi;
            if (k_sigma > 0.0f) {
                float a0 = R[k][0] * s[0];
                float a1 = R[k][1] * s[1];
                float a2 = R[k][2] * s[2];
                float skk = (a0 * a0 + a1 * a1) + a2 * a2;
                float r = (k_sigma * sqrtf(skk)) * inv_h[k];
                flo = ceilf(u - r);
                fhi = floorf(u + r);
            } else {
                float f = floorf(u);
                flo = f - (float)box_half;
                fhi = f + (float)box_half;
            }
            float D = (float)dims[k];
            if (flo < 0.0f) flo = 0.0f;
            if (flo > D) flo = D;
            if (fhi > D - 1.0f) fhi = D - 1.0f;
            if (fhi < -1.0f) fhi = -1.0f;
            box[6 * g + k] = (int32_t)flo;
            box[6 * g + 3 + k] = (int32_t)fhi;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O2. Tile pairs.  Every 8^3 voxel tile that meets a non-empty box gives   */
/* one (tile, gid) pair; tile = (tz*Ty + ty)*Tx + tx with T = ceil(D/8).     */
/* The canonical order is ascending (tile, gid).  This replaces the paper's */
/* scatter into the volume (Alg. 1, final accumulation) by a gather per     */
/* tile; the set of (Gaussian, voxel) contributions is unchanged.           */
/* Returns the pair count; writes pairs[2*P] (tile, gid) and                */
/* tile_begin[T+1] when the pointers are non-null.                          */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_tile_pairs(const int32_t *box, int64_t n, const int32_t dims[3],
                       uint32_t *pairs, int64_t *tile_begin)
{
    int64_t Tx = (dims[0] + 7) / 8, Ty = (dims[1] + 7) / 8, Tz = (dims[2] + 7) / 8;
    int64_t T = Tx * Ty * Tz;
    int64_t P = 0;
    for (int64_t g = 0; g < n; ++g) {
        const int32_t *b = box + 6 * g;
        if (b[0] > b[3] || b[1] > b[4] || b[2] > b[5]) continue;
        P += (int64_t)((b[3] >> 3) - (b[0] >> 3) + 1) * ((b[4] >> 3) - (b[1] >> 3) + 1) *
             ((b[5] >> 3) - (b[2] >> 3) + 1);
    }
    if (!pairs && !tile_begin) return P;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(P > 0 ? P : 1));
    int64_t p = 0;
    for (int64_t g = 0; g < n; ++g) {
        const int32_t *b = box + 6 * g;
        if (b[0] > b[3] || b[1] > b[4] || b[2] > b[5]) continue;
        for (int32_t tz = b[2] >> 3; tz <= (b[5] >> 3); ++tz)
            for (int32_t ty = b[1] >> 3; ty <= (b[4] >> 3); ++ty)
                for (int32_t tx = b[0] >> 3; tx <= (b[3] >> 3); ++tx) {
                    uint64_t tile = (uint64_t)((tz * Ty + ty) * Tx + tx);
                    keys[p++] = (tile << 32) | (uint64_t)g;
                }
    }
    qsort(keys, (size_t)P, sizeof(uint64_t), cmp_u64);
    if (pairs)
        for (int64_t i = 0; i < P; ++i) {
            pairs[2 * i] = (uint32_t)(keys[i] >> 32);
            pairs[2 * i + 1] = (uint32_t)(keys[i] & 0xffffffffu);
        }
    if (tile_begin) {
        int64_t i = 0;
        for (int64_t t = 0; t <= T; ++t) {
            while (i < P && (int64_t)(keys[i] >> 32) < t) ++i;
            tile_begin[t] = i;
        }
    }
    free(keys);
    return P;
}

/* ------------------------------------------------------------------------ */
/* Gaussian shape in binary64.  Sigma = R diag(s^2) R^T with R the rotation */
/* of the normalised quaternion (w, x, y, z); the precision matrix is       */
/* Q = Sigma^-1 = R diag(s^-2) R^T (sec. 4.1, eq. for G(p, mu, Sigma); the  */
/* anisotropic form is the variant of App. D.2).                            */
/* ------------------------------------------------------------------------ */
static void rot_f64(const double q[4], double R[3][3], double qh[4], double *qn)
{
    double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    *qn = sqrt(n2);
    if (n2 == 0.0) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
        qh[0] = 1.0; qh[1] = qh[2] = qh[3] = 0.0;
        return;
    }
    double w = q[0] / *qn, x = q[1] / *qn, y = q[2] / *qn, z = q[3] / *qn;
    qh[0] = w; qh[1] = x; qh[2] = y; qh[3] = z;
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

static void precision_matrix(const double *s, const double *q, double Q[3][3])
{
    double R[3][3], qh[4], qn;
    rot_f64(q, R, qh, &qn);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += R[a][j] * R[b][j] / (s[j] * s[j]);
            Q[a][b] = acc;
        }
}

static inline double gauss_at(const double Q[3][3], const double d[3])
{
    double m = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m += d[a] * Q[a][b] * d[b];
    return exp(-0.5 * m);
}

static inline int in_box(const int32_t *b, int64_t i, int64_t j, int64_t k)
{
    return i >= b[0] && i <= b[3] && j >= b[1] && j <= b[4] && k >= b[2] && k <= b[5];
}

/* ------------------------------------------------------------------------ */
/* O3a. Voxelization by brute force: every Gaussian at every voxel, kept    */
/* where the voxel lies in that Gaussian's box.  V(p) = sum_i G(p, mu_i,    */
/* Sigma_i) * I_i (sec. 4.1, Direct Reconstruction) with the confinement    */
/* and validity mask of Alg. 1.  V is overwritten.                          */
/* ------------------------------------------------------------------------ */
void orc_voxelize_brute(const double *mu, const double *scale, const double *quat,
                        const double *density, int64_t n, const int32_t dims[3],
                        const double glo[3], const double inv_h[3], const int32_t *box,
                        double *V)
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    double (*Q)[3][3] = malloc(sizeof(double[3][3]) * (size_t)(n > 0 ? n : 1));
    for (int64_t g = 0; g < n; ++g) precision_matrix(scale + 3 * g, quat + 4 * g, Q[g]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double p[3] = {glo[0] + (i + 0.5) / inv_h[0], glo[1] + (j + 0.5) / inv_h[1],
                               glo[2] + (k + 0.5) / inv_h[2]};
                double acc = 0.0;
                for (int64_t g = 0; g < n; ++g) {
                    if (!in_box(box + 6 * g, i, j, k)) continue;
                    double d[3] = {p[0] - mu[3 * g], p[1] - mu[3 * g + 1], p[2] - mu[3 * g + 2]};
                    acc += gauss_at(Q[g], d) * density[g];
                }
                V[(k * ny + j) * nx + i] = acc;
            }
    free(Q);
}

/* O3b. The same sum restricted to each box (sec. 4.1 confinement): loops  */
/* over the box only.  Parallel over z-slabs; each slab sums its Gaussians  */
/* in gid order.                                                            */
void orc_voxelize_box(const double *mu, const double *scale, const double *quat,
                      const double *density, int64_t n, const int32_t dims[3],
                      const double glo[3], const double inv_h[3], const int32_t *box,
                      double *V)
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    double (*Q)[3][3] = malloc(sizeof(double[3][3]) * (size_t)(n > 0 ? n : 1));
    for (int64_t g = 0; g < n; ++g) precision_matrix(scale + 3 * g, quat + 4 * g, Q[g]);
    memset(V, 0, sizeof(double) * (size_t)(nx * ny * nz));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nz; ++k) {
        for (int64_t g = 0; g < n; ++g) {
            const int32_t *b = box + 6 * g;
            if (k < b[2] || k > b[5]) continue;
            for (int64_t j = b[1]; j <= b[4]; ++j)
                for (int64_t i = b[0]; i <= b[3]; ++i) {
                    double d[3] = {glo[0] + (i + 0.5) / inv_h[0] - mu[3 * g],
                                   glo[1] + (j + 0.5) / inv_h[1] - mu[3 * g + 1],
                                   glo[2] + (k + 0.5) / inv_h[2] - mu[3 * g + 2]};
                    V[(k * ny + j) * nx + i] += gauss_at(Q[g], d) * density[g];
                }
        }
    }
    free(Q);
}

/* ------------------------------------------------------------------------ */
/* O8. Gradient of a loss L(V) with respect to the Gaussian parameters,     */
/* given dL/dV, with the boxes held fixed.  The paper obtains it by         */
/* automatic differentiation through the aligned evaluation (sec. 4.1,      */
/* Discretize and Align); here it is the chain rule written out:            */
/*   drho = sum w G,  dmu = rho Q m1,  dQ = -rho/2 M2,                      */
/*   with w = dL/dV, d = x - mu, m1 = sum w G d, M2 = sum w G d d^T;        */
/*   Q = R L R^T with L = diag(s^-2): ds_j = -2 s_j^-3 (R^T dQ R)_jj,       */
/*   dR = 2 dQ R L, dq_hat = <dR, dR/dq_hat>, dq = (I - qh qh^T) dq_hat/|q|.*/
/* A zero quaternion is the identity rotation with zero gradient.           */
/* ------------------------------------------------------------------------ */
void orc_voxelize_grad(const double *mu, const double *scale, const double *quat,
                       const double *density, int64_t n, const int32_t dims[3],
                       const double glo[3], const double inv_h[3], const int32_t *box,
                       const double *dV, double *dmu, double *dscale, double *dquat,
                       double *ddensity)
{
    int64_t nx = dims[0], ny = dims[1];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < n; ++g) {
        const double *s = scale + 3 * g;
        double R[3][3], qh[4], qn, Q[3][3];
        rot_f64(quat + 4 * g, R, qh, &qn);
        precision_matrix(s, quat + 4 * g, Q);
        const int32_t *b = box + 6 * g;
        double M0 = 0.0, m1[3] = {0, 0, 0}, M2[3][3] = {{0}};
        for (int64_t k = b[2]; k <= b[5]; ++k)
            for (int64_t j = b[1]; j <= b[4]; ++j)
                for (int64_t i = b[0]; i <= b[3]; ++i) {
                    double d[3] = {glo[0] + (i + 0.5) / inv_h[0] - mu[3 * g],
                                   glo[1] + (j + 0.5) / inv_h[1] - mu[3 * g + 1],
                                   glo[2] + (k + 0.5) / inv_h[2] - mu[3 * g + 2]};
                    double wG = dV[(k * ny + j) * nx + i] * gauss_at(Q, d);
                    M0 += wG;
                    for (int a = 0; a < 3; ++a) {
                        m1[a] += wG * d[a];
                        for (int c = 0; c < 3; ++c) M2[a][c] += wG * d[a] * d[c];
                    }
                }
        double rho = density[g];
        ddensity[g] = M0;
        for (int a = 0; a < 3; ++a) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) acc += Q[a][c] * m1[c];
            dmu[3 * g + a] = rho * acc;
        }
        double dQ[3][3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) dQ[a][c] = -0.5 * rho * M2[a][c];
        /* dL/dL_jj = (R^T dQ R)_jj and dL/ds_j = dL/dL_jj * d(s_j^-2)/ds_j */
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) acc += R[a][j] * dQ[a][c] * R[c][j];
            dscale[3 * g + j] = acc * (-2.0 / (s[j] * s[j] * s[j]));
        }
        double *dq = dquat + 4 * g;
        if (qn == 0.0) {
            dq[0] = dq[1] = dq[2] = dq[3] = 0.0;
            continue;
        }
        double dR[3][3];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += dQ[a][c] * R[c][j];
                dR[a][j] = 2.0 * acc / (s[j] * s[j]);
            }
        double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
        /* partial derivatives of the nine entries of R(w, x, y, z) */
        double dRdq[4][3][3] = {
            {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}},
            {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}},
            {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}},
            {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}}};
        double dqh[4];
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int j = 0; j < 3; ++j) acc += dR[a][j] * dRdq[c][a][j];
            dqh[c] = acc;
        }
        double proj = qh[0] * dqh[0] + qh[1] * dqh[1] + qh[2] * dqh[2] + qh[3] * dqh[3];
        for (int c = 0; c < 4; ++c) dq[c] = (dqh[c] - qh[c] * proj) / qn;
    }
}

/* ------------------------------------------------------------------------ */
/* Acquisition geometry.  The paper leaves the projection operator T        */
/* abstract (sec. 4.3, P_hat = T(V)).  The operator of record is a          */
/* trilinear ray march: for ray r with unit direction d and c the point of  */
/* the ray nearest the world origin (the isocentre),                        */
/*   P_hat_r = ell * dt * sum_{k in Z} Vbar(c + k dt d),                    */
/* where Vbar is the trilinear interpolant of V on voxel centres with zero  */
/* outside the grid.  views[12*j] = {a[3], det[3], e_u[3], e_v[3]}: a is    */
/* the ray direction (parallel, kind 0) or the source point (cone, kind 1); */
/* pixel (iu, iv) sits at det + (iu - (nu-1)/2) e_u + (iv - (nv-1)/2) e_v.  */
/* Fan beam (kind 2), the slice stacks of the paper's fan-beam experiments  */
/* (sec. 5.1, Tabs. 2-3): every detector row is a 2-D fan with its own      */
/* source, a + (iv - (nv-1)/2) e_v, the central row's source shifted with   */
/* the row.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t kind, n_views, nu, nv;
    const float *views;
    double step, length_scale;
} orc_geom;

static void ray_of(const orc_geom *G, int64_t j, int64_t iu, int64_t iv, double c[3], double d[3])
{
    const float *v = G->views + 12 * j;
    double au = (double)iu - 0.5 * (double)(G->nu - 1);
    double av = (double)iv - 0.5 * (double)(G->nv - 1);
    double pix[3], o[3];
    for (int a = 0; a < 3; ++a) pix[a] = (double)v[3 + a] + au * (double)v[6 + a] + av * (double)v[9 + a];
    if (G->kind == 0) {
        for (int a = 0; a < 3; ++a) { d[a] = v[a]; o[a] = pix[a]; }
    } else if (G->kind == 1) {
        for (int a = 0; a < 3; ++a) { d[a] = pix[a] - (double)v[a]; o[a] = v[a]; }
    } else {
        for (int a = 0; a < 3; ++a) {
            o[a] = (double)v[a] + av * (double)v[9 + a];
            d[a] = pix[a] - o[a];
        }
    }
    double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] /= nd;
    double od = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    for (int a = 0; a < 3; ++a) c[a] = o[a] - od * d[a];
}

/* k-range that contains every sample with a non-zero interpolant: the      */
/* interpolant vanishes unless -1 < u_a < D_a on every axis.  The range is  */
/* padded by two samples; out-of-grid taps read as zero, so padding only   */
/* adds zero terms.  Returns 0 when the ray misses the support.             */
static int k_range(const double c[3], const double d[3], const int32_t dims[3],
                   const double glo[3], const double inv_h[3], double dt, int64_t *k0, int64_t *k1)
{
    double tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double uc = (c[a] - glo[a]) * inv_h[a] - 0.5;
        double du = d[a] * inv_h[a];
        if (du == 0.0) {
            if (!(uc > -1.0 && uc < (double)dims[a])) return 0;
            continue;
        }
        double t0 = (-1.0 - uc) / du, t1 = ((double)dims[a] - uc) / du;
        if (t0 > t1) { double tt = t0; t0 = t1; t1 = tt; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    if (!(tmin < tmax)) return 0;
    *k0 = (int64_t)floor(tmin / dt) - 2;
    *k1 = (int64_t)ceil(tmax / dt) + 2;
    return 1;
}

static inline double vox_or_zero(const double *V, const int32_t dims[3], int64_t i, int64_t j, int64_t k)
{
    if (i < 0 || j < 0 || k < 0 || i >= dims[0] || j >= dims[1] || k >= dims[2]) return 0.0;
    return V[(k * dims[1] + j) * dims[0] + i];
}

/* Trilinear interpolant at voxel coordinate u: sum over the eight          */
/* surrounding voxel centres of V * prod_a (1 - |u_a - i_a|).               */
static double trilinear(const double *V, const int32_t dims[3], const double u[3])
{
    double fl[3], f[3];
    for (int a = 0; a < 3; ++a) { fl[a] = floor(u[a]); f[a] = u[a] - fl[a]; }
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
        double w = (ox ? f[0] : 1 - f[0]) * (oy ? f[1] : 1 - f[1]) * (oz ? f[2] : 1 - f[2]);
        acc += w * vox_or_zero(V, dims, (int64_t)fl[0] + ox, (int64_t)fl[1] + oy, (int64_t)fl[2] + oz);
    }
    return acc;
}

/* O4. Forward projection P_hat = T(V) (sec. 4.3) as the ray march above.   */
void orc_project(const double *V, const int32_t dims[3], const double glo[3], const double inv_h[3],
                 int32_t kind, int32_t n_views, int32_t nu, int32_t nv, const float *views,
                 double step, double length_scale, double *proj)
{
    orc_geom G = {kind, n_views, nu, nv, views, step, length_scale};
    int64_t nrays = (int64_t)n_views * nu * nv;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrays; ++r) {
        int64_t j = r / ((int64_t)nu * nv), iv = (r / nu) % nv, iu = r % nu;
        double c[3], d[3];
        ray_of(&G, j, iu, iv, c, d);
        int64_t k0, k1;
        double acc = 0.0;
        if (k_range(c, d, dims, glo, inv_h, step, &k0, &k1)) {
            for (int64_t k = k0; k <= k1; ++k) {
                double t = (double)k * step, u[3];
                for (int a = 0; a < 3; ++a) u[a] = (c[a] + t * d[a] - glo[a]) * inv_h[a] - 0.5;
                acc += trilinear(V, dims, u);
            }
        }
        proj[r] = length_scale * step * acc;
    }
}

/* O7. The exact transpose of O4: (A^T g)(i) = ell dt sum_r g_r sum_k      */
/* w_i(c_r + k dt d_r), w_i the trilinear weight of voxel i.  Each thread  */
/* scatters into its own copy of the volume; the copies are then summed.   */
void orc_backproject(const double *proj, const int32_t dims[3], const double glo[3],
                     const double inv_h[3], int32_t kind, int32_t n_views, int32_t nu, int32_t nv,
                     const float *views, double step, double length_scale, double *V)
{
    orc_geom G = {kind, n_views, nu, nv, views, step, length_scale};
    int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t nrays = (int64_t)n_views * nu * nv;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nthr * (size_t)nvox, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + (size_t)tid * (size_t)nvox;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nrays; ++r) {
            int64_t j = r / ((int64_t)nu * nv), iv = (r / nu) % nv, iu = r % nu;
            double c[3], d[3];
            ray_of(&G, j, iu, iv, c, d);
            int64_t k0, k1;
            if (!k_range(c, d, dims, glo, inv_h, step, &k0, &k1)) continue;
            double gr = length_scale * step * proj[r];
            for (int64_t k = k0; k <= k1; ++k) {
                double t = (double)k * step, u[3], fl[3], f[3];
                for (int a = 0; a < 3; ++a) {
                    u[a] = (c[a] + t * d[a] - glo[a]) * inv_h[a] - 0.5;
                    fl[a] = floor(u[a]);
                    f[a] = u[a] - fl[a];
                }
                for (int cc = 0; cc < 8; ++cc) {
                    int ox = cc & 1, oy = (cc >> 1) & 1, oz = (cc >> 2) & 1;
                    int64_t i = (int64_t)fl[0] + ox, jj = (int64_t)fl[1] + oy, kk = (int64_t)fl[2] + oz;
                    if (i < 0 || jj < 0 || kk < 0 || i >= dims[0] || jj >= dims[1] || kk >= dims[2]) continue;
                    double w = (ox ? f[0] : 1 - f[0]) * (oy ? f[1] : 1 - f[1]) * (oz ? f[2] : 1 - f[2]);
                    mine[(kk * dims[1] + jj) * dims[0] + i] += gr * w;
                }
            }
        }
    }
    for (int64_t i = 0; i < nvox; ++i) {
        double acc = 0.0;
        for (int t = 0; t < nthr; ++t) acc += part[(size_t)t * (size_t)nvox + (size_t)i];
        V[i] = acc;
    }
    free(part);
}

/* ------------------------------------------------------------------------ */
/* O5. Siddon projector: the exact length of the ray inside each voxel      */
/* (voxels as constant-valued cells [glo + i h, glo + (i+1) h]), summed     */
/* with the voxel values, times ell (Siddon 1985).  The line is the same    */
/* infinite line as in O4.  Crossing parameters of every cell plane are     */
/* gathered, sorted, and each interval is attributed to the cell holding    */
/* its midpoint.  It checks the geometry of the ray march and is the        */
/* reference of the library's exact-path projector and its transpose.       */
/* ------------------------------------------------------------------------ */
static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Segments of ray (c, d) inside the grid: cells[q] (flat index, or -1 when */
/* the midpoint falls outside by rounding) and lengths len[q]; ts holds at  */
/* least dims[0] + dims[1] + dims[2] + 6 doubles.  Returns the count.       */
static int64_t siddon_segments(const double c[3], const double d[3], const int32_t dims[3],
                               const double glo[3], const double inv_h[3], double *ts,
                               int64_t *cells, double *len)
{
    double tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double lo = glo[a], hi = glo[a] + (double)dims[a] / inv_h[a];
        if (d[a] == 0.0) {
            if (!(c[a] > lo && c[a] < hi)) return 0;
            continue;
        }
        double t0 = (lo - c[a]) / d[a], t1 = (hi - c[a]) / d[a];
        if (t0 > t1) { double tt = t0; t0 = t1; t1 = tt; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    if (!(tmin < tmax)) return 0;
    int64_t m = 0, k = 0;
    ts[m++] = tmin;
    ts[m++] = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        for (int64_t p = 0; p <= dims[a]; ++p) {
            double t = (glo[a] + (double)p / inv_h[a] - c[a]) / d[a];
            if (t > tmin && t < tmax) ts[m++] = t;
        }
    }
    qsort(ts, (size_t)m, sizeof(double), cmp_dbl);
    for (int64_t q = 0; q + 1 < m; ++q) {
        double l = ts[q + 1] - ts[q];
        if (l <= 0.0) continue;
        double tm = 0.5 * (ts[q] + ts[q + 1]);
        int64_t idx[3], inside = 1;
        for (int a = 0; a < 3; ++a) {
            idx[a] = (int64_t)floor((c[a] + tm * d[a] - glo[a]) * inv_h[a]);
            if (idx[a] < 0 || idx[a] >= dims[a]) inside = 0;
        }
        cells[k] = inside ? (idx[2] * dims[1] + idx[1]) * dims[0] + idx[0] : -1;
        len[k] = l;
        ++k;
    }
    return k;
}

void orc_project_siddon(const double *V, const int32_t dims[3], const double glo[3],
                        const double inv_h[3], int32_t kind, int32_t n_views, int32_t nu, int32_t nv,
                        const float *views, double length_scale, double *proj)
{
    orc_geom G = {kind, n_views, nu, nv, views, 1.0, length_scale};
    int64_t nrays = (int64_t)n_views * nu * nv;
    int64_t cap = (int64_t)dims[0] + dims[1] + dims[2] + 6;
#pragma omp parallel
    {
        double *ts = malloc(sizeof(double) * (size_t)cap), *len = malloc(sizeof(double) * (size_t)cap);
        int64_t *cells = malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nrays; ++r) {
            int64_t j = r / ((int64_t)nu * nv), iv = (r / nu) % nv, iu = r % nu;
            double c[3], d[3];
            ray_of(&G, j, iu, iv, c, d);
            int64_t k = siddon_segments(c, d, dims, glo, inv_h, ts, cells, len);
            double acc = 0.0;
            for (int64_t q = 0; q < k; ++q)
                if (cells[q] >= 0) acc += len[q] * V[cells[q]];
            proj[r] = length_scale * acc;
        }
        free(ts); free(len); free(cells);
    }
}

/* Transpose of orc_project_siddon: V[i] = ell * sum over rays r and their  */
/* segments in cell i of len * proj[r].  Rays are taken one after another.  */
void orc_backproject_siddon(const double *proj, const int32_t dims[3], const double glo[3],
                            const double inv_h[3], int32_t kind, int32_t n_views, int32_t nu, int32_t nv,
                            const float *views, double length_scale, double *V)
{
    orc_geom G = {kind, n_views, nu, nv, views, 1.0, length_scale};
    int64_t nrays = (int64_t)n_views * nu * nv;
    int64_t cap = (int64_t)dims[0] + dims[1] + dims[2] + 6;
    int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    double *ts = malloc(sizeof(double) * (size_t)cap), *len = malloc(sizeof(double) * (size_t)cap);
    int64_t *cells = malloc(sizeof(int64_t) * (size_t)cap);
    for (int64_t i = 0; i < nvox; ++i) V[i] = 0.0;
    for (int64_t r = 0; r < nrays; ++r) {
        int64_t j = r / ((int64_t)nu * nv), iv = (r / nu) % nv, iu = r % nu;
        double c[3], d[3];
        ray_of(&G, j, iu, iv, c, d);
        int64_t k = siddon_segments(c, d, dims, glo, inv_h, ts, cells, len);
        for (int64_t q = 0; q < k; ++q)
            if (cells[q] >= 0) V[cells[q]] += length_scale * len[q] * proj[r];
    }
    free(ts); free(len); free(cells);
}

/* ------------------------------------------------------------------------ */
/* O6. L1 projection loss (sec. 4.3 objective, the L1 term) as a mean over  */
/* all M = views * pixels, and its gradient g = sign(P_hat - y)/M with      */
/* sign(0) = 0.  Returns the loss; g may be null.                           */
/* ------------------------------------------------------------------------ */
double orc_l1(const double *proj, const float *target, int64_t m, double *g)
{
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r = proj[i] - (double)target[i];
        acc += fabs(r);
        if (g) g[i] = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / (double)m;
    }
    return acc / (double)m;
}

/* ------------------------------------------------------------------------ */
/* Adam step (the optimiser of sec. 5.1, Implementation Details), projected */
/* onto p >= lower (the reconstruction keeps densities in R+, sec. 4.1, and */
/* scales positive):                                                        */
/*   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,                         */
/*   p <- max(p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), lower). */
/* The moments are not affected by the projection.  lower = -inf gives the  */
/* plain step.                                                              */
/* ------------------------------------------------------------------------ */
void orc_adam(double *p, const double *g, double *m, double *v, int64_t n, double lr, double b1,
              double b2, double eps, int64_t t, double lower)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double next = p[i] - lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
        p[i] = next < lower ? lower : next;
    }
}

/* ------------------------------------------------------------------------ */
/* PSNR (App. C.1): 10 log10(MAX^2 / MSE) with MAX the largest ground-truth */
/* value and MSE the mean over all voxels.                                  */
/* ------------------------------------------------------------------------ */
double orc_psnr(const double *x, const double *gt, int64_t n)
{
    double mx = -INFINITY, se = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (gt[i] > mx) mx = gt[i];
        double e = x[i] - gt[i];
        se += e * e;
    }
    return 10.0 * log10(mx * mx / (se / (double)n));
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (for single-thread timings). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* O9. FDK (Feldkamp-Davis-Kress) for a full circular cone-beam scan on a   */
/* flat detector, the textbook filtered backprojection (Kak & Slaney, the  */
/* reference the paper cites in sec. 4.1); the paper uses an FBP/FDK        */
/* volume to initialise Gaussian positions (Fig. 4 caption) and as a        */
/* baseline.  Per view j (source s, detector plane with unit normal n from  */
/* the source side, D = (det - s).n, R = -s.n):                             */
/*  1. p_w = p * D / |pix - s|              (cosine weight)                 */
/*  2. q = ramp filter of p_w along e_u: spacing tau = |e_u| R / D,         */
/*     q(i) = (1/tau) [p_w(i)/4 - sum_{k odd} p_w(i-k) / (k^2 pi^2)]        */
/*  3. f(x) += (dbeta / 2) (R / U)^2 q(a(x), b(x)), U = (x - s).n, (a, b)   */
/*     the detector position of the ray s -> x, bilinear in q, zero outside.*/
/* The result is divided by length_scale (projections carry that factor).   */
/* Fan beam (kind 2): 2-D fan-beam FBP of each slice is the same three      */
/* steps with the row's own source s_b = s + b e_v: in step 1 |pix - s_b|   */
/* has no e_v part; in step 3 x is read from the row b whose fan plane      */
/* holds it, b = ((x - s).m) / (e_v.m) with m = (det - s) x e_u, R and U    */
/* taken from s_b.                                                          */
/* ------------------------------------------------------------------------ */
static void view_frame(const float *v, double s[3], double det[3], double eu[3], double ev[3],
                       double n[3], double *D, double *R)
{
    for (int a = 0; a < 3; ++a) { s[a] = v[a]; det[a] = v[3 + a]; eu[a] = v[6 + a]; ev[a] = v[9 + a]; }
    n[0] = eu[1] * ev[2] - eu[2] * ev[1];
    n[1] = eu[2] * ev[0] - eu[0] * ev[2];
    n[2] = eu[0] * ev[1] - eu[1] * ev[0];
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) n[a] /= nn;
    double dd = (det[0] - s[0]) * n[0] + (det[1] - s[1]) * n[1] + (det[2] - s[2]) * n[2];
    if (dd < 0) { for (int a = 0; a < 3; ++a) n[a] = -n[a]; dd = -dd; }
    *D = dd;
    *R = -(s[0] * n[0] + s[1] * n[1] + s[2] * n[2]);
}

/* Step 2 alone: the discrete Ram-Lak filter of one row p[nu] with sample  */
/* spacing tau, the samples of the band-limited ramp |w| (Kak & Slaney,     */
/* ch. 3): h(0) = 1/(4 tau^2), h(k) = 0 for even k != 0 and                 */
/* -1/(k^2 pi^2 tau^2) for odd k, convolved with spacing tau; samples       */
/* beyond the row are zero.                                                 */
void orc_ramp_filter(const double *p, int64_t nu, double tau, double *q)
{
    for (int64_t i = 0; i < nu; ++i) {
        double acc = 0.25 * p[i];
        for (int64_t k = 1; k < nu; k += 2) {
            double w = 1.0 / ((double)k * (double)k * M_PI * M_PI);
            if (i - k >= 0) acc -= w * p[i - k];
            if (i + k < nu) acc -= w * p[i + k];
        }
        q[i] = acc / tau;
    }
}

void orc_fdk(const float *proj, int32_t kind, int32_t n_views, int32_t nu, int32_t nv, const float *views,
             double arc, double length_scale, const int32_t dims[3], const double glo[3],
             const double inv_h[3], double *V)
{
    int fan = kind == 2;
    int64_t npix = (int64_t)nu * nv;
    double *q = malloc(sizeof(double) * (size_t)(n_views * npix));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jr = 0; jr < (int64_t)n_views * nv; ++jr) {
        int64_t j = jr / nv, iv = jr % nv;
        double s[3], det[3], eu[3], ev[3], n[3], D, R;
        view_frame(views + 12 * j, s, det, eu, ev, n, &D, &R);
        double pu = sqrt(eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2]);
        double tau = pu * R / D;
        double *row = malloc(sizeof(double) * (size_t)nu);
        for (int64_t iu = 0; iu < nu; ++iu) {
            double au = (double)iu - 0.5 * (nu - 1), av = (double)iv - 0.5 * (nv - 1), r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double src = fan ? s[a] + av * ev[a] : s[a];
                double d = det[a] + au * eu[a] + av * ev[a] - src;
                r2 += d * d;
            }
            row[iu] = (double)proj[(j * nv + iv) * nu + iu] * D / sqrt(r2);
        }
        orc_ramp_filter(row, nu, tau, q + (j * nv + iv) * nu);
        free(row);
    }
    double dbeta = arc / (double)n_views;
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t jj = 0; jj < ny; ++jj)
            for (int64_t i = 0; i < nx; ++i) {
                double x[3] = {glo[0] + (i + 0.5) / inv_h[0], glo[1] + (jj + 0.5) / inv_h[1],
                               glo[2] + (k + 0.5) / inv_h[2]};
                double acc = 0.0;
                for (int64_t j = 0; j < n_views; ++j) {
                    double s[3], det[3], eu[3], ev[3], n[3], D, R;
                    view_frame(views + 12 * j, s, det, eu, ev, n, &D, &R);
                    if (fan) {
                        double w[3] = {det[0] - s[0], det[1] - s[1], det[2] - s[2]};
                        double m[3] = {w[1] * eu[2] - w[2] * eu[1], w[2] * eu[0] - w[0] * eu[2],
                                       w[0] * eu[1] - w[1] * eu[0]};
                        double em = ev[0] * m[0] + ev[1] * m[1] + ev[2] * m[2];
                        double b = ((x[0] - s[0]) * m[0] + (x[1] - s[1]) * m[1] + (x[2] - s[2]) * m[2]) / em;
                        for (int a = 0; a < 3; ++a) s[a] += b * ev[a];
                        R = -(s[0] * n[0] + s[1] * n[1] + s[2] * n[2]);
                    }
                    double r[3] = {x[0] - s[0], x[1] - s[1], x[2] - s[2]};
                    double U = r[0] * n[0] + r[1] * n[1] + r[2] * n[2];
                    if (!(U > 0)) continue;
                    double hit[3];
                    for (int a = 0; a < 3; ++a) hit[a] = s[a] + (D / U) * r[a] - det[a];
                    double uu = eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2];
                    double vv = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
                    double a_pix = (hit[0] * eu[0] + hit[1] * eu[1] + hit[2] * eu[2]) / uu + 0.5 * (nu - 1);
                    double b_pix = (hit[0] * ev[0] + hit[1] * ev[1] + hit[2] * ev[2]) / vv + 0.5 * (nv - 1);
                    double fa = floor(a_pix), fb = floor(b_pix), wa = a_pix - fa, wb = b_pix - fb;
                    double val = 0.0;
                    for (int c = 0; c < 4; ++c) {
                        int64_t ia = (int64_t)fa + (c & 1), ib = (int64_t)fb + (c >> 1);
                        if (ia < 0 || ib < 0 || ia >= nu || ib >= nv) continue;
                        double w = ((c & 1) ? wa : 1 - wa) * ((c >> 1) ? wb : 1 - wb);
                        val += w * q[(j * nv + ib) * nu + ia];
                    }
                    acc += (R / U) * (R / U) * val;
                }
                V[(k * ny + jj) * nx + i] = 0.5 * dbeta * acc / length_scale;
            }
    free(q);
}

/* ------------------------------------------------------------------------ */
/* Initial Gaussians drawn from a volume (the paper places the initial      */
/* Gaussians from an FBP volume, Fig. 4 caption).  Voxels above             */
/* thresh_frac * max(f) are drawn with probability proportional to f, with  */
/* replacement: sample i takes the first voxel v (x fastest) whose          */
/* cumulative weight exceeds u_i0 * W.  Its mean is the voxel centre plus   */
/* (u_i1..3 - 1/2) voxel, isotropic scale `scale`, identity rotation and    */
/* density f(v).  uniforms [n][4] in [0, 1).  Returns the number of voxels  */
/* above the threshold.                                                     */
/* ------------------------------------------------------------------------ */
int64_t orc_init_from_volume(const float *f, const int32_t dims[3], const double glo[3],
                             const double inv_h[3], double thresh_frac, int64_t n,
                             const double *uniforms, double scale, double *mu, double *sc,
                             double *quat, double *rho, int64_t *voxel)
{
    int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    double mx = -INFINITY;
    for (int64_t v = 0; v < nvox; ++v) if (f[v] > mx) mx = f[v];
    double tau = thresh_frac * mx;
    double *cdf = malloc(sizeof(double) * (size_t)nvox);
    double run = 0.0;
    int64_t above = 0;
    for (int64_t v = 0; v < nvox; ++v) {
        if ((double)f[v] > tau) { run += (double)f[v]; ++above; }
        cdf[v] = run;
    }
    for (int64_t i = 0; i < n; ++i) {
        double target = uniforms[4 * i] * run;
        int64_t lo = 0, hi = nvox - 1;  /* first v with cdf[v] > target */
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        int64_t v = lo;
        voxel[i] = v;
        int64_t x = v % dims[0], y = (v / dims[0]) % dims[1], z = v / ((int64_t)dims[0] * dims[1]);
        int64_t idx[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            mu[3 * i + a] = glo[a] + (idx[a] + 0.5 + (uniforms[4 * i + 1 + a] - 0.5)) / inv_h[a];
            sc[3 * i + a] = scale;
        }
        quat[4 * i] = 1.0; quat[4 * i + 1] = quat[4 * i + 2] = quat[4 * i + 3] = 0.0;
        rho[i] = (double)f[v];
    }
    free(cdf);
    return above;
}
