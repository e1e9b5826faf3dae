// Per-Gaussian preparation: truncation box (bit-exact binary32 definition),
// exponent coefficients in voxel units, floored position and residual, and the
// number of 8^3 tiles the box touches.
//
// Paper: sec. 4.1 (Gaussian Effect Confinement, Discretize and Align) and the
// set-up steps of Alg. 1: the floored anchor floor(mu), the residual
// Delta mu = mu - floor(mu), and the validity clamp to the volume.
#include "internal.h"

namespace dgr {
namespace {

#pragma clang fp contract(off)

// One correctly rounded binary32 operation, computed in binary64 and rounded
// once.  binary64 carries more than 2*24+2 bits, so the double rounding is
// innocuous for +, -, *, / and sqrt: the result equals the binary32 IEEE
// operation, whatever the compiler does with float division or sqrt.
__device__ __forceinline__ float f_add(float a, float b) { return (float)((double)a + (double)b); }
__device__ __forceinline__ float f_sub(float a, float b) { return (float)((double)a - (double)b); }
__device__ __forceinline__ float f_mul(float a, float b) { return (float)((double)a * (double)b); }
__device__ __forceinline__ float f_div(float a, float b) { return (float)((double)a / (double)b); }
__device__ __forceinline__ float f_sqrt(float a) { return (float)__dsqrt_rn((double)a); }

// Rotation of the normalised quaternion, binary32 definition of the box.
__device__ void rot32(float w, float x, float y, float z, float R[3][3]) {
    float n2 = f_add(f_add(f_add(f_mul(w, w), f_mul(x, x)), f_mul(y, y)), f_mul(z, z));
    if (n2 == 0.0f) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = (i == j) ? 1.0f : 0.0f;
        return;
    }
    float m = f_sqrt(n2);
    float a = f_div(w, m), b = f_div(x, m), c = f_div(y, m), d = f_div(z, m);
    R[0][0] = f_sub(1.0f, f_mul(2.0f, f_add(f_mul(c, c), f_mul(d, d))));
    R[0][1] = f_mul(2.0f, f_sub(f_mul(b, c), f_mul(a, d)));
    R[0][2] = f_mul(2.0f, f_add(f_mul(b, d), f_mul(a, c)));
    R[1][0] = f_mul(2.0f, f_add(f_mul(b, c), f_mul(a, d)));
    R[1][1] = f_sub(1.0f, f_mul(2.0f, f_add(f_mul(b, b), f_mul(d, d))));
    R[1][2] = f_mul(2.0f, f_sub(f_mul(c, d), f_mul(a, b)));
    R[2][0] = f_mul(2.0f, f_sub(f_mul(b, d), f_mul(a, c)));
    R[2][1] = f_mul(2.0f, f_add(f_mul(c, d), f_mul(a, b)));
    R[2][2] = f_sub(1.0f, f_mul(2.0f, f_add(f_mul(b, b), f_mul(c, c))));
}

__global__ __launch_bounds__(256) void prep_kernel(
    const float *__restrict__ mu, const float *__restrict__ scale, const float *__restrict__ quat,
    const float *__restrict__ density, int64_t n, DevGrid g, float k_sigma, int box_half,
    GaussRec *__restrict__ rec, uint32_t *__restrict__ tile_count, int32_t *__restrict__ box_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float m3[3] = {mu[3 * i], mu[3 * i + 1], mu[3 * i + 2]};
    const float s3[3] = {scale[3 * i], scale[3 * i + 1], scale[3 * i + 2]};
    const float q4[4] = {quat[4 * i], quat[4 * i + 1], quat[4 * i + 2], quat[4 * i + 3]};
    const int dims[3] = {g.nx, g.ny, g.nz};

    // ---- truncation box (binary32 definition) ----
    float R[3][3];
    rot32(q4[0], q4[1], q4[2], q4[3], R);
    int lo[3], hi[3];
    bool empty = false;
    for (int k = 0; k < 3; ++k) {
        float u = f_sub(f_mul(f_sub(m3[k], g.lo[k]), g.inv_h[k]), 0.5f);
        float flo, fhi;
        if (k_sigma > 0.0f) {
            float a0 = f_mul(R[k][0], s3[0]);
            float a1 = f_mul(R[k][1], s3[1]);
            float a2 = f_mul(R[k][2], s3[2]);
            float skk = f_add(f_add(f_mul(a0, a0), f_mul(a1, a1)), f_mul(a2, a2));
            float r = f_mul(f_mul(k_sigma, f_sqrt(skk)), g.inv_h[k]);
            flo = ceilf(f_sub(u, r));
            fhi = floorf(f_add(u, r));
        } else {
            float f = floorf(u);
            flo = f_sub(f, (float)box_half);
            fhi = f_add(f, (float)box_half);
        }
        float D = (float)dims[k];
        if (flo < 0.0f) flo = 0.0f;
        if (flo > D) flo = D;
        if (fhi > D - 1.0f) fhi = D - 1.0f;
        if (fhi < -1.0f) fhi = -1.0f;
        lo[k] = (int)flo;
        hi[k] = (int)fhi;
        empty |= lo[k] > hi[k];
    }
    if (box_out) {
        for (int k = 0; k < 3; ++k) {
            box_out[6 * i + k] = lo[k];
            box_out[6 * i + 3 + k] = hi[k];
        }
    }
    if (tile_count) {
        uint32_t c = 0;
        if (!empty)
            c = (uint32_t)((hi[0] >> 3) - (lo[0] >> 3) + 1) * (uint32_t)((hi[1] >> 3) - (lo[1] >> 3) + 1) *
                (uint32_t)((hi[2] >> 3) - (lo[2] >> 3) + 1);
        tile_count[i] = c;
    }
    if (!rec) return;

    // ---- shape in binary64: Q = R diag(s^-2) R^T, in voxel units ----
    double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
    double n2 = w * w + x * x + y * y + z * z;
    double Rd[3][3];
    if (n2 == 0.0) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Rd[a][b] = (a == b) ? 1.0 : 0.0;
    } else {
        double inv = 1.0 / sqrt(n2);
        w *= inv; x *= inv; y *= inv; z *= inv;
        Rd[0][0] = 1 - 2 * (y * y + z * z); Rd[0][1] = 2 * (x * y - w * z); Rd[0][2] = 2 * (x * z + w * y);
        Rd[1][0] = 2 * (x * y + w * z); Rd[1][1] = 1 - 2 * (x * x + z * z); Rd[1][2] = 2 * (y * z - w * x);
        Rd[2][0] = 2 * (x * z - w * y); Rd[2][1] = 2 * (y * z + w * x); Rd[2][2] = 1 - 2 * (x * x + y * y);
    }
    double il[3];
    for (int j = 0; j < 3; ++j) il[j] = 1.0 / ((double)s3[j] * (double)s3[j]);
    double Q[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = Rd[a][0] * Rd[b][0] * il[0] + Rd[a][1] * Rd[b][1] * il[1] + Rd[a][2] * Rd[b][2] * il[2];
            Q[a][b] = acc / ((double)g.inv_h[a] * (double)g.inv_h[b]);
        }
    const double L2E = 1.4426950408889634;  // log2(e): exp(-x/2) = exp2(-x/2 * log2 e)
    GaussRec r;
    for (int a = 0; a < 3; ++a) {
        double u = ((double)m3[a] - (double)g.lo[a]) * (double)g.inv_h[a] - 0.5;
        double f = floor(u);
        float uf = (float)(u - f);
        if (uf >= 1.0f) {  // residual rounded up to 1
            f += 1.0;
            uf = 0.0f;
        }
        r.ui[a] = (int32_t)f;
        r.uf[a] = uf;
        r.box[a] = ((uint32_t)lo[a] & 0xffffu) | ((uint32_t)(hi[a] & 0xffff) << 16);
    }
    r.rho = density[i];
    r.k00 = (float)(-0.5 * L2E * Q[0][0]);
    r.k11 = (float)(-0.5 * L2E * Q[1][1]);
    r.k22 = (float)(-0.5 * L2E * Q[2][2]);
    r.k01 = (float)(-L2E * Q[0][1]);
    r.k02 = (float)(-L2E * Q[0][2]);
    r.k12 = (float)(-L2E * Q[1][2]);
    rec[i] = r;
}

}  // namespace

dgr_status launch_prep(const float *mu, const float *scale, const float *quat,
                       const float *density, int64_t n, const dgr_grid *grid,
                       const dgr_trunc *trunc, GaussRec *rec, uint32_t *tile_count,
                       int32_t *box_out, hipStream_t st) {
    if (n == 0) return DGR_OK;
    int64_t blocks = (n + 255) / 256;
    prep_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(
        mu, scale, quat, density, n, dev_grid(grid), trunc->k_sigma, trunc->box_half, rec,
        tile_count, box_out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

}  // namespace dgr

using namespace dgr;

extern "C" dgr_status dgr_bbox(const float *mu, const float *scale, const float *quat, int64_t n,
                               const dgr_grid *grid, const dgr_trunc *trunc, int32_t *box,
                               void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_trunc(trunc)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n = %lld out of range", (long long)n);
    if (n == 0) return DGR_OK;
    DGR_CHECK(mu && scale && quat && box, "null pointer argument");
    return launch_prep(mu, scale, quat, nullptr, n, grid, trunc, nullptr, nullptr, box,
                       as_stream(stream));
}
