// The paper's full objective (sec. 4.3; weights in App. D.1):
//   L = w1 L1(P_hat, P) + w2 L_SSIM(P_hat, P) + w3 L_TV(V)
// L1 = mean |P_hat - P|; L_SSIM = 1 - mean SSIM over every view and pixel
// (App. C.2 formula; 11 x 11 Gaussian window, sigma 1.5, normalised, zero
// padding outside the detector, C1 = (0.01 R)^2, C2 = (0.03 R)^2 with
// R = max P); L_TV = mean over voxels of the absolute forward differences
// along the three axes.
//
// SSIM gradient.  With the local moments m1 = G*x, my = G*y, m2 = G*x^2,
// mxy = G*xy and S = A B / (C D) (A = 2 m1 my + C1, B = 2 (mxy - m1 my) + C2,
// C = m1^2 + my^2 + C1, D = m2 - m1^2 + G*y^2 - my^2 + C2):
//   dS/dm1 = S (2my/A - 2my/B - 2m1/C + 2m1/D),  dS/dm2 = -S/D,  dS/dmxy = 2S/B,
//   dL_SSIM/dx = -(1/M) [G*(dS/dm1) + 2x G*(dS/dm2) + y G*(dS/dmxy)]
// (the window is symmetric, so blurring is its own adjoint).  Variances are
// differences of second moments of line integrals of order 10, which cancel
// in binary32, so the moments and the SSIM terms are binary64.  The three
// maps (dS/dm1, dS/dm2, dS/dmxy, order 1/R) are stored and blurred in
// binary32: they need no cancellation, and halving their bytes halves the
// traffic between the two passes.
//
// Kernels, all HBM-bound stencils: ssim_fwd (one work-group per 32 x 16
// pixel tile with an 11-pixel halo in LDS: moments, SSIM, the three maps,
// the L1 term and its gradient), ssim_bwd (blur of the maps, SSIM gradient
// added into dL/dP_hat), tv (7-point stencil, gradient added into dL/dV).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr int kWin = 11, kHalf = 5;
constexpr int kTX = 32, kTY = 16;
constexpr int kHX = kTX + 2 * kHalf, kHY = kTY + 2 * kHalf;
constexpr int kObjBlocks = 1024;

struct Win {
    double w[kWin];
};
struct WinF {
    float w[kWin];
};

Win gauss_window() {
    Win W;
    double s = 0.0;
    for (int k = 0; k < kWin; ++k) {
        const double t = k - kHalf;
        W.w[k] = std::exp(-t * t / (2.0 * 1.5 * 1.5));
        s += W.w[k];
    }
    for (int k = 0; k < kWin; ++k) W.w[k] /= s;
    return W;
}

__device__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void max_partial(const float *__restrict__ a, int64_t n, float *__restrict__ part) {
    __shared__ float sh[256];
    float m = -3.0e38f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmaxf(m, a[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void max_final(const float *__restrict__ part, int nb, float range,
                                                 double *__restrict__ rng) {
    __shared__ float sh[256];
    float m = -3.0e38f;
    for (int i = threadIdx.x; i < nb; i += 256) m = fmaxf(m, part[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *rng = range > 0.0f ? (double)range : (double)sh[0];
}

// grid (tiles_u, tiles_v, n_views)
__global__ __launch_bounds__(256) void ssim_fwd(const float *__restrict__ x, const float *__restrict__ y, int nv,
                                                int nu, Win W, const double *__restrict__ rng, float g1,
                                                float *__restrict__ maps, int64_t M, float *__restrict__ dproj,
                                                double *__restrict__ part) {
    __shared__ float sx[kHY][kHX], sy[kHY][kHX];
    __shared__ double hs[5][kHY][kTX];
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int j = blockIdx.z;
    const int u0 = blockIdx.x * kTX - kHalf, v0 = blockIdx.y * kTY - kHalf;
    const float *xv = x + (int64_t)j * nv * nu, *yv = y + (int64_t)j * nv * nu;
    for (int e = t; e < kHY * kHX; e += 256) {
        const int r = e / kHX, c = e - r * kHX;
        const int iv = v0 + r, iu = u0 + c;
        const bool in = iv >= 0 && iu >= 0 && iv < nv && iu < nu;
        sx[r][c] = in ? xv[(int64_t)iv * nu + iu] : 0.0f;
        sy[r][c] = in ? yv[(int64_t)iv * nu + iu] : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < kHY * kTX; e += 256) {
        const int r = e / kTX, c = e - r * kTX;
        double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const double a = sx[r][c + k], b = sy[r][c + k], w = W.w[k];
            m[0] += w * a;
            m[1] += w * b;
            m[2] += w * a * a;
            m[3] += w * b * b;
            m[4] += w * a * b;
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) hs[q][r][c] = m[q];
    }
    __syncthreads();
    const double R = *rng;
    const double C1 = (0.01 * R) * (0.01 * R), C2 = (0.03 * R) * (0.03 * R);
    double s_abs = 0.0, s_ssim = 0.0;
    for (int e = t; e < kTY * kTX; e += 256) {
        const int r = e / kTX, c = e - r * kTX;
        const int iv = v0 + kHalf + r, iu = u0 + kHalf + c;
        if (iv >= nv || iu >= nu) continue;
        double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kWin; ++k)
#pragma unroll
            for (int q = 0; q < 5; ++q) m[q] += W.w[k] * hs[q][r + k][c];
        const double mx = m[0], my = m[1];
        const double A = 2.0 * mx * my + C1;
        const double B = 2.0 * (m[4] - mx * my) + C2;
        const double Cc = mx * mx + my * my + C1;
        const double D = (m[2] - mx * mx) + (m[3] - my * my) + C2;
        const double S = A * B / (Cc * D);
        const int64_t pix = ((int64_t)j * nv + iv) * nu + iu;
        maps[pix] = (float)(S * (2.0 * my / A - 2.0 * my / B - 2.0 * mx / Cc + 2.0 * mx / D));
        maps[M + pix] = (float)(-S / D);
        maps[2 * M + pix] = (float)(2.0 * S / B);
        const float res = sx[r + kHalf][c + kHalf] - sy[r + kHalf][c + kHalf];
        dproj[pix] = res > 0.0f ? g1 : (res < 0.0f ? -g1 : 0.0f);
        s_abs += fabs((double)res);
        s_ssim += S;
    }
    s_abs = block_sum(s_abs, red);
    s_ssim = block_sum(s_ssim, red);
    if (t == 0) {
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[2 * b] = s_abs;
        part[2 * b + 1] = s_ssim;
    }
}

// dproj += g2 * (G*a + 2 x G*b + y G*c), g2 = -w2 / M
__global__ __launch_bounds__(256) void ssim_bwd(const float *__restrict__ maps, int64_t M, const float *__restrict__ x,
                                                const float *__restrict__ y, int nv, int nu, WinF W, double g2,
                                                float *__restrict__ dproj) {
    __shared__ float sm[3][kHY][kHX];
    __shared__ float hs[3][kHY][kTX];
    const int t = threadIdx.x;
    const int j = blockIdx.z;
    const int u0 = blockIdx.x * kTX - kHalf, v0 = blockIdx.y * kTY - kHalf;
    const int64_t base = (int64_t)j * nv * nu;
    for (int e = t; e < kHY * kHX; e += 256) {
        const int r = e / kHX, c = e - r * kHX;
        const int iv = v0 + r, iu = u0 + c;
        const bool in = iv >= 0 && iu >= 0 && iv < nv && iu < nu;
        const int64_t pix = base + (int64_t)iv * nu + iu;
#pragma unroll
        for (int q = 0; q < 3; ++q) sm[q][r][c] = in ? maps[q * M + pix] : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < kHY * kTX; e += 256) {
        const int r = e / kTX, c = e - r * kTX;
        float m[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < kWin; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q) m[q] += W.w[k] * sm[q][r][c + k];
#pragma unroll
        for (int q = 0; q < 3; ++q) hs[q][r][c] = m[q];
    }
    __syncthreads();
    for (int e = t; e < kTY * kTX; e += 256) {
        const int r = e / kTX, c = e - r * kTX;
        const int iv = v0 + kHalf + r, iu = u0 + kHalf + c;
        if (iv >= nv || iu >= nu) continue;
        float m[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < kWin; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q) m[q] += W.w[k] * hs[q][r + k][c];
        const int64_t pix = base + (int64_t)iv * nu + iu;
        const double xv = x[pix], yv = y[pix];
        dproj[pix] = (float)((double)dproj[pix] + g2 * ((double)m[0] + 2.0 * xv * (double)m[1] + yv * (double)m[2]));
    }
}

// loss[0] = w1 L1 + w2 L_SSIM, loss[1] = L1, loss[2] = L_SSIM
__global__ __launch_bounds__(256) void ssim_final(const double *__restrict__ part, int nb, int64_t M, float w1,
                                                  float w2, float *__restrict__ loss) {
    __shared__ double red[256];
    double a = 0.0, s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        s += part[2 * i + 1];
    }
    a = block_sum(a, red);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        const double l1 = a / (double)M, ls = 1.0 - s / (double)M;
        loss[0] = (float)((double)w1 * l1 + (double)w2 * ls);
        loss[1] = (float)l1;
        loss[2] = (float)ls;
    }
}

// dV += w3/N * d(sum |forward differences|)/dV; block partials of the sum.
__global__ __launch_bounds__(256) void tv_kernel(const float *__restrict__ V, int nx, int ny, int nz, float g3,
                                                 float *__restrict__ dV, double *__restrict__ part) {
    __shared__ double red[256];
    const int64_t N = (int64_t)nx * ny * nz, plane = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const int64_t z = i / plane, rem = i - z * plane;
        const int y = (int)(rem / nx), x = (int)(rem - (int64_t)y * nx);
        const float v = V[i];
        float g = 0.0f;
        const int64_t step[3] = {1, nx, plane};
        const bool hi[3] = {x + 1 < nx, y + 1 < ny, z + 1 < nz};
        const bool lo[3] = {x > 0, y > 0, z > 0};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (hi[a]) {
                const float d = V[i + step[a]] - v;
                acc += fabs((double)d);
                g -= d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            }
            if (lo[a]) {
                const float d = v - V[i - step[a]];
                g += d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            }
        }
        dV[i] += g3 * g;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void tv_final(const double *__restrict__ part, int nb, int64_t N,
                                                float *__restrict__ loss) {
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) a += part[i];
    a = block_sum(a, red);
    if (threadIdx.x == 0) *loss = (float)(a / (double)N);
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_projection_loss_workspace(int32_t n_views, int32_t nv, int32_t nu) {
    if (n_views < 1 || nv < 1 || nu < 1) return 0;
    const int64_t M = (int64_t)n_views * nv * nu;
    const int64_t tiles = (int64_t)((nu + kTX - 1) / kTX) * ((nv + kTY - 1) / kTY) * n_views;
    Carver c(nullptr);
    c.take<float>(3 * M);
    c.take<double>(2 * tiles);
    c.take<float>(kObjBlocks);
    c.take<double>(1);
    return c.off;
}

extern "C" dgr_status dgr_projection_loss(const float *proj, const float *target, int32_t n_views, int32_t nv,
                                          int32_t nu, float w_l1, float w_ssim, float range, float *loss,
                                          float *dproj, void *ws, size_t ws_bytes, void *stream) {
    DGR_CHECK(proj && target && loss && dproj && ws, "null pointer argument");
    DGR_CHECK(n_views >= 1 && nv >= 1 && nu >= 1 && n_views <= 65535 && nv <= 65535,
              "sizes must be >= 1 (n_views, nv <= 65535)");
    DGR_CHECK(std::isfinite(w_l1) && std::isfinite(w_ssim) && std::isfinite(range), "weights must be finite");
    if (ws_bytes < dgr_projection_loss_workspace(n_views, nv, nu)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = as_stream(stream);
    const int64_t M = (int64_t)n_views * nv * nu;
    const dim3 grid((unsigned)((nu + kTX - 1) / kTX), (unsigned)((nv + kTY - 1) / kTY), (unsigned)n_views);
    const int64_t tiles = (int64_t)grid.x * grid.y * grid.z;
    Carver c(ws);
    float *maps = c.take<float>(3 * M);
    double *part = c.take<double>(2 * tiles);
    float *mpart = c.take<float>(kObjBlocks);
    double *rng = c.take<double>(1);
    const Win W = gauss_window();
    const int mb = (int)std::min<int64_t>(kObjBlocks, (M + 255) / 256);
    max_partial<<<mb, 256, 0, st>>>(target, M, mpart);
    DGR_LAUNCH_CHECK();
    max_final<<<1, 256, 0, st>>>(mpart, mb, range, rng);
    DGR_LAUNCH_CHECK();
    ssim_fwd<<<grid, 256, 0, st>>>(proj, target, nv, nu, W, rng, (float)((double)w_l1 / (double)M), maps, M, dproj,
                                   part);
    DGR_LAUNCH_CHECK();
    WinF Wf;
    for (int k = 0; k < kWin; ++k) Wf.w[k] = (float)W.w[k];
    ssim_bwd<<<grid, 256, 0, st>>>(maps, M, proj, target, nv, nu, Wf, -(double)w_ssim / (double)M, dproj);
    DGR_LAUNCH_CHECK();
    ssim_final<<<1, 256, 0, st>>>(part, (int)tiles, M, w_l1, w_ssim, loss);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_tv_workspace(void) { return align_up(sizeof(double) * kObjBlocks); }

extern "C" dgr_status dgr_tv(const float *volume, const dgr_grid *grid, float w_tv, float *loss, float *dvolume,
                             void *ws, size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    DGR_CHECK(volume && loss && dvolume && ws, "null pointer argument");
    DGR_CHECK(std::isfinite(w_tv), "w_tv must be finite");
    if (ws_bytes < dgr_tv_workspace()) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t N = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    double *part = static_cast<double *>(ws);
    const int nb = (int)std::min<int64_t>(kObjBlocks, (N + 255) / 256);
    tv_kernel<<<nb, 256, 0, st>>>(volume, grid->dims[0], grid->dims[1], grid->dims[2], (float)((double)w_tv / (double)N),
                                  dvolume, part);
    DGR_LAUNCH_CHECK();
    tv_final<<<1, 256, 0, st>>>(part, nb, N, loss);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
