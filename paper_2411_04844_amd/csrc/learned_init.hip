// Learned initialisation, around the U-Net: the input pooling, the training
// targets built from a converged Gaussian set, and the Gaussian set drawn from
// the network's output fields.
//
// Training targets on a grid (per voxel v, from the converged parameters of a
// plain DGR run and their voxelization V*):
//   t_d = V*(v) / input_scale
//   t_o = 1 if the mean of some Gaussian lies in v, else 0
//   t_s = mean over those Gaussians of log(geometric-mean scale / voxel size)
// The network's output (o_d, o_s, o_o) is drawn from the same way the plain
// initialisation draws from an FDK volume (inverse CDF with replacement): the
// voxel weight is sigmoid(o_o), the mean is jittered uniformly over the
// voxel, the isotropic scale is exp(o_s) voxels (clamped to [0.25, 8]) and
// the density is max(o_d, 0) * input_scale, before the least-squares
// density scale fitted to the projections.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr double kLogFix = 16777216.0;  // 2^24: fixed-point scale of the log-scale sums

__global__ __launch_bounds__(256) void pool2_f32(const float *__restrict__ in, int nx, int ny, int nz,
                                                 float *__restrict__ out) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const int64_t n = (int64_t)cx * cy * cz;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % cx), y = (int)((i / cx) % cy), z = (int)(i / ((int64_t)cx * cy));
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const int64_t v = ((int64_t)(2 * z + (k >> 2)) * ny + (2 * y + ((k >> 1) & 1))) * nx + 2 * x + (k & 1);
        s += in[v];
    }
    out[i] = 0.125f * s;
}

__global__ __launch_bounds__(256) void zero_fields(unsigned *__restrict__ cnt, long long *__restrict__ lsum,
                                                   int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    cnt[i] = 0u;
    lsum[i] = 0ll;
}

__global__ __launch_bounds__(256) void scatter_means(const float *__restrict__ mu, const float *__restrict__ scale,
                                                     int64_t n, DevGrid g, unsigned *__restrict__ cnt,
                                                     long long *__restrict__ lsum) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int idx[3];
    double ls = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double u = ((double)mu[3 * i + a] - (double)g.lo[a]) * (double)g.inv_h[a];
        if (!(u >= 0.0 && u < (double)(a == 0 ? g.nx : a == 1 ? g.ny : g.nz))) return;
        idx[a] = (int)u;
        ls += log(fmax((double)scale[3 * i + a] * (double)g.inv_h[a], 1e-30));
    }
    const int64_t v = ((int64_t)idx[2] * g.ny + idx[1]) * g.nx + idx[0];
    atomicAdd(&cnt[v], 1u);
    atomicAdd(reinterpret_cast<unsigned long long *>(&lsum[v]),
              (unsigned long long)__double2ll_rn(ls / 3.0 * kLogFix));
}

__global__ __launch_bounds__(256) void finish_targets(const float *__restrict__ vol, int64_t n, float inv_in,
                                                      const unsigned *__restrict__ cnt,
                                                      const long long *__restrict__ lsum,
                                                      float *__restrict__ tgt) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const unsigned c = cnt[v];
    tgt[3 * v] = vol[v] * inv_in;
    tgt[3 * v + 1] = c ? (float)((double)lsum[v] / kLogFix / (double)c) : 0.0f;
    tgt[3 * v + 2] = c ? 1.0f : 0.0f;
}

__global__ __launch_bounds__(256) void occupancy_weights(const float *__restrict__ out, int64_t n,
                                                         float *__restrict__ w) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    w[v] = 1.0f / (1.0f + expf(-out[3 * v + 2]));
}

__global__ __launch_bounds__(256) void draw_from_fields(const double *__restrict__ excl, const double *__restrict__ W,
                                                        const float *__restrict__ out, int64_t nvox, DevGrid g,
                                                        int64_t n, const float *__restrict__ uni, float in_scale,
                                                        float *__restrict__ mu, float *__restrict__ sc,
                                                        float *__restrict__ quat, float *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double target = (double)uni[4 * i] * *W;
    int64_t lo = 1, hi = nvox;  // first j with excl[j] > target (excl[nvox] = W)
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const double c = mid < nvox ? excl[mid] : *W;
        if (c > target) hi = mid;
        else lo = mid + 1;
    }
    const int64_t v = lo - 1;
    const int64_t idx[3] = {v % g.nx, (v / g.nx) % g.ny, v / ((int64_t)g.nx * g.ny)};
    const float s_vox = fminf(fmaxf(expf(out[3 * v + 1]), 0.25f), 8.0f);
    for (int a = 0; a < 3; ++a) {
        mu[3 * i + a] = (float)(g.lo[a] + ((double)idx[a] + 0.5 + ((double)uni[4 * i + 1 + a] - 0.5)) / (double)g.inv_h[a]);
        sc[3 * i + a] = s_vox / g.inv_h[a];
    }
    quat[4 * i] = 1.0f;
    quat[4 * i + 1] = quat[4 * i + 2] = quat[4 * i + 3] = 0.0f;
    rho[i] = fmaxf(out[3 * v], 0.0f) * in_scale;
}

unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" dgr_status dgr_pool2_f32(const float *in, const int32_t dims[3], float *out, void *stream) {
    DGR_CHECK(in && out && dims, "null pointer argument");
    DGR_CHECK(dims[0] >= 2 && dims[1] >= 2 && dims[2] >= 2 && dims[0] % 2 == 0 && dims[1] % 2 == 0 &&
                  dims[2] % 2 == 0 && dims[0] <= 16384 && dims[1] <= 16384 && dims[2] <= 16384,
              "dims must be even and in [2, 16384]");
    const int64_t n = (int64_t)(dims[0] / 2) * (dims[1] / 2) * (dims[2] / 2);
    pool2_f32<<<nblk(n), 256, 0, as_stream(stream)>>>(in, dims[0], dims[1], dims[2], out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_unet_targets_workspace(const dgr_grid *grid) {
    if (check_grid(grid) != DGR_OK) return 0;
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(nullptr);
    c.take<unsigned>(nvox);
    c.take<long long>(nvox);
    return c.off;
}

extern "C" dgr_status dgr_unet_targets(const float *mu, const float *scale, int64_t n, const dgr_grid *grid,
                                       const float *volume, float input_scale, float *target, void *ws,
                                       size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    DGR_CHECK(volume && target && ws && (n == 0 || (mu && scale)), "null pointer argument");
    DGR_CHECK(std::isfinite(input_scale) && input_scale > 0.0f, "input_scale must be > 0");
    if (ws_bytes < dgr_unet_targets_workspace(grid)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(ws);
    unsigned *cnt = c.take<unsigned>(nvox);
    long long *lsum = c.take<long long>(nvox);
    zero_fields<<<nblk(nvox), 256, 0, st>>>(cnt, lsum, nvox);
    DGR_LAUNCH_CHECK();
    if (n > 0) {
        scatter_means<<<nblk(n), 256, 0, st>>>(mu, scale, n, dev_grid(grid), cnt, lsum);
        DGR_LAUNCH_CHECK();
    }
    finish_targets<<<nblk(nvox), 256, 0, st>>>(volume, nvox, 1.0f / input_scale, cnt, lsum, target);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_init_from_unet_workspace(const dgr_grid *grid) {
    if (check_grid(grid) != DGR_OK) return 0;
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(nullptr);
    c.take<float>(nvox);
    c.take<double>(nvox);
    c.take<double>(scan_f64_blocks(nvox));
    c.take<double>(1);
    return c.off;
}

extern "C" dgr_status dgr_init_from_unet(const float *out, const dgr_grid *grid, int64_t n, const float *uniforms,
                                         float input_scale, float *mu, float *scale, float *quat, float *density,
                                         void *ws, size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if (n == 0) return DGR_OK;
    DGR_CHECK(out && uniforms && mu && scale && quat && density && ws, "null pointer argument");
    DGR_CHECK(std::isfinite(input_scale) && input_scale > 0.0f, "input_scale must be > 0");
    if (ws_bytes < dgr_init_from_unet_workspace(grid)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(ws);
    float *w = c.take<float>(nvox);
    double *excl = c.take<double>(nvox);
    double *blk = c.take<double>(scan_f64_blocks(nvox));
    double *W = c.take<double>(1);
    occupancy_weights<<<nblk(nvox), 256, 0, st>>>(out, nvox, w);
    DGR_LAUNCH_CHECK();
    if ((s = exclusive_scan_f64(w, excl, nvox, blk, W, st)) != DGR_OK) return s;
    draw_from_fields<<<nblk(n), 256, 0, st>>>(excl, W, out, nvox, dev_grid(grid), n, uniforms, input_scale, mu,
                                              scale, quat, density);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
