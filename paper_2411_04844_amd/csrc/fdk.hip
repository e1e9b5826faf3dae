// FDK reconstruction, PSNR and the FDK-driven initialisation of Gaussians.
//
// The paper places its initial Gaussians from an FBP/FDK volume (Fig. 4
// caption; FDK is also its baseline row in Tab. 1) and reports PSNR
// (App. C.1).  FDK here is the textbook Feldkamp algorithm for a full circular
// cone-beam scan on a flat detector: cosine weighting, a Ram-Lak ramp filter
// along each detector row, and a voxel-driven weighted backprojection.  For a
// stack of fan-beam slices (each row with its own source) the same three
// steps, taken with the row's source, are 2-D fan-beam FBP of every slice.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Per-view frame: detector normal n (source side -> detector), D = (det - s).n,
// R = -s.n (isocentre depth), e_u / |e_u|^2 and e_v / |e_v|^2.  Fan beam:
// the row position of a point x is (x - s).m_n with m_n = m / (e_v.m),
// m = (det - s) x e_u (zero if e_v lies in the fan plane), and the row's
// source is s + b e_v; D is the same for every row.
struct FdkView {
    double s[3], det[3], n[3], eu_n[3], ev_n[3], ev[3], m_n[3];
    double D, R, tau;  // tau: detector pitch along u at the isocentre
};

__global__ void fdk_frames(const float *__restrict__ views, int n_views, FdkView *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_views) return;
    const float *v = views + 12 * (int64_t)j;
    FdkView f;
    double eu[3], ev[3];
    for (int a = 0; a < 3; ++a) {
        f.s[a] = v[a];
        f.det[a] = v[3 + a];
        eu[a] = v[6 + a];
        ev[a] = v[9 + a];
    }
    double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) n[a] /= nn;
    double D = (f.det[0] - f.s[0]) * n[0] + (f.det[1] - f.s[1]) * n[1] + (f.det[2] - f.s[2]) * n[2];
    if (D < 0.0) {
        for (int a = 0; a < 3; ++a) n[a] = -n[a];
        D = -D;
    }
    const double uu = eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2];
    const double vv = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
    const double w[3] = {f.det[0] - f.s[0], f.det[1] - f.s[1], f.det[2] - f.s[2]};
    const double m[3] = {w[1] * eu[2] - w[2] * eu[1], w[2] * eu[0] - w[0] * eu[2], w[0] * eu[1] - w[1] * eu[0]};
    const double em = ev[0] * m[0] + ev[1] * m[1] + ev[2] * m[2];
    for (int a = 0; a < 3; ++a) {
        f.n[a] = n[a];
        f.eu_n[a] = eu[a] / uu;
        f.ev_n[a] = ev[a] / vv;
        f.ev[a] = ev[a];
        f.m_n[a] = em != 0.0 ? m[a] / em : 0.0;
    }
    f.D = D;
    f.R = -(f.s[0] * n[0] + f.s[1] * n[1] + f.s[2] * n[2]);
    f.tau = sqrt(uu) * f.R / D;
    out[j] = f;
}

// One work-group per (detector row, view): cosine weight, then the discrete
// Ram-Lak filter q(i) = (1/tau) [p(i)/4 - sum_{k odd} (p(i-k) + p(i+k)) / (k^2 pi^2)].
// The row and the sum are kept in binary64: the taps cancel strongly inside
// a uniform object.  Only q is rounded to binary32.
__global__ __launch_bounds__(256) void fdk_filter(const float *__restrict__ proj, const float *__restrict__ views,
                                                  const FdkView *__restrict__ frames, int nu, int nv, int fan,
                                                  float *__restrict__ q) {
    extern __shared__ double row[];
    const int iv = blockIdx.x, j = blockIdx.y;
    const FdkView &f = frames[j];
    const float *v = views + 12 * (int64_t)j;
    const float *src = proj + ((int64_t)j * nv + iv) * nu;
    // fan beam: the row's source moves with the row, so the source-to-pixel
    // vector has no e_v part
    const double av = fan ? 0.0 : (double)iv - 0.5 * (nv - 1);
    for (int i = threadIdx.x; i < nu; i += 256) {
        const double au = (double)i - 0.5 * (nu - 1);
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double d = (double)v[3 + a] + au * (double)v[6 + a] + av * (double)v[9 + a] - f.s[a];
            r2 += d * d;
        }
        row[i] = (double)src[i] * f.D / sqrt(r2);
    }
    __syncthreads();
    const double c = 1.0 / (kPi * kPi);
    float *dst = q + ((int64_t)j * nv + iv) * nu;
    for (int i = threadIdx.x; i < nu; i += 256) {
        double acc = 0.0;
        for (int k = 1; k < nu; k += 2) {
            const double l = i - k >= 0 ? row[i - k] : 0.0;
            const double r = i + k < nu ? row[i + k] : 0.0;
            acc += (c / ((double)k * (double)k)) * (l + r);
        }
        dst[i] = (float)((0.25 * row[i] - acc) / f.tau);
    }
}

// Voxel-driven backprojection: f(x) = (dbeta/2) sum_j (R/U)^2 q_j(a, b) / ell,
// U = (x - s).n, (a, b) the detector position of the ray s -> x (binary64
// geometry), q bilinear and zero outside the detector.  Fan beam: s is the
// source of the (continuous) row b that holds x, and R = -s.n that row's.
__global__ __launch_bounds__(256) void fdk_backproject(const float *__restrict__ q,
                                                       const FdkView *__restrict__ frames, int n_views,
                                                       int nu, int nv, int fan, DevGrid g, double weight,
                                                       float *__restrict__ V) {
    const int64_t total = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t z = i / ((int64_t)g.nx * g.ny), rem = i - z * (int64_t)g.nx * g.ny;
        const int64_t y = rem / g.nx, xi = rem - y * g.nx;
        const double x[3] = {g.lo[0] + (xi + 0.5) / (double)g.inv_h[0], g.lo[1] + (y + 0.5) / (double)g.inv_h[1],
                             g.lo[2] + (z + 0.5) / (double)g.inv_h[2]};
        double acc = 0.0;
        for (int j = 0; j < n_views; ++j) {
            const FdkView &f = frames[j];
            double sv[3];
            if (fan) {
                const double b = (x[0] - f.s[0]) * f.m_n[0] + (x[1] - f.s[1]) * f.m_n[1] + (x[2] - f.s[2]) * f.m_n[2];
                for (int a = 0; a < 3; ++a) sv[a] = f.s[a] + b * f.ev[a];
            } else {
                for (int a = 0; a < 3; ++a) sv[a] = f.s[a];
            }
            const double r[3] = {x[0] - sv[0], x[1] - sv[1], x[2] - sv[2]};
            const double U = r[0] * f.n[0] + r[1] * f.n[1] + r[2] * f.n[2];
            if (!(U > 0.0)) continue;
            const double t = f.D / U;
            double hit[3];
            for (int a = 0; a < 3; ++a) hit[a] = sv[a] + t * r[a] - f.det[a];
            const double ap = hit[0] * f.eu_n[0] + hit[1] * f.eu_n[1] + hit[2] * f.eu_n[2] + 0.5 * (nu - 1);
            const double bp = hit[0] * f.ev_n[0] + hit[1] * f.ev_n[1] + hit[2] * f.ev_n[2] + 0.5 * (nv - 1);
            const double fa = floor(ap), fb = floor(bp);
            // both taps of an axis outside the detector: nothing to add
            if (!(fa >= -1.0 && fb >= -1.0 && fa <= (double)(nu - 1) && fb <= (double)(nv - 1))) continue;
            const float wa = (float)(ap - fa), wb = (float)(bp - fb);
            const int ia = (int)fa, ib = (int)fb;  // in [-1, nu - 1] x [-1, nv - 1]
            const float *qj = q + (int64_t)j * nv * nu;
            const bool a0 = ia >= 0, a1 = ia + 1 < nu, b0 = ib >= 0, b1 = ib + 1 < nv;
            const float q00 = (a0 && b0) ? qj[(int64_t)ib * nu + ia] : 0.0f;
            const float q10 = (a1 && b0) ? qj[(int64_t)ib * nu + ia + 1] : 0.0f;
            const float q01 = (a0 && b1) ? qj[(int64_t)(ib + 1) * nu + ia] : 0.0f;
            const float q11 = (a1 && b1) ? qj[(int64_t)(ib + 1) * nu + ia + 1] : 0.0f;
            const float lo = fmaf(wa, q10 - q00, q00), hi = fmaf(wa, q11 - q01, q01);
            const double val = (double)fmaf(wb, hi - lo, lo);
            const double Rv = -(sv[0] * f.n[0] + sv[1] * f.n[1] + sv[2] * f.n[2]);
            const double m = Rv / U;
            acc += m * m * val;
        }
        V[i] = (float)(acc * weight);
    }
}

// ---- reductions with a fixed order (block partials, then one block) -------
__device__ double block_sum_d(double v) {
    __shared__ double sh[256];
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

__device__ float block_max_f(float v) {
    __shared__ float sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

constexpr int kRedBlocks = 1024;

// part[b] = (sum (x - gt)^2, max gt) over a grid-stride slice
__global__ __launch_bounds__(256) void psnr_partial(const float *__restrict__ x, const float *__restrict__ gt,
                                                    int64_t n, double *__restrict__ part) {
    double se = 0.0;
    float mx = -3.0e38f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double e = (double)x[i] - (double)gt[i];
        se += e * e;
        mx = fmaxf(mx, gt[i]);
    }
    se = block_sum_d(se);
    mx = block_max_f(mx);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = se;
        part[2 * blockIdx.x + 1] = (double)mx;
    }
}

__global__ __launch_bounds__(256) void psnr_final(const double *__restrict__ part, int nb, int64_t n,
                                                  double *__restrict__ out) {
    double se = 0.0;
    float mx = -3.0e38f;
    for (int b = threadIdx.x; b < nb; b += 256) {
        se += part[2 * b];
        mx = fmaxf(mx, (float)part[2 * b + 1]);
    }
    se = block_sum_d(se);
    mx = block_max_f(mx);
    if (threadIdx.x == 0) {
        const double mse = se / (double)n;
        out[0] = 10.0 * log10((double)mx * (double)mx / mse);
        out[1] = mse;
        out[2] = (double)mx;
    }
}

__global__ __launch_bounds__(256) void max_partial(const float *__restrict__ x, int64_t n, float *__restrict__ part) {
    float mx = -3.0e38f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        mx = fmaxf(mx, x[i]);
    mx = block_max_f(mx);
    if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// weights w = f if f > frac * max(f) else 0
__global__ __launch_bounds__(256) void threshold_weights(const float *__restrict__ f, int64_t n,
                                                         const float *__restrict__ part, int nb, float frac,
                                                         float *__restrict__ w) {
    __shared__ float tau;
    if (threadIdx.x == 0) {
        float mx = -3.0e38f;
        for (int b = 0; b < nb; ++b) mx = fmaxf(mx, part[b]);
        tau = (float)((double)frac * (double)mx);
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = f[i] > tau ? f[i] : 0.0f;
}

// Sample i: the voxel whose cumulative-weight interval holds u_i0 * W (first
// v with cdf_incl[v] > target, cdf_incl[v] = excl[v + 1]), jittered by u_i1..3.
__global__ __launch_bounds__(256) void draw_gaussians(const double *__restrict__ excl, const double *__restrict__ W,
                                                      const float *__restrict__ f, int64_t nvox, DevGrid g,
                                                      int64_t n, const float *__restrict__ uni, float scale,
                                                      float *__restrict__ mu, float *__restrict__ sc,
                                                      float *__restrict__ quat, float *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double target = (double)uni[4 * i] * *W;
    // first j in [1, nvox] with incl(j - 1) = excl[j] > target (excl[nvox] = W)
    int64_t lo = 1, hi = nvox;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const double c = mid < nvox ? excl[mid] : *W;
        if (c > target) hi = mid;
        else lo = mid + 1;
    }
    const int64_t v = lo - 1;
    const int64_t x = v % g.nx, y = (v / g.nx) % g.ny, z = v / ((int64_t)g.nx * g.ny);
    const int64_t idx[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        mu[3 * i + a] = (float)(g.lo[a] + ((double)idx[a] + 0.5 + ((double)uni[4 * i + 1 + a] - 0.5)) / (double)g.inv_h[a]);
        sc[3 * i + a] = scale;
    }
    quat[4 * i] = 1.0f;
    quat[4 * i + 1] = quat[4 * i + 2] = quat[4 * i + 3] = 0.0f;
    rho[i] = f[v];
}

__global__ __launch_bounds__(256) void dot2_partial(const float *__restrict__ a, const float *__restrict__ b,
                                                    int64_t n, double *__restrict__ part) {
    double ab = 0.0, aa = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double x = a[i];
        ab += x * (double)b[i];
        aa += x * x;
    }
    ab = block_sum_d(ab);
    aa = block_sum_d(aa);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ab;
        part[2 * blockIdx.x + 1] = aa;
    }
}

// kappa = <a, b> / <a, a>; density *= kappa.  One work-group.
__global__ __launch_bounds__(256) void apply_scale(const double *__restrict__ part, int nb, float *__restrict__ rho,
                                                   int64_t n, double *__restrict__ kappa_out) {
    double ab = 0.0, aa = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        ab += part[2 * b];
        aa += part[2 * b + 1];
    }
    ab = block_sum_d(ab);
    aa = block_sum_d(aa);
    const double kappa = aa > 0.0 ? ab / aa : 0.0;
    if (threadIdx.x == 0 && kappa_out) *kappa_out = kappa;
    for (int64_t i = threadIdx.x; i < n; i += 256) rho[i] = (float)((double)rho[i] * kappa);
}

unsigned red_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + 255) / 256)); }

dgr_status check_fdk_geometry(const dgr_geometry *geom) {
    dgr_status s = check_geometry(geom);
    if (s != DGR_OK) return s;
    DGR_CHECK(geom->kind == DGR_CONE || geom->kind == DGR_FAN, "FDK needs a cone-beam or fan-beam geometry");
    DGR_CHECK(geom->nu <= 8192, "FDK rows are staged in LDS as binary64: nu <= 8192");
    return DGR_OK;
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_fdk_workspace(const dgr_grid *grid, const dgr_geometry *geom) {
    if (check_grid(grid) != DGR_OK || check_fdk_geometry(geom) != DGR_OK) return 0;
    Carver c(nullptr);
    c.take<FdkView>(geom->n_views);
    c.take<float>((int64_t)geom->n_views * geom->nu * geom->nv);
    return c.off;
}

extern "C" dgr_status dgr_fdk(const float *proj, const dgr_grid *grid, const dgr_geometry *geom, float arc,
                              float *volume, void *ws, size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_fdk_geometry(geom)) != DGR_OK) return s;
    DGR_CHECK(proj && volume && ws, "null pointer argument");
    DGR_CHECK(std::isfinite(arc) && arc > 0.0f, "arc must be > 0");
    if (ws_bytes < dgr_fdk_workspace(grid, geom)) return fail(DGR_ERR_WORKSPACE, "workspace too small for FDK");
    hipStream_t st = as_stream(stream);
    Carver c(ws);
    FdkView *frames = c.take<FdkView>(geom->n_views);
    float *q = c.take<float>((int64_t)geom->n_views * geom->nu * geom->nv);
    fdk_frames<<<dim3((geom->n_views + 63) / 64), dim3(64), 0, st>>>(geom->views, geom->n_views, frames);
    DGR_LAUNCH_CHECK();
    fdk_filter<<<dim3(geom->nv, geom->n_views), dim3(256), sizeof(double) * geom->nu, st>>>(
        proj, geom->views, frames, geom->nu, geom->nv, geom->kind == DGR_FAN, q);
    DGR_LAUNCH_CHECK();
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    const double weight = 0.5 * ((double)arc / geom->n_views) / (double)geom->length_scale;
    fdk_backproject<<<dim3((unsigned)std::min<int64_t>((nvox + 255) / 256, 65536)), dim3(256), 0, st>>>(
        q, frames, geom->n_views, geom->nu, geom->nv, geom->kind == DGR_FAN, dev_grid(grid), weight, volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_reduce_workspace(void) { return align_up(sizeof(double) * 2 * kRedBlocks); }

extern "C" dgr_status dgr_psnr(const float *x, const float *gt, int64_t n, double *out, void *ws,
                               size_t ws_bytes, void *stream) {
    DGR_CHECK(n >= 1, "n must be >= 1");
    DGR_CHECK(x && gt && out && ws, "null pointer argument");
    if (ws_bytes < dgr_reduce_workspace()) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    double *part = static_cast<double *>(ws);
    const unsigned nb = red_blocks(n);
    psnr_partial<<<dim3(nb), dim3(256), 0, st>>>(x, gt, n, part);
    DGR_LAUNCH_CHECK();
    psnr_final<<<1, 256, 0, st>>>(part, (int)nb, n, out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_init_workspace(const dgr_grid *grid) {
    if (check_grid(grid) != DGR_OK) return 0;
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(nullptr);
    c.take<float>(kRedBlocks);
    c.take<float>(nvox);
    c.take<double>(nvox);
    c.take<double>(scan_f64_blocks(nvox));
    c.take<double>(1);
    return c.off;
}

extern "C" dgr_status dgr_init_from_volume(const float *volume, const dgr_grid *grid, float thresh_frac,
                                           int64_t n, const float *uniforms, float scale, float *mu,
                                           float *scale_out, float *quat, float *density, void *ws,
                                           size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    if (n == 0) return DGR_OK;
    DGR_CHECK(volume && uniforms && mu && scale_out && quat && density && ws, "null pointer argument");
    DGR_CHECK(std::isfinite(thresh_frac) && std::isfinite(scale) && scale > 0.0f, "bad threshold or scale");
    if (ws_bytes < dgr_init_workspace(grid)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    Carver c(ws);
    float *part = c.take<float>(kRedBlocks);
    float *w = c.take<float>(nvox);
    double *excl = c.take<double>(nvox);
    double *blk = c.take<double>(scan_f64_blocks(nvox));
    double *W = c.take<double>(1);
    const unsigned nb = red_blocks(nvox);
    max_partial<<<dim3(nb), dim3(256), 0, st>>>(volume, nvox, part);
    DGR_LAUNCH_CHECK();
    threshold_weights<<<dim3(nb), dim3(256), 0, st>>>(volume, nvox, part, (int)nb, thresh_frac, w);
    DGR_LAUNCH_CHECK();
    if ((s = exclusive_scan_f64(w, excl, nvox, blk, W, st)) != DGR_OK) return s;
    draw_gaussians<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(
        excl, W, volume, nvox, dev_grid(grid), n, uniforms, scale, mu, scale_out, quat, density);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" dgr_status dgr_fit_density_scale(const float *p1, const float *target, int64_t m, float *density,
                                            int64_t n, double *kappa, void *ws, size_t ws_bytes,
                                            void *stream) {
    DGR_CHECK(m >= 1 && n >= 0, "bad sizes");
    DGR_CHECK(p1 && target && (n == 0 || density) && ws, "null pointer argument");
    if (ws_bytes < dgr_reduce_workspace()) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    double *part = static_cast<double *>(ws);
    const unsigned nb = red_blocks(m);
    dot2_partial<<<dim3(nb), dim3(256), 0, st>>>(p1, target, m, part);
    DGR_LAUNCH_CHECK();
    apply_scale<<<1, 256, 0, st>>>(part, (int)nb, density, n, kappa);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
