// Binary64 path used only to check gradients by central finite differences.
//
// dgr_voxelize_f64: the volume of sec. 4.1 (eq. for V(p), boxes of the
// truncation rule) evaluated in binary64 from the binary32 parameters.
//
// dgr_fd_l1_f64: for each requested (Gaussian g, component c, step h), the
// change of the mean-L1 projection loss (sec. 4.3) when parameter c of g moves
// by +h and by -h, with g's box held fixed.  Only g's box changes the volume,
// and the projector is linear, so
//   L(theta +- h) - L(theta) = (1/M) sum_{rays r crossing the box}
//                              ( |res_r + (A dV+-)_r| - |res_r| ),
//   res = A V - y,  dV+- = rho' G(.; theta') - rho G(.; theta) on the box.
// Summing only over the crossing rays avoids cancelling against the full loss.
// Components: 0-2 mean x,y,z; 3-5 scale; 6-9 quaternion w,x,y,z; 10 density.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace dgr {
namespace {

struct Gauss64 {
    double mu[3];
    double Q[3][3];  // precision matrix, world units
    double rho;
};

__device__ void make_gauss(const double mu[3], const double s[3], const double q[4], double rho,
                           Gauss64 &G) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double n2 = w * w + x * x + y * y + z * z;
    double R[3][3];
    if (n2 == 0.0) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) R[a][b] = (a == b) ? 1.0 : 0.0;
    } else {
        const double inv = 1.0 / sqrt(n2);
        w *= inv; x *= inv; y *= inv; z *= inv;
        R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
        R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
        R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += R[a][j] * R[b][j] / (s[j] * s[j]);
            G.Q[a][b] = acc;
        }
    for (int a = 0; a < 3; ++a) G.mu[a] = mu[a];
    G.rho = rho;
}

__device__ __forceinline__ double eval_gauss(const Gauss64 &G, const double p[3]) {
    const double d0 = p[0] - G.mu[0], d1 = p[1] - G.mu[1], d2 = p[2] - G.mu[2];
    const double m = d0 * (G.Q[0][0] * d0 + 2.0 * (G.Q[0][1] * d1 + G.Q[0][2] * d2)) +
                     d1 * (G.Q[1][1] * d1 + 2.0 * G.Q[1][2] * d2) + d2 * G.Q[2][2] * d2;
    return G.rho * exp(-0.5 * m);
}

__device__ void load_params(const float *mu, const float *scale, const float *quat,
                            const float *density, int64_t g, double m[3], double s[3], double q[4],
                            double *rho) {
    for (int a = 0; a < 3; ++a) {
        m[a] = mu[3 * g + a];
        s[a] = scale[3 * g + a];
    }
    for (int a = 0; a < 4; ++a) q[a] = quat[4 * g + a];
    *rho = density[g];
}

// ---- binary64 voxelization: one thread per voxel of each tile, gid order ----
__global__ __launch_bounds__(256) void voxelize_tiles_f64(
    const float *__restrict__ mu, const float *__restrict__ scale, const float *__restrict__ quat,
    const float *__restrict__ density, const GaussRec *__restrict__ rec,
    const uint32_t *__restrict__ gid, const uint32_t *__restrict__ tile_begin,
    const VoxHeader *__restrict__ hdr, int64_t cap, DevGrid g, int Tx, int Ty, double *__restrict__ V) {
    const int64_t tile = blockIdx.x;
    const int tx = (int)(tile % Tx), ty = (int)((tile / Tx) % Ty), tz = (int)(tile / ((int64_t)Tx * Ty));
    const int t = threadIdx.x;
    const int vx = tx * 8 + (t & 7), vy = ty * 8 + ((t >> 3) & 7);
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (int half = 0; half < 2; ++half) {
        const int vz = tz * 8 + (t >> 6) + 4 * half;
        if (vx >= g.nx || vy >= g.ny || vz >= g.nz) continue;
        const int64_t out = vz * plane + (int64_t)vy * g.nx + vx;
        if (hdr->total > (uint64_t)cap) {
            V[out] = __builtin_nan("");
            continue;
        }
        const double p[3] = {g.lo[0] + (vx + 0.5) / (double)g.inv_h[0],
                             g.lo[1] + (vy + 0.5) / (double)g.inv_h[1],
                             g.lo[2] + (vz + 0.5) / (double)g.inv_h[2]};
        double acc = 0.0;
        for (uint32_t i = tile_begin[tile]; i < tile_begin[tile + 1]; ++i) {
            const uint32_t k = gid[i];
            const GaussRec &r = rec[k];
            if (vx < box_lo(r.box[0]) || vx > box_hi(r.box[0]) || vy < box_lo(r.box[1]) ||
                vy > box_hi(r.box[1]) || vz < box_lo(r.box[2]) || vz > box_hi(r.box[2]))
                continue;
            double m[3], s[3], q[4], rho;
            load_params(mu, scale, quat, density, k, m, s, q, &rho);
            Gauss64 G;
            make_gauss(m, s, q, rho, G);
            acc += eval_gauss(G, p);
        }
        V[out] = acc;
    }
}

// ---- finite-difference kernel --------------------------------------------------
struct FdJob {
    int32_t gid, comp;
    double h;
};

struct Geom64 {
    int kind, n_views, nu, nv;
    const float *views;
    double step, scale;
};

__device__ void ray64(const Geom64 &G, int j, int iu, int iv, double c[3], double d[3]) {
    const float *v = G.views + 12 * (int64_t)j;
    const double au = (double)iu - 0.5 * (G.nu - 1), av = (double)iv - 0.5 * (G.nv - 1);
    double o[3];
    for (int a = 0; a < 3; ++a) {
        const double pix = (double)v[3 + a] + au * (double)v[6 + a] + av * (double)v[9 + a];
        if (G.kind == DGR_PARALLEL) {
            d[a] = v[a];
            o[a] = pix;
        } else {
            const double src = G.kind == DGR_FAN ? (double)v[a] + av * (double)v[9 + a] : (double)v[a];
            d[a] = pix - src;
            o[a] = src;
        }
    }
    const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] /= nd;
    const double od = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    for (int a = 0; a < 3; ++a) c[a] = o[a] - od * d[a];
}

// k-range (samples c + k step d) whose voxel coordinate lies in [lo, hi]
// on every axis; false if empty.
__device__ bool krange64(const double c[3], const double d[3], const DevGrid &g, double step,
                         const double lo[3], const double hi[3], int64_t *k0, int64_t *k1) {
    double tmin = -1e300, tmax = 1e300;
    for (int a = 0; a < 3; ++a) {
        const double uc = (c[a] - g.lo[a]) * (double)g.inv_h[a] - 0.5;
        const double du = d[a] * (double)g.inv_h[a] * step;
        if (du == 0.0) {
            if (!(uc >= lo[a] && uc <= hi[a])) return false;
            continue;
        }
        const double t0 = (lo[a] - uc) / du, t1 = (hi[a] - uc) / du;
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    }
    if (!(tmin <= tmax) || tmin < -1e9 || tmax > 1e9) return false;
    *k0 = (int64_t)ceil(tmin);
    *k1 = (int64_t)floor(tmax);
    return *k0 <= *k1;
}

// trilinear interpolant of a [nz][ny][nx] field (offset o3) at voxel coordinate u
__device__ double trilin64(const double *F, const int n3[3], const int o3[3], const double u[3]) {
    double fl[3], f[3];
    for (int a = 0; a < 3; ++a) {
        fl[a] = floor(u[a]);
        f[a] = u[a] - fl[a];
    }
    double acc = 0.0;
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = (cc >> 2) & 1;
        const int i = (int)fl[0] + ox - o3[0], j = (int)fl[1] + oy - o3[1], k = (int)fl[2] + oz - o3[2];
        if (i < 0 || j < 0 || k < 0 || i >= n3[0] || j >= n3[1] || k >= n3[2]) continue;
        const double w = (ox ? f[0] : 1 - f[0]) * (oy ? f[1] : 1 - f[1]) * (oz ? f[2] : 1 - f[2]);
        acc += w * F[((int64_t)k * n3[1] + j) * n3[0] + i];
    }
    return acc;
}

// dV+- on g's box: dvol[job][2][bz][by][bx]
__global__ __launch_bounds__(256) void fd_delta_volumes(
    const float *__restrict__ mu, const float *__restrict__ scale, const float *__restrict__ quat,
    const float *__restrict__ density, const int32_t *__restrict__ box, const FdJob *__restrict__ jobs,
    DevGrid g, int64_t box_cap, double *__restrict__ dvol) {
    const int jb = blockIdx.y;
    const FdJob J = jobs[jb];
    const int32_t *b = box + 6 * (int64_t)J.gid;
    const int bx = b[3] - b[0] + 1, by = b[4] - b[1] + 1, bz = b[5] - b[2] + 1;
    if (bx <= 0 || by <= 0 || bz <= 0) return;
    const int64_t nbox = (int64_t)bx * by * bz;
    double m[3], s[3], q[4], rho;
    load_params(mu, scale, quat, density, J.gid, m, s, q, &rho);
    Gauss64 G0, Gp, Gm;
    make_gauss(m, s, q, rho, G0);
    for (int sgn = 0; sgn < 2; ++sgn) {
        double mm[3] = {m[0], m[1], m[2]}, ss[3] = {s[0], s[1], s[2]}, qq[4] = {q[0], q[1], q[2], q[3]};
        double rr = rho;
        const double hh = sgn == 0 ? J.h : -J.h;
        if (J.comp < 3) mm[J.comp] += hh;
        else if (J.comp < 6) ss[J.comp - 3] += hh;
        else if (J.comp < 10) qq[J.comp - 6] += hh;
        else rr += hh;
        make_gauss(mm, ss, qq, rr, sgn == 0 ? Gp : Gm);
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nbox && i < box_cap;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % bx), y = (int)((i / bx) % by), z = (int)(i / ((int64_t)bx * by));
        const double p[3] = {g.lo[0] + (b[0] + x + 0.5) / (double)g.inv_h[0],
                             g.lo[1] + (b[1] + y + 0.5) / (double)g.inv_h[1],
                             g.lo[2] + (b[2] + z + 0.5) / (double)g.inv_h[2]};
        const double v0 = eval_gauss(G0, p);
        dvol[((int64_t)jb * 2 + 0) * box_cap + i] = eval_gauss(Gp, p) - v0;
        dvol[((int64_t)jb * 2 + 1) * box_cap + i] = eval_gauss(Gm, p) - v0;
    }
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// One work-group per (job, view): every detector pixel whose ray crosses the
// box's cell region contributes |res + dP+-| - |res|.  out[job][view][2].
__global__ __launch_bounds__(256) void fd_rays(const double *__restrict__ V, DevGrid g, Geom64 G,
                                               const float *__restrict__ target,
                                               const int32_t *__restrict__ box,
                                               const FdJob *__restrict__ jobs,
                                               const double *__restrict__ dvol, int64_t box_cap,
                                               double *__restrict__ out) {
    __shared__ double sh[4];
    const int jb = blockIdx.y, j = blockIdx.x;
    const FdJob J = jobs[jb];
    const int32_t *b = box + 6 * (int64_t)J.gid;
    const int n3b[3] = {b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
    double sp = 0.0, sm = 0.0;
    const bool nonempty = n3b[0] > 0 && n3b[1] > 0 && n3b[2] > 0;
    const bool too_big = nonempty && (int64_t)n3b[0] * n3b[1] * n3b[2] > box_cap;
    if (nonempty && !too_big) {
        const int o3b[3] = {b[0], b[1], b[2]};
        const int n3v[3] = {g.nx, g.ny, g.nz};
        const int o3v[3] = {0, 0, 0};
        const double *dp = dvol + ((int64_t)jb * 2 + 0) * box_cap;
        const double *dm = dvol + ((int64_t)jb * 2 + 1) * box_cap;
        // cells that can touch the box: voxel coordinate in [lo - 1, hi + 1]
        const double blo[3] = {b[0] - 1.0, b[1] - 1.0, b[2] - 1.0};
        const double bhi[3] = {b[3] + 1.0, b[4] + 1.0, b[5] + 1.0};
        const double slo[3] = {-1.0, -1.0, -1.0};
        const double shi[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
        int iu0, iu1, iv0, iv1;
        shadow_rect(G.kind, G.views + 12 * (int64_t)j, G.nu, G.nv, g, blo, bhi, &iu0, &iu1, &iv0, &iv1);
        const int wu = iu1 - iu0 + 1, wv = iv1 - iv0 + 1;
        const int64_t npix = (wu > 0 && wv > 0) ? (int64_t)wu * wv : 0;
        for (int64_t pix = threadIdx.x; pix < npix; pix += 256) {
            const int iu = iu0 + (int)(pix % wu), iv = iv0 + (int)(pix / wu);
            double c[3], d[3];
            ray64(G, j, iu, iv, c, d);
            int64_t q0, q1;
            if (!krange64(c, d, g, G.step, blo, bhi, &q0, &q1)) continue;
            double dpp = 0.0, dmm = 0.0;
            for (int64_t k = q0; k <= q1; ++k) {
                double u[3];
                for (int a = 0; a < 3; ++a)
                    u[a] = (c[a] + (double)k * G.step * d[a] - g.lo[a]) * (double)g.inv_h[a] - 0.5;
                dpp += trilin64(dp, n3b, o3b, u);
                dmm += trilin64(dm, n3b, o3b, u);
            }
            if (dpp == 0.0 && dmm == 0.0) continue;
            int64_t k0, k1;
            double acc = 0.0;
            if (krange64(c, d, g, G.step, slo, shi, &k0, &k1))
                for (int64_t k = k0; k <= k1; ++k) {
                    double u[3];
                    for (int a = 0; a < 3; ++a)
                        u[a] = (c[a] + (double)k * G.step * d[a] - g.lo[a]) * (double)g.inv_h[a] - 0.5;
                    acc += trilin64(V, n3v, o3v, u);
                }
            const double res = G.scale * acc - (double)target[((int64_t)j * G.nv + iv) * G.nu + iu];
            sp += fabs(res + G.scale * dpp) - fabs(res);
            sm += fabs(res + G.scale * dmm) - fabs(res);
        }
    }
    sp = block_sum(sp, sh);
    sm = block_sum(sm, sh);
    if (too_big) sp = sm = __builtin_nan("");  // a box larger than box_cap is reported, not skipped
    if (threadIdx.x == 0) {
        out[((int64_t)jb * G.n_views + j) * 2 + 0] = sp;
        out[((int64_t)jb * G.n_views + j) * 2 + 1] = sm;
    }
}

// Loss changes of each job: the per-view sums added in view order in
// binary64 and divided by M (one thread per job and sign).
__global__ __launch_bounds__(256) void fd_sum_views(const double *__restrict__ per_view, int n_jobs, int n_views,
                                                    double inv_m, double *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;  // job * 2 + sign
    if (i >= 2 * n_jobs) return;
    const int jb = i >> 1, sg = i & 1;
    double acc = 0.0;
    for (int j = 0; j < n_views; ++j) acc += per_view[((int64_t)jb * n_views + j) * 2 + sg];
    out[i] = acc * inv_m;
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_voxelize_f64_workspace(int64_t n, int64_t max_pairs, const dgr_grid *grid) {
    return dgr_voxelize_workspace(n, max_pairs, grid);
}

extern "C" dgr_status dgr_voxelize_f64(const float *mu, const float *scale, const float *quat,
                                       const float *density, int64_t n, const dgr_grid *grid,
                                       const dgr_trunc *trunc, double *volume, void *ws,
                                       size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_trunc(trunc)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n out of range");
    DGR_CHECK(n == 0 || (mu && scale && quat && density), "null parameter pointer");
    DGR_CHECK(volume && ws, "null volume or workspace");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const int64_t cap = vox_ws_capacity(ws_bytes, n, grid);
    if (cap < 0) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    VoxWs w = carve_vox_ws(ws, n, cap, grid);
    hipStream_t st = as_stream(stream);
    int which = 0;
    if ((s = enqueue_binning(mu, scale, quat, density, n, grid, trunc, w, &which, st)) != DGR_OK) return s;
    const int Tx = (grid->dims[0] + 7) / 8, Ty = (grid->dims[1] + 7) / 8;
    voxelize_tiles_f64<<<dim3((unsigned)w.tiles), dim3(256), 0, st>>>(
        mu, scale, quat, density, w.rec, w.val[which], w.tile_begin, w.hdr, w.cap, dev_grid(grid), Tx, Ty,
        volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_fd_l1_f64_workspace(int64_t n, int32_t n_jobs, int64_t box_cap,
                                          const dgr_geometry *geom) {
    if (n < 0 || n_jobs < 0 || box_cap < 1 || !geom || geom->n_views < 1) return 0;
    Carver c(nullptr);
    c.take<int32_t>(6 * std::max<int64_t>(n, 1));
    c.take<FdJob>(std::max(n_jobs, 1));
    c.take<double>((int64_t)std::max(n_jobs, 1) * 2 * box_cap);
    c.take<double>((int64_t)std::max(n_jobs, 1) * geom->n_views * 2);
    return c.off;
}

extern "C" dgr_status dgr_fd_l1_f64(const double *volume, const dgr_grid *grid,
                                    const dgr_geometry *geom, const float *target, const float *mu,
                                    const float *scale, const float *quat, const float *density,
                                    int64_t n, const dgr_trunc *trunc, const int32_t *job_gid,
                                    const int32_t *job_comp, const double *job_h, int32_t n_jobs,
                                    int64_t box_cap, double *out, void *ws, size_t ws_bytes,
                                    void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_geometry(geom)) != DGR_OK) return s;
    if ((s = check_trunc(trunc)) != DGR_OK) return s;
    DGR_CHECK(n >= 1 && n < (int64_t(1) << 31), "n out of range");
    DGR_CHECK(n_jobs >= 1 && n_jobs <= 65535, "n_jobs out of range");
    DGR_CHECK(box_cap >= 1, "box_cap must be >= 1");
    DGR_CHECK(volume && target && mu && scale && quat && density && job_gid && job_comp && job_h && out,
              "null pointer argument");
    DGR_CHECK(ws != nullptr, "null workspace");
    if (ws_bytes < dgr_fd_l1_f64_workspace(n, n_jobs, box_cap, geom))
        return fail(DGR_ERR_WORKSPACE, "workspace too small for the finite-difference jobs");
    hipStream_t st = as_stream(stream);
    Carver c(ws);
    int32_t *box = c.take<int32_t>(6 * n);
    FdJob *jobs = c.take<FdJob>(n_jobs);
    double *dvol = c.take<double>((int64_t)n_jobs * 2 * box_cap);
    double *per_view = c.take<double>((int64_t)n_jobs * geom->n_views * 2);
    if ((s = launch_prep(mu, scale, quat, nullptr, n, grid, trunc, nullptr, nullptr, box, st)) != DGR_OK)
        return s;
    // the job table (host arrays) is packed and copied to the workspace
    std::vector<FdJob> hj(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        DGR_CHECK(job_gid[i] >= 0 && job_gid[i] < n && job_comp[i] >= 0 && job_comp[i] <= 10,
                  "job %d: bad gid or component", i);
        hj[i] = FdJob{job_gid[i], job_comp[i], job_h[i]};
    }
    DGR_TRY_HIP(hipMemcpyAsync(jobs, hj.data(), sizeof(FdJob) * n_jobs, hipMemcpyHostToDevice, st));
    const DevGrid g = dev_grid(grid);
    fd_delta_volumes<<<dim3(64, n_jobs), dim3(256), 0, st>>>(mu, scale, quat, density, box, jobs, g, box_cap, dvol);
    DGR_LAUNCH_CHECK();
    Geom64 G{geom->kind, geom->n_views, geom->nu, geom->nv, geom->views, (double)geom->step,
             (double)geom->length_scale * (double)geom->step};
    fd_rays<<<dim3(geom->n_views, n_jobs), dim3(256), 0, st>>>(volume, g, G, target, box, jobs, dvol, box_cap,
                                                               per_view);
    DGR_LAUNCH_CHECK();
    const double m = (double)geom->n_views * geom->nu * geom->nv;
    fd_sum_views<<<dim3((unsigned)((2 * n_jobs + 255) / 256)), dim3(256), 0, st>>>(per_view, n_jobs, geom->n_views,
                                                                                 1.0 / m, out);
    DGR_LAUNCH_CHECK();
    DGR_TRY_HIP(hipStreamSynchronize(st));  // the host job table goes out of scope
    return DGR_OK;
}
