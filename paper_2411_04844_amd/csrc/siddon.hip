// Exact-path (Siddon) projection and its transpose.
//
// The projection of a ray is length_scale times the sum over voxels of the
// length of the ray inside the voxel times the voxel value, the voxels being
// constant-valued cells [lo + i h, lo + (i + 1) h] (Siddon's exact
// radiological path; the paper leaves the projector abstract, sec. 4.3).  The
// rays are those of the ray march: the same views, kinds and lines.  One
// thread walks one ray in binary64: the entry and exit of the grid box, then
// the cell planes in increasing order of the ray parameter, one axis at a
// time; the segment between two consecutive crossings belongs to the cell
// that holds its midpoint.  The transpose walks the same segments and adds
// length_scale * proj * length to each cell in a binary64 workspace (hardware
// binary64 atomics), which is rounded to binary32 at the end.
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

struct SidGeom {
    int kind, n_views, nu, nv;
    const float *views;
    double ell;
};

// Point of the line nearest the world origin and unit direction of the ray
// through pixel (iu, iv) of view j (the ray march's definitions).
__device__ void ray_world(const SidGeom &G, int j, int iu, int iv, double c[3], double d[3]) {
    const float *v = G.views + 12 * (int64_t)j;
    const double au = (double)iu - 0.5 * (double)(G.nu - 1);
    const double av = (double)iv - 0.5 * (double)(G.nv - 1);
    double o[3];
    for (int a = 0; a < 3; ++a) {
        const double pix = (double)v[3 + a] + au * (double)v[6 + a] + av * (double)v[9 + a];
        if (G.kind == DGR_PARALLEL) {
            d[a] = (double)v[a];
            o[a] = pix;
        } else {
            o[a] = G.kind == DGR_FAN ? (double)v[a] + av * (double)v[9 + a] : (double)v[a];
            d[a] = pix - o[a];
        }
    }
    const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] /= nd;
    const double od = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    for (int a = 0; a < 3; ++a) c[a] = o[a] - od * d[a];
}

// Calls f(cell, length) for every segment of the ray inside the grid.  The
// walk visits at most nx + ny + nz + 3 crossings; the loop is capped at that
// count plus a margin whatever the rounding.
template <class F>
__device__ void walk(const DevGrid &g, const double c[3], const double d[3], F &&f) {
    const int dims[3] = {g.nx, g.ny, g.nz};
    double lo[3], h[3];
    double tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        lo[a] = (double)g.lo[a];
        h[a] = 1.0 / (double)g.inv_h[a];
        const double hi = lo[a] + (double)dims[a] / (double)g.inv_h[a];
        if (d[a] == 0.0) {
            if (!(c[a] > lo[a] && c[a] < hi)) return;
            continue;
        }
        double t0 = (lo[a] - c[a]) / d[a], t1 = (hi - c[a]) / d[a];
        if (t0 > t1) {
            const double tt = t0;
            t0 = t1;
            t1 = tt;
        }
        tmin = fmax(tmin, t0);
        tmax = fmin(tmax, t1);
    }
    if (!(tmin < tmax)) return;
    int p[3], s[3];
    double tn[3], inv_d[3];
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            s[a] = 0;
            p[a] = 0;
            inv_d[a] = 0.0;
            tn[a] = INFINITY;
            continue;
        }
        s[a] = d[a] > 0.0 ? 1 : -1;
        inv_d[a] = 1.0 / d[a];
        // first plane beyond the entry point along the direction of travel
        const double u = (c[a] + tmin * d[a] - lo[a]) * (double)g.inv_h[a];
        p[a] = s[a] > 0 ? (int)floor(u) + 1 : (int)ceil(u) - 1;
        tn[a] = (lo[a] + (double)p[a] * h[a] - c[a]) * inv_d[a];
        for (int k = 0; k < 2 && !(tn[a] > tmin); ++k) {  // entry rounded onto a plane
            p[a] += s[a];
            tn[a] = (lo[a] + (double)p[a] * h[a] - c[a]) * inv_d[a];
        }
    }
    double t = tmin;
    const int cap = dims[0] + dims[1] + dims[2] + 16;
    for (int it = 0; it < cap && t < tmax; ++it) {
        const double tnext = fmin(fmin(tn[0], tn[1]), fmin(tn[2], tmax));
        if (tnext > t) {
            const double tm = 0.5 * (t + tnext);
            int idx[3];
            bool inside = true;
            for (int a = 0; a < 3; ++a) {
                idx[a] = (int)floor((c[a] + tm * d[a] - lo[a]) * (double)g.inv_h[a]);
                inside = inside && idx[a] >= 0 && idx[a] < dims[a];
            }
            if (inside) f(((int64_t)idx[2] * g.ny + idx[1]) * g.nx + idx[0], tnext - t);
        }
        for (int a = 0; a < 3; ++a)
            if (tn[a] == tnext) {
                p[a] += s[a];
                tn[a] = (lo[a] + (double)p[a] * h[a] - c[a]) * inv_d[a];
            }
        t = tnext;
    }
}

__global__ __launch_bounds__(256) void siddon_project(const float *__restrict__ V, DevGrid g, SidGeom G,
                                                      float *__restrict__ proj) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nrays = (int64_t)G.n_views * G.nu * G.nv;
    if (r >= nrays) return;
    const int j = (int)(r / ((int64_t)G.nu * G.nv));
    const int rem = (int)(r - (int64_t)j * G.nu * G.nv);
    const int iv = rem / G.nu, iu = rem - iv * G.nu;
    double c[3], d[3];
    ray_world(G, j, iu, iv, c, d);
    double acc = 0.0;
    walk(g, c, d, [&](int64_t cell, double len) { acc += len * (double)V[cell]; });
    proj[r] = (float)(G.ell * acc);
}

__global__ __launch_bounds__(256) void siddon_backproject(const float *__restrict__ proj, DevGrid g, SidGeom G,
                                                          double *__restrict__ acc) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nrays = (int64_t)G.n_views * G.nu * G.nv;
    if (r >= nrays) return;
    const double w = G.ell * (double)proj[r];
    if (w == 0.0) return;
    const int j = (int)(r / ((int64_t)G.nu * G.nv));
    const int rem = (int)(r - (int64_t)j * G.nu * G.nv);
    const int iv = rem / G.nu, iu = rem - iv * G.nu;
    double c[3], d[3];
    ray_world(G, j, iu, iv, c, d);
    walk(g, c, d, [&](int64_t cell, double len) { unsafeAtomicAdd(acc + cell, w * len); });
}

__global__ __launch_bounds__(256) void fill_f64(double *__restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = 0.0;
}

__global__ __launch_bounds__(256) void round_f64(const double *__restrict__ x, int64_t n, float *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] = (float)x[i];
}

SidGeom sid_geom(const dgr_geometry *G) {
    return SidGeom{G->kind, G->n_views, G->nu, G->nv, G->views, (double)G->length_scale};
}

unsigned ray_blocks(const dgr_geometry *G) {
    return (unsigned)(((int64_t)G->n_views * G->nu * G->nv + 255) / 256);
}

unsigned stride_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" dgr_status dgr_project_siddon(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                                         float *proj, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_geometry(geom)) != DGR_OK) return s;
    DGR_CHECK(volume && proj, "null volume or projection pointer");
    siddon_project<<<dim3(ray_blocks(geom)), dim3(256), 0, as_stream(stream)>>>(volume, dev_grid(grid),
                                                                               sid_geom(geom), proj);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_backproject_siddon_workspace(const dgr_grid *grid) {
    if (check_grid(grid) != DGR_OK) return 0;
    return align_up(sizeof(double) * (size_t)grid->dims[0] * grid->dims[1] * grid->dims[2]);
}

extern "C" dgr_status dgr_backproject_siddon(const float *proj, const dgr_grid *grid, const dgr_geometry *geom,
                                             float *volume, void *ws, size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_geometry(geom)) != DGR_OK) return s;
    DGR_CHECK(proj && volume && ws, "null pointer argument");
    DGR_CHECK(reinterpret_cast<uintptr_t>(ws) % kAlign == 0, "workspace must be 256-byte aligned");
    if (ws_bytes < dgr_backproject_siddon_workspace(grid))
        return fail(DGR_ERR_WORKSPACE, "workspace too small for the exact-path backprojection");
    hipStream_t st = as_stream(stream);
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    double *acc = static_cast<double *>(ws);
    fill_f64<<<dim3(stride_blocks(nvox)), dim3(256), 0, st>>>(acc, nvox);
    DGR_LAUNCH_CHECK();
    siddon_backproject<<<dim3(ray_blocks(geom)), dim3(256), 0, st>>>(proj, dev_grid(grid), sid_geom(geom), acc);
    DGR_LAUNCH_CHECK();
    round_f64<<<dim3(stride_blocks(nvox)), dim3(256), 0, st>>>(acc, nvox, volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
