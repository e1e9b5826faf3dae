// Internal declarations shared by the libdgr.so translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "dgr.h"

namespace dgr {

// ---- error plumbing --------------------------------------------------------
dgr_status fail(dgr_status s, const char *fmt, ...);

#define DGR_TRY_HIP(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::dgr::fail(DGR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define DGR_CHECK(cond, ...)                                         \
    do {                                                             \
        if (!(cond)) return ::dgr::fail(DGR_ERR_INVALID_ARG, __VA_ARGS__); \
    } while (0)

// Kernel launches report launch failures through hipGetLastError().
#define DGR_LAUNCH_CHECK() DGR_TRY_HIP(hipGetLastError())

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

dgr_status check_grid(const dgr_grid *g);
dgr_status check_trunc(const dgr_trunc *t);
dgr_status check_geometry(const dgr_geometry *g);

// ---- workspace carving -----------------------------------------------------
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *p) : base(static_cast<char *>(p)) {}
    template <class T>
    T *take(size_t count) {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += align_up(count * sizeof(T));
        return p;
    }
};

// ---- per-Gaussian record written by the prep kernel ------------------------
// Continuous voxel position u = ui + uf with ui = floor(u) (the paper's
// floored index) and uf in [0, 1) (its residual Delta mu), the exponent
// coefficients of exp2, and the packed truncation box.  64 bytes.
struct alignas(16) GaussRec {
    int32_t ui[3];
    float rho;
    float uf[3];
    float k00;      // exponent = k00 dx^2 + k11 dy^2 + k22 dz^2
    float k11, k22; //          + k01 dx dy + k02 dx dz + k12 dy dz  (log2 units)
    float k01, k02;
    float k12;
    uint32_t box[3];  // (lo & 0xffff) | (hi << 16), hi = -1 stored as 0xffff
};
static_assert(sizeof(GaussRec) == 64, "record must be 64 bytes");

__host__ __device__ inline int box_lo(uint32_t b) { return (int)(int16_t)(b & 0xffffu); }
__host__ __device__ inline int box_hi(uint32_t b) { return (int)(int16_t)(b >> 16); }

struct DevGrid {
    int nx, ny, nz;
    float lo[3];
    float inv_h[3];
};
inline DevGrid dev_grid(const dgr_grid *g) {
    DevGrid d;
    d.nx = g->dims[0];
    d.ny = g->dims[1];
    d.nz = g->dims[2];
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = g->lo[a];
        d.inv_h[a] = g->inv_h[a];
    }
    return d;
}

// Inclusive detector rectangle (pixel indices, widened by one pixel) that
// contains the shadow of the box [ulo, uhi] (continuous voxel coordinates) in
// one view (`view` = the 12 floats of the view).  A box is convex, so its
// shadow lies in the bounding rectangle of its projected corners.  If a corner
// cannot be projected (behind a cone source, or a ray parallel to the
// detector) the whole detector is returned.  An empty rectangle has iu0 > iu1.
// Fan beam: a point x belongs to the row whose fan plane holds it, row
// position b = ((x - a).m)/(e_v.m) with m = (det - a) x e_u, and is projected
// from that row's source a + b e_v.  When e_v is orthogonal to e_u and to
// det - a this splits into a linear map along e_v and a perspective map of
// the box's orthogonal projection onto the fan plane, so the corners still
// bound the shadow; other views get the whole detector.
__device__ inline void shadow_rect(int kind, const float *view, int nu, int nv, const DevGrid &g,
                                   const double ulo[3], const double uhi[3], int *iu0, int *iu1,
                                   int *iv0, int *iv1) {
    double A[3], D0[3], eu[3], ev[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = view[a];
        D0[a] = view[3 + a];
        eu[a] = view[6 + a];
        ev[a] = view[9 + a];
    }
    const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2],
                         eu[0] * ev[1] - eu[1] * ev[0]};
    const double uu = eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2];
    const double vv = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
    const double uv = eu[0] * ev[0] + eu[1] * ev[1] + eu[2] * ev[2];
    const double det2 = uu * vv - uv * uv;
    double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
    bool ok = det2 > 0.0;
    double m[3] = {0.0, 0.0, 0.0}, em = 0.0;
    if (kind == DGR_FAN && ok) {
        const double w[3] = {D0[0] - A[0], D0[1] - A[1], D0[2] - A[2]};
        m[0] = w[1] * eu[2] - w[2] * eu[1];
        m[1] = w[2] * eu[0] - w[0] * eu[2];
        m[2] = w[0] * eu[1] - w[1] * eu[0];
        em = ev[0] * m[0] + ev[1] * m[1] + ev[2] * m[2];
        const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        const double ew = ev[0] * w[0] + ev[1] * w[1] + ev[2] * w[2];
        // orthogonality to 1e-6 (binary32 views of an exact geometry are
        // orthogonal to about 1e-7); the widening by one pixel absorbs the rest
        ok = fabs(uv) <= 1e-6 * sqrt(uu * vv) && fabs(ew) <= 1e-6 * sqrt(ww * vv) && fabs(em) > 0.0;
    }
    for (int c = 0; c < 8 && ok; ++c) {
        double X[3], dir[3], src[3];
        for (int a = 0; a < 3; ++a) {
            const double u = ((c >> a) & 1) ? uhi[a] : ulo[a];
            X[a] = (double)g.lo[a] + (u + 0.5) / (double)g.inv_h[a];
        }
        const double brow = kind == DGR_FAN
            ? ((X[0] - A[0]) * m[0] + (X[1] - A[1]) * m[1] + (X[2] - A[2]) * m[2]) / em : 0.0;
        for (int a = 0; a < 3; ++a) {
            src[a] = A[a] + brow * ev[a];
            dir[a] = kind == DGR_PARALLEL ? A[a] : X[a] - src[a];
        }
        const double den = n[0] * dir[0] + n[1] * dir[1] + n[2] * dir[2];
        if (!(fabs(den) > 1e-300)) { ok = false; break; }
        const double t = (n[0] * (D0[0] - X[0]) + n[1] * (D0[1] - X[1]) + n[2] * (D0[2] - X[2])) / den;
        if (kind != DGR_PARALLEL && !(t > -1.0)) { ok = false; break; }  // corner behind the source
        double P[3];
        for (int a = 0; a < 3; ++a) P[a] = X[a] + t * dir[a] - D0[a];
        const double pu = P[0] * eu[0] + P[1] * eu[1] + P[2] * eu[2];
        const double pv = P[0] * ev[0] + P[1] * ev[1] + P[2] * ev[2];
        const double ca = (pu * vv - pv * uv) / det2, cb = (pv * uu - pu * uv) / det2;
        amin = fmin(amin, ca); amax = fmax(amax, ca);
        bmin = fmin(bmin, cb); bmax = fmax(bmax, cb);
    }
    *iu0 = 0; *iu1 = nu - 1; *iv0 = 0; *iv1 = nv - 1;
    if (ok) {
        const double cu = 0.5 * (nu - 1), cv = 0.5 * (nv - 1);
        const double a0 = floor(amin + cu) - 1.0, a1 = ceil(amax + cu) + 1.0;
        const double b0 = floor(bmin + cv) - 1.0, b1 = ceil(bmax + cv) + 1.0;
        if (a1 < 0.0 || b1 < 0.0 || a0 > nu - 1.0 || b0 > nv - 1.0) {
            *iu0 = 1; *iu1 = 0; *iv0 = 1; *iv1 = 0;  // empty
            return;
        }
        *iu0 = (int)fmax(0.0, a0); *iu1 = (int)fmin((double)(nu - 1), a1);
        *iv0 = (int)fmax(0.0, b0); *iv1 = (int)fmin((double)(nv - 1), b1);
    }
}

// Enqueue the prep kernel: records + tile counts (and optional int32 boxes).
dgr_status launch_prep(const float *mu, const float *scale, const float *quat,
                       const float *density, int64_t n, const dgr_grid *grid,
                       const dgr_trunc *trunc, GaussRec *rec, uint32_t *tile_count,
                       int32_t *box_out, hipStream_t st);

// ---- voxelization workspace -----------------------------------------------
struct VoxHeader {
    uint32_t overflow;   // set by the emit kernel when pairs > capacity
    uint32_t pad0;
    uint64_t total;      // pair count of the last binning
};

struct VoxWs {
    VoxHeader *hdr;
    GaussRec *rec;
    uint32_t *count;     // tiles per Gaussian
    uint64_t *offset;    // exclusive scan of count
    uint64_t *scan_blk;  // block partials of the scan
    uint32_t *key[2];
    uint32_t *val[2];
    uint32_t *hist;      // radix histograms [256][nblk]
    uint32_t *tile_begin;
    int64_t cap;
    int64_t n;
    int64_t tiles;
    int radix_blocks;
    size_t bytes;
};

VoxWs carve_vox_ws(void *ws, int64_t n, int64_t cap, const dgr_grid *grid);
int64_t vox_ws_capacity(size_t ws_bytes, int64_t n, const dgr_grid *grid);

// Binning: prep -> count scan -> emit -> stable radix sort -> tile ranges.
// On return (enqueued) key/val[*which] hold the sorted pairs.
dgr_status enqueue_binning(const float *mu, const float *scale, const float *quat,
                           const float *density, int64_t n, const dgr_grid *grid,
                           const dgr_trunc *trunc, VoxWs &w, int *which, hipStream_t st);
dgr_status enqueue_count_only(const float *mu, const float *scale, const float *quat, int64_t n,
                              const dgr_grid *grid, const dgr_trunc *trunc, VoxWs &w,
                              hipStream_t st);

// Exclusive prefix sum of binary32 values in binary64; *total gets the sum.
// blk needs scan_f64_blocks(n) entries.
int64_t scan_f64_blocks(int64_t n);
dgr_status exclusive_scan_f64(const float *in, double *out, int64_t n, double *blk, double *total,
                              hipStream_t st);
// uint32 exclusive scan (sums below 2^32); blk needs scan_f64_blocks(n) entries.
dgr_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *blk, uint32_t *total,
                              hipStream_t st);

inline int64_t tiles_of(const dgr_grid *g) {
    return (int64_t)((g->dims[0] + 7) / 8) * ((g->dims[1] + 7) / 8) * ((g->dims[2] + 7) / 8);
}

}  // namespace dgr
