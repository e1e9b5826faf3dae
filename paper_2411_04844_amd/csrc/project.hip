// Forward projection P_hat = T(V) (sec. 4.3) as a trilinear ray march, the
// fused L1 data term of the objective (sec. 4.3), and the exact transpose
// (backprojection).
//
//   P_hat[r] = length_scale * step * sum_{k in Z} Vbar(c_r + k step d_r)
//
// d_r is the unit ray direction, c_r the point of the ray nearest the world
// origin, and Vbar the trilinear interpolant of V on voxel centres, zero
// outside the grid.
//
// Sample positions.  Per-ray set-up (direction, anchor, advance) runs in
// binary64.  Sample k sits at u_k = I(kb) + (f(kb) + (k - kb) * du), where
// kb = 32 * floor(k / 32), I(kb) is the integer part of the binary64 position
// cu + kb * du and f(kb) its residual (the floor / residual split of the
// paper's Discretize and Align step), and the bracket is evaluated in binary32.
// The offsets stay below ~17 voxels, so positions are within ~2e-6 voxel of
// exact on any grid, and the anchor depends only on (ray, k): the projector and
// the backprojector evaluate every sample at the same position.
//
// Forward: one thread per ray; the volume is read from a copy with a two-voxel
// zero border, so the eight taps of any sample in the support need no test.
// Backward: one work-group per 16^3-cell brick accumulates, over all views, the
// samples whose trilinear cell lies in the brick into a 17^3 LDS tile (no
// global atomics); the tiles are then summed per voxel.  The LDS sums are
// 64-bit fixed point: every contribution is scaled by a power of two S chosen
// from max|proj| so that it fits in 32 bits, truncated to an integer and added
// with ds_add_u64.  On gfx950 that is ~20x faster than ds_add_f32, and integer
// addition makes the result independent of the order of the adds.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr int kPad = 2;
constexpr int kRayTile = 16;  // 16 x 16 detector pixels per work-group (forward)
constexpr int kB = 16;        // brick edge in cells (backward)
constexpr int kBT = kB + 1;   // brick tile edge in voxels
constexpr int kBT3 = kBT * kBT * kBT;

struct PadDims {
    int px, py, pz;  // padded extents
    int64_t plane;   // px * py
};

inline PadDims pad_dims(const dgr_grid *g) {
    PadDims p;
    p.px = g->dims[0] + 2 * kPad;
    p.py = g->dims[1] + 2 * kPad;
    p.pz = g->dims[2] + 2 * kPad;
    p.plane = (int64_t)p.px * p.py;
    return p;
}

inline int64_t pad_count(const dgr_grid *g) {
    PadDims p = pad_dims(g);
    return p.plane * p.pz;
}

struct Bricks {
    int nx, ny, nz;
    __host__ __device__ int64_t count() const { return (int64_t)nx * ny * nz; }
};

inline Bricks bricks_of(const dgr_grid *g) {
    // cells floor(u) range over [-1, dims-1]: dims + 1 values per axis
    Bricks b;
    b.nx = (g->dims[0] + 1 + kB - 1) / kB;
    b.ny = (g->dims[1] + 1 + kB - 1) / kB;
    b.nz = (g->dims[2] + 1 + kB - 1) / kB;
    return b;
}

__global__ __launch_bounds__(256) void pad_volume(const float *__restrict__ V, DevGrid g, PadDims p,
                                                  float *__restrict__ out) {
    const int64_t total = p.plane * p.pz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        int64_t z = i / p.plane, rem = i - z * p.plane;
        int64_t y = rem / p.px, x = rem - y * p.px;
        x -= kPad; y -= kPad; z -= kPad;
        float v = 0.0f;
        if (x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz)
            v = V[(z * g.ny + y) * g.nx + x];
        out[i] = v;
    }
}

struct GeomDev {
    int kind, n_views, nu, nv;
    const float *views;
    double step;
    float scale;  // length_scale * step
};

struct Ray {
    double cu[3];  // padded voxel coordinate of the anchor c
    double du[3];  // voxel-coordinate advance per sample
};

// Unit direction and anchor of the ray through pixel (iu, iv) of view j, in
// binary64.  1/|d| comes from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ void ray_geom(const GeomDev &G, const DevGrid &g, int j, int iu, int iv,
                                         Ray &r) {
    const float *v = G.views + 12 * (int64_t)j;
    const double au = (double)iu - 0.5 * (double)(G.nu - 1);
    const double av = (double)iv - 0.5 * (double)(G.nv - 1);
    double d[3], o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double pix = fma(av, (double)v[9 + a], fma(au, (double)v[6 + a], (double)v[3 + a]));
        if (G.kind == DGR_PARALLEL) {
            d[a] = (double)v[a];
            o[a] = pix;
        } else {
            d[a] = pix - (double)v[a];
            o[a] = (double)v[a];
        }
    }
    const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double y = __builtin_amdgcn_rsq(n2);
    y = y * (1.5 - 0.5 * n2 * y * y);
    y = y * (1.5 - 0.5 * n2 * y * y);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= y;
    const double od = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double c = o[a] - od * d[a];
        r.cu[a] = (c - (double)g.lo[a]) * (double)g.inv_h[a] + (kPad - 0.5);
        r.du[a] = d[a] * ((double)g.inv_h[a] * G.step);
    }
}

// Samples k in [*k0, *k1] are those with lo <= u_a <= hi on every axis (padded
// coordinates), computed exactly in binary64.  False if there are none.
__device__ bool k_interval(const Ray &r, const double lo[3], const double hi[3], int *k0, int *k1) {
    double tmin = -1e300, tmax = 1e300;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.du[a] == 0.0) {
            if (!(r.cu[a] >= lo[a] && r.cu[a] <= hi[a])) return false;
            continue;
        }
        double t0 = (lo[a] - r.cu[a]) / r.du[a], t1 = (hi[a] - r.cu[a]) / r.du[a];
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    }
    const double kk0 = ceil(tmin), kk1 = floor(tmax);
    // Supports beyond +-2^30 samples of the anchor are treated as misses.
    if (!(kk0 <= kk1) || kk0 < -1073741824.0 || kk1 > 1073741824.0) return false;
    *k0 = (int)kk0;
    *k1 = (int)kk1;
    return true;
}

__device__ __forceinline__ bool support_range(const Ray &r, const DevGrid &g, int *k0, int *k1) {
    // support of the interpolant: -1 <= u <= dims  (padded: 1 .. dims + 2)
    const double lo[3] = {kPad - 1.0, kPad - 1.0, kPad - 1.0};
    const double hi[3] = {(double)g.nx + kPad, (double)g.ny + kPad, (double)g.nz + kPad};
    return k_interval(r, lo, hi, k0, k1);
}

constexpr int kSeg = 32;  // samples per re-anchored segment (a power of two)

__device__ __forceinline__ void seg_base(const Ray &r, int kb, int ib[3], float bf[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = r.cu[a] + (double)kb * r.du[a];
        const double f = floor(u);
        ib[a] = (int)f;
        bf[a] = (float)(u - f);
    }
}

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

__device__ __forceinline__ f2u ld2(const float *p) { return *reinterpret_cast<const f2u *>(p); }

// The floors are clamped so that every tap stays inside the padded volume: a
// no-op for every sample of the support (whose taps lie in [0, dims + 3]); it
// only guards the buffer against non-finite geometry.

__device__ float march(const float *__restrict__ vp, const PadDims &p, const Ray &r, int k0, int k1) {
    const float dux = (float)r.du[0], duy = (float)r.du[1], duz = (float)r.du[2];
    const int px = p.px;
    const int plane = (int)p.plane;
    float acc = 0.0f;
    for (int k = k0; k <= k1;) {
        const int kb = k & ~(kSeg - 1);
        const int kend = min(kb + kSeg - 1, k1);
        int ib[3];
        float b[3];
        seg_base(r, kb, ib, b);
        // relative clamp bounds keep every absolute floor in [0, dims + 2]
        const float lx = (float)(-ib[0]), ly = (float)(-ib[1]), lz = (float)(-ib[2]);
        const float hx = (float)(p.px - 2 - ib[0]), hy = (float)(p.py - 2 - ib[1]),
                    hz = (float)(p.pz - 2 - ib[2]);
        const float *vb = vp + (((int64_t)ib[2] * p.py + ib[1]) * px + ib[0]);
        for (int m = k - kb; m <= kend - kb; ++m) {
            const float fm = (float)m;
            const float ux = fmaf(fm, dux, b[0]), uy = fmaf(fm, duy, b[1]), uz = fmaf(fm, duz, b[2]);
            const float flx = __builtin_amdgcn_fmed3f(floorf(ux), lx, hx);
            const float fly = __builtin_amdgcn_fmed3f(floorf(uy), ly, hy);
            const float flz = __builtin_amdgcn_fmed3f(floorf(uz), lz, hz);
            const float wx = ux - flx, wy = uy - fly, wz = uz - flz;
            const int idx = ((int)flz * p.py + (int)fly) * px + (int)flx;
            const f2u a00 = ld2(vb + idx), a10 = ld2(vb + idx + px);
            const f2u a01 = ld2(vb + idx + plane), a11 = ld2(vb + idx + plane + px);
            const float c00 = fmaf(wx, a00.y - a00.x, a00.x);
            const float c10 = fmaf(wx, a10.y - a10.x, a10.x);
            const float c01 = fmaf(wx, a01.y - a01.x, a01.x);
            const float c11 = fmaf(wx, a11.y - a11.x, a11.x);
            const float c0 = fmaf(wy, c10 - c00, c00);
            const float c1 = fmaf(wy, c11 - c01, c01);
            acc += fmaf(wz, c1 - c0, c0);
        }
        k = kend + 1;
    }
    return acc;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// mode 0: write P_hat; mode 1: fused L1 (loss partial per work-group + dproj).
template <int MODE>
__global__ __launch_bounds__(256) void project_rays(const float *__restrict__ vp, PadDims p, DevGrid g,
                                                    GeomDev G, int tiles_u, int tiles_v,
                                                    const float *__restrict__ target,
                                                    float *__restrict__ out, float inv_m,
                                                    float *__restrict__ partial) {
    const int64_t b = blockIdx.x;
    const int per_view = tiles_u * tiles_v;
    const int j = (int)(b / per_view);
    const int rem = (int)(b - (int64_t)j * per_view);
    const int tv = rem / tiles_u, tu = rem - tv * tiles_u;
    const int iu = tu * kRayTile + (threadIdx.x & (kRayTile - 1));
    const int iv = tv * kRayTile + (threadIdx.x / kRayTile);
    const bool live = iu < G.nu && iv < G.nv;
    float val = 0.0f;
    if (live) {
        Ray r;
        ray_geom(G, g, j, iu, iv, r);
        int k0, k1;
        if (support_range(r, g, &k0, &k1)) val = march(vp, p, r, k0, k1);
        val *= G.scale;
    }
    const int64_t ri = ((int64_t)j * G.nv + iv) * G.nu + iu;
    if (MODE == 0) {
        if (live) out[ri] = val;
        return;
    }
    float absr = 0.0f;
    if (live) {
        const float res = val - target[ri];
        out[ri] = res > 0.0f ? inv_m : (res < 0.0f ? -inv_m : 0.0f);
        absr = fabsf(res);
    }
    __shared__ float ws[4];
    absr = wave_sum(absr);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = absr;
    __syncthreads();
    if (threadIdx.x == 0) partial[b] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Sum of the work-group partials in binary64, fixed order; loss = sum / M.
__global__ __launch_bounds__(256) void finish_loss(const float *__restrict__ partial, int64_t nb,
                                                   double inv_m, float *__restrict__ loss) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) acc += (double)partial[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] * inv_m);
}

// ---- backprojection ---------------------------------------------------------

// Detector rectangle (pixel indices, inclusive, widened by one pixel) that
// contains the shadow of every brick's cell box, per (brick, view).  A box is
// convex, so its shadow lies in the bounding rectangle of its eight projected
// corners.  If a corner cannot be projected (behind the source, or a ray
// parallel to the detector) the whole detector is used.
__global__ __launch_bounds__(256) void brick_rects(GeomDev G, DevGrid g, Bricks bk,
                                                   ushort4 *__restrict__ rect) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nb = bk.count();
    if (i >= nb * G.n_views) return;
    const int j = (int)(i / nb);
    const int64_t b = i - (int64_t)j * nb;
    const int bx = (int)(b % bk.nx), by = (int)((b / bk.nx) % bk.ny), bz = (int)(b / ((int64_t)bk.nx * bk.ny));
    const int cb[3] = {bx * kB - 1, by * kB - 1, bz * kB - 1};
    const float *v = G.views + 12 * (int64_t)j;
    double A[3], D0[3], eu[3], ev[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = v[a];
        D0[a] = v[3 + a];
        eu[a] = v[6 + a];
        ev[a] = v[9 + a];
    }
    const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2],
                         eu[0] * ev[1] - eu[1] * ev[0]};
    const double uu = eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2];
    const double vv = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
    const double uv = eu[0] * ev[0] + eu[1] * ev[1] + eu[2] * ev[2];
    const double det2 = uu * vv - uv * uv;
    double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
    bool ok = det2 > 0.0;
    for (int c = 0; c < 8 && ok; ++c) {
        double X[3];
        for (int a = 0; a < 3; ++a) {
            const double ucell = (double)(cb[a] + (((c >> a) & 1) ? kB : 0));  // cell box corner, u
            X[a] = (double)g.lo[a] + (ucell + 0.5) / (double)g.inv_h[a];
        }
        double dir[3], P[3];
        if (G.kind == DGR_PARALLEL) {
            for (int a = 0; a < 3; ++a) dir[a] = A[a];
        } else {
            for (int a = 0; a < 3; ++a) dir[a] = X[a] - A[a];
        }
        const double den = n[0] * dir[0] + n[1] * dir[1] + n[2] * dir[2];
        if (!(fabs(den) > 1e-300)) { ok = false; break; }
        const double num = n[0] * (D0[0] - X[0]) + n[1] * (D0[1] - X[1]) + n[2] * (D0[2] - X[2]);
        const double t = num / den;
        if (G.kind == DGR_CONE && !(t > -1.0)) { ok = false; break; }  // corner behind the source
        for (int a = 0; a < 3; ++a) P[a] = X[a] + t * dir[a] - D0[a];
        const double pu = P[0] * eu[0] + P[1] * eu[1] + P[2] * eu[2];
        const double pv = P[0] * ev[0] + P[1] * ev[1] + P[2] * ev[2];
        const double ca = (pu * vv - pv * uv) / det2, cbv = (pv * uu - pu * uv) / det2;
        amin = fmin(amin, ca); amax = fmax(amax, ca);
        bmin = fmin(bmin, cbv); bmax = fmax(bmax, cbv);
    }
    int iu0 = 0, iu1 = G.nu - 1, iv0 = 0, iv1 = G.nv - 1;
    if (ok) {
        const double cu = 0.5 * (G.nu - 1), cv = 0.5 * (G.nv - 1);
        iu0 = (int)fmax(0.0, floor(amin + cu) - 1.0);
        iu1 = (int)fmin((double)(G.nu - 1), ceil(amax + cu) + 1.0);
        iv0 = (int)fmax(0.0, floor(bmin + cv) - 1.0);
        iv1 = (int)fmin((double)(G.nv - 1), ceil(bmax + cv) + 1.0);
        if (iu0 > iu1 || iv0 > iv1) { iu0 = 1; iu1 = 0; iv0 = 1; iv1 = 0; }  // empty
    }
    rect[i] = make_ushort4((unsigned short)iu0, (unsigned short)iu1, (unsigned short)iv0, (unsigned short)iv1);
}

// max |proj| as the bit pattern of a non-negative float (bit order = value order).
__global__ __launch_bounds__(256) void zero_u32(unsigned *__restrict__ p) { *p = 0u; }

__global__ __launch_bounds__(256) void absmax_bits(const float *__restrict__ x, int64_t n,
                                                   unsigned *__restrict__ out) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(x[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Fixed-point scale: the largest power of two S with |proj| * |scale| * S < 2^30.
__device__ __forceinline__ float fixed_scale(const unsigned *maxbits, float scale) {
    const float mc = __uint_as_float(*maxbits) * fabsf(scale);
    if (!(mc > 0.0f) || !(mc < 3.0e38f)) return 1.0f;
    int e;
    frexpf(mc, &e);  // mc < 2^e
    return ldexpf(1.0f, 30 - e);
}

// One work-group per brick.  For every view, each thread takes candidate rays
// of the brick's shadow rectangle, finds the samples whose trilinear cell lies
// in the brick (cell test on the same binary32 position as the projector), and
// adds the eight weighted values, in fixed point, into the LDS tile.
__global__ __launch_bounds__(256) void backproject_bricks(const float *__restrict__ proj, DevGrid g,
                                                          GeomDev G, Bricks bk,
                                                          const ushort4 *__restrict__ rect,
                                                          float eps, const unsigned *__restrict__ maxbits,
                                                          long long *__restrict__ staging) {
    __shared__ unsigned long long tile[kBT3];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t nb = bk.count();
    const int bx = (int)(b % bk.nx), by = (int)((b / bk.nx) % bk.ny), bz = (int)(b / ((int64_t)bk.nx * bk.ny));
    // brick cells in padded coordinates: [c0, c0 + kB)
    const int c0x = bx * kB - 1 + kPad, c0y = by * kB - 1 + kPad, c0z = bz * kB - 1 + kPad;
    // The candidate k-range is exact in binary64 for the brick grown by eps, a
    // bound on |binary32 position - binary64 position|; the cell test on the
    // binary32 position then assigns every sample to exactly one brick.
    const double blo[3] = {c0x - (double)eps, c0y - (double)eps, c0z - (double)eps};
    const double bhi[3] = {c0x + kB + (double)eps, c0y + kB + (double)eps, c0z + kB + (double)eps};
    const float gs = G.scale * fixed_scale(maxbits, G.scale);  // |proj * gs| < 2^30
    for (int e = t; e < kBT3; e += 256) tile[e] = 0ull;
    __syncthreads();
    for (int j = 0; j < G.n_views; ++j) {
        const ushort4 rc = rect[(int64_t)j * nb + b];
        const int nu_r = (int)rc.y - (int)rc.x + 1, nv_r = (int)rc.w - (int)rc.z + 1;
        const int ncand = (nu_r > 0 && nv_r > 0) ? nu_r * nv_r : 0;
        for (int c = t; c < ncand; c += 256) {
            const int iv = (int)rc.z + c / nu_r, iu = (int)rc.x + c % nu_r;
            const float gr = gs * proj[((int64_t)j * G.nv + iv) * G.nu + iu];
            if (gr == 0.0f) continue;
            Ray r;
            ray_geom(G, g, j, iu, iv, r);
            int k0, k1;
            if (!k_interval(r, blo, bhi, &k0, &k1)) continue;
            const float dux = (float)r.du[0], duy = (float)r.du[1], duz = (float)r.du[2];
            for (int k = k0; k <= k1;) {
                const int kb = k & ~(kSeg - 1);
                const int kend = min(kb + kSeg - 1, k1);
                int ib[3];
                float bs[3];
                seg_base(r, kb, ib, bs);
                const int ox = c0x - ib[0], oy = c0y - ib[1], oz = c0z - ib[2];
                for (int m = k - kb; m <= kend - kb; ++m) {
                    const float fm = (float)m;
                    const float ux = fmaf(fm, dux, bs[0]), uy = fmaf(fm, duy, bs[1]), uz = fmaf(fm, duz, bs[2]);
                    const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
                    const int lx = (int)flx - ox, ly = (int)fly - oy, lz = (int)flz - oz;
                    if ((unsigned)lx >= (unsigned)kB || (unsigned)ly >= (unsigned)kB ||
                        (unsigned)lz >= (unsigned)kB)
                        continue;
                    const float wx = ux - flx, wy = uy - fly, wz = uz - flz;
                    const float z1 = gr * wz, z0 = gr - z1;
                    const float y01 = z0 * wy, y00 = z0 - y01, y11 = z1 * wy, y10 = z1 - y11;
                    const float a0 = y00 * wx, a1 = y01 * wx, a2 = y10 * wx, a3 = y11 * wx;
                    unsigned long long *q = tile + (lz * kBT + ly) * kBT + lx;
                    atomicAdd(q, (unsigned long long)(long long)(int)(y00 - a0));
                    atomicAdd(q + 1, (unsigned long long)(long long)(int)a0);
                    atomicAdd(q + kBT, (unsigned long long)(long long)(int)(y01 - a1));
                    atomicAdd(q + kBT + 1, (unsigned long long)(long long)(int)a1);
                    atomicAdd(q + kBT * kBT, (unsigned long long)(long long)(int)(y10 - a2));
                    atomicAdd(q + kBT * kBT + 1, (unsigned long long)(long long)(int)a2);
                    atomicAdd(q + kBT * kBT + kBT, (unsigned long long)(long long)(int)(y11 - a3));
                    atomicAdd(q + kBT * kBT + kBT + 1, (unsigned long long)(long long)(int)a3);
                }
                k = kend + 1;
            }
        }
    }
    __syncthreads();
    long long *out = staging + b * kBT3;
    for (int e = t; e < kBT3; e += 256) out[e] = (long long)tile[e];
}

// Each voxel lies in one or two brick tiles per axis (tiles overlap by one
// voxel on their faces); its value is the exact integer sum of those tile
// entries divided by the fixed-point scale.
__global__ __launch_bounds__(256) void gather_bricks(const long long *__restrict__ staging, DevGrid g,
                                                     Bricks bk, const unsigned *__restrict__ maxbits,
                                                     float scale, float *__restrict__ V) {
    const double inv_s = 1.0 / (double)fixed_scale(maxbits, scale);
    const int64_t total = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t z = i / ((int64_t)g.nx * g.ny), rem = i - z * (int64_t)g.nx * g.ny;
        const int y = (int)(rem / g.nx), x = (int)(rem - (int64_t)y * g.nx);
        const int vv[3] = {x, y, (int)z};
        int nb[3], bb[3][2], ll[3][2];
        for (int a = 0; a < 3; ++a) {
            const int s = vv[a] + 1;  // local index in brick b is s - kB * b
            bb[a][0] = s / kB;
            ll[a][0] = s - kB * bb[a][0];
            nb[a] = 1;
            if (ll[a][0] == 0 && bb[a][0] > 0) {
                bb[a][1] = bb[a][0] - 1;
                ll[a][1] = kB;
                nb[a] = 2;
            }
        }
        long long acc = 0;
        for (int iz = 0; iz < nb[2]; ++iz)
            for (int iy = 0; iy < nb[1]; ++iy)
                for (int ix = 0; ix < nb[0]; ++ix) {
                    const int64_t brick = ((int64_t)bb[2][iz] * bk.ny + bb[1][iy]) * bk.nx + bb[0][ix];
                    acc += staging[brick * kBT3 + (ll[2][iz] * kBT + ll[1][iy]) * kBT + ll[0][ix]];
                }
        V[i] = (float)((double)acc * inv_s);
    }
}

// ---- workspace and entry points ------------------------------------------------
struct ProjWs {
    float *vpad;
    float *partial;
    long long *staging;
    ushort4 *rect;
    unsigned *maxbits;
    size_t bytes;
};

int64_t ray_blocks(const dgr_geometry *G, int *tu, int *tv) {
    *tu = (G->nu + kRayTile - 1) / kRayTile;
    *tv = (G->nv + kRayTile - 1) / kRayTile;
    return (int64_t)G->n_views * (*tu) * (*tv);
}

ProjWs carve_proj_ws(void *ws, const dgr_grid *grid, const dgr_geometry *geom) {
    // The forward pass uses vpad + partial; the backward pass staging + rect.
    // The two share the front of the workspace.
    ProjWs w;
    int tu, tv;
    Carver f(ws);
    w.vpad = f.take<float>(pad_count(grid));
    w.partial = f.take<float>(ray_blocks(geom, &tu, &tv));
    Carver b(ws);
    const Bricks bk = bricks_of(grid);
    w.staging = b.take<long long>(bk.count() * kBT3);
    w.rect = b.take<ushort4>(bk.count() * geom->n_views);
    w.maxbits = b.take<unsigned>(1);
    w.bytes = std::max(f.off, b.off);
    return w;
}

GeomDev geom_dev(const dgr_geometry *G) {
    GeomDev d;
    d.kind = G->kind;
    d.n_views = G->n_views;
    d.nu = G->nu;
    d.nv = G->nv;
    d.views = G->views;
    d.step = (double)G->step;
    d.scale = (float)((double)G->length_scale * (double)G->step);
    return d;
}

dgr_status check_proj(const dgr_grid *grid, const dgr_geometry *geom, void *ws, size_t ws_bytes) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_geometry(geom)) != DGR_OK) return s;
    DGR_CHECK(pad_count(grid) < (int64_t(1) << 31), "padded volume exceeds 2^31 voxels");
    {
        // Bound the samples per ray: the support's diagonal over the step.
        double diag2 = 0.0, min_inv = 1e300;
        for (int a = 0; a < 3; ++a) {
            diag2 += (double)(grid->dims[a] + 3) * (grid->dims[a] + 3);
            min_inv = std::min(min_inv, (double)grid->inv_h[a]);
        }
        double samples = std::sqrt(diag2) / ((double)geom->step * min_inv);
        DGR_CHECK(samples <= (double)(1 << 20), "step too small: %.3g samples per ray (limit 2^20)",
                  samples);
    }
    DGR_CHECK(ws != nullptr, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = carve_proj_ws(nullptr, grid, geom).bytes;
    if (ws_bytes < need)
        return fail(DGR_ERR_WORKSPACE, "workspace holds %zu bytes, projection needs %zu", ws_bytes, need);
    return DGR_OK;
}

unsigned grid_stride_blocks(int64_t n) {
    return (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_project_workspace(const dgr_grid *grid, const dgr_geometry *geom) {
    if (check_grid(grid) != DGR_OK || check_geometry(geom) != DGR_OK) return 0;
    return carve_proj_ws(nullptr, grid, geom).bytes;
}

template <int MODE>
static dgr_status project_impl(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                               const float *target, float *loss, float *out, void *ws,
                               size_t ws_bytes, void *stream) {
    dgr_status s = check_proj(grid, geom, ws, ws_bytes);
    if (s != DGR_OK) return s;
    DGR_CHECK(volume && out, "null volume or output pointer");
    if (MODE == 1) DGR_CHECK(target && loss, "null target or loss pointer");
    hipStream_t st = as_stream(stream);
    ProjWs w = carve_proj_ws(ws, grid, geom);
    PadDims p = pad_dims(grid);
    DevGrid g = dev_grid(grid);
    pad_volume<<<dim3(grid_stride_blocks(pad_count(grid))), dim3(256), 0, st>>>(volume, g, p, w.vpad);
    DGR_LAUNCH_CHECK();
    int tu, tv;
    const int64_t nb = ray_blocks(geom, &tu, &tv);
    const double m = (double)geom->n_views * geom->nu * geom->nv;
    project_rays<MODE><<<dim3((unsigned)nb), dim3(256), 0, st>>>(
        w.vpad, p, g, geom_dev(geom), tu, tv, target, out, (float)(1.0 / m), w.partial);
    DGR_LAUNCH_CHECK();
    if (MODE == 1) {
        finish_loss<<<1, 256, 0, st>>>(w.partial, nb, 1.0 / m, loss);
        DGR_LAUNCH_CHECK();
    }
    return DGR_OK;
}

extern "C" dgr_status dgr_project(const float *volume, const dgr_grid *grid, const dgr_geometry *geom,
                                  float *proj, void *ws, size_t ws_bytes, void *stream) {
    return project_impl<0>(volume, grid, geom, nullptr, nullptr, proj, ws, ws_bytes, stream);
}

extern "C" dgr_status dgr_project_l1(const float *volume, const dgr_grid *grid,
                                     const dgr_geometry *geom, const float *target, float *loss,
                                     float *dproj, void *ws, size_t ws_bytes, void *stream) {
    return project_impl<1>(volume, grid, geom, target, loss, dproj, ws, ws_bytes, stream);
}

extern "C" dgr_status dgr_backproject(const float *proj, const dgr_grid *grid,
                                      const dgr_geometry *geom, float *volume, void *ws,
                                      size_t ws_bytes, void *stream) {
    dgr_status s = check_proj(grid, geom, ws, ws_bytes);
    if (s != DGR_OK) return s;
    DGR_CHECK(proj && volume, "null projection or volume pointer");
    hipStream_t st = as_stream(stream);
    ProjWs w = carve_proj_ws(ws, grid, geom);
    DevGrid g = dev_grid(grid);
    const Bricks bk = bricks_of(grid);
    const GeomDev G = geom_dev(geom);
    const int64_t nrect = bk.count() * geom->n_views;
    brick_rects<<<dim3((unsigned)((nrect + 255) / 256)), dim3(256), 0, st>>>(G, g, bk, w.rect);
    DGR_LAUNCH_CHECK();
    // Bound on |binary32 - binary64| sample positions: offsets within a segment
    // stay below kSeg * |du| + 1 voxel, each coordinate sees a few binary32
    // roundings of that size; a factor 8 of margin on top.
    const double du_max = (double)geom->step *
                          std::max((double)grid->inv_h[0], std::max((double)grid->inv_h[1], (double)grid->inv_h[2]));
    const float eps = (float)(8.0 * std::ldexp(kSeg * du_max + 2.0, -24) + 1e-6);
    const int64_t nproj = (int64_t)geom->n_views * geom->nu * geom->nv;
    zero_u32<<<1, 1, 0, st>>>(w.maxbits);
    DGR_LAUNCH_CHECK();
    absmax_bits<<<dim3((unsigned)std::min<int64_t>((nproj + 255) / 256, 4096)), dim3(256), 0, st>>>(
        proj, nproj, w.maxbits);
    DGR_LAUNCH_CHECK();
    backproject_bricks<<<dim3((unsigned)bk.count()), dim3(256), 0, st>>>(proj, g, G, bk, w.rect, eps,
                                                                         w.maxbits, w.staging);
    DGR_LAUNCH_CHECK();
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    gather_bricks<<<dim3(grid_stride_blocks(nvox)), dim3(256), 0, st>>>(w.staging, g, bk, w.maxbits,
                                                                        G.scale, volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
