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
// binary64 and is then rounded to 64-bit fixed point with 32 fractional bits:
// U_k = U_c + k * DU.  The integer part (high word) is the floor used for the
// taps, the low word times 2^-32 is the trilinear weight.  Integer steps are
// exact, so sample k has the same position in every kernel and every brick,
// from any starting sample, and stays within ~5e-8 voxel of the binary64
// position; no periodic re-anchoring is needed.
// Forward: one thread per ray; the volume is read from a copy with a two-voxel
// zero border, so the eight taps of any sample in the support need no test.
// Backward: each ray is set up once per view batch into a table row; one
// work-group per 20 x 20 x 6-cell brick accumulates, over all views, the
// samples whose trilinear cell lies in the brick into a 21 x 21 x 7 LDS tile
// (flat bricks: for nearly horizontal rays the detector footprint of a brick
// shrinks while the samples per ray grow; 37 KB of LDS, four work-groups per
// CU; no global atomics); the tiles are then summed per voxel.  The LDS sums are
// 64-bit fixed point: the weights of the samples of one ray in one cell are
// summed in registers, scaled by a power of two S chosen from max|proj| so that
// the sum fits in 32 bits, converted to an integer (within one unit) and added
// with ds_add_u64.
// Integer addition makes the result independent of the order of the adds
// between rays (the order within a ray is fixed).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr int kPad = 2;
constexpr int kXcd = 8;     // MI355X: work-groups are dealt round-robin to 8 XCDs
// Backprojection bricks: kBX x kBY x kBZ cells (<= 32 each: 5-bit local
// cells in the ray records), tiles one voxel larger per axis.
#ifndef DGR_BRICK_X
#define DGR_BRICK_X 20
#endif
#ifndef DGR_BRICK_Y
#define DGR_BRICK_Y 20
#endif
#ifndef DGR_BRICK_Z
#define DGR_BRICK_Z 6
#endif
#ifndef DGR_BP_WAVES
#define DGR_BP_WAVES 4
#endif
constexpr int kBX = DGR_BRICK_X, kBY = DGR_BRICK_Y, kBZ = DGR_BRICK_Z;
constexpr int kTBX = kBX + 1, kTBY = kBY + 1, kTBZ = kBZ + 1;
constexpr int kBT3 = kTBX * kTBY * kTBZ;
static_assert(kBX <= 32 && kBY <= 32 && kBZ <= 32, "local cells are 5-bit");

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
    b.nx = (g->dims[0] + 1 + kBX - 1) / kBX;
    b.ny = (g->dims[1] + 1 + kBY - 1) / kBY;
    b.nz = (g->dims[2] + 1 + kBZ - 1) / kBZ;
    return b;
}

// Zero-bordered copy of V, [z][y][x], two voxels of zeros on every side, so
// the eight taps of any sample in the support need no bounds test.
__global__ __launch_bounds__(256) void pad_volume(const float *__restrict__ V, DevGrid g, PadDims p,
                                                  float *__restrict__ out) {
    const int64_t total = p.plane * p.pz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        int64_t z = i / p.plane, rem = i - z * p.plane;
        int64_t y = rem / p.px, x = rem - y * p.px;
        x -= kPad;
        y -= kPad;
        z -= kPad;
        out[i] = (x >= 0 && y >= 0 && z >= 0 && x < g.nx && y < g.ny && z < g.nz)
                     ? V[(z * g.ny + y) * g.nx + x] : 0.0f;
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
    long long U[3];   // cu in 32.32 fixed point
    long long DU[3];  // du in 32.32 fixed point
};

constexpr double kTwo32 = 4294967296.0;
constexpr float kInv32 = 2.3283064365386963e-10f;  // 2^-32
constexpr double kMaxK = 4194304.0;                 // |k| limit (2^22) for fixed-point exactness


// Unit direction and anchor of the ray through pixel (iu, iv) of view j, in
// binary64 (fan beam: the source of row iv is a + av e_v).  1/|d| comes from
// the hardware estimate refined by two Newton steps.
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
            const double src = G.kind == DGR_FAN ? fma(av, (double)v[9 + a], (double)v[a]) : (double)v[a];
            d[a] = pix - src;
            o[a] = src;
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
        // |cu| < 2^30 keeps U and every in-range position below 2^62 (the
        // caller treats larger anchors as misses through k_interval's guard)
        const double cu_c = fmin(fmax(r.cu[a], -1073741824.0), 1073741824.0);
        r.U[a] = __double2ll_rn(cu_c * kTwo32);
        r.DU[a] = __double2ll_rn(r.du[a] * kTwo32);
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
    // Samples beyond +-2^22 of the anchor, or anchors beyond 2^30 voxels, are
    // treated as misses (absurdly placed grids); this keeps the fixed-point
    // positions within 2^-10 voxel of the binary64 ones.
    if (!(kk0 <= kk1) || kk0 < -kMaxK || kk1 > kMaxK) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(fabs(r.cu[a]) < 1073741824.0)) return false;
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

// Every sample of the support range has its floor in [0, dims + 2] (padded),
// because the fixed-point position is within 2^-10 voxel of the binary64 one
// that defined the range; its eight taps are therefore inside the padded copy.

// Trilinear value of one sample from 8 taps at q (x fastest; strides sy, sz).
__device__ __forceinline__ float trilinear(const float *q, int sy, int sz, float wx, float wy, float wz) {
    const float c00 = fmaf(wx, q[1] - q[0], q[0]);
    const float c10 = fmaf(wx, q[sy + 1] - q[sy], q[sy]);
    const float c01 = fmaf(wx, q[sz + 1] - q[sz], q[sz]);
    const float c11 = fmaf(wx, q[sz + sy + 1] - q[sz + sy], q[sz + sy]);
    const float c0 = fmaf(wy, c10 - c00, c00);
    const float c1 = fmaf(wy, c11 - c01, c01);
    return fmaf(wz, c1 - c0, c0);
}

// Samples a..e of ray r, taps read from a volume whose element (0, 0, 0) is
// the padded voxel o (strides sy, sz): the LDS box or the padded copy itself.
__device__ __forceinline__ void march_span(const float *vol, int sy, int sz, const int o[3], const Ray &r,
                                           int a, int e, float &acc) {
    long long ux = r.U[0] + (long long)a * r.DU[0] - ((long long)o[0] << 32);
    long long uy = r.U[1] + (long long)a * r.DU[1] - ((long long)o[1] << 32);
    long long uz = r.U[2] + (long long)a * r.DU[2] - ((long long)o[2] << 32);
    for (int k = a; k <= e; ++k) {
        const int lx = (int)(ux >> 32), ly = (int)(uy >> 32), lz = (int)(uz >> 32);
        const float wx = (float)(unsigned)ux * kInv32;
        const float wy = (float)(unsigned)uy * kInv32;
        const float wz = (float)(unsigned)uz * kInv32;
        acc += trilinear(vol + (int64_t)lz * sz + (int64_t)ly * sy + lx, sy, sz, wx, wy, wz);
        ux += r.DU[0];
        uy += r.DU[1];
        uz += r.DU[2];
    }
}

// march_span over the LDS box: the tap's byte offset (cells within the box, so
// every term is below 2^24) takes two 24-bit multiplies per sample instead of
// two full-width multiplies and a scaling of each term.
// PLANAR: the ray has no advance in z and a whole-voxel z position, so every
// sample's z weight is 0 and the trilinear value is the bilinear one of the
// lower plane, bit for bit (its last lerp adds 0 times a finite difference):
// four taps instead of eight.
template <bool PLANAR>
__device__ __forceinline__ void march_box(const float *box, int sy, int sz, const int o[3], const Ray &r,
                                          int a, int e, float &acc) {
    const unsigned sy4 = 4u * (unsigned)sy, sz4 = 4u * (unsigned)sz;  // byte strides
    long long ux = r.U[0] + (long long)a * r.DU[0] - ((long long)o[0] << 32);
    long long uy = r.U[1] + (long long)a * r.DU[1] - ((long long)o[1] << 32);
    long long uz = r.U[2] + (long long)a * r.DU[2] - ((long long)o[2] << 32);
    for (int k = a; k <= e; ++k) {
        const int lx = (int)(ux >> 32), ly = (int)(uy >> 32), lz = (int)(uz >> 32);
        const float wx = (float)(unsigned)ux * kInv32;
        const float wy = (float)(unsigned)uy * kInv32;
        const float wz = PLANAR ? 0.0f : (float)(unsigned)uz * kInv32;
        const unsigned off = __umul24((unsigned)lz, sz4) + __umul24((unsigned)ly, sy4) + ((unsigned)lx << 2);
        const float *q = reinterpret_cast<const float *>(reinterpret_cast<const char *>(box) + off);
        if (PLANAR) {
            const float c00 = fmaf(wx, q[1] - q[0], q[0]);
            const float c10 = fmaf(wx, q[sy + 1] - q[sy], q[sy]);
            acc += fmaf(wy, c10 - c00, c00);
        } else {
            acc += trilinear(q, sy, sz, wx, wy, wz);
        }
        ux += r.DU[0];
        uy += r.DU[1];
        if (!PLANAR) uz += r.DU[2];
    }
}

// Minimum / maximum over the 64 lanes of a wave (all lanes active), returned
// wave-uniform: DPP exchanges within each row of 16 lanes (lane ^ 1, lane ^ 2,
// then the mirrored lane of the half row and of the row), then the four rows'
// lane 0 through readlane.  No LDS traffic, unlike a shuffle.
__device__ __forceinline__ int row_dpp(int v, int ctrl) {
    switch (ctrl) {  // the control must be a constant
        case 0: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 1: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 2: return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
        default: return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false); // row_mirror
    }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v = min(v, row_dpp(v, c));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v = max(v, row_dpp(v, c));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Forward projection, one work-group per 16 x 16 pixel bundle of one view.
// The bundle's rays are marched in chunks of kFwdChunk samples: for each chunk
// the work-group finds the box of cells its samples touch (sample positions
// are affine in k, so the floors at the two ends of each ray's span bound
// them), copies that box of the padded volume into LDS with coalesced rows,
// and reads the eight taps of every sample from LDS.  The box is stored dense
// (x fastest, its own extents as strides), so any shape up to the box
// capacity fits: rays of a cone-beam bundle are nearly parallel (about 16 x
// 16 x 13 cells for an 8-voxel chunk at 45 degrees), a fan-beam bundle's 16
// rows span 16 slices.  A chunk whose box exceeds the capacity reads its taps
// from the padded copy instead.  Work-groups are numbered so each XCD (which
// receives every 8th dispatched work-group) runs a contiguous range of
// bundles.
// NR rays per thread: a cone-beam work-group takes two 16 x 16 bundles side
// by side in u (32 x 16 pixels), so the block-wide bound reductions, the
// barriers and the row-wise staging of each box are shared by twice the
// samples (70 VGPRs; a 22 KB box, so that seven work-groups fit a CU).  Fan
// and parallel beams take one bundle with a larger box (28 KB, five
// work-groups per CU): a fan bundle's 16 rows make taller boxes, and a chunk
// that overflows reads its taps from HBM; 7,000 cells balance the two on the
// fan-beam scans (a larger box costs a work-group per CU).
// mode 0: write P_hat; mode 1: fused L1 (loss partial per work-group + dproj).
constexpr int kBun = 16;  // bundle edge (pixels)
constexpr int box_cap(int nr) { return nr == 1 ? 7000 : 5600; }  // LDS box (cells)
constexpr int kFwdChunk = 16;    // samples per chunk

__device__ __forceinline__ void block_bounds(int v[6], int (*red)[8], int wave, int lane) {
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = wave_min(v[i]);
#pragma unroll
    for (int i = 3; i < 6; ++i) v[i] = wave_max(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) red[wave][i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = min(min(red[0][i], red[1][i]), min(red[2][i], red[3][i]));
#pragma unroll
    for (int i = 3; i < 6; ++i) v[i] = max(max(red[0][i], red[1][i]), max(red[2][i], red[3][i]));
}

// Copies the box of nx x ny x nz padded voxels at src (strides px, plane) into
// LDS, dense with x fastest.  Box element q is cell (q mod nx, (q / nx) mod
// ny, q / (nx ny)); the quotients come from binary32 reciprocals, exact here:
// (q + 1/2) / n_a lies at least 1/(2 n_a) from an integer and its rounding
// error (reciprocal and fused product) is below (q + 1/2) / n_a * 2^-23,
// smaller for q < 2^22.  Offsets are 32-bit (the padded copy holds fewer than
// 2^31 voxels); kSmall: the padded plane is below 2^24 voxels, so their
// products take 24-bit multiplies.  Each thread issues kStage loads before its
// first LDS write, so the loads overlap.
template <bool kSmall>
__device__ __forceinline__ void stage_box(float *box, const float *__restrict__ src, int nx, int ny, int nz,
                                          unsigned px, unsigned plane) {
    const int n = nx * ny * nz;
    const float inx = 1.0f / (float)nx, iny = 1.0f / (float)ny;
    const float hnx = 0.5f * inx, hny = 0.5f * iny;  // exact halves
    constexpr int kStage = 4;
    for (int q0 = threadIdx.x; q0 < n; q0 += 256 * kStage) {
        float v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int q = q0 + u * 256;
            if (q < n) {
                const int rq = (int)fmaf((float)q, inx, hnx);
                const int lz = (int)fmaf((float)rq, iny, hny);
                const int lx = q - __mul24(rq, nx), ly = rq - __mul24(lz, ny);
                const unsigned off = kSmall ? __umul24((unsigned)lz, plane) + __umul24((unsigned)ly, px) + (unsigned)lx
                                            : (unsigned)lz * plane + (unsigned)ly * px + (unsigned)lx;
                v[u] = src[off];
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u)
            if (q0 + u * 256 < n) box[q0 + u * 256] = v[u];
    }
}

template <int MODE, int NR>
__global__ __launch_bounds__(256) void project_bundles(const float *__restrict__ vp, PadDims p, DevGrid g,
                                                       GeomDev G, int tiles_u, int tiles_v, int64_t nb,
                                                       const float *__restrict__ target,
                                                       float *__restrict__ out, float inv_m,
                                                       float *__restrict__ partial) {
    constexpr int kCap = box_cap(NR);
    __shared__ float box[kCap];
    __shared__ int red[2][4][8];
    const int64_t per_xcd = (nb + kXcd - 1) / kXcd;
    const int64_t b = (int64_t)(blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd;
    if (b >= nb) return;  // whole work-group
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per_view = tiles_u * tiles_v;
    const int j = (int)(b / per_view);
    const int rem = (int)(b - (int64_t)j * per_view);
    const int tv = rem / tiles_u, tu = rem - tv * tiles_u;
    const int iv = tv * kBun + (t / kBun);
    // ray q of this thread: pixel (iu[q], iv), bundle q of the tile
    int iu[NR], k0[NR], k1[NR];
    bool live[NR], ok[NR];
    Ray r[NR];
    int kr[6] = {0x7fffffff, 0, 0, -0x7fffffff, 0, 0};
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        iu[q] = tu * (kBun * NR) + q * kBun + (t & (kBun - 1));
        live[q] = iu[q] < G.nu && iv < G.nv;
        ok[q] = false;
        k0[q] = 0;
        k1[q] = -1;
        if (live[q]) {
            ray_geom(G, g, j, iu[q], iv, r[q]);
            ok[q] = support_range(r[q], g, &k0[q], &k1[q]);
        }
        if (ok[q]) {
            kr[0] = min(kr[0], k0[q]);
            kr[3] = max(kr[3], k1[q]);
        }
    }
    // one ray per thread (fan and parallel beams): the wave marches the
    // lower plane only where all of its rays are planar (see march_box)
    bool planar = false;
    if constexpr (NR == 1) planar = __ballot(!ok[0] || (r[0].DU[2] == 0 && (unsigned)r[0].U[2] == 0u)) == __ballot(1);
    block_bounds(kr, red[1], wave, lane);
    const int kmin = kr[0], kmax = kr[3];
    const int sy = (int)p.px, sz = (int)p.plane;
    float acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = 0.0f;
    int it = 0;
    for (int K = kmin; K <= kmax; K += kFwdChunk, ++it) {
        const int Ke = min(K + kFwdChunk - 1, kmax);
        int a[NR], e[NR];
        bool has[NR];
        int bb[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -0x7fffffff, -0x7fffffff, -0x7fffffff};
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            a[q] = max(K, k0[q]);
            e[q] = min(Ke, k1[q]);
            has[q] = ok[q] && a[q] <= e[q];
            if (has[q]) {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const int fa = (int)((r[q].U[ax] + (long long)a[q] * r[q].DU[ax]) >> 32);
                    const int fe = (int)((r[q].U[ax] + (long long)e[q] * r[q].DU[ax]) >> 32);
                    bb[ax] = min(bb[ax], min(fa, fe));
                    bb[3 + ax] = max(bb[3 + ax], max(fa, fe));
                }
            }
        }
        block_bounds(bb, red[it & 1], wave, lane);  // alternate buffers: no reuse race
        // No ray of the work-group has a sample in this chunk (the union of
        // the rays' sample ranges can have gaps): the bounds are still the
        // sentinels.  The test is uniform over the work-group.
        if (bb[0] > bb[3]) continue;
        const int o[3] = {bb[0], bb[1], bb[2]};
        const int nx = bb[3] - bb[0] + 2, ny = bb[4] - bb[1] + 2, nz = bb[5] - bb[2] + 2;
        if ((int64_t)nx * ny * nz <= kCap) {
            // taps of the chunk: padded voxels o .. o + n - 1, inside the padded
            // copy
            const float *src = vp + ((int64_t)o[2] * p.py + o[1]) * p.px + o[0];
            if (p.plane < (int64_t(1) << 24))
                stage_box<true>(box, src, nx, ny, nz, (unsigned)p.px, (unsigned)p.plane);
            else
                stage_box<false>(box, src, nx, ny, nz, (unsigned)p.px, (unsigned)p.plane);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (has[q]) {
                    if (NR == 1 && planar)
                        march_box<true>(box, nx, nx * ny, o, r[q], a[q], e[q], acc[q]);
                    else
                        march_box<false>(box, nx, nx * ny, o, r[q], a[q], e[q], acc[q]);
                }
            __syncthreads();
        } else {
            const int o0[3] = {0, 0, 0};
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (has[q]) march_span(vp, sy, sz, o0, r[q], a[q], e[q], acc[q]);
        }
    }
    float absr = 0.0f;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const float val = acc[q] * G.scale;
        const int64_t ri = ((int64_t)j * G.nv + iv) * G.nu + iu[q];
        if (MODE == 0) {
            if (live[q]) out[ri] = val;
        } else if (live[q]) {
            const float res = val - target[ri];
            out[ri] = res > 0.0f ? inv_m : (res < 0.0f ? -inv_m : 0.0f);
            absr += fabsf(res);
        }
    }
    if (MODE == 0) return;
    __shared__ float ws[4];
    absr = wave_sum(absr);
    if (lane == 0) ws[wave] = absr;
    __syncthreads();
    if (t == 0) partial[b] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Sum of the work-group partials in binary64, fixed order; loss = sum / M.
// One work-group of 1024 threads; each thread keeps eight independent sums
// so that eight loads are in flight at a time.
__global__ __launch_bounds__(1024) void finish_loss(const float *__restrict__ partial, int64_t nb,
                                                    double inv_m, float *__restrict__ loss) {
    __shared__ double s[1024];
    constexpr int kU = 8;
    double acc[kU] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t i = threadIdx.x;
    for (; i + (kU - 1) * 1024 < nb; i += kU * 1024) {
        float p[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) p[u] = partial[i + u * 1024];
#pragma unroll
        for (int u = 0; u < kU; ++u) acc[u] += (double)p[u];
    }
    for (; i < nb; i += 1024) acc[0] += (double)partial[i];
    s[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] * inv_m);
}

// ---- backprojection ---------------------------------------------------------

// Detector rectangle that contains the shadow of each brick's cell box, per
// (brick, view) (see shadow_rect).
__global__ __launch_bounds__(256) void brick_rects(GeomDev G, DevGrid g, Bricks bk,
                                                   ushort4 *__restrict__ rect) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nb = bk.count();
    if (i >= nb * G.n_views) return;
    const int j = (int)(i / nb);
    const int64_t b = i - (int64_t)j * nb;
    const int bx = (int)(b % bk.nx), by = (int)((b / bk.nx) % bk.ny), bz = (int)(b / ((int64_t)bk.nx * bk.ny));
    // the brick's cells span voxel coordinates [c0, c0 + kB] (unpadded)
    const double ulo[3] = {(double)(bx * kBX - 1), (double)(by * kBY - 1), (double)(bz * kBZ - 1)};
    const double uhi[3] = {ulo[0] + kBX, ulo[1] + kBY, ulo[2] + kBZ};
    int iu0, iu1, iv0, iv1;
    shadow_rect(G.kind, G.views + 12 * (int64_t)j, G.nu, G.nv, g, ulo, uhi, &iu0, &iu1, &iv0, &iv1);
    if (iu0 > iu1 || iv0 > iv1) { iu0 = 1; iu1 = 0; iv0 = 1; iv1 = 0; }
    rect[i] = make_ushort4((unsigned short)iu0, (unsigned short)iu1, (unsigned short)iv0, (unsigned short)iv1);
}

// max |proj| as the bit pattern of a non-negative float (bit order = value order).
__global__ __launch_bounds__(256) void zero_u32x2(unsigned *__restrict__ p) {
    if (threadIdx.x < 2) p[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void absmax_bits(const float *__restrict__ x, int64_t n,
                                                   unsigned *__restrict__ out) {
    // 16-byte loads (four in flight per thread) over the aligned body, then
    // the ragged head and tail; one atomic per wave
    float m = 0.0f;
    const int64_t head = std::min<int64_t>(n, (int64_t)((16 - (reinterpret_cast<uintptr_t>(x) & 15)) & 15) / 4);
    const int64_t nv = (n - head) / 4;
    const float4 *xv = reinterpret_cast<const float4 *>(x + head);
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < nv; i += 4 * stride) {
        float4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = xv[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            m = fmaxf(m, fmaxf(fmaxf(fabsf(a[u].x), fabsf(a[u].y)), fmaxf(fabsf(a[u].z), fabsf(a[u].w))));
    }
    for (; i < nv; i += stride) {
        const float4 a = xv[i];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))));
    }
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < head) m = fmaxf(m, fabsf(x[t]));
    const int64_t tail = head + 4 * nv + t;
    if (tail < n) m = fmaxf(m, fabsf(x[tail]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Fixed-point scale, in binary64: the largest power of two S with
// |proj| * |scale| * S * 2^headroom < 2^30, so that a sum of up to 2^headroom
// weighted values still converts to a 32-bit integer.  S ranges over
// 2^-128 ... 2^(180 - headroom), beyond binary32, so it is kept in binary64
// and a value is scaled as (double)proj * (scale * S), one rounding to
// binary32 (exact products: a binary32 times a binary32 times a power of two).
__device__ __forceinline__ double fixed_scale(const unsigned *maxbits, float scale, int headroom) {
    const float mc = __uint_as_float(*maxbits) * fabsf(scale);
    if (!(mc > 0.0f) || !(mc < 3.0e38f)) return 1.0;
    int e;
    frexpf(mc, &e);  // mc < 2^e
    return ldexp(1.0, 30 - e - headroom);
}

// ---- fixed-point mode and scale of the backprojection ------------------------
// Two tile formats.  The 64-bit tile holds one exact sum per tile point.  The
// packed tile holds the sums of two neighbouring points along x in the two
// 32-bit halves of one 64-bit word, so a cell visit takes four LDS adds
// instead of eight.  A view adds at most B * max|value| to one half, where B
// bounds the rays through the block of eight cells around a tile point times
// the trilinear weight one ray can give it (view_weight_bound); the scale
// makes that at most half of the 32-bit range, and after every view each word
// with a half beyond the other half of the range is moved into the brick's
// 64-bit staging sums, so no half can overflow.  (The bound is far above the
// sums of real data, so few words are moved.)  Where B is large (a unit above
// 2^-21 of the largest value) the 64-bit tile is used.
struct BpScale {
    double s;         // fixed-point scale: gr = proj * length_scale * step * s
    double inv_s;     // 1 / s
    int packed;       // 1: packed tile (backproject_bricks<true, .>), 0: 64-bit tile
    int drain_above;  // packed: a word is moved when a half exceeds this in magnitude
};
constexpr double kHalfCap = 2147483648.0 - 134217728.0;  // 2^31 - 2^27: the margin covers the
                                                         // rounding of at most 2^16 flushes
constexpr double kPackedMaxBound = 512.0;                // 2^31 / 2 * 2^-21 (one bit for the drain margin)

// Upper bound, for view j, on the sum over its rays of the trilinear weight
// that one tile point can receive.  A ray gives weight to point p only from
// samples in the eight cells around p, a box of half-widths h inside the ball
// of radius R = |h| about p; along a unit direction d some axis a has
// |d_a| / h_a >= 1 / R, so consecutive samples are at least step / R apart in
// that axis's voxel units and the ray's weights at p (bounded by the hat
// function of that axis) sum to at most R / step + 1.  The rays through the
// ball hit the detector inside a disk of radius rho:
//  * parallel: rho = R / |cos| of the angle between the rays and the detector
//    normal;
//  * cone (and each row of a fan, within its plane): the rays through the
//    ball lie within alpha = asin(R / dist) of the ray to its centre, and the
//    central projection onto the plane at distance Dn moves by at most
//    Dn / cos^2(theta) per radian at angle theta from the normal, so rho =
//    alpha Dn / cos^2(theta_max + 2 alpha) with theta_max the largest angle of
//    a pixel ray (a detector corner) and dist the distance from the source to
//    the box of tile points.
// A disk of radius rho holds at most (floor(2 rho / l) + 1) (floor(2 rho /
// |e_v|) + 1) pixel centres, l the distance between pixel columns.  A fan's
// rows are translates of the central row by multiples of e_v; the planes of
// at most floor(2 R / |e_v . n0|) + 1 of them meet the ball (n0 the central
// plane's normal).  Infinity where no bound is found.
__device__ double view_weight_bound(const GeomDev &G, const DevGrid &g, int j) {
    const double kInf = __longlong_as_double(0x7ff0000000000000ll);
    const float *v = G.views + 12 * (int64_t)j;
    double A[3], D0[3], eu[3], ev[3], h[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = v[a];
        D0[a] = v[3 + a];
        eu[a] = v[6 + a];
        ev[a] = v[9 + a];
        h[a] = 1.0 / (double)g.inv_h[a];
    }
    auto dot = [](const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    const double R = sqrt(dot(h, h));
    const double W = R / G.step + 1.0;
    const double uu = dot(eu, eu), vv = dot(ev, ev), uv = dot(eu, ev);
    const double area2 = uu * vv - uv * uv;
    if (!(area2 > 0.0)) return kInf;
    const double area = sqrt(area2), lu = area / sqrt(vv);
    const double n[3] = {(eu[1] * ev[2] - eu[2] * ev[1]) / area, (eu[2] * ev[0] - eu[0] * ev[2]) / area,
                         (eu[0] * ev[1] - eu[1] * ev[0]) / area};
    const double cu = 0.5 * (G.nu - 1), cv = 0.5 * (G.nv - 1);
    const double npix = (double)G.nu * G.nv;
    auto in_disk = [&](double rho) {
        return fmin((floor(2.0 * rho / lu) + 1.0) * (floor(2.0 * rho / sqrt(vv)) + 1.0), npix);
    };
    // distance from point x to the box of tile points (voxel centres of the
    // indices -1 ... dims: the corners of the support's cells)
    auto box_dist = [&](const double *x) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double b0 = (double)g.lo[a] - 0.5 * h[a];
            const double b1 = (double)g.lo[a] + ((a == 0 ? g.nx : (a == 1 ? g.ny : g.nz)) + 0.5) * h[a];
            const double e = x[a] < b0 ? b0 - x[a] : (x[a] > b1 ? x[a] - b1 : 0.0);
            d2 += e * e;
        }
        return sqrt(d2);
    };
    double count;
    if (G.kind == DGR_PARALLEL) {
        const double c = fabs(dot(A, n)) / sqrt(dot(A, A));
        if (!(c > 1e-6)) return kInf;
        count = in_disk(R / c);
    } else if (G.kind == DGR_CONE) {
        const double w[3] = {D0[0] - A[0], D0[1] - A[1], D0[2] - A[2]};
        const double Dn = fabs(dot(w, n));
        const double dist = box_dist(A);
        if (!(Dn > 0.0) || !(dist > 1.0001 * R)) return kInf;
        const double alpha = asin(R / dist);
        double cmin = 1.0;  // cosine of the largest pixel-ray angle
        for (int c = 0; c < 4; ++c) {
            const double su = (c & 1) ? cu : -cu, sv = (c & 2) ? cv : -cv;
            double p[3];
            for (int a = 0; a < 3; ++a) p[a] = w[a] + su * eu[a] + sv * ev[a];
            cmin = fmin(cmin, fabs(dot(p, n)) / sqrt(dot(p, p)));
        }
        const double th = acos(fmin(1.0, cmin)) + 2.0 * alpha;
        if (!(th < 1.5)) return kInf;
        const double ct = cos(th);
        count = in_disk(alpha * Dn / (ct * ct));
    } else {
        const double w[3] = {D0[0] - A[0], D0[1] - A[1], D0[2] - A[2]};
        double n0[3] = {eu[1] * w[2] - eu[2] * w[1], eu[2] * w[0] - eu[0] * w[2], eu[0] * w[1] - eu[1] * w[0]};
        const double nn = sqrt(dot(n0, n0));
        if (!(nn > 0.0)) return kInf;
        for (int a = 0; a < 3; ++a) n0[a] /= nn;
        const double off = fabs(dot(ev, n0));
        const double rows = off > 0.0 ? fmin(floor(2.0 * R / off) + 1.0, (double)G.nv) : (double)G.nv;
        // in-plane normal of the detector line, and the distance to it
        const double wu = dot(w, eu) / uu;
        double m[3] = {w[0] - wu * eu[0], w[1] - wu * eu[1], w[2] - wu * eu[2]};
        const double Dn = sqrt(dot(m, m));
        // every row's source lies within cv |e_v| of the central one
        const double dist = box_dist(A) - cv * sqrt(vv);
        if (!(Dn > 0.0) || !(dist > 1.0001 * R)) return kInf;
        for (int a = 0; a < 3; ++a) m[a] /= Dn;
        const double alpha = asin(R / dist);
        double cmin = 1.0;
        for (int c = 0; c < 2; ++c) {
            const double su = c ? cu : -cu;
            double p[3];
            for (int a = 0; a < 3; ++a) p[a] = w[a] + su * eu[a];
            cmin = fmin(cmin, fabs(dot(p, m)) / sqrt(dot(p, p)));
        }
        const double th = acos(fmin(1.0, cmin)) + 2.0 * alpha;
        if (!(th < 1.5)) return kInf;
        const double ct = cos(th);
        const double rho = alpha * Dn / (ct * ct);
        count = fmin(rows * (floor(2.0 * rho / sqrt(uu)) + 1.0), npix);
    }
    const double B = count * W;
    return B == B ? B : kInf;
}

// max over views of view_weight_bound, as the bit pattern of a non-negative
// float (out), and each view's bound (per_view, if not null; 3e38 where
// none is found)
__global__ __launch_bounds__(256) void view_bound(GeomDev G, DevGrid g, unsigned *__restrict__ out,
                                                  float *__restrict__ per_view) {
    const int j = (int)(blockIdx.x * 256 + threadIdx.x);
    if (j >= G.n_views) return;
    const float b = (float)fmin(view_weight_bound(G, g, j), 3.0e38);
    const unsigned bits = __float_as_uint(b) + (b < 3.0e38f ? 1u : 0u);  // one ulp up: never below the bound
    if (out) atomicMax(out, bits);
    if (per_view) per_view[j] = __uint_as_float(bits);
}

// Mode and scale from max |proj| and the weight bound (one thread).
__global__ void bp_scale(const unsigned *__restrict__ words, float scale, int headroom,
                         BpScale *__restrict__ sc) {
    const double mc = (double)__uint_as_float(words[0]) * fabs((double)scale);
    const double B = (double)__uint_as_float(words[1]);
    BpScale r;
    r.packed = B <= kPackedMaxBound ? 1 : 0;
    r.drain_above = (int)(0.5 * kHalfCap);
    if (!(mc > 0.0) || !(mc < 3.0e38)) {
        r.s = 1.0;  // all values zero (or not finite)
    } else if (r.packed) {
        r.s = fmin(0.5 * kHalfCap / (B * mc), ldexp(1.0, 28) / mc);
        r.drain_above = (int)floor(kHalfCap - B * mc * r.s);
    } else {
        r.s = fixed_scale(words, scale, headroom);
    }
    r.inv_s = 1.0 / r.s;
    *sc = r;
}

// ---- per-ray table of the backprojection -------------------------------------
// Every ray is set up once per view batch (binary64 geometry, fixed-point
// anchor and advance, the scaled projection value) and read by each brick its
// shadow rectangle holds, instead of once per brick (a ray crosses about 30
// bricks of the 256^3 workload).  48 bytes per ray, 16-byte aligned.
struct alignas(16) RayTab {
    long long U[3];   // anchor, padded voxel coordinates, 32.32 fixed point
    unsigned dlo[3];  // low words of the advance per sample
    unsigned meta;    // [0, 9): high words of the advance, 3-bit two's complement per axis;
                      // bit 31: no sample of the ray lies in the support, or g = 0
    float gr;         // projection value times length_scale * step * the fixed-point scale
    unsigned pad;
};
static_assert(sizeof(RayTab) == 48, "ray table rows are 48 bytes");
constexpr unsigned kRayMiss = 0x80000000u;
// Table budget per batch of views (bytes): 360 views of 512^2 fit one batch;
// larger scans are backprojected in several batches that add into the same
// integer tiles.
constexpr int64_t kRayTableBudget = int64_t(6) << 30;

// One thread per ray of views j0 ... (nrays rays in all).
__global__ __launch_bounds__(256) void ray_table(const float *__restrict__ proj, GeomDev G, DevGrid g,
                                                 int j0, int64_t nrays, const BpScale *__restrict__ sc,
                                                 RayTab *__restrict__ tab) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nrays) return;
    const int64_t per_view = (int64_t)G.nu * G.nv;
    const int jl = (int)(i / per_view);
    const int64_t pix = i - (int64_t)jl * per_view;
    const int iv = (int)(pix / G.nu), iu = (int)(pix - (int64_t)iv * G.nu);
    const int j = j0 + jl;
    const double gs = (double)G.scale * sc->s;
    const float gr = (float)(gs * (double)proj[(int64_t)j * per_view + pix]);
    Ray r;
    ray_geom(G, g, j, iu, iv, r);
    int k0, k1;
    // a ray with no sample in the support (or beyond the fixed-point limits of
    // support_range) is a miss for the projector, and so for its transpose
    const bool hit = gr != 0.0f && support_range(r, g, &k0, &k1);
    RayTab t;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        t.U[a] = r.U[a];
        t.dlo[a] = (unsigned)r.DU[a];
    }
    t.meta = (((unsigned)(r.DU[0] >> 32) & 7u)) | (((unsigned)(r.DU[1] >> 32) & 7u) << 3) |
             (((unsigned)(r.DU[2] >> 32) & 7u) << 6) | (hit ? 0u : kRayMiss);
    t.gr = gr;
    t.pad = 0u;
    tab[i] = t;
}

// Samples k whose fixed-point position lies in [lo, hi] on every axis with an
// advance, from binary32 estimates: a superset, whose ends the caller tests
// exactly.  t = (lo - U) / DU: both integers rounded to binary32 (through
// binary64, total error below 2^-24 each), the hardware reciprocal within one
// ulp and the product rounded keep the relative error of t below 5 * 2^-24;
// the interval is widened by four times that plus 2^-10.  Axes without
// advance are left to the caller.
__device__ bool k_interval_fixed(const long long U[3], const long long DU[3], const long long lo[3],
                                 const long long hi[3], int *k0, int *k1) {
    float tmin = -3.0e38f, tmax = 3.0e38f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (DU[a] == 0) continue;
        const float inv = __builtin_amdgcn_rcpf((float)(double)DU[a]);
        const float t0 = (float)(double)(lo[a] - U[a]) * inv, t1 = (float)(double)(hi[a] - U[a]) * inv;
        tmin = fmaxf(tmin, fminf(t0, t1));
        tmax = fminf(tmax, fmaxf(t0, t1));
    }
    const float slack = 0x1p-10f + 1.2e-6f * fmaxf(fabsf(tmin), fabsf(tmax));
    tmin -= slack;
    tmax += slack;
    if (!(tmin <= tmax) || tmin < -(float)kMaxK || tmax > (float)kMaxK) return false;
    *k0 = (int)ceilf(tmin);
    *k1 = (int)floorf(tmax);
    return *k0 <= *k1;
}

// ---- brick backprojection ---------------------------------------------------
// One work-group per brick, two phases repeated until every view is done.
//  1. Ray set-up: each thread takes one candidate pixel of a view's shadow
//     rectangle, computes its ray and the exact range [k0, k1] of samples whose
//     trilinear cell lies in the brick, and appends a 32-byte record to an LDS
//     queue, plus one entry per segment of at most L = 2^seg_shift
//     consecutive samples.
//  2. March: the work-group's lanes take the queued segments in order, so every
//     lane runs (nearly) the same number of samples whatever the chord lengths
//     of the rays, and add the eight weighted values of each sample, in fixed
//     point, into the LDS tile.
// The queue holds one chunk of 256 candidates and is emptied by the march;
// each wave's table rows for the next chunk are in flight during its part of
// the march, and it sets those rays up as soon as that part is done, while
// the other waves still march.
constexpr int kChunk = 256;     // candidates per set-up pass (one per thread)
constexpr int kRayCap = 256;    // queued rays (one chunk)
constexpr int kSegCap = 2048;   // queued segments (>= kChunk * kMaxSeg)
constexpr int kMaxSeg = 8;      // segments per ray (the host sizes L for this)
static_assert(kSegCap >= kChunk * kMaxSeg && kRayCap >= kChunk, "a chunk must fit an empty queue");

struct alignas(16) RayRec {  // 32 bytes
    unsigned ulo[3];  // low words of the brick-relative 32.32 position of sample k0
    float gr;         // weighted projection value, scaled to fixed point
    unsigned dlo[3];  // low words of the 32.32 advance per sample
    unsigned meta;    // [0,15): high words of the position, 5 bits per axis, in [0, 32)
                      // [15,24): high words of the advance, 3-bit two's complement
                      // [24,32): number of samples - 1
};

__device__ __forceinline__ bool in_brick(long long x, long long y, long long z) {
    return (unsigned long long)x < ((unsigned long long)kBX << 32) &&
           (unsigned long long)y < ((unsigned long long)kBY << 32) &&
           (unsigned long long)z < ((unsigned long long)kBZ << 32);
}

// Exclusive prefix sum over the 64 lanes of a wave (all lanes active) and the
// wave total: a Hillis-Steele scan within each row of 16 lanes by DPP row
// shifts (lanes shifted in from outside the row add 0), then the row totals
// carried across rows by the DPP row broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_excl_scan(int v, int *total) {
    int incl = v;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, false);  // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, false);  // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, false);  // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, false);  // row_shr:8
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
    *total = __builtin_amdgcn_readlane(incl, 63);
    return incl - v;
}

// Adds the eight corner values e of the cell whose lower corner is tile entry
// `cell` (x fastest); hi is the high word of all eight (the sign of e).
__device__ __forceinline__ void flush_cell(unsigned long long *tile, unsigned cell, const float (&e)[8],
                                           unsigned hi) {
    constexpr unsigned sy = kTBX, sz = kTBX * kTBY;
    unsigned long long *q = tile + cell;
    const unsigned long long h = (unsigned long long)hi << 32;
    atomicAdd(q, h | (unsigned)(int)e[0]);
    atomicAdd(q + 1, h | (unsigned)(int)e[1]);
    atomicAdd(q + sy, h | (unsigned)(int)e[2]);
    atomicAdd(q + sy + 1, h | (unsigned)(int)e[3]);
    atomicAdd(q + sz, h | (unsigned)(int)e[4]);
    atomicAdd(q + sz + 1, h | (unsigned)(int)e[5]);
    atomicAdd(q + sz + sy, h | (unsigned)(int)e[6]);
    atomicAdd(q + sz + sy + 1, h | (unsigned)(int)e[7]);
}

// Packed tile: word (x, y, z), x < kBX, holds tile points (x, y, z) and
// (x + 1, y, z) in its low and high 32 bits (two's complement halves of one
// 64-bit sum: the low half's sign carries into the high half, and is taken
// back out when the word is drained).
constexpr int kPX = kBX, kPXY = kBX * kTBY, kPW3 = kBX * kTBY * kTBZ;

__device__ __forceinline__ unsigned long long pack_pair(float e0, float e1) {
    const int lo = (int)e0, hi = (int)e1;
    return ((unsigned long long)(unsigned)(hi + (lo >> 31)) << 32) | (unsigned)lo;
}

// Adds the eight corner values of in-brick cell `word` (the word of its lower
// corner) as four pairs along x.
__device__ __forceinline__ void flush_packed(unsigned long long *tile, unsigned word, const float (&e)[8]) {
    unsigned long long *q = tile + word;
    atomicAdd(q, pack_pair(e[0], e[1]));
    atomicAdd(q + kPX, pack_pair(e[2], e[3]));
    atomicAdd(q + kPXY, pack_pair(e[4], e[5]));
    atomicAdd(q + kPXY + kPX, pack_pair(e[6], e[7]));
}

// Adds the four lower-plane corner values of in-brick cell `word` (planar
// rays, whose upper-plane values are zero) as two pairs along x.
__device__ __forceinline__ void flush_planar(unsigned long long *tile, unsigned word, const float (&e)[4]) {
    unsigned long long *q = tile + word;
    atomicAdd(q, pack_pair(e[0], e[1]));
    atomicAdd(q + kPX, pack_pair(e[2], e[3]));
}

// Tile entry (packed: word) of the lower corner of in-brick cell (x, y, z):
// 24-bit products.
template <bool PACKED>
__device__ __forceinline__ unsigned cell_index(long long ux, long long uy, long long uz) {
    constexpr unsigned sy = PACKED ? kPX : kTBX, sz = PACKED ? kPXY : kTBX * kTBY;
    return __umul24((unsigned)(uz >> 32), sz) + (__umul24((unsigned)(uy >> 32), sy) + (unsigned)(ux >> 32));
}

// Phase 2 over the queued segments: lane i of wave w takes segments
// w * 64 + i, w * 64 + i + 256, ...  Consecutive samples of a ray often share
// their trilinear cell (about two per cell at half-voxel steps); a lane sums
// their eight corner weights in registers and adds them to the tile once per
// cell visit.  The fixed-point scale leaves room for the largest number of
// samples one cell can hold.
// PLANE_OK: the launch may hold planar rays (fan beams whose rows lie on voxel
// centre planes: no advance in z and a whole-voxel z position).  Their
// samples' z weights are exactly 0, so the upper-plane corner values stay at
// the accumulators' start of +-1/2 and add the integer 0: where every active
// lane of a wave holds a planar ray, the wave marches the lower plane only
// (four corner values, two packed adds per cell visit), with a tile equal to
// the general march's bit for bit.
template <bool PACKED, bool PLANE_OK>
__device__ __forceinline__ void march_segments(unsigned long long *tile, const RayRec *rays,
                                               const unsigned short *segs, int nsegs, int seg_shift) {
    const int t = threadIdx.x;
    // Lane order within each block of 256 segments is strided by 8: a ray's
    // segments are queued together and neighbouring pixels one after the
    // other, so lanes side by side take segments about two rays apart and
    // rarely add into the same LDS word at once.  (Strides 2 ... 64 were
    // timed; on 16^3 bricks 8 gave the fewest LDS bank conflicts, 3 % faster
    // than 32; on the flat bricks 4 ... 16 are within 0.5 %.)
    // The last, partial block of 256 is taken in order instead, so waves
    // beyond its segments skip it and leave their issue slots to the other
    // work-groups of the CU.
    const int perm = ((t & 31) << 3) | (t >> 5);
    for (int base = 0; base < nsegs; base += 256) {
        const int s = base + (nsegs - base >= 256 ? perm : t);
        if (s >= nsegs) continue;
        const unsigned e = segs[s];
        const RayRec rec = rays[e >> 3];
        const int seg = (int)(e & 7u);
        const unsigned m = rec.meta;
        long long ux = (long long)(((unsigned long long)(m & 31u) << 32) | rec.ulo[0]);
        long long uy = (long long)(((unsigned long long)((m >> 5) & 31u) << 32) | rec.ulo[1]);
        long long uz = (long long)(((unsigned long long)((m >> 10) & 31u) << 32) | rec.ulo[2]);
        const long long dx = (long long)(((unsigned long long)(long long)((int)(m << 14) >> 29) << 32) | rec.dlo[0]);
        const long long dy = (long long)(((unsigned long long)(long long)((int)(m << 11) >> 29) << 32) | rec.dlo[1]);
        const long long dz = (long long)(((unsigned long long)(long long)((int)(m << 8) >> 29) << 32) | rec.dlo[2]);
        const int n = (int)(m >> 24) + 1;
        const int k_off = seg << seg_shift;
        const int cnt = min(1 << seg_shift, n - k_off);
        ux += (long long)k_off * dx;
        uy += (long long)k_off * dy;
        uz += (long long)k_off * dz;
        const float gr = rec.gr;
        // Fixed-point conversion (64-bit tile): every corner value of a ray
        // has the sign of gr, so the high word of its 64-bit integer is the
        // sign of gr.  The accumulators start at +1 or -1, so the truncated
        // integer is at least 1 or at most -1 (never 0, whose high word would
        // be 0 for either sign); it lies within one unit of the value, on
        // average half a unit away from zero, with opposite signs for the two
        // signs of gr.  Packed tile: the accumulators start at +-1/2, so the
        // truncation rounds to the nearest integer (each half carries its own
        // sign).
        const float gr32 = gr * kInv32;  // exact: a power-of-two scale
        const unsigned hi = gr < 0.0f ? 0xffffffffu : 0u;
        const float a_init = PACKED ? (gr < 0.0f ? -0.5f : 0.5f) : (gr < 0.0f ? -1.0f : 1.0f);
        unsigned cell = cell_index<PACKED>(ux, uy, uz);
        if (PACKED && PLANE_OK && __ballot(dz == 0 && (unsigned)uz == 0u) == __ballot(1)) {
            // the same products as below with fz = 0: z0 = gr, z1 = 0
            float acc4[4] = {a_init, a_init, a_init, a_init};
            for (int i = 0; i < cnt; ++i) {
                const unsigned here = cell_index<PACKED>(ux, uy, uz);
                const float fx = (float)(unsigned)ux, fy = (float)(unsigned)uy;
                ux += dx;
                uy += dy;
                if (here != cell) {
                    flush_planar(tile, cell, acc4);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc4[c] = a_init;
                    cell = here;
                }
                const float wy = fy * kInv32;
                const float y01 = gr * wy, y00 = fmaf(-gr, wy, gr);
                const float wx = fx * kInv32, ox = fmaf(-fx, kInv32, 1.0f);
                acc4[0] = fmaf(y00, ox, acc4[0]);
                acc4[1] = fmaf(y00, wx, acc4[1]);
                acc4[2] = fmaf(y01, ox, acc4[2]);
                acc4[3] = fmaf(y01, wx, acc4[3]);
            }
            flush_planar(tile, cell, acc4);
            continue;
        }
        float acc[8] = {a_init, a_init, a_init, a_init, a_init, a_init, a_init, a_init};
        for (int i = 0; i < cnt; ++i) {
            const unsigned here = cell_index<PACKED>(ux, uy, uz);
            // 2^32 times the trilinear weights of the upper corners
            const float fx = (float)(unsigned)ux, fy = (float)(unsigned)uy, fz = (float)(unsigned)uz;
            ux += dx;
            uy += dy;
            uz += dz;
            if (here != cell) {
                if (PACKED)
                    flush_packed(tile, cell, acc);
                else
                    flush_cell(tile, cell, acc, hi);
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = a_init;
                cell = here;
            }
            // Every corner value has the sign of gr (or is 0), so the high
            // word above holds: z1 = gr 2^-32 fz with fz <= 2^32 is at most gr
            // in magnitude, and each lower-corner factor is formed as
            // fma(-z, w, z) = z (1 - w), rounded once from the exact value,
            // with 0 <= w <= 1.  (Where gr 2^-32 is subnormal a residue of the
            // wrong sign below 2^-94 is possible; added to an accumulator of
            // magnitude >= 1 it rounds away.)
            const float z1 = gr32 * fz, z0 = fmaf(-gr32, fz, gr);
            const float wy = fy * kInv32;
            const float y01 = z0 * wy, y11 = z1 * wy, y00 = fmaf(-z0, wy, z0), y10 = fmaf(-z1, wy, z1);
            const float wx = fx * kInv32, ox = fmaf(-fx, kInv32, 1.0f);
            acc[0] = fmaf(y00, ox, acc[0]);
            acc[1] = fmaf(y00, wx, acc[1]);
            acc[2] = fmaf(y01, ox, acc[2]);
            acc[3] = fmaf(y01, wx, acc[3]);
            acc[4] = fmaf(y10, ox, acc[4]);
            acc[5] = fmaf(y10, wx, acc[5]);
            acc[6] = fmaf(y11, ox, acc[6]);
            acc[7] = fmaf(y11, wx, acc[7]);
        }
        if (PACKED)
            flush_packed(tile, cell, acc);
        else
            flush_cell(tile, cell, acc, hi);
    }
}

// seg_shift: log2 of the samples per segment, chosen on the host so that no ray
// in a brick has more than kMaxSeg segments (and no more than 256 samples).
// Four work-groups per CU (37 KB of LDS each, <= 128 VGPRs): the extra waves
// overlap one work-group's LDS adds with another's arithmetic.  Both
// instances are launched; the one whose tile format sc->packed does not name
// returns at once.  The 64-bit tile is written to (accumulate: loaded from
// and written to) the brick's staging sums at the end; the packed tile's
// words are added into them when a half nears the end of its range (checked
// after every view) and at the end.
// PLANE_OK: the planar march where a wave's rays allow it (launched for fan
// beams; the other instances compile it out).
template <bool PACKED, bool PLANE_OK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DGR_BP_WAVES, DGR_BP_WAVES))) void backproject_bricks(
    const RayTab *__restrict__ tab, int j0, int nj, GeomDev G, Bricks bk, const ushort4 *__restrict__ rect,
    int seg_shift, int accumulate, const BpScale *__restrict__ sc, long long *__restrict__ staging) {
    constexpr int kTile = PACKED ? kPW3 : kBT3;
    __shared__ unsigned long long tile[kTile];
    __shared__ RayRec rays[kRayCap];
    __shared__ unsigned short segs[kSegCap];
    __shared__ int q_rays, q_segs;
    if (sc->packed != (PACKED ? 1 : 0)) return;
    const int t = threadIdx.x, lane = t & 63;
    const int64_t nb = bk.count();
    const int64_t b = blockIdx.x;
    const int bx = (int)(b % bk.nx), by = (int)((b / bk.nx) % bk.ny), bz = (int)(b / ((int64_t)bk.nx * bk.ny));
    // brick cells in padded coordinates: [c0, c0 + kB)
    const int c0x = bx * kBX - 1 + kPad, c0y = by * kBY - 1 + kPad, c0z = bz * kBZ - 1 + kPad;
    const long long C0x = (long long)c0x << 32, C0y = (long long)c0y << 32, C0z = (long long)c0z << 32;
    // Bounds of the candidate k-range: the brick's cells in fixed point (a
    // sample is in the brick iff its fixed-point cell is); the range from the
    // binary32 estimate is a superset of the samples in the brick, which form
    // one run of k (each axis test is an interval of the exact integer
    // positions), and the run's ends are found by testing the cells.
    const long long blo[3] = {C0x, C0y, C0z};
    const long long bhi[3] = {C0x + ((long long)kBX << 32), C0y + ((long long)kBY << 32),
                              C0z + ((long long)kBZ << 32)};
    const int64_t per_view = (int64_t)G.nu * G.nv;
    long long *out = staging + b * kBT3;
    if (PACKED) {
        for (int e = t; e < kTile; e += 256) tile[e] = 0ull;
        // the staging sums start at zero; the loop's barriers (work-group
        // release and acquire) order these stores before every drain's
        // atomics on the same words, which this work-group alone touches
        if (!accumulate)
            for (int e = t; e < kBT3; e += 256) out[e] = 0;
    } else {
        for (int e = t; e < kBT3; e += 256) tile[e] = accumulate ? (unsigned long long)out[e] : 0ull;
    }
    // packed: moves the two halves of a word into the staging sums of its two
    // tile points with non-returning 64-bit atomics (the brick's sums are its
    // own, so the atomics meet no other work-group; they only spare the wait
    // of a read-modify-write) and clears the word: every word (all) or those
    // with a half beyond drain_above
    const int drain_above = PACKED ? sc->drain_above : 0;
    auto drain = [&](bool all) {
        for (int w = t; w < kPW3; w += 256) {
            const unsigned long long p = tile[w];
            const int lo = (int)(unsigned)p;
            const int hi = (int)((long long)(p - (unsigned long long)(long long)lo) >> 32);
            if (all ? p != 0ull : (abs(lo) > drain_above || abs(hi) > drain_above)) {
                tile[w] = 0ull;
                const int z = w / kPXY, r = w - z * kPXY;
                const int y = r / kPX, x = r - y * kPX;
                unsigned long long *q = reinterpret_cast<unsigned long long *>(out + (z * kTBY + y) * kTBX + x);
                if (lo != 0) atomicAdd(q, (unsigned long long)(long long)lo);
                if (hi != 0) atomicAdd(q + 1, (unsigned long long)(long long)hi);
            }
        }
    };
    if (t == 0) {
        q_rays = 0;
        q_segs = 0;
    }
    __syncthreads();
    // Ray set-up (phase 1), in two parts: the table row of candidate c of view
    // j's rectangle rc, and from that row the record and the number of the
    // ray's samples in the brick (0: none).
    auto row_of = [&](int j, const ushort4 &rc, float inu, long long c) -> int64_t {
        const int nu_r = (int)rc.y - (int)rc.x + 1;
        // c / nu_r from a binary32 reciprocal, exact for c < 2^22 (as in the
        // forward staging); integer division beyond
        int row, col;
        if (c < (1 << 22)) {
            row = (int)fmaf((float)c, inu, 0.5f * inu);
            col = (int)c - row * nu_r;
        } else {
            row = (int)(c / nu_r);
            col = (int)(c - (long long)row * nu_r);
        }
        const int iv = (int)rc.z + row, iu = (int)rc.x + col;
        return (int64_t)(j - j0) * per_view + (int64_t)iv * G.nu + iu;
    };
    auto finish = [&](const RayTab &rt, RayRec &rec) -> int {
        int n = 0;
        if (rt.meta & kRayMiss) return 0;
        long long DU[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            DU[a] = (long long)(((unsigned long long)(long long)((int)(rt.meta << (29 - 3 * a)) >> 29) << 32) |
                                rt.dlo[a]);
        const float gr = rt.gr;
        // an axis without advance keeps one fixed-point cell for every
        // sample: test it once (the interval estimate cannot bound it)
        const bool still_ok =
            (DU[0] != 0 || (unsigned long long)(rt.U[0] - C0x) < ((unsigned long long)kBX << 32)) &&
            (DU[1] != 0 || (unsigned long long)(rt.U[1] - C0y) < ((unsigned long long)kBY << 32)) &&
            (DU[2] != 0 || (unsigned long long)(rt.U[2] - C0z) < ((unsigned long long)kBZ << 32));
        int k0, k1;
        if (still_ok && k_interval_fixed(rt.U, DU, blo, bhi, &k0, &k1)) {
            long long ux = rt.U[0] + (long long)k0 * DU[0] - C0x;
            long long uy = rt.U[1] + (long long)k0 * DU[1] - C0y;
            long long uz = rt.U[2] + (long long)k0 * DU[2] - C0z;
            while (k0 <= k1 && !in_brick(ux, uy, uz)) {
                ++k0;
                ux += DU[0];
                uy += DU[1];
                uz += DU[2];
            }
            if (k0 <= k1) {
                long long vx = rt.U[0] + (long long)k1 * DU[0] - C0x;
                long long vy = rt.U[1] + (long long)k1 * DU[1] - C0y;
                long long vz = rt.U[2] + (long long)k1 * DU[2] - C0z;
                while (!in_brick(vx, vy, vz)) {  // stops at k0 at the latest
                    --k1;
                    vx -= DU[0];
                    vy -= DU[1];
                    vz -= DU[2];
                }
                n = k1 - k0 + 1;
                rec.ulo[0] = (unsigned)ux;
                rec.ulo[1] = (unsigned)uy;
                rec.ulo[2] = (unsigned)uz;
                rec.dlo[0] = rt.dlo[0];
                rec.dlo[1] = rt.dlo[1];
                rec.dlo[2] = rt.dlo[2];
                rec.gr = gr;
                rec.meta = (unsigned)(ux >> 32) | ((unsigned)(uy >> 32) << 5) | ((unsigned)(uz >> 32) << 10) |
                           ((rt.meta & 0x1ffu) << 15) | ((unsigned)(n - 1) << 24);
            }
        }
        return n;
    };
    // The candidates of all views are taken 256 at a time (one per thread;
    // consecutive pixels of a rectangle, so the projection reads coalesce):
    // the chunk starting at candidate cb of view j.  advance() moves to the
    // next chunk, skipping empty rectangles; j == n_views when done.
    const int jend = j0 + nj;
    int j = j0 - 1;
    long long cb = -kChunk, ncand = 0;  // a rectangle may hold up to 2^32 pixels
    float inu = 1.0f;  // 1 / rectangle width
    ushort4 rc = make_ushort4(1, 0, 1, 0), rc_next = rect[(int64_t)j0 * nb + b];
    auto advance = [&]() {
        cb += kChunk;
        while (cb >= ncand) {
            if (++j >= jend) return;
            rc = rc_next;
            if (j + 1 < jend) rc_next = rect[(int64_t)(j + 1) * nb + b];  // prefetch
            const int nu_r = (int)rc.y - (int)rc.x + 1, nv_r = (int)rc.w - (int)rc.z + 1;
            ncand = (nu_r > 0 && nv_r > 0) ? (long long)nu_r * nv_r : 0;
            inu = nu_r > 0 ? 1.0f / (float)nu_r : 1.0f;
            cb = 0;
        }
    };
    RayRec rec;
    int n = 0;
    advance();
    if (j < jend && cb + t < ncand) n = finish(tab[row_of(j, rc, inu, cb + t)], rec);
    while (j < jend) {
        // ---- queue the chunk's rays and segments (the queue is empty)
        const int nseg = (n + (1 << seg_shift) - 1) >> seg_shift;
        const unsigned long long mask = __ballot(n > 0);
        const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
        int seg_tot;
        const int seg_pre = wave_excl_scan(nseg, &seg_tot);
        int rbase = 0, sbase = 0;
        if (lane == 0 && mask != 0ull) {
            rbase = atomicAdd(&q_rays, __popcll(mask));
            sbase = atomicAdd(&q_segs, seg_tot);
        }
        rbase = __builtin_amdgcn_readlane(rbase, 0);
        sbase = __builtin_amdgcn_readlane(sbase, 0);
        if (n > 0) {
            const int slot = rbase + rank;
            rays[slot] = rec;
            for (int q = 0; q < nseg; ++q) segs[sbase + seg_pre + q] = (unsigned short)((slot << 3) | q);
        }
        __syncthreads();
        const int ns = q_segs;
        // ---- phase 2; each wave loads the table rows of its candidates of
        // the next chunk before its part of the march and sets them up after
        // it, while the other waves finish their segments
        const int j_marched = j;
        advance();
        const bool have = j < jend && cb + t < ncand;
        // (unconditional load, row 0 for lanes without a candidate: no
        // branch, so nothing waits for the load before the march)
        const RayTab rt_next = tab[have ? row_of(j, rc, inu, cb + t) : 0];
        march_segments<PACKED, PLANE_OK>(tile, rays, segs, ns, seg_shift);
        n = have ? finish(rt_next, rec) : 0;
        __syncthreads();
        if (t == 0) {
            q_rays = 0;
            q_segs = 0;
        }
        if (PACKED && j != j_marched && j < jend) drain(false);  // view j_marched is complete
                                                                   // (the last drain follows the loop)
        __syncthreads();
    }
    if (PACKED) {
        drain(true);
    } else {
        for (int e = t; e < kBT3; e += 256) out[e] = (long long)tile[e];
    }
}

// Each voxel lies in one or two brick tiles per axis (tiles overlap by one
// voxel on their faces); its value is the exact integer sum of those tile
// entries divided by the fixed-point scale.
__global__ __launch_bounds__(256) void gather_bricks(const long long *__restrict__ staging, DevGrid g,
                                                     Bricks bk, const BpScale *__restrict__ sc,
                                                     float *__restrict__ V) {
    const double inv_s = sc->inv_s;
    const int64_t total = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t z = i / ((int64_t)g.nx * g.ny), rem = i - z * (int64_t)g.nx * g.ny;
        const int y = (int)(rem / g.nx), x = (int)(rem - (int64_t)y * g.nx);
        const int vv[3] = {x, y, (int)z};
        int nb[3], bb[3][2], ll[3][2];
        for (int a = 0; a < 3; ++a) {
            const int kb = a == 0 ? kBX : (a == 1 ? kBY : kBZ);
            const int s = vv[a] + 1;  // local index in brick b is s - kb * b
            bb[a][0] = s / kb;
            ll[a][0] = s - kb * bb[a][0];
            nb[a] = 1;
            if (ll[a][0] == 0 && bb[a][0] > 0) {
                bb[a][1] = bb[a][0] - 1;
                ll[a][1] = kb;
                nb[a] = 2;
            }
        }
        long long acc = 0;
        for (int iz = 0; iz < nb[2]; ++iz)
            for (int iy = 0; iy < nb[1]; ++iy)
                for (int ix = 0; ix < nb[0]; ++ix) {
                    const int64_t brick = ((int64_t)bb[2][iz] * bk.ny + bb[1][iy]) * bk.nx + bb[0][ix];
                    acc += staging[brick * kBT3 + (ll[2][iz] * kTBY + ll[1][iy]) * kTBX + ll[0][ix]];
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
    unsigned *maxbits;  // [0]: max |proj| (float bits), [1]: view weight bound (float bits)
    BpScale *scale;
    RayTab *tab;
    int batch_views;  // views per backprojection batch (ray table rows: batch_views * nu * nv)
    size_t bytes;
};

// rays per thread of the forward work-groups (see project_bundles): two for
// cone beams, one for fan and parallel beams
inline int fwd_rays_per_thread(const dgr_geometry *G) { return G->kind == DGR_CONE ? 2 : 1; }

// Forward work-groups of a scan with nr rays per thread: tiles of (16 nr) x 16
// pixels.
int64_t ray_blocks(const dgr_geometry *G, int *tu, int *tv, int nr) {
    *tu = (G->nu + kBun * nr - 1) / (kBun * nr);
    *tv = (G->nv + kBun - 1) / kBun;
    return (int64_t)G->n_views * (*tu) * (*tv);
}

ProjWs carve_proj_ws(void *ws, const dgr_grid *grid, const dgr_geometry *geom) {
    // The forward pass uses vpad + partial; the backward pass staging + rect.
    // The two share the front of the workspace.
    ProjWs w;
    int tu, tv;
    Carver f(ws);
    w.vpad = f.take<float>(pad_count(grid));
    w.partial = f.take<float>(ray_blocks(geom, &tu, &tv, fwd_rays_per_thread(geom)));
    Carver b(ws);
    const Bricks bk = bricks_of(grid);
    w.staging = b.take<long long>(bk.count() * kBT3);
    w.rect = b.take<ushort4>(bk.count() * geom->n_views);
    w.maxbits = b.take<unsigned>(2);
    w.scale = b.take<BpScale>(1);
    const int64_t row_bytes = (int64_t)geom->nu * geom->nv * (int64_t)sizeof(RayTab);
    const int64_t fit = std::max<int64_t>(1, kRayTableBudget / std::max<int64_t>(row_bytes, 1));
    const int64_t nbatch = (geom->n_views + fit - 1) / fit;  // equal batches
    w.batch_views = (int)((geom->n_views + nbatch - 1) / nbatch);
    w.tab = b.take<RayTab>((int64_t)w.batch_views * geom->nu * geom->nv);
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
    const int nr = fwd_rays_per_thread(geom);
    const int64_t nb = ray_blocks(geom, &tu, &tv, nr);
    const double m = (double)geom->n_views * geom->nu * geom->nv;
    const int64_t launched = (nb + kXcd - 1) / kXcd * kXcd;
    if (nr == 2)
        project_bundles<MODE, 2><<<dim3((unsigned)launched), dim3(256), 0, st>>>(
            w.vpad, p, g, geom_dev(geom), tu, tv, nb, target, out, (float)(1.0 / m), w.partial);
    else
        project_bundles<MODE, 1><<<dim3((unsigned)launched), dim3(256), 0, st>>>(
            w.vpad, p, g, geom_dev(geom), tu, tv, nb, target, out, (float)(1.0 / m), w.partial);
    DGR_LAUNCH_CHECK();
    if (MODE == 1) {
        finish_loss<<<1, 1024, 0, st>>>(w.partial, nb, 1.0 / m, loss);
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

extern "C" dgr_status dgr_backproject_weight_bound(const dgr_grid *grid, const dgr_geometry *geom,
                                                   float *bound, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_geometry(geom)) != DGR_OK) return s;
    DGR_CHECK(bound, "null bound pointer");
    view_bound<<<dim3((unsigned)((geom->n_views + 255) / 256)), dim3(256), 0, as_stream(stream)>>>(
        geom_dev(geom), dev_grid(grid), nullptr, bound);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" dgr_status dgr_backproject(const float *proj, const dgr_grid *grid,
                                      const dgr_geometry *geom, float *volume, void *ws,
                                      size_t ws_bytes, void *stream) {
    dgr_status s = check_proj(grid, geom, ws, ws_bytes);
    if (s != DGR_OK) return s;
    DGR_CHECK(proj && volume, "null projection or volume pointer");
    // Samples of one ray inside a brick: its chord is at most the brick's
    // diagonal, and samples are step * min(inv_h) cells apart or more.  The
    // queue records hold at most 256 samples per ray and advances below 4
    // cells per sample per axis (3-bit high words).
    double min_inv = 1e300, max_inv = 0.0;
    for (int a = 0; a < 3; ++a) {
        min_inv = std::min(min_inv, (double)grid->inv_h[a]);
        max_inv = std::max(max_inv, (double)grid->inv_h[a]);
    }
    const double step_min = (double)geom->step * min_inv;
    const double chord = std::sqrt((double)kBX * kBX + (double)kBY * kBY + (double)kBZ * kBZ);
    const int max_n = (int)std::min(1e9, std::floor(chord * 1.0001 / step_min) + 2.0);
    DGR_CHECK(max_n <= 256, "backprojection needs step >= %.3g voxel (got %.4g)", chord / 254.0, step_min);
    DGR_CHECK((double)geom->step * max_inv <= 3.9, "backprojection needs step <= 3.9 voxels");
    int seg_shift = 3;  // segments of 2^seg_shift samples, at most kMaxSeg of them per ray
    while ((kMaxSeg << seg_shift) < max_n) ++seg_shift;
    // samples of one ray inside one unit cell: at most sqrt(3) / step + 1
    const int per_cell = (int)std::floor(std::sqrt(3.0) * 1.0001 / step_min) + 1;
    int headroom = 0;
    while ((1 << headroom) < per_cell) ++headroom;
    hipStream_t st = as_stream(stream);
    ProjWs w = carve_proj_ws(ws, grid, geom);
    DevGrid g = dev_grid(grid);
    const Bricks bk = bricks_of(grid);
    const GeomDev G = geom_dev(geom);
    const int64_t nrect = bk.count() * geom->n_views;
    brick_rects<<<dim3((unsigned)((nrect + 255) / 256)), dim3(256), 0, st>>>(G, g, bk, w.rect);
    DGR_LAUNCH_CHECK();
    const int64_t nproj = (int64_t)geom->n_views * geom->nu * geom->nv;
    zero_u32x2<<<1, 64, 0, st>>>(w.maxbits);
    DGR_LAUNCH_CHECK();
    absmax_bits<<<dim3((unsigned)std::min<int64_t>((nproj / 4 + 255) / 256 + 1, 2048)), dim3(256), 0, st>>>(
        proj, nproj, w.maxbits);
    DGR_LAUNCH_CHECK();
    view_bound<<<dim3((unsigned)((geom->n_views + 255) / 256)), dim3(256), 0, st>>>(G, g, w.maxbits + 1,
                                                                                   nullptr);
    DGR_LAUNCH_CHECK();
    bp_scale<<<1, 1, 0, st>>>(w.maxbits, G.scale, headroom, w.scale);
    DGR_LAUNCH_CHECK();
    // views in batches whose ray table fits the budget; each batch adds into
    // the integer tiles of the previous ones
    for (int j0 = 0; j0 < geom->n_views; j0 += w.batch_views) {
        const int nj = std::min(w.batch_views, geom->n_views - j0);
        const int64_t nrays = (int64_t)nj * geom->nu * geom->nv;
        ray_table<<<dim3((unsigned)((nrays + 255) / 256)), dim3(256), 0, st>>>(proj, G, g, j0, nrays, w.scale,
                                                                              w.tab);
        DGR_LAUNCH_CHECK();
        // the instance whose tile format the scale kernel did not choose returns
        // at once; fan beams take the packed instance with the planar march
        if (geom->kind == DGR_FAN)
            backproject_bricks<true, true><<<dim3((unsigned)bk.count()), dim3(256), 0, st>>>(
                w.tab, j0, nj, G, bk, w.rect, seg_shift, j0 > 0 ? 1 : 0, w.scale, w.staging);
        else
            backproject_bricks<true, false><<<dim3((unsigned)bk.count()), dim3(256), 0, st>>>(
                w.tab, j0, nj, G, bk, w.rect, seg_shift, j0 > 0 ? 1 : 0, w.scale, w.staging);
        DGR_LAUNCH_CHECK();
        backproject_bricks<false, false><<<dim3((unsigned)bk.count()), dim3(256), 0, st>>>(
            w.tab, j0, nj, G, bk, w.rect, seg_shift, j0 > 0 ? 1 : 0, w.scale, w.staging);
        DGR_LAUNCH_CHECK();
    }
    const int64_t nvox = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    gather_bricks<<<dim3(grid_stride_blocks(nvox)), dim3(256), 0, st>>>(w.staging, g, bk, w.scale, volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
