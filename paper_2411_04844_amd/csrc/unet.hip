// Learned initialisation: a 3-D U-Net that maps a one-channel volume (an FDK
// reconstruction) to per-voxel density, log-scale and occupancy fields, from
// which an initial Gaussian set is drawn.  The paper initialises its Gaussians
// from an FBP/FDK volume (Fig. 4 caption) or at random; the network proposes
// a better-placed set, and the plain initialisation remains the fallback.
//
// Architecture (base width B = 32; extents divisible by 8):
//   enc1 = relu(conv3(x; 1 -> B))                       D
//   enc2 = relu(conv3(pool(enc1); B -> 2B))             D/2
//   enc3 = relu(conv3(pool(enc2); 2B -> 4B))            D/4
//   bott = relu(conv3(pool(enc3); 4B -> 8B))            D/8
//   dec3 = relu(conv3([up(bott), enc3]; 12B -> 4B))     D/4
//   dec2 = relu(conv3([up(dec3), enc2]; 6B -> 2B))      D/2
//   dec1 = relu(conv3([up(dec2), enc1]; 3B -> B))       D
//   out  = head(dec1; B -> 3)                           1x1x1
// conv3: 3x3x3 cross-correlation, zero padding 1, tap t = 9(dz+1)+3(dy+1)+(dx+1).
// pool: 2x2x2 mean; up: nearest 2x; [a, b]: channel concatenation.
//
// Numerics: activations, activation gradients and the weights fed to the
// matrix cores are bfloat16 (round to nearest even); every product is
// accumulated in binary32 (MFMA f32 accumulators); weight gradients and the
// head are binary32.
//
// Data layout: channels-last [z][y][x][c].  Each skip concatenation is one
// buffer: the encoder writes its output straight into the channel slice that
// the decoder reads, so concatenation costs nothing.
//
// Kernels:
//   conv3_tile   implicit GEMM (M = voxels, N = output channels,
//                K = 27 x input channels) on v_mfma_f32_16x16x32_bf16 over
//                16 x 4 x 4 voxel tiles whose halo is staged in LDS once per
//                32-channel block and read by all 27 taps (two LDS reads per
//                three taps along x, the middle one formed by DPP row
//                shifts); weights in a fragment-major layout, so that a wave
//                reads each B fragment as 1 KB in one piece, prefetched one
//                (dz, dy) row ahead.  The data gradient is the same kernel
//                with transposed, tap-reversed weights.
//   conv3_wgrad  dW[t] = dY^T shift_t(X): K = voxels; per 16 x 4 x 4 voxel
//                tile dY and the x-shifted X halo are transposed into LDS
//                (bank-swizzled columns) and 9 taps share each dY fragment;
//                the next tile's loads are in flight during the current
//                tile's MFMAs; split over chunks of tiles into binary32
//                partials summed in a fixed order, all work-groups of a chunk
//                on one XCD.
//   conv1_*      the 1-channel first layer on the VALU (K = 27).
//   pooling, upsampling (with the ReLU masks of the backward fused in), the
//   1x1 head and the loss are elementwise VALU kernels.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

typedef unsigned short u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16 f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }

struct Vol {
    int nx, ny, nz;
    int64_t V;
};

// Voxel v's coordinates.  32-bit division: the network's volumes have extents
// of at most 1024, so v < 2^30.
__device__ __forceinline__ void vox_coords(const Vol &d, int64_t v, int *x, int *y, int *z) {
    const unsigned plane = (unsigned)d.nx * (unsigned)d.ny, uv = (unsigned)v;
    const unsigned zz = uv / plane, r = uv - zz * plane;
    const unsigned yy = r / (unsigned)d.nx;
    *z = (int)zz;
    *y = (int)yy;
    *x = (int)(r - yy * (unsigned)d.nx);
}

// i / n for an element index of a launch: 32-bit division where i fits.
__device__ __forceinline__ int64_t idx_div(int64_t i, int n) {
    return i < 0xffffffffLL ? (int64_t)((unsigned)i / (unsigned)n) : i / n;
}

// ---- implicit-GEMM 3x3x3 convolution on the matrix cores ---------------------
// M = voxels, N = output channels, K = 27 taps x input channels, on
// v_mfma_f32_16x16x32_bf16: lane l of a wave holds rows (voxels) l%16 of A
// and columns l%16 of B with the 8-element K slice 8 (l/16) .. 8 (l/16) + 7
// of each 32-channel block, and D[4 (l/16) + i][l%16] of each 16x16 tile.
// x: bf16 [V][xs] (channels 0..cin-1 used); w: bf16 [27][cout][cin];
// y: bf16 [V][ys] (channels 0..cout-1 written).  cin % 32 == 0, xs % 8 == 0,
// ys % 8 == 0, pointers 16-byte aligned.
// Work-group: a 16 x 4 x 4 voxel tile (x fastest) x 16*NT output channels.
// For each 32-channel K block the tile's 18 x 6 x 6 halo of x is staged in
// LDS once ([hz][hy][hx], 32 channels per voxel at a pitch of 40 u16 so the
// 16-byte reads of 16 neighbouring voxels fall in distinct banks; zeros
// outside the volume), and all 27 taps read their A fragments there: wave w
// owns the tile's z-slice w, whose 4 rows of 16 voxels are its 4 M tiles;
// lane (r, g) reads voxel (r + dx, m + dy, w + dz) of the halo.  B fragments
// (weights) come from memory (small, cached).
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;  // 648 voxels
constexpr int kHPitch = 40;             // u16 per halo voxel (32 used)

// Index of weight (tap t, output channel o, input channel c) of a cout x cin
// layer in the fragment-major layout: per tap, 32-channel input block and
// 16-channel output block, the 1 KB B fragment of v_mfma_f32_16x16x32_bf16 in
// lane order (lane 16 g + r holds output channel 16 ob + r and input channels
// 32 kb + 8 g .. + 7), so that a wave reads a fragment as 1 KB in one piece.
// The plain layout [27][cout][cin] puts a fragment's 16 rows cin apart.
__host__ __device__ __forceinline__ int64_t frag_index(int t, int o, int c, int cout, int cin) {
    const int64_t f = ((int64_t)t * (cin >> 5) + (c >> 5)) * (cout >> 4) + (o >> 4);
    return f * 512 + (((c & 31) >> 3) * 16 + (o & 15)) * 8 + (c & 7);
}

// The A fragment one voxel to the right: lane r of each row of 16 takes
// lane r + 1 of lo (DPP row shift left), lane 15 takes lane 14 of hi (row
// shift right), lo and hi being the fragments at offsets 0 and 2 in x.
__device__ __forceinline__ bf16x8 mid_fragment(const bf16x8 &lo, const bf16x8 &hi) {
    const u32x4 a = __builtin_bit_cast(u32x4, lo), b = __builtin_bit_cast(u32x4, hi);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int edge = __builtin_amdgcn_update_dpp(0, (int)b[k], 0x111, 0xF, 0xF, false);  // row_shr:1
        o[k] = (unsigned)__builtin_amdgcn_update_dpp(edge, (int)a[k], 0x101, 0xF, 0xF, false);  // row_shl:1
    }
    return __builtin_bit_cast(bf16x8, o);
}

// The 27 taps run as 9 (dz, dy) rows of 3: per row a wave reads its A
// fragments at dx = -1 and dx = +1 from the halo and forms dx = 0 from them
// with two DPP moves per register, two LDS reads for three taps.  FRAG: the
// weights are in the fragment-major layout.
template <int NT, bool FRAG>
__global__ __launch_bounds__(256) void conv3_tile(const u16 *__restrict__ x, int xs, Vol d, int cin,
                                                  const u16 *__restrict__ w,
                                                  const float *__restrict__ bias, int cout, int relu,
                                                  u16 *__restrict__ y, int ys) {
    __shared__ __attribute__((aligned(16))) u16 halo[kHalo * kHPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ntx = (d.nx + kTX - 1) / kTX, nty = (d.ny + kTY - 1) / kTY;
    int tile = blockIdx.x;
    const int tx = tile % ntx;
    tile /= ntx;
    const int ty = tile % nty, tz = tile / nty;
    const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
    const int co0 = blockIdx.y * (16 * NT);
    // per tap and per output block of 16: strides between B fragments (u16)
    const int64_t tstride = FRAG ? (int64_t)(cin >> 5) * (cout >> 4) * 512 : (int64_t)cout * cin;
    const int64_t nstride = FRAG ? 512 : (int64_t)16 * cin;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // 16-byte halo loads per thread (the last partial), issued kBatch at a time
    // before their LDS stores: all at once, or in two batches for the
    // 64-channel instance, which holds 64 accumulator registers besides
    constexpr int kLoads = (kHalo * 4 + 255) / 256;
    constexpr int kBatch = NT >= 4 ? (kLoads + 1) / 2 : kLoads;
    for (int kb = 0; kb < cin; kb += 32) {
#pragma unroll
        for (int u0 = 0; u0 < kLoads; u0 += kBatch) {
            u32x4 val[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = threadIdx.x + 256 * (u0 + u);
                const int hv = q >> 2, c8 = (q & 3) * 8;
                const int hx = hv % kHX, hr = hv / kHX;
                const int hy = hr % kHY, hz = hr / kHY;
                const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
                val[u] = u32x4{0u, 0u, 0u, 0u};
                if (u0 + u < kLoads && q < kHalo * 4 && gx >= 0 && gy >= 0 && gz >= 0 && gx < d.nx && gy < d.ny &&
                    gz < d.nz)
                    val[u] =
                        *reinterpret_cast<const u32x4 *>(x + (((int64_t)gz * d.ny + gy) * d.nx + gx) * xs + kb + c8);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = threadIdx.x + 256 * (u0 + u);
                if (u0 + u < kLoads && q < kHalo * 4)
                    *reinterpret_cast<u32x4 *>(halo + (q >> 2) * kHPitch + (q & 3) * 8) = val[u];
            }
        }
        __syncthreads();
        const u16 *wk = FRAG ? w + ((int64_t)(kb >> 5) * (cout >> 4) + (co0 >> 4)) * 512 + lane * 8
                             : w + (int64_t)(co0 + r) * cin + kb + 8 * g;
        // B fragments of the three taps of row p; those of row p + 1 are
        // loaded before row p's MFMAs
        bf16x8 b[3][NT];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                b[dx][n] = *reinterpret_cast<const bf16x8 *>(wk + (int64_t)dx * tstride + n * nstride);
#pragma unroll 1
        for (int p = 0; p < 9; ++p) {
            const int dz = p / 3 - 1, dy = p % 3 - 1;
            bf16x8 bn[3][NT];
            if (p < 8) {
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        bn[dx][n] = *reinterpret_cast<const bf16x8 *>(wk + (int64_t)(3 * p + 3 + dx) * tstride +
                                                                     n * nstride);
            }
            bf16x8 a[3][4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                // halo x index r (dx = -1) and r + 2 (dx = +1)
                const int hv = ((wave + 1 + dz) * kHY + (m + 1 + dy)) * kHX + r;
                a[0][m] = *reinterpret_cast<const bf16x8 *>(halo + hv * kHPitch + 8 * g);
                a[2][m] = *reinterpret_cast<const bf16x8 *>(halo + (hv + 2) * kHPitch + 8 * g);
                a[1][m] = mid_fragment(a[0][m], a[2][m]);
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[dx][m], b[dx][n], acc[m][n], 0, 0, 0);
            if (p < 8) {
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int n = 0; n < NT; ++n) b[dx][n] = bn[dx][n];
            }
        }
        __syncthreads();
    }
    // lane holds D[4 g + i][r] of tile (m, n): voxel (x0 + 4 g + i, y0 + m,
    // z0 + wave), channel co0 + 16 n + r
    const int gz = z0 + wave;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = co0 + n * 16 + r;
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int gy = y0 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gx = x0 + 4 * g + i;
                if (gx < d.nx && gy < d.ny && gz < d.nz) {
                    float val = acc[m][n][i] + bb;
                    if (relu) val = fmaxf(val, 0.0f);
                    y[(((int64_t)gz * d.ny + gy) * d.nx + gx) * ys + co] = f2bf(val);
                }
            }
        }
    }
}

// ---- weight gradient ------------------------------------------------------------
// dW[t][co][ci] = sum_v dY[v][co] X[v + t][ci]: K = voxels.  Work-groups:
// 3 shifts (dx) x (cout / 32) x (cin / 32) channel blocks for each chunk of
// the 16 x 4 x 4 voxel tiles (the tiles of conv3_tile).  Per tile a work-group
// stages, transposed in LDS, dY of the tile's 256 voxels ([co][v], v = x +
// 16 (y + 4 z)) and X over the tile's (dy, dz) halo shifted by its dx
// ([ci][hz][hy][x], 6 x 6 rows of 16), so that the 8-voxel K slice of a lane
// is contiguous and 16-byte aligned in both; then wave w, owning the 16x16
// sub-tile (co0 + 16 (w / 2), ci0 + 16 (w % 2)), runs the 9 (dy, dz) taps x 8
// K blocks of 32 voxels = 72 MFMAs per tile, each dY fragment read once for
// the 9 taps.  Loaders take 8 channels of 4 consecutive voxels (along x) and
// write, per channel, the 4 voxels as one 64-bit LDS word.
constexpr int kWgPitchA = 256 + 8;      // u16 per dY row (one channel, 256 voxels)
constexpr int kWgPitchB = 6 * 6 * 16 + 8;  // u16 per X row (one channel, 6 x 6 x 16 voxels)

// Column swizzle of the transposed tiles: row c (a channel) stores its 16-byte
// chunks (8 voxels) XOR-ed with 2 ((c / 8) mod 4), so that the four loader
// lanes of a voxel group, whose channel octets put their rows 8 apart (the
// same LDS banks for any 16-byte-aligned pitch), write different banks.  The
// XOR stays inside aligned groups of 8 chunks.
__device__ __forceinline__ int wg_swz(int row, int col) { return col ^ (((row >> 3) & 3) << 4); }

__device__ __forceinline__ void store_transposed(u16 *dst, int pitch, int c8, int vg, const u32x4 (&q)[4]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int sh = (j & 1) * 16;
        const unsigned long long w =
            (unsigned long long)((q[0][j >> 1] >> sh) & 0xffffu) |
            ((unsigned long long)((q[1][j >> 1] >> sh) & 0xffffu) << 16) |
            ((unsigned long long)((q[2][j >> 1] >> sh) & 0xffffu) << 32) |
            ((unsigned long long)((q[3][j >> 1] >> sh) & 0xffffu) << 48);
        *reinterpret_cast<unsigned long long *>(dst + (c8 + j) * pitch + wg_swz(c8 + j, vg)) = w;
    }
}

__device__ __forceinline__ u32x4 load8(const u16 *p, const Vol &d, int gx, int gy, int gz, int s) {
    if (gx < 0 || gy < 0 || gz < 0 || gx >= d.nx || gy >= d.ny || gz >= d.nz) return u32x4{0u, 0u, 0u, 0u};
    return *reinterpret_cast<const u32x4 *>(p + (((int64_t)gz * d.ny + gy) * d.nx + gx) * s);
}

// One-dimensional grid of ncombo x (nc rounded up to a multiple of 8)
// work-groups, ncombo = 3 shifts x (cout / 32) x (cin / 32).  The dispatcher
// deals work-groups round-robin to the 8 XCDs, so XCD L mod 8 runs work-groups
// L, L + 8, ...; they are given, in order, every combination of chunk
// 8 k + L mod 8 for k = 0, 1, ...: the combinations of a chunk read the same
// tiles of X and dY, which then stay in that XCD's L2.
constexpr int kXcds = 8;

// Two waves per SIMD (the LDS holds two work-groups per CU): the registers
// that carry the next tile's loads fit in the 256 that leaves each wave.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void conv3_wgrad(const u16 *__restrict__ x, int xs, Vol d, int cin,
                                                   const u16 *__restrict__ dy, int dys, int cout, int nc,
                                                   float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) u16 At[32 * kWgPitchA];  // [co][v]
    __shared__ __attribute__((aligned(16))) u16 Bt[32 * kWgPitchB];  // [ci][hz][hy][x]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int n_ci = cin / 32, n_co = cout / 32;
    const int ncombo = 3 * n_co * n_ci;
    const int slot = (int)(blockIdx.x / kXcds);
    const int chunk = (slot / ncombo) * kXcds + (int)(blockIdx.x % kXcds);
    if (chunk >= nc) return;  // whole work-group
    int blk = slot % ncombo;
    const int ib = blk % n_ci;
    blk /= n_ci;
    const int cb = blk % n_co;
    const int dx = blk / n_co - 1;
    const int ntx = (d.nx + kTX - 1) / kTX, nty = (d.ny + kTY - 1) / kTY, ntz = (d.nz + kTZ - 1) / kTZ;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    const int64_t t_begin = ntiles * chunk / nc, t_end = ntiles * (chunk + 1) / nc;
    const int msub = (wave >> 1) * 16, nsub = (wave & 1) * 16;
    f32x4 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // Loader tasks of a tile: dY, 64 groups of 4 voxels (same row) x 4 channel
    // octets, one per thread; X, the halo rows (hz, hy) shifted by dx, 144
    // groups x 4 octets, two or three per thread.  The next tile's loads are
    // issued before the current tile's MFMAs and held in registers.
    const int c8 = (tid & 3) * 8;  // 8 channels of every loader task (task = tid mod 4)
    const int vga = (tid >> 2) * 4;  // dY: tile voxels vga .. vga + 3
    u32x4 qa[4], qb[3][4];
    auto load_tile = [&](int64_t tile) {
        const int tx = (int)(tile % ntx), ty = (int)((tile / ntx) % nty), tz = (int)(tile / ((int64_t)ntx * nty));
        const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
        const int lx = vga & 15, ly = (vga >> 4) & 3, lz = vga >> 6;
#pragma unroll
        for (int i = 0; i < 4; ++i) qa[i] = load8(dy + cb * 32 + c8, d, x0 + lx + i, y0 + ly, z0 + lz, dys);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int task = tid + 256 * u;
            if (task < 144 * 4) {
                const int vg = (task >> 2) * 4;  // halo voxels vg .. vg + 3 (same row of 16)
                const int hx = vg & 15, hr = vg >> 4, hy = hr % 6, hz = hr / 6;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    qb[u][i] = load8(x + ib * 32 + c8, d, x0 + hx + i + dx, y0 + hy - 1, z0 + hz - 1, xs);
            }
        }
    };
    if (t_begin < t_end) load_tile(t_begin);
    for (int64_t tile = t_begin; tile < t_end; ++tile) {
        store_transposed(At, kWgPitchA, c8, vga, qa);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int task = tid + 256 * u;
            if (task < 144 * 4) store_transposed(Bt, kWgPitchB, c8, (task >> 2) * 4, qb[u]);
        }
        __syncthreads();
        if (tile + 1 < t_end) load_tile(tile + 1);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            // K block kk: tile voxels 32 kk .. 32 kk + 31, i.e. rows (y, z) =
            // (2 kk, 2 kk + 1) in units of 16; lane g takes row 2 kk + g / 2,
            // x = 8 (g % 2) .. + 7
            const bf16x8 a =
                *reinterpret_cast<const bf16x8 *>(At + (msub + r) * kWgPitchA + wg_swz(msub + r, kk * 32 + 8 * g));
            const int row = 2 * kk + (g >> 1);  // = y + 4 z of the tile
            const int ly = row & 3, lz = row >> 2, xo = 8 * (g & 1);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int dz = k / 3 - 1, dyy = k % 3 - 1;
                const int hrow = (lz + 1 + dz) * 6 + (ly + 1 + dyy);
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8 *>(Bt + (nsub + r) * kWgPitchB + wg_swz(nsub + r, hrow * 16 + xo));
                acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds D[4 g + i][r] of each tap: co = cb*32 + msub + 4g + i, ci = ib*32 + nsub + r
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int t = (k / 3) * 9 + (k % 3) * 3 + (dx + 1);  // (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
        float *out = part + ((int64_t)chunk * 27 + t) * cout * cin;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = cb * 32 + msub + 4 * g + i, ci = ib * 32 + nsub + r;
            out[(int64_t)co * cin + ci] = acc[k][i];
        }
    }
}

// out[i] = sum_{c < n_chunks} part[c][i] (fixed order).
__global__ __launch_bounds__(256) void sum_chunks(const float *__restrict__ part, int n_chunks, int64_t n,
                                                  float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    // eight running sums (chunks c = u mod 8), so that eight loads are in
    // flight, added in a fixed order at the end
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int c = 0;
    for (; c + 8 <= n_chunks; c += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += part[(int64_t)(c + u) * n + i];
    for (int u = 0; c < n_chunks; ++c, ++u) s[u] += part[(int64_t)c * n + i];
    out[i] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Per-channel sums of a bf16 [V][s] slice (channels 0..C-1), C <= 256 and a
// multiple of 8: part[block][c] over the block's voxel range.  Each thread
// reads 8 channels per voxel; lanes = 256 / (C / 8) threads share a channel
// octet, taking every lanes-th voxel, and their sums are added in a fixed
// order at the end (threads beyond lanes x C / 8 compute sums nobody reads).
constexpr int kSumBlocks = 1024;
__global__ __launch_bounds__(256) void channel_sums(const u16 *__restrict__ a, int s, int C, int64_t V,
                                                    float *__restrict__ part) {
    __shared__ float red[256 * 8];
    // thread: 8 channels c8 .. c8 + 7 (one 16-byte load per voxel) of every
    // lanes-th voxel of the block's range (C % 8 == 0, s % 8 == 0)
    const int groups = C / 8;
    const int c8 = (threadIdx.x % groups) * 8, j = threadIdx.x / groups, lanes = 256 / groups;
    const int64_t per = (V + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * per, v1 = min(V, v0 + per);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t v = v0 + j; v < v1; v += lanes) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(a + v * s + c8);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += bf2f((u16)(q[k >> 1] >> (16 * (k & 1))));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x * 8 + k] = acc[k];
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += 256) {
        float t = 0.0f;
        for (int q = 0; q < lanes; ++q) t += red[(q * groups + c / 8) * 8 + c % 8];
        part[(int64_t)blockIdx.x * C + c] = t;
    }
}

// ---- first layer (one input channel) on the VALU ------------------------------------
// y[v][c] = relu(b[c] + sum_t W[t][c] x[v + t]) for c < B (bf16 out, stride ys).
__global__ __launch_bounds__(256) void conv1_fwd(const float *__restrict__ x, Vol d,
                                                 const float *__restrict__ W /*[27][B]*/,
                                                 const float *__restrict__ b, int B,
                                                 u16 *__restrict__ y, int ys) {
    __shared__ float sw[27 * 256];
    __shared__ float sb[256];
    for (int i = threadIdx.x; i < 27 * B; i += 256) sw[i] = W[i];
    for (int i = threadIdx.x; i < B; i += 256) sb[i] = b[i];
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= d.V) return;
    int px, py, pz;
    vox_coords(d, v, &px, &py, &pz);
    float nb[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int xx = px + t % 3 - 1, yy = py + (t / 3) % 3 - 1, zz = pz + t / 9 - 1;
        const bool in = xx >= 0 && yy >= 0 && zz >= 0 && xx < d.nx && yy < d.ny && zz < d.nz;
        nb[t] = in ? x[((int64_t)zz * d.ny + yy) * d.nx + xx] : 0.0f;
    }
    // 8 channels per 16-byte store (B % 8 == 0, ys % 8 == 0)
    for (int c8 = 0; c8 < B; c8 += 8) {
        u32x4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c8 + 2 * k;
            float a0 = sb[c], a1 = sb[c + 1];
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                a0 = fmaf(sw[t * B + c], nb[t], a0);
                a1 = fmaf(sw[t * B + c + 1], nb[t], a1);
            }
            o[k] = (unsigned)f2bf(fmaxf(a0, 0.0f)) | ((unsigned)f2bf(fmaxf(a1, 0.0f)) << 16);
        }
        *reinterpret_cast<u32x4 *>(y + v * ys + c8) = o;
    }
}

// part[block][t][c] = sum over the block's voxels of dy[v][c] x[v + t]; the
// block walks its share of the 16 x 4 x 4 voxel tiles, stages each tile's
// 18 x 6 x 6 halo of x in LDS, and its 256 threads are 8 voxel lanes x 32
// channel lanes (B <= 32 per pass): per voxel one dy value times the 27
// halo values at constant offsets.
__global__ __launch_bounds__(256) void conv1_wgrad(const float *__restrict__ x, Vol d,
                                                   const u16 *__restrict__ dy, int dys, int B,
                                                   float *__restrict__ part) {
    __shared__ float xh[kHalo];
    __shared__ float red[8][27][32];
    const int c = threadIdx.x & 31, j = threadIdx.x >> 5;
    const int ntx = (d.nx + kTX - 1) / kTX, nty = (d.ny + kTY - 1) / kTY, ntz = (d.nz + kTZ - 1) / kTZ;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    const int64_t t_begin = ntiles * blockIdx.x / gridDim.x, t_end = ntiles * (blockIdx.x + 1) / gridDim.x;
    for (int cb = 0; cb < B; cb += 32) {
        float acc[27];
#pragma unroll
        for (int t = 0; t < 27; ++t) acc[t] = 0.0f;
        for (int64_t tile = t_begin; tile < t_end; ++tile) {
            const int tx = (int)(tile % ntx), ty = (int)((tile / ntx) % nty), tz = (int)(tile / ((int64_t)ntx * nty));
            const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
            __syncthreads();  // the previous tile's halo has been read
            for (int q = threadIdx.x; q < kHalo; q += 256) {
                const int hx = q % kHX, hr = q / kHX, hy = hr % kHY, hz = hr / kHY;
                const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
                xh[q] = (gx >= 0 && gy >= 0 && gz >= 0 && gx < d.nx && gy < d.ny && gz < d.nz)
                            ? x[((int64_t)gz * d.ny + gy) * d.nx + gx] : 0.0f;
            }
            __syncthreads();
            if (cb + c < B) {
                // runs of 4 voxels along x (64 per tile, 8 per thread): per
                // (dz, dy) six halo values serve the run's 3 x 4 products
                for (int run = j; run < kTX * kTY * kTZ / 4; run += 8) {
                    const int lx = (run & 3) * 4, ly = (run >> 2) & 3, lz = run >> 4;
                    const int gy = y0 + ly, gz = z0 + lz;
                    float gv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int gx = x0 + lx + i;
                        gv[i] = (gx < d.nx && gy < d.ny && gz < d.nz)
                                    ? bf2f(dy[(((int64_t)gz * d.ny + gy) * d.nx + gx) * dys + cb + c])
                                    : 0.0f;
                    }
#pragma unroll
                    for (int pz = 0; pz < 3; ++pz)
#pragma unroll
                        for (int py = 0; py < 3; ++py) {
                            const float *hb = xh + ((lz + pz) * kHY + ly + py) * kHX + lx;
                            float h[6];
#pragma unroll
                            for (int q = 0; q < 6; ++q) h[q] = hb[q];
#pragma unroll
                            for (int px = 0; px < 3; ++px) {
                                const int t = pz * 9 + py * 3 + px;
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[t] = fmaf(gv[i], h[i + px], acc[t]);
                            }
                        }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 27; ++t) red[j][t][c] = acc[t];
        __syncthreads();
        for (int i = threadIdx.x; i < 27 * 32; i += 256) {
            const int t = i / 32, cc = i % 32;
            float s = 0.0f;
            for (int jj = 0; jj < 8; ++jj) s += red[jj][t][cc];
            if (cb + cc < B) part[((int64_t)blockIdx.x * 27 + t) * B + cb + cc] = s;
        }
        __syncthreads();
    }
}

// ---- weights -----------------------------------------------------------------------------
// wb[t][o][i] = bf16(W[t][o][i]); wt[t][i][o] = bf16(W[26 - t][o][i]) (the data
// gradient is a convolution of dY with these transposed, tap-reversed weights).
__global__ __launch_bounds__(256) void cast_weights(const float *__restrict__ W, int cout, int cin,
                                                    u16 *__restrict__ wb, u16 *__restrict__ wt) {
    const int64_t n = 27LL * cout * cin;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int t = (int)(i / ((int64_t)cout * cin));
    const int rem = (int)(i - (int64_t)t * cout * cin);
    const int o = rem / cin, ci = rem - o * cin;
    const u16 h = f2bf(W[i]);
    // fragment-major (frag_index): wb for the forward (cout x cin), wt, with
    // the taps reversed and the channel roles swapped, for the data gradient
    wb[frag_index(t, o, ci, cout, cin)] = h;
    wt[frag_index(26 - t, ci, o, cin, cout)] = h;
}

// ---- pooling, upsampling, skip gradients ---------------------------------------------------
// One thread per (coarse voxel, 8-channel group).  Fine volume d (even
// extents), coarse volume dc = d / 2.
__device__ __forceinline__ int64_t fine_child(const Vol &d, int cx, int cy, int cz, int k) {
    return ((int64_t)(2 * cz + (k >> 2)) * d.ny + (2 * cy + ((k >> 1) & 1))) * d.nx + 2 * cx + (k & 1);
}

__global__ __launch_bounds__(256) void pool2_fwd(const u16 *__restrict__ a, int as, Vol d, Vol dc, int C,
                                                 u16 *__restrict__ out) {
    const int groups = C / 8;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= dc.V * groups) return;
    const int64_t p = idx_div(i, groups);
    const int c8 = (int)(i - p * groups) * 8;
    int cx, cy, cz;
    vox_coords(dc, p, &cx, &cy, &cz);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(a + fine_child(d, cx, cy, cz, k) * as + c8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[2 * j] += bf2f((u16)(q[j] & 0xffffu));
            s[2 * j + 1] += bf2f((u16)(q[j] >> 16));
        }
    }
    u32x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (unsigned)f2bf(0.125f * s[2 * j]) | ((unsigned)f2bf(0.125f * s[2 * j + 1]) << 16);
    *reinterpret_cast<u32x4 *>(out + p * C + c8) = o;
}

// out slice [V][os] channels 0..C-1 = src[parent][c]
__global__ __launch_bounds__(256) void up2_fwd(const u16 *__restrict__ src, Vol d, Vol dc, int C,
                                               u16 *__restrict__ out, int os) {
    const int groups = C / 8;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= dc.V * groups) return;
    const int64_t p = idx_div(i, groups);
    const int c8 = (int)(i - p * groups) * 8;
    int cx, cy, cz;
    vox_coords(dc, p, &cx, &cy, &cz);
    const u32x4 q = *reinterpret_cast<const u32x4 *>(src + p * C + c8);
    for (int k = 0; k < 8; ++k) *reinterpret_cast<u32x4 *>(out + fine_child(d, cx, cy, cz, k) * os + c8) = q;
}

// dpre[p][c] = (sum of the 8 children of dcat[.][c]) * (act[p][c] > 0)
__global__ __launch_bounds__(256) void up2_bwd_relu(const u16 *__restrict__ dcat, int ds, Vol d, Vol dc,
                                                    int C, const u16 *__restrict__ act,
                                                    u16 *__restrict__ dpre) {
    const int groups = C / 8;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= dc.V * groups) return;
    const int64_t p = idx_div(i, groups);
    const int c8 = (int)(i - p * groups) * 8;
    int cx, cy, cz;
    vox_coords(dc, p, &cx, &cy, &cz);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(dcat + fine_child(d, cx, cy, cz, k) * ds + c8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[2 * j] += bf2f((u16)(q[j] & 0xffffu));
            s[2 * j + 1] += bf2f((u16)(q[j] >> 16));
        }
    }
    const u32x4 m = *reinterpret_cast<const u32x4 *>(act + p * C + c8);
    u32x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float a0 = bf2f((u16)(m[j] & 0xffffu)) > 0.0f ? s[2 * j] : 0.0f;
        const float a1 = bf2f((u16)(m[j] >> 16)) > 0.0f ? s[2 * j + 1] : 0.0f;
        o[j] = (unsigned)f2bf(a0) | ((unsigned)f2bf(a1) << 16);
    }
    *reinterpret_cast<u32x4 *>(dpre + p * C + c8) = o;
}

// dpre[v][c] = (dskip[v][c] + dpool[parent(v)][c] / 8) * (act[v][c] > 0);
// dskip: slice of the concatenation gradient (stride ds), act: encoder output
// (stride as).  One thread per (fine voxel, 8-channel group).
__global__ __launch_bounds__(256) void skip_bwd_relu(const u16 *__restrict__ dskip, int ds,
                                                     const u16 *__restrict__ dpool, Vol d, Vol dc, int C,
                                                     const u16 *__restrict__ act, int as,
                                                     u16 *__restrict__ dpre) {
    const int groups = C / 8;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= d.V * groups) return;
    const int64_t v = idx_div(i, groups);
    const int c8 = (int)(i - v * groups) * 8;
    int px, py, pz;
    vox_coords(d, v, &px, &py, &pz);
    const int64_t p = ((int64_t)(pz >> 1) * dc.ny + (py >> 1)) * dc.nx + (px >> 1);
    const u32x4 qs = *reinterpret_cast<const u32x4 *>(dskip + v * ds + c8);
    const u32x4 qp = *reinterpret_cast<const u32x4 *>(dpool + p * C + c8);
    const u32x4 m = *reinterpret_cast<const u32x4 *>(act + v * as + c8);
    u32x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float a0 = bf2f((u16)(qs[j] & 0xffffu)) + 0.125f * bf2f((u16)(qp[j] & 0xffffu));
        float a1 = bf2f((u16)(qs[j] >> 16)) + 0.125f * bf2f((u16)(qp[j] >> 16));
        if (!(bf2f((u16)(m[j] & 0xffffu)) > 0.0f)) a0 = 0.0f;
        if (!(bf2f((u16)(m[j] >> 16)) > 0.0f)) a1 = 0.0f;
        o[j] = (unsigned)f2bf(a0) | ((unsigned)f2bf(a1) << 16);
    }
    *reinterpret_cast<u32x4 *>(dpre + v * C + c8) = o;
}

// ---- head (1x1x1, B -> 3) and loss -----------------------------------------------------
__global__ __launch_bounds__(256) void head_fwd(const u16 *__restrict__ a, int B, int64_t V,
                                                const float *__restrict__ Wh, const float *__restrict__ bh,
                                                float *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    float o0 = bh[0], o1 = bh[1], o2 = bh[2];
    // the voxel's B channels as 16-byte vectors (B % 8 == 0), in channel order
    for (int c8 = 0; c8 < B; c8 += 8) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(a + v * B + c8);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c8 + k;
            const float h = bf2f((u16)(q[k >> 1] >> (16 * (k & 1))));
            o0 = fmaf(Wh[c], h, o0);
            o1 = fmaf(Wh[B + c], h, o1);
            o2 = fmaf(Wh[2 * B + c], h, o2);
        }
    }
    out[3 * v] = o0;
    out[3 * v + 1] = o1;
    out[3 * v + 2] = o2;
}

// dpre[v][c] = (sum_o dout[v][o] Wh[o][c]) * (a[v][c] > 0); block partials of
// dWh[o][c] = sum_v dout[v][o] a[v][c] and dbh[o].  256 threads = 256 / B voxel
// lanes x B channels (B = 32), summed in a fixed order at the end.
__global__ __launch_bounds__(256) void head_bwd(const u16 *__restrict__ a, int B, int64_t V,
                                                const float *__restrict__ Wh, const float *__restrict__ dout,
                                                u16 *__restrict__ dpre, float *__restrict__ part) {
    // thread: channel octet c8 .. c8 + 7 (16-byte loads and stores) of every
    // lanes-th voxel of the block's range; B % 8 == 0 and B / 8 divides 256
    __shared__ float red[256 * 27];
    const int groups = B / 8;
    const int c8 = (threadIdx.x % groups) * 8, j = threadIdx.x / groups, lanes = 256 / groups;
    const int64_t per = (V + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * per, v1 = min(V, v0 + per);
    float gs[3][8], bs[3] = {0.0f, 0.0f, 0.0f}, w[3][8];
#pragma unroll
    for (int o = 0; o < 3; ++o)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            gs[o][k] = 0.0f;
            w[o][k] = Wh[o * B + c8 + k];
        }
    for (int64_t v = v0 + j; v < v1; v += lanes) {
        const float d0 = dout[3 * v], d1 = dout[3 * v + 1], d2 = dout[3 * v + 2];
        const u32x4 q = *reinterpret_cast<const u32x4 *>(a + v * B + c8);
        u32x4 r;
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            unsigned packed = 0u;
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int k = 2 * k2 + h2;
                const float h = bf2f((u16)(q[k2] >> (16 * h2)));
                gs[0][k] = fmaf(d0, h, gs[0][k]);
                gs[1][k] = fmaf(d1, h, gs[1][k]);
                gs[2][k] = fmaf(d2, h, gs[2][k]);
                const float sv = fmaf(d0, w[0][k], fmaf(d1, w[1][k], d2 * w[2][k]));
                packed |= (unsigned)f2bf(h > 0.0f ? sv : 0.0f) << (16 * h2);
            }
            r[k2] = packed;
        }
        *reinterpret_cast<u32x4 *>(dpre + v * B + c8) = r;
        bs[0] += d0;
        bs[1] += d1;
        bs[2] += d2;
    }
    float *mine = red + threadIdx.x * 27;
#pragma unroll
    for (int o = 0; o < 3; ++o) {
#pragma unroll
        for (int k = 0; k < 8; ++k) mine[o * 8 + k] = gs[o][k];
        mine[24 + o] = bs[o];
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * (3 * B + 3);
    for (int e = threadIdx.x; e < 3 * B + 3; e += 256) {
        float t = 0.0f;
        if (e < 3 * B) {  // weight (o, c)
            const int o = e / B, c = e - o * B;
            for (int qq = 0; qq < lanes; ++qq) t += red[(qq * groups + c / 8) * 27 + o * 8 + c % 8];
        } else {  // bias o: the threads of octet 0 saw every voxel of the range
            for (int qq = 0; qq < lanes; ++qq) t += red[(qq * groups) * 27 + 24 + (e - 3 * B)];
        }
        out[e] = t;
    }
}

// part[block] = sum of per-voxel losses (binary64); dout = dL/dout.
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ out,
                                                   const float *__restrict__ tgt, int64_t V,
                                                   float *__restrict__ dout, double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    const float inv_v = (float)(1.0 / (double)V);
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const float od = out[3 * v], os = out[3 * v + 1], oo = out[3 * v + 2];
        const float td = tgt[3 * v], ts = tgt[3 * v + 1], to = tgt[3 * v + 2];
        const float ed = od - td, es = os - ts;
        const float sp = fmaxf(oo, 0.0f) + log1pf(expf(-fabsf(oo)));  // softplus
        acc += (double)(ed * ed) + (double)(to * es * es) + (double)(sp - to * oo);
        dout[3 * v] = 2.0f * ed * inv_v;
        dout[3 * v + 1] = 2.0f * to * es * inv_v;
        dout[3 * v + 2] = (1.0f / (1.0f + expf(-oo)) - to) * inv_v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void loss_final(const double *__restrict__ part, int nb, int64_t V,
                                                  float *__restrict__ loss) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(sh[0] / (double)V);
}

// out[i] = sum over blocks of part[block][i], n entries: one work-group per
// entry, a fixed-order tree over the block partials.
__global__ __launch_bounds__(256) void sum_parts(const float *__restrict__ part, int nb, int n,
                                                 float *__restrict__ out) {
    __shared__ float sh[256];
    const int i = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(int64_t)b * n + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sh[0];
}

// ---- host side -----------------------------------------------------------------------------
unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Layer {
    int cin, cout;
    int64_t w_off, b_off;  // offsets in the flat parameter vector
};

struct Net {
    int B;
    Vol d[4];  // levels 1..4 (index 0..3)
    Layer L[8];  // enc1 enc2 enc3 bott dec3 dec2 dec1 head
    int64_t n_params;
};

enum { ENC1, ENC2, ENC3, BOTT, DEC3, DEC2, DEC1, HEAD };

bool make_net(const int32_t dims[3], int B, Net *n) {
    if (B != 32) return false;  // the 32/64/128/256 network
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 8 || dims[a] % 8 != 0 || dims[a] > 1024) return false;
    n->B = B;
    for (int l = 0; l < 4; ++l) {
        n->d[l].nx = dims[0] >> l;
        n->d[l].ny = dims[1] >> l;
        n->d[l].nz = dims[2] >> l;
        n->d[l].V = (int64_t)n->d[l].nx * n->d[l].ny * n->d[l].nz;
    }
    const int io[8][2] = {{1, B}, {B, 2 * B}, {2 * B, 4 * B}, {4 * B, 8 * B},
                          {12 * B, 4 * B}, {6 * B, 2 * B}, {3 * B, B}, {B, 3}};
    int64_t off = 0;
    for (int l = 0; l < 8; ++l) {
        Layer &L = n->L[l];
        L.cin = io[l][0];
        L.cout = io[l][1];
        L.w_off = off;
        off += (int64_t)(l == HEAD ? 1 : 27) * L.cin * L.cout;
        L.b_off = off;
        off += L.cout;
    }
    n->n_params = off;
    return true;
}

// Buffers in the workspace (bf16 unless noted).  Concatenations:
//   cat1 [V1][3B] = up(dec2) 2B | enc1 B;  cat2 [V2][6B] = up(dec3) 4B | enc2 2B;
//   cat3 [V3][12B] = up(bott) 8B | enc3 4B.
struct UWs {
    u16 *wb[7], *wt[7];  // conv weights [27][cout][cin] and transposed/reversed
    u16 *cat1, *cat2, *cat3, *p2, *p3, *p4, *bott, *dec3, *dec2, *dec1;
    u16 *g_dec1, *g_cat1, *g_dec2, *g_cat2, *g_dec3, *g_cat3, *g_bott, *g_p4, *g_enc3, *g_p3, *g_enc2,
        *g_p2, *g_enc1;
    float *part;      // weight-gradient partials
    int64_t part_n;   // floats in part
    double *lpart;    // loss partials
    size_t bytes;
};

constexpr int kLossBlocks = 1024;
constexpr int kHeadBlocks = 1024;
constexpr int kConv1Blocks = 2048;

// Voxel-tile chunks of the weight gradient: about 8 tiles of 256 voxels each.
int wgrad_chunks(int64_t V) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, V / 2048)); }

UWs carve_unet(void *base, const Net &n) {
    UWs w;
    Carver c(base);
    const int B = n.B;
    const int64_t V1 = n.d[0].V, V2 = n.d[1].V, V3 = n.d[2].V, V4 = n.d[3].V;
    for (int l = ENC2; l <= DEC1; ++l) {
        const int64_t nw = 27LL * n.L[l].cin * n.L[l].cout;
        w.wb[l] = c.take<u16>(nw);
        w.wt[l] = c.take<u16>(nw);
    }
    w.wb[ENC1] = w.wt[ENC1] = nullptr;
    w.cat1 = c.take<u16>(V1 * 3 * B);
    w.cat2 = c.take<u16>(V2 * 6 * B);
    w.cat3 = c.take<u16>(V3 * 12 * B);
    w.p2 = c.take<u16>(V2 * B);
    w.p3 = c.take<u16>(V3 * 2 * B);
    w.p4 = c.take<u16>(V4 * 4 * B);
    w.bott = c.take<u16>(V4 * 8 * B);
    w.dec3 = c.take<u16>(V3 * 4 * B);
    w.dec2 = c.take<u16>(V2 * 2 * B);
    w.dec1 = c.take<u16>(V1 * B);
    w.g_dec1 = c.take<u16>(V1 * B);
    w.g_cat1 = c.take<u16>(V1 * 3 * B);
    w.g_dec2 = c.take<u16>(V2 * 2 * B);
    w.g_cat2 = c.take<u16>(V2 * 6 * B);
    w.g_dec3 = c.take<u16>(V3 * 4 * B);
    w.g_cat3 = c.take<u16>(V3 * 12 * B);
    w.g_bott = c.take<u16>(V4 * 8 * B);
    w.g_p4 = c.take<u16>(V4 * 4 * B);
    w.g_enc3 = c.take<u16>(V3 * 4 * B);
    w.g_p3 = c.take<u16>(V3 * 2 * B);
    w.g_enc2 = c.take<u16>(V2 * 2 * B);
    w.g_p2 = c.take<u16>(V2 * B);
    w.g_enc1 = c.take<u16>(V1 * B);
    int64_t pn = (int64_t)kConv1Blocks * 27 * B;
    pn = std::max<int64_t>(pn, (int64_t)kHeadBlocks * (3 * B + 3));
    pn = std::max<int64_t>(pn, (int64_t)kSumBlocks * 8 * B);
    const int lev[7] = {0, 1, 2, 3, 2, 1, 0};
    for (int l = ENC2; l <= DEC1; ++l)
        pn = std::max<int64_t>(pn, (int64_t)wgrad_chunks(n.d[lev[l]].V) * 27 * n.L[l].cin * n.L[l].cout);
    w.part = c.take<float>(pn);
    w.part_n = pn;
    w.lpart = c.take<double>(kLossBlocks);
    w.bytes = c.off;
    return w;
}

dgr_status check_unet(const int32_t dims[3], int B, Net *n, void *ws, size_t ws_bytes) {
    DGR_CHECK(dims != nullptr, "dims is null");
    DGR_CHECK(make_net(dims, B, n),
              "U-Net needs base width 32 and extents that are multiples of 8 in [8, 1024]");
    DGR_CHECK(ws != nullptr, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t need = carve_unet(nullptr, *n).bytes;
    if (ws_bytes < need) return fail(DGR_ERR_WORKSPACE, "workspace holds %zu bytes, U-Net needs %zu", ws_bytes, need);
    return DGR_OK;
}

// frag: w is in the fragment-major layout (the library's casts), else plain
// [27][cout][cin].
dgr_status launch_conv(const u16 *x, int xs, const Vol &d, int cin, const u16 *w, const float *bias,
                       int cout, int relu, u16 *y, int ys, hipStream_t st, bool frag = true) {
    const int64_t tiles = (int64_t)((d.nx + kTX - 1) / kTX) * ((d.ny + kTY - 1) / kTY) * ((d.nz + kTZ - 1) / kTZ);
    // output channels per work-group: 64 where they divide, else 32; 16 where
    // that leaves fewer than two work-groups per CU (the deep levels: 16^3
    // voxels are 16 tiles), trading fragment reuse for parallelism
    int per = cout % 64 == 0 ? 64 : 32;
    if (frag && tiles * (cout / per) < 512) per = 16;
    const dim3 grid((unsigned)tiles, (unsigned)(cout / per));
    if (per == 16)
        conv3_tile<1, true><<<grid, dim3(256), 0, st>>>(x, xs, d, cin, w, bias, cout, relu, y, ys);
    else if (per == 64 && frag)
        conv3_tile<4, true><<<grid, dim3(256), 0, st>>>(x, xs, d, cin, w, bias, cout, relu, y, ys);
    else if (frag)
        conv3_tile<2, true><<<grid, dim3(256), 0, st>>>(x, xs, d, cin, w, bias, cout, relu, y, ys);
    else if (per == 64)
        conv3_tile<4, false><<<grid, dim3(256), 0, st>>>(x, xs, d, cin, w, bias, cout, relu, y, ys);
    else
        conv3_tile<2, false><<<grid, dim3(256), 0, st>>>(x, xs, d, cin, w, bias, cout, relu, y, ys);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

// dW (binary32 [27][cout][cin]) and db ([cout]) of one conv3 layer.
dgr_status launch_wgrad(const u16 *x, int xs, const Vol &d, int cin, const u16 *dy, int cout, float *part,
                        float *dW, float *db, hipStream_t st) {
    const int nc = wgrad_chunks(d.V);
    const int64_t blocks = (int64_t)3 * (cout / 32) * (cin / 32) * ((nc + kXcds - 1) / kXcds * kXcds);
    conv3_wgrad<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(x, xs, d, cin, dy, cout, cout, nc, part);
    DGR_LAUNCH_CHECK();
    const int64_t n = 27LL * cout * cin;
    sum_chunks<<<blocks_for(n), 256, 0, st>>>(part, nc, n, dW);
    DGR_LAUNCH_CHECK();
    channel_sums<<<kSumBlocks, 256, 0, st>>>(dy, cout, cout, d.V, part);
    DGR_LAUNCH_CHECK();
    sum_parts<<<cout, 256, 0, st>>>(part, kSumBlocks, cout, db);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

dgr_status up_level(const u16 *src, const Vol &fine, const Vol &coarse, int C, u16 *cat, int cs,
                    hipStream_t st) {
    up2_fwd<<<blocks_for(coarse.V * (C / 8)), 256, 0, st>>>(src, fine, coarse, C, cat, cs);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

dgr_status pool_level(const u16 *a, int as, const Vol &fine, const Vol &coarse, int C, u16 *out,
                      hipStream_t st) {
    pool2_fwd<<<blocks_for(coarse.V * (C / 8)), 256, 0, st>>>(a, as, fine, coarse, C, out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

}  // namespace
}  // namespace dgr

using namespace dgr;

#define DGR_RET(expr)                      \
    do {                                   \
        dgr_status s_ = (expr);            \
        if (s_ != DGR_OK) return s_;       \
    } while (0)

extern "C" int64_t dgr_unet_param_count(int32_t base) {
    const int32_t dims[3] = {8, 8, 8};
    Net n;
    if (!make_net(dims, base, &n)) return -1;
    return n.n_params;
}

extern "C" size_t dgr_unet_workspace(const int32_t dims[3], int32_t base) {
    Net n;
    if (!dims || !make_net(dims, base, &n)) return 0;
    return carve_unet(nullptr, n).bytes;
}

extern "C" dgr_status dgr_unet_forward(const float *params, const float *input, const int32_t dims[3],
                                       int32_t base, float *out, void *ws, size_t ws_bytes, void *stream) {
    Net n;
    DGR_RET(check_unet(dims, base, &n, ws, ws_bytes));
    DGR_CHECK(params && input && out, "null pointer argument");
    hipStream_t st = as_stream(stream);
    UWs w = carve_unet(ws, n);
    const int B = n.B;
    for (int l = ENC2; l <= DEC1; ++l) {
        const Layer &L = n.L[l];
        cast_weights<<<blocks_for(27LL * L.cin * L.cout), 256, 0, st>>>(params + L.w_off, L.cout, L.cin,
                                                                         w.wb[l], w.wt[l]);
        DGR_LAUNCH_CHECK();
    }
    const Vol &d1 = n.d[0], &d2 = n.d[1], &d3 = n.d[2], &d4 = n.d[3];
    auto P = [&](int l) { return params + n.L[l].w_off; };
    auto Bi = [&](int l) { return params + n.L[l].b_off; };
    // encoder (encoder outputs live in the concatenation buffers' skip slices)
    conv1_fwd<<<blocks_for(d1.V), 256, 0, st>>>(input, d1, P(ENC1), Bi(ENC1), B, w.cat1 + 2 * B, 3 * B);
    DGR_LAUNCH_CHECK();
    DGR_RET(pool_level(w.cat1 + 2 * B, 3 * B, d1, d2, B, w.p2, st));
    DGR_RET(launch_conv(w.p2, B, d2, B, w.wb[ENC2], Bi(ENC2), 2 * B, 1, w.cat2 + 4 * B, 6 * B, st));
    DGR_RET(pool_level(w.cat2 + 4 * B, 6 * B, d2, d3, 2 * B, w.p3, st));
    DGR_RET(launch_conv(w.p3, 2 * B, d3, 2 * B, w.wb[ENC3], Bi(ENC3), 4 * B, 1, w.cat3 + 8 * B, 12 * B, st));
    DGR_RET(pool_level(w.cat3 + 8 * B, 12 * B, d3, d4, 4 * B, w.p4, st));
    DGR_RET(launch_conv(w.p4, 4 * B, d4, 4 * B, w.wb[BOTT], Bi(BOTT), 8 * B, 1, w.bott, 8 * B, st));
    // decoder
    DGR_RET(up_level(w.bott, d3, d4, 8 * B, w.cat3, 12 * B, st));
    DGR_RET(launch_conv(w.cat3, 12 * B, d3, 12 * B, w.wb[DEC3], Bi(DEC3), 4 * B, 1, w.dec3, 4 * B, st));
    DGR_RET(up_level(w.dec3, d2, d3, 4 * B, w.cat2, 6 * B, st));
    DGR_RET(launch_conv(w.cat2, 6 * B, d2, 6 * B, w.wb[DEC2], Bi(DEC2), 2 * B, 1, w.dec2, 2 * B, st));
    DGR_RET(up_level(w.dec2, d1, d2, 2 * B, w.cat1, 3 * B, st));
    DGR_RET(launch_conv(w.cat1, 3 * B, d1, 3 * B, w.wb[DEC1], Bi(DEC1), B, 1, w.dec1, B, st));
    head_fwd<<<blocks_for(d1.V), 256, 0, st>>>(w.dec1, B, d1.V, P(HEAD), Bi(HEAD), out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" dgr_status dgr_unet_backward(const float *params, const float *input, const int32_t dims[3],
                                        int32_t base, const float *dout, float *grad, void *ws,
                                        size_t ws_bytes, void *stream) {
    Net n;
    DGR_RET(check_unet(dims, base, &n, ws, ws_bytes));
    DGR_CHECK(params && input && dout && grad, "null pointer argument");
    hipStream_t st = as_stream(stream);
    UWs w = carve_unet(ws, n);
    const int B = n.B;
    const Vol &d1 = n.d[0], &d2 = n.d[1], &d3 = n.d[2], &d4 = n.d[3];
    auto G = [&](int l) { return grad + n.L[l].w_off; };
    auto Gb = [&](int l) { return grad + n.L[l].b_off; };
    // head
    head_bwd<<<kHeadBlocks, 256, 0, st>>>(w.dec1, B, d1.V, params + n.L[HEAD].w_off, dout, w.g_dec1, w.part);
    DGR_LAUNCH_CHECK();
    sum_parts<<<3 * B + 3, 256, 0, st>>>(w.part, kHeadBlocks, 3 * B + 3, G(HEAD));
    DGR_LAUNCH_CHECK();
    // dec1: input cat1, output grad g_dec1 (pre-activation)
    DGR_RET(launch_wgrad(w.cat1, 3 * B, d1, 3 * B, w.g_dec1, B, w.part, G(DEC1), Gb(DEC1), st));
    DGR_RET(launch_conv(w.g_dec1, B, d1, B, w.wt[DEC1], nullptr, 3 * B, 0, w.g_cat1, 3 * B, st));
    up2_bwd_relu<<<blocks_for(d2.V * (2 * B / 8)), 256, 0, st>>>(w.g_cat1, 3 * B, d1, d2, 2 * B, w.dec2, w.g_dec2);
    DGR_LAUNCH_CHECK();
    // dec2
    DGR_RET(launch_wgrad(w.cat2, 6 * B, d2, 6 * B, w.g_dec2, 2 * B, w.part, G(DEC2), Gb(DEC2), st));
    DGR_RET(launch_conv(w.g_dec2, 2 * B, d2, 2 * B, w.wt[DEC2], nullptr, 6 * B, 0, w.g_cat2, 6 * B, st));
    up2_bwd_relu<<<blocks_for(d3.V * (4 * B / 8)), 256, 0, st>>>(w.g_cat2, 6 * B, d2, d3, 4 * B, w.dec3, w.g_dec3);
    DGR_LAUNCH_CHECK();
    // dec3
    DGR_RET(launch_wgrad(w.cat3, 12 * B, d3, 12 * B, w.g_dec3, 4 * B, w.part, G(DEC3), Gb(DEC3), st));
    DGR_RET(launch_conv(w.g_dec3, 4 * B, d3, 4 * B, w.wt[DEC3], nullptr, 12 * B, 0, w.g_cat3, 12 * B, st));
    up2_bwd_relu<<<blocks_for(d4.V * (8 * B / 8)), 256, 0, st>>>(w.g_cat3, 12 * B, d3, d4, 8 * B, w.bott, w.g_bott);
    DGR_LAUNCH_CHECK();
    // bottleneck: input p4
    DGR_RET(launch_wgrad(w.p4, 4 * B, d4, 4 * B, w.g_bott, 8 * B, w.part, G(BOTT), Gb(BOTT), st));
    DGR_RET(launch_conv(w.g_bott, 8 * B, d4, 8 * B, w.wt[BOTT], nullptr, 4 * B, 0, w.g_p4, 4 * B, st));
    // enc3: its output feeds cat3 (skip) and pool -> bott
    skip_bwd_relu<<<blocks_for(d3.V * (4 * B / 8)), 256, 0, st>>>(w.g_cat3 + 8 * B, 12 * B, w.g_p4, d3, d4,
                                                                   4 * B, w.cat3 + 8 * B, 12 * B, w.g_enc3);
    DGR_LAUNCH_CHECK();
    DGR_RET(launch_wgrad(w.p3, 2 * B, d3, 2 * B, w.g_enc3, 4 * B, w.part, G(ENC3), Gb(ENC3), st));
    DGR_RET(launch_conv(w.g_enc3, 4 * B, d3, 4 * B, w.wt[ENC3], nullptr, 2 * B, 0, w.g_p3, 2 * B, st));
    // enc2
    skip_bwd_relu<<<blocks_for(d2.V * (2 * B / 8)), 256, 0, st>>>(w.g_cat2 + 4 * B, 6 * B, w.g_p3, d2, d3,
                                                                   2 * B, w.cat2 + 4 * B, 6 * B, w.g_enc2);
    DGR_LAUNCH_CHECK();
    DGR_RET(launch_wgrad(w.p2, B, d2, B, w.g_enc2, 2 * B, w.part, G(ENC2), Gb(ENC2), st));
    DGR_RET(launch_conv(w.g_enc2, 2 * B, d2, 2 * B, w.wt[ENC2], nullptr, B, 0, w.g_p2, B, st));
    // enc1 (first layer, VALU)
    skip_bwd_relu<<<blocks_for(d1.V * (B / 8)), 256, 0, st>>>(w.g_cat1 + 2 * B, 3 * B, w.g_p2, d1, d2, B,
                                                               w.cat1 + 2 * B, 3 * B, w.g_enc1);
    DGR_LAUNCH_CHECK();
    conv1_wgrad<<<kConv1Blocks, 256, 0, st>>>(input, d1, w.g_enc1, B, B, w.part);
    DGR_LAUNCH_CHECK();
    sum_parts<<<27 * B, 256, 0, st>>>(w.part, kConv1Blocks, 27 * B, G(ENC1));
    DGR_LAUNCH_CHECK();
    channel_sums<<<kSumBlocks, 256, 0, st>>>(w.g_enc1, B, B, d1.V, w.part);
    DGR_LAUNCH_CHECK();
    sum_parts<<<B, 256, 0, st>>>(w.part, kSumBlocks, B, Gb(ENC1));
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_unet_loss_workspace(void) { return align_up(sizeof(double) * kLossBlocks); }

extern "C" dgr_status dgr_unet_loss(const float *out, const float *target, int64_t n_voxels, float *loss,
                                    float *dout, void *ws, size_t ws_bytes, void *stream) {
    DGR_CHECK(n_voxels >= 1, "n_voxels must be >= 1");
    DGR_CHECK(out && target && loss && dout && ws, "null pointer argument");
    if (ws_bytes < dgr_unet_loss_workspace()) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    hipStream_t st = as_stream(stream);
    double *part = static_cast<double *>(ws);
    const int nb = (int)std::min<int64_t>(kLossBlocks, (n_voxels + 255) / 256);
    loss_kernel<<<nb, 256, 0, st>>>(out, target, n_voxels, dout, part);
    DGR_LAUNCH_CHECK();
    loss_final<<<1, 256, 0, st>>>(part, nb, n_voxels, loss);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

// ---- single layers, for tests -----------------------------------------------------------------
extern "C" dgr_status dgr_conv3_forward(const uint16_t *x, int32_t x_stride, const int32_t dims[3],
                                        int32_t cin, const uint16_t *w, const float *bias, int32_t cout,
                                        int32_t relu, uint16_t *y, int32_t y_stride, void *stream) {
    DGR_CHECK(x && w && y && dims, "null pointer argument");
    DGR_CHECK(cin >= 32 && cin % 32 == 0 && cout >= 32 && cout % 32 == 0, "cin and cout must be multiples of 32");
    DGR_CHECK(x_stride >= cin && x_stride % 8 == 0 && y_stride >= cout && y_stride % 8 == 0,
              "strides must cover the channels and be multiples of 8");
    DGR_CHECK(((uintptr_t)x | (uintptr_t)w | (uintptr_t)y) % 16 == 0, "pointers must be 16-byte aligned");
    Vol d{dims[0], dims[1], dims[2], (int64_t)dims[0] * dims[1] * dims[2]};
    DGR_CHECK(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1, "dims must be >= 1");
    return launch_conv(reinterpret_cast<const u16 *>(x), x_stride, d, cin, reinterpret_cast<const u16 *>(w),
                       bias, cout, relu, reinterpret_cast<u16 *>(y), y_stride, as_stream(stream), false);
}

extern "C" size_t dgr_conv3_grad_workspace(const int32_t dims[3], int32_t cin, int32_t cout) {
    if (!dims || cin < 1 || cout < 1) return 0;
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    const int64_t pn = std::max<int64_t>((int64_t)wgrad_chunks(V) * 27 * cin * cout, (int64_t)kSumBlocks * cout);
    return align_up(sizeof(float) * pn) + 2 * align_up(sizeof(u16) * 27 * cin * cout);
}

extern "C" dgr_status dgr_conv3_backward(const uint16_t *x, int32_t x_stride, const int32_t dims[3],
                                         int32_t cin, const float *w, const uint16_t *dy, int32_t cout,
                                         float *dw, float *db, uint16_t *dx, void *ws, size_t ws_bytes,
                                         void *stream) {
    DGR_CHECK(x && w && dy && dw && db && dx && dims && ws, "null pointer argument");
    DGR_CHECK(cin >= 32 && cin % 32 == 0 && cout >= 32 && cout % 32 == 0 && cout <= 256,
              "cin and cout must be multiples of 32, cout <= 256");
    DGR_CHECK(x_stride >= cin && x_stride % 8 == 0, "x stride must cover cin and be a multiple of 8");
    DGR_CHECK(((uintptr_t)x | (uintptr_t)dy | (uintptr_t)dx) % 16 == 0, "pointers must be 16-byte aligned");
    DGR_CHECK(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1, "dims must be >= 1");
    if (ws_bytes < dgr_conv3_grad_workspace(dims, cin, cout)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = as_stream(stream);
    Vol d{dims[0], dims[1], dims[2], (int64_t)dims[0] * dims[1] * dims[2]};
    const int64_t V = d.V;
    Carver c(ws);
    float *part = c.take<float>(std::max<int64_t>((int64_t)wgrad_chunks(V) * 27 * cin * cout, (int64_t)kSumBlocks * cout));
    u16 *wb = c.take<u16>(27LL * cin * cout);
    u16 *wt = c.take<u16>(27LL * cin * cout);
    cast_weights<<<blocks_for(27LL * cin * cout), 256, 0, st>>>(w, cout, cin, wb, wt);
    DGR_LAUNCH_CHECK();
    DGR_RET(launch_wgrad(reinterpret_cast<const u16 *>(x), x_stride, d, cin, reinterpret_cast<const u16 *>(dy),
                         cout, part, dw, db, st));
    return launch_conv(reinterpret_cast<const u16 *>(dy), cout, d, cout, wt, nullptr, cin, 0,
                       reinterpret_cast<u16 *>(dx), cin, st);
}
