// Tile binning of truncation boxes: per-Gaussian tile counts -> exclusive scan
// -> (tile, gid) emission in gid order -> stable LSD radix sort on the tile
// key -> per-tile ranges.  The result is the unique list ordered by
// (tile, gid), so every tile later sums its Gaussians in ascending index.
//
// This replaces the scatter-add of the paper's Alg. 1 (final accumulation step)
// by a gather per 8^3 tile; the set of (Gaussian, voxel) contributions is the
// same.
#include <algorithm>

#include "internal.h"

namespace dgr {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 2048;  // elements per scan / sort block
constexpr int kRounds = kTile / kThreads;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <class T>
__device__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan over the 256 threads of a block; *total receives the sum.
template <class T>
__device__ T block_exclusive_scan(T v, T *total) {
    __shared__ T wsum[kThreads / 64];
    T inc = wave_inclusive_scan(v);
    if (lane_id() == 63) wsum[wave_id()] = inc;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave_id()) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// ---- device-wide exclusive scan (three kernels) ----------------------------
template <class Tin, class Tout>
__global__ __launch_bounds__(kThreads) void scan_reduce(const Tin *__restrict__ in, int64_t n,
                                                        Tout *__restrict__ blk) {
    int64_t base = (int64_t)blockIdx.x * kTile;
    Tout s = 0;
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        int64_t j = base + i;
        if (j < n) s += (Tout)in[j];
    }
    Tout tot;
    block_exclusive_scan<Tout>(s, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place; the grand total
// goes to *total (may be null).
template <class Tout, class Ttot>
__global__ __launch_bounds__(kThreads) void scan_top(Tout *__restrict__ blk, int64_t nb,
                                                     Ttot *__restrict__ total) {
    Tout carry = 0;
    for (int64_t c = 0; c < nb; c += kThreads) {
        int64_t j = c + threadIdx.x;
        Tout v = j < nb ? blk[j] : 0;
        Tout tot;
        Tout ex = block_exclusive_scan<Tout>(v, &tot);
        if (j < nb) blk[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = (Ttot)carry;
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kThreads) void scan_apply(const Tin *__restrict__ in, int64_t n,
                                                       const Tout *__restrict__ blk,
                                                       Tout *__restrict__ out) {
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kRounds;
    Tin v[kRounds];
    Tout s = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        int64_t j = base + r;
        v[r] = j < n ? in[j] : (Tin)0;
        s += (Tout)v[r];
    }
    Tout tot;
    Tout run = blk[blockIdx.x] + block_exclusive_scan<Tout>(s, &tot);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        int64_t j = base + r;
        if (j < n) out[j] = run;
        run += (Tout)v[r];
    }
}

template <class Tin, class Tout, class Ttot>
dgr_status exclusive_scan(const Tin *in, Tout *out, int64_t n, Tout *blk, Ttot *total,
                          hipStream_t st) {
    int64_t nb = std::max<int64_t>(1, (n + kTile - 1) / kTile);
    scan_reduce<Tin, Tout><<<dim3((unsigned)nb), dim3(kThreads), 0, st>>>(in, n, blk);
    DGR_LAUNCH_CHECK();
    scan_top<Tout, Ttot><<<dim3(1), dim3(kThreads), 0, st>>>(blk, nb, total);
    DGR_LAUNCH_CHECK();
    scan_apply<Tin, Tout><<<dim3((unsigned)nb), dim3(kThreads), 0, st>>>(in, n, blk, out);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

// ---- pair emission -----------------------------------------------------------
__global__ __launch_bounds__(kThreads) void emit_pairs(const GaussRec *__restrict__ rec,
                                                       const uint32_t *__restrict__ count,
                                                       const uint64_t *__restrict__ offset,
                                                       int64_t n, int64_t cap, int Tx, int Ty,
                                                       VoxHeader *__restrict__ hdr,
                                                       uint32_t *__restrict__ key,
                                                       uint32_t *__restrict__ val) {
    int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (hdr->total > (uint64_t)cap) {
        if (g == 0) hdr->overflow = 1u;
        return;
    }
    if (g >= n || count[g] == 0) return;
    const GaussRec &r = rec[g];
    uint64_t o = offset[g];
    const int x0 = box_lo(r.box[0]) >> 3, x1 = box_hi(r.box[0]) >> 3;
    const int y0 = box_lo(r.box[1]) >> 3, y1 = box_hi(r.box[1]) >> 3;
    const int z0 = box_lo(r.box[2]) >> 3, z1 = box_hi(r.box[2]) >> 3;
    for (int tz = z0; tz <= z1; ++tz)
        for (int ty = y0; ty <= y1; ++ty)
            for (int tx = x0; tx <= x1; ++tx) {
                key[o] = (uint32_t)((tz * Ty + ty) * Tx + tx);
                val[o] = (uint32_t)g;
                ++o;
            }
}

__device__ __forceinline__ uint64_t pair_count(const VoxHeader *hdr, int64_t cap) {
    uint64_t t = hdr->total;
    return t > (uint64_t)cap ? 0 : t;
}

// ---- stable LSD radix sort, 8-bit digits -----------------------------------------
__global__ __launch_bounds__(kThreads) void radix_hist(const uint32_t *__restrict__ keys,
                                                       const VoxHeader *__restrict__ hdr,
                                                       int64_t cap, int nblk, int shift,
                                                       uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t P = (int64_t)pair_count(hdr, cap);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        int64_t j = base + i;
        if (j < P) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// hist holds the exclusive scan of the digit-major histogram, i.e. the first
// output slot of (digit, block).  Within a block elements are placed in input
// order, so the sort is stable.
__global__ __launch_bounds__(kThreads) void radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, const VoxHeader *__restrict__ hdr,
    int64_t cap, int nblk, int shift, const uint32_t *__restrict__ hist) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    const int t = threadIdx.x, lane = lane_id(), w = wave_id();
    run[t] = hist[(int64_t)t * nblk + blockIdx.x];
    const int64_t P = (int64_t)pair_count(hdr, cap);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRounds; ++r) {
        for (int ww = 0; ww < kThreads / 64; ++ww) wcnt[ww][t] = 0;
        __syncthreads();
        const int64_t j = base + (int64_t)r * kThreads + t;
        const bool valid = j < P;
        uint32_t k = valid ? kin[j] : 0u;
        uint32_t v = valid ? vin[j] : 0u;
        uint32_t d = (k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t o = run[d] + rank;
            for (int ww = 0; ww < w; ++ww) o += wcnt[ww][d];
            kout[o] = k;
            vout[o] = v;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int ww = 0; ww < kThreads / 64; ++ww) add += wcnt[ww][t];
        run[t] += add;
        __syncthreads();
    }
}

// tile_begin[t] = first sorted pair with tile >= t, for t in [0, T].
__global__ __launch_bounds__(kThreads) void tile_ranges(const uint32_t *__restrict__ keys,
                                                        const VoxHeader *__restrict__ hdr,
                                                        int64_t cap, int64_t T,
                                                        uint32_t *__restrict__ tile_begin) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t P = (int64_t)pair_count(hdr, cap);
    if (i > P) return;
    const int64_t k = (i < P) ? (int64_t)keys[i] : T;
    const int64_t kp = (i == 0) ? -1 : (int64_t)keys[i - 1];
    for (int64_t t = kp + 1; t <= k; ++t) tile_begin[t] = (uint32_t)i;
}

__global__ void zero_total(VoxHeader *hdr) { hdr->total = 0; }

int key_bits(int64_t T) {
    int b = 0;
    while (b < 32 && (int64_t(1) << b) < T) ++b;
    return std::max(b, 1);
}

}  // namespace

int64_t scan_f64_blocks(int64_t n) { return std::max<int64_t>(1, (n + kTile - 1) / kTile) + 1; }

dgr_status exclusive_scan_f64(const float *in, double *out, int64_t n, double *blk, double *total,
                              hipStream_t st) {
    return exclusive_scan<float, double, double>(in, out, n, blk, total, st);
}

dgr_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *blk, uint32_t *total,
                              hipStream_t st) {
    return exclusive_scan<uint32_t, uint32_t, uint32_t>(in, out, n, blk, total, st);
}

VoxWs carve_vox_ws(void *ws, int64_t n, int64_t cap, const dgr_grid *grid) {
    VoxWs w{};
    Carver c(ws);
    const int64_t nn = std::max<int64_t>(n, 1);
    w.n = n;
    w.cap = cap;
    w.tiles = tiles_of(grid);
    w.radix_blocks = (int)std::max<int64_t>(1, (cap + kTile - 1) / kTile);
    w.hdr = c.take<VoxHeader>(1);
    w.rec = c.take<GaussRec>(nn);
    w.count = c.take<uint32_t>(nn);
    w.offset = c.take<uint64_t>(nn);
    int64_t scan_blocks = std::max<int64_t>((nn + kTile - 1) / kTile,
                                            ((int64_t)256 * w.radix_blocks + kTile - 1) / kTile);
    w.scan_blk = c.take<uint64_t>(scan_blocks + 1);
    w.tile_begin = c.take<uint32_t>(w.tiles + 1);
    w.hist = c.take<uint32_t>((int64_t)256 * w.radix_blocks);
    for (int i = 0; i < 2; ++i) {
        w.key[i] = c.take<uint32_t>(std::max<int64_t>(cap, 1));
        w.val[i] = c.take<uint32_t>(std::max<int64_t>(cap, 1));
    }
    w.bytes = c.off;
    return w;
}

int64_t vox_ws_capacity(size_t ws_bytes, int64_t n, const dgr_grid *grid) {
    if (carve_vox_ws(nullptr, n, 0, grid).bytes > ws_bytes) return -1;
    int64_t lo = 0, hi = (int64_t(1) << 31) - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (carve_vox_ws(nullptr, n, mid, grid).bytes <= ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

dgr_status enqueue_count_only(const float *mu, const float *scale, const float *quat, int64_t n,
                              const dgr_grid *grid, const dgr_trunc *trunc, VoxWs &w,
                              hipStream_t st) {
    dgr_status s = launch_prep(mu, scale, quat, nullptr, n, grid, trunc, nullptr, w.count,
                               nullptr, st);
    if (s != DGR_OK) return s;
    zero_total<<<1, 1, 0, st>>>(w.hdr);
    DGR_LAUNCH_CHECK();
    if (n == 0) return DGR_OK;
    return exclusive_scan<uint32_t, uint64_t, uint64_t>(w.count, w.offset, n, w.scan_blk, &w.hdr->total, st);
}

dgr_status enqueue_binning(const float *mu, const float *scale, const float *quat,
                           const float *density, int64_t n, const dgr_grid *grid,
                           const dgr_trunc *trunc, VoxWs &w, int *which, hipStream_t st) {
    dgr_status s;
    zero_total<<<1, 1, 0, st>>>(w.hdr);
    DGR_LAUNCH_CHECK();
    if (n > 0) {
        s = launch_prep(mu, scale, quat, density, n, grid, trunc, w.rec, w.count, nullptr, st);
        if (s != DGR_OK) return s;
        s = exclusive_scan<uint32_t, uint64_t, uint64_t>(w.count, w.offset, n, w.scan_blk, &w.hdr->total, st);
        if (s != DGR_OK) return s;
        const int Tx = (grid->dims[0] + 7) / 8, Ty = (grid->dims[1] + 7) / 8;
        emit_pairs<<<dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st>>>(
            w.rec, w.count, w.offset, n, w.cap, Tx, Ty, w.hdr, w.key[0], w.val[0]);
        DGR_LAUNCH_CHECK();
    }
    const int bits = key_bits(w.tiles);
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_hist<<<dim3(w.radix_blocks), dim3(kThreads), 0, st>>>(w.key[cur], w.hdr, w.cap,
                                                                   w.radix_blocks, shift, w.hist);
        DGR_LAUNCH_CHECK();
        s = exclusive_scan<uint32_t, uint32_t, uint32_t>(w.hist, w.hist, (int64_t)256 * w.radix_blocks,
                                                         reinterpret_cast<uint32_t *>(w.scan_blk),
                                                         (uint32_t *)nullptr, st);
        if (s != DGR_OK) return s;
        radix_scatter<<<dim3(w.radix_blocks), dim3(kThreads), 0, st>>>(
            w.key[cur], w.val[cur], w.key[cur ^ 1], w.val[cur ^ 1], w.hdr, w.cap, w.radix_blocks,
            shift, w.hist);
        DGR_LAUNCH_CHECK();
        cur ^= 1;
    }
    const int64_t nthreads = w.cap + 1;
    tile_ranges<<<dim3((unsigned)((nthreads + kThreads - 1) / kThreads)), dim3(kThreads), 0, st>>>(
        w.key[cur], w.hdr, w.cap, w.tiles, w.tile_begin);
    DGR_LAUNCH_CHECK();
    *which = cur;
    return DGR_OK;
}

}  // namespace dgr
