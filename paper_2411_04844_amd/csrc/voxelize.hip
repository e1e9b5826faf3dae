// Forward voxelization (sec. 4.2 Fast Volume Reconstruction, Alg. 1):
// V(p) = sum_g rho_g exp(-1/2 d^T Q_g d), d = p - mu_g, over the voxel centres
// p in each Gaussian's truncation box.
//
// One wavefront owns one 8^3 tile (four per work-group); each lane owns one
// row of 8 voxels along x (lane = 8 z + y) and keeps their sums in registers.
// The tile's Gaussians arrive as a gid-sorted list from the binning step and
// are read wave-uniformly (through the scalar cache) and added in list order,
// so the result does not depend on scheduling.  Per Gaussian only the rows
// inside its box take part, and only the x range of the box within the tile
// is evaluated: the exponent along a row is a quadratic in dx,
// e = base(dy, dz) + dx (k00 dx + b(dy, dz)).  The quadratic form uses the
// paper's split of the position into the floored anchor and its residual
// (Discretize and Align, sec. 4.1): d = (i - floor(u)) - (u - floor(u)), which
// keeps d accurate to ~1e-6 voxel in binary32 on large grids.
#include <algorithm>

#include "internal.h"

namespace dgr {
namespace {

__global__ __launch_bounds__(256) void voxelize_tiles(const GaussRec *__restrict__ rec,
                                                      const uint32_t *__restrict__ gid,
                                                      const uint32_t *__restrict__ tile_begin,
                                                      const VoxHeader *__restrict__ hdr,
                                                      int64_t cap, int64_t tiles, DevGrid g, int Tx, int Ty,
                                                      float *__restrict__ V) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= tiles) return;  // whole wavefront
    const int lane = threadIdx.x & 63;
    const int tx = (int)(tile % Tx), ty = (int)((tile / Tx) % Ty), tz = (int)(tile / ((int64_t)Tx * Ty));
    const int ox = tx * 8, oy = ty * 8, oz = tz * 8;
    const int ly = lane & 7, lz = lane >> 3;
    const int vy = oy + ly, vz = oz + lz;
    const int64_t plane = (int64_t)g.nx * g.ny;
    const bool row_in = vy < g.ny && vz < g.nz;
    float *row = V + (int64_t)vz * plane + (int64_t)vy * g.nx + ox;
    const int nxr = min(8, g.nx - ox);  // voxels of the row inside the grid

    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (hdr->total > (uint64_t)cap) {  // pair list incomplete: poison the tile
        const float nan = __builtin_nanf("");
#pragma unroll
        for (int x = 0; x < 8; ++x) acc[x] = nan;
    } else {
        const uint32_t beg = tile_begin[tile], end = tile_begin[tile + 1];
        for (uint32_t c = beg; c < end; ++c) {
            const uint32_t gi = __builtin_amdgcn_readfirstlane(gid[c]);
            const GaussRec r = rec[gi];
            const int by0 = box_lo(r.box[1]), by1 = box_hi(r.box[1]);
            const int bz0 = box_lo(r.box[2]), bz1 = box_hi(r.box[2]);
            // x range of the box inside the tile (uniform over the wave)
            const int xa = max(box_lo(r.box[0]) - ox, 0), xb = min(box_hi(r.box[0]) - ox, 7);
            if (vy < by0 || vy > by1 || vz < bz0 || vz > bz1 || xa > xb) continue;
            const float dy = (float)(vy - r.ui[1]) - r.uf[1];
            const float dz = (float)(vz - r.ui[2]) - r.uf[2];
            const float base = dy * (r.k11 * dy + r.k12 * dz) + r.k22 * dz * dz;
            const float bl = r.k01 * dy + r.k02 * dz;
            const float dx0 = (float)(ox - r.ui[0]) - r.uf[0];
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                if (x >= xa && x <= xb) {  // uniform
                    const float dx = dx0 + (float)x;
                    acc[x] += r.rho * __builtin_amdgcn_exp2f(base + dx * (r.k00 * dx + bl));
                }
            }
        }
    }
    if (!row_in) return;
#pragma unroll
    for (int x = 0; x < 8; ++x)
        if (x < nxr) row[x] = acc[x];
}

dgr_status check_vox_args(const float *mu, const float *scale, const float *quat, int64_t n,
                          const dgr_grid *grid, const dgr_trunc *trunc, void *ws) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_trunc(trunc)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n = %lld out of range [0, 2^31)", (long long)n);
    DGR_CHECK(n == 0 || (mu && scale && quat), "null parameter pointer");
    DGR_CHECK(ws != nullptr, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    return DGR_OK;
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_voxelize_workspace(int64_t n, int64_t max_pairs, const dgr_grid *grid) {
    if (check_grid(grid) != DGR_OK || n < 0 || max_pairs < 0 || max_pairs >= (int64_t(1) << 31))
        return 0;
    return carve_vox_ws(nullptr, n, max_pairs, grid).bytes;
}

extern "C" dgr_status dgr_voxelize_plan(const float *mu, const float *scale, const float *quat,
                                        int64_t n, const dgr_grid *grid, const dgr_trunc *trunc,
                                        int64_t *n_pairs_host, void *ws, size_t ws_bytes,
                                        void *stream) {
    dgr_status s = check_vox_args(mu, scale, quat, n, grid, trunc, ws);
    if (s != DGR_OK) return s;
    DGR_CHECK(n_pairs_host != nullptr, "n_pairs_host is null");
    VoxWs w = carve_vox_ws(ws, n, 0, grid);
    if (w.bytes > ws_bytes)
        return fail(DGR_ERR_WORKSPACE, "workspace holds %zu bytes, plan needs %zu", ws_bytes, w.bytes);
    hipStream_t st = as_stream(stream);
    // Read any overflow left by an earlier voxelization before the count.
    VoxHeader before;
    DGR_TRY_HIP(hipMemcpyAsync(&before, w.hdr, sizeof(before), hipMemcpyDeviceToHost, st));
    if ((s = enqueue_count_only(mu, scale, quat, n, grid, trunc, w, st)) != DGR_OK) return s;
    uint64_t total = 0;
    DGR_TRY_HIP(hipMemcpyAsync(&total, &w.hdr->total, sizeof(total), hipMemcpyDeviceToHost, st));
    DGR_TRY_HIP(hipStreamSynchronize(st));
    *n_pairs_host = (int64_t)total;
    if (before.overflow) {
        uint32_t zero = 0;
        DGR_TRY_HIP(hipMemcpyAsync(&w.hdr->overflow, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
        DGR_TRY_HIP(hipStreamSynchronize(st));
        return fail(DGR_ERR_CAPACITY, "an earlier voxelization overflowed its pair capacity");
    }
    return DGR_OK;
}

extern "C" dgr_status dgr_voxelize(const float *mu, const float *scale, const float *quat,
                                   const float *density, int64_t n, const dgr_grid *grid,
                                   const dgr_trunc *trunc, float *volume, void *ws,
                                   size_t ws_bytes, void *stream) {
    dgr_status s = check_vox_args(mu, scale, quat, n, grid, trunc, ws);
    if (s != DGR_OK) return s;
    DGR_CHECK(volume != nullptr, "volume is null");
    DGR_CHECK(n == 0 || density != nullptr, "density is null");
    int64_t cap = vox_ws_capacity(ws_bytes, n, grid);
    if (cap < 0)
        return fail(DGR_ERR_WORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes,
                    carve_vox_ws(nullptr, n, 0, grid).bytes);
    VoxWs w = carve_vox_ws(ws, n, cap, grid);
    hipStream_t st = as_stream(stream);
    int which = 0;
    if ((s = enqueue_binning(mu, scale, quat, density, n, grid, trunc, w, &which, st)) != DGR_OK)
        return s;
    const int Tx = (grid->dims[0] + 7) / 8, Ty = (grid->dims[1] + 7) / 8;
    voxelize_tiles<<<dim3((unsigned)((w.tiles + 3) / 4)), dim3(256), 0, st>>>(
        w.rec, w.val[which], w.tile_begin, w.hdr, w.cap, w.tiles, dev_grid(grid), Tx, Ty, volume);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" dgr_status dgr_bin(const float *mu, const float *scale, const float *quat, int64_t n,
                              const dgr_grid *grid, const dgr_trunc *trunc, uint32_t *pairs,
                              uint32_t *tile_begin, void *ws, size_t ws_bytes, void *stream) {
    dgr_status s = check_vox_args(mu, scale, quat, n, grid, trunc, ws);
    if (s != DGR_OK) return s;
    DGR_CHECK(pairs && tile_begin, "null output pointer");
    int64_t cap = vox_ws_capacity(ws_bytes, n, grid);
    if (cap < 0) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    VoxWs w = carve_vox_ws(ws, n, cap, grid);
    hipStream_t st = as_stream(stream);
    int which = 0;
    // density is not needed for binning; the records' rho slot reads mu.
    if ((s = enqueue_binning(mu, scale, quat, mu, n, grid, trunc, w, &which, st)) != DGR_OK) return s;
    uint64_t total = 0;
    DGR_TRY_HIP(hipMemcpyAsync(&total, &w.hdr->total, sizeof(total), hipMemcpyDeviceToHost, st));
    DGR_TRY_HIP(hipStreamSynchronize(st));
    if (total > (uint64_t)cap)
        return fail(DGR_ERR_CAPACITY, "%llu pairs exceed the capacity %lld", (unsigned long long)total,
                    (long long)cap);
    if (total > 0) {
        DGR_TRY_HIP(hipMemcpy2DAsync(pairs, 2 * sizeof(uint32_t), w.key[which], sizeof(uint32_t),
                                     sizeof(uint32_t), total, hipMemcpyDeviceToDevice, st));
        DGR_TRY_HIP(hipMemcpy2DAsync(pairs + 1, 2 * sizeof(uint32_t), w.val[which],
                                     sizeof(uint32_t), sizeof(uint32_t), total,
                                     hipMemcpyDeviceToDevice, st));
    }
    DGR_TRY_HIP(hipMemcpyAsync(tile_begin, w.tile_begin, sizeof(uint32_t) * (w.tiles + 1),
                               hipMemcpyDeviceToDevice, st));
    return DGR_OK;
}
