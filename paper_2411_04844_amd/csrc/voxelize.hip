// Forward voxelization (sec. 4.2 Fast Volume Reconstruction, Alg. 1):
// V(p) = sum_g rho_g exp(-1/2 d^T Q_g d), d = p - mu_g, over the voxel centres
// p in each Gaussian's truncation box.
//
// One 256-thread work-group owns one 8^3 tile; each thread owns two voxels
// (z and z+4) and keeps their sums in registers.  The tile's Gaussians arrive
// as a gid-sorted list from the binning step; they are staged through LDS in
// chunks of 256, converted to tile-relative coordinates, and added in list
// order, so the result does not depend on scheduling.  The quadratic form uses
// the paper's split of the position into the floored anchor and its residual
// (Discretize and Align, sec. 4.1): d = (i - floor(u)) - (u - floor(u)), which
// keeps d accurate to ~1e-6 voxel in binary32 on large grids.
#include <algorithm>

#include "internal.h"

namespace dgr {
namespace {

struct alignas(16) TileRec {
    float ux, uy, uz, rho;
    float k00, k11, k22, k01;
    float k02, k12;
    int bx0, bx1, by0, by1, bz0, bz1;
};
static_assert(sizeof(TileRec) == 64, "tile record must be 64 bytes");

__global__ __launch_bounds__(256) void voxelize_tiles(const GaussRec *__restrict__ rec,
                                                      const uint32_t *__restrict__ gid,
                                                      const uint32_t *__restrict__ tile_begin,
                                                      const VoxHeader *__restrict__ hdr,
                                                      int64_t cap, DevGrid g, int Tx, int Ty,
                                                      float *__restrict__ V) {
    __shared__ TileRec S[256];
    const int64_t tile = blockIdx.x;
    const int tx = (int)(tile % Tx), ty = (int)((tile / Tx) % Ty), tz = (int)(tile / ((int64_t)Tx * Ty));
    const int ox = tx * 8, oy = ty * 8, oz = tz * 8;
    const int t = threadIdx.x;
    const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const float fx = (float)lx, fy = (float)ly, fz0 = (float)lz, fz1 = (float)(lz + 4);
    const int64_t vx = ox + lx, vy = oy + ly, vz0 = oz + lz, vz1 = oz + lz + 4;
    const int64_t plane = (int64_t)g.nx * g.ny;
    const bool store_xy = vx < g.nx && vy < g.ny;

    if (hdr->total > (uint64_t)cap) {  // pair list incomplete: poison the tile
        const float nan = __builtin_nanf("");
        if (store_xy && vz0 < g.nz) V[vz0 * plane + vy * g.nx + vx] = nan;
        if (store_xy && vz1 < g.nz) V[vz1 * plane + vy * g.nx + vx] = nan;
        return;
    }
    const uint32_t beg = tile_begin[tile], end = tile_begin[tile + 1];
    float acc0 = 0.0f, acc1 = 0.0f;
    for (uint32_t c = beg; c < end; c += 256) {
        const int m = (int)min<uint32_t>(256u, end - c);
        if (t < m) {
            const GaussRec r = rec[gid[c + t]];
            TileRec s;
            s.ux = (float)(r.ui[0] - ox) + r.uf[0];
            s.uy = (float)(r.ui[1] - oy) + r.uf[1];
            s.uz = (float)(r.ui[2] - oz) + r.uf[2];
            s.rho = r.rho;
            s.k00 = r.k00; s.k11 = r.k11; s.k22 = r.k22;
            s.k01 = r.k01; s.k02 = r.k02; s.k12 = r.k12;
            s.bx0 = box_lo(r.box[0]) - ox; s.bx1 = box_hi(r.box[0]) - ox;
            s.by0 = box_lo(r.box[1]) - oy; s.by1 = box_hi(r.box[1]) - oy;
            s.bz0 = box_lo(r.box[2]) - oz; s.bz1 = box_hi(r.box[2]) - oz;
            S[t] = s;
        }
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            const TileRec &s = S[j];
            const bool inxy = lx >= s.bx0 && lx <= s.bx1 && ly >= s.by0 && ly <= s.by1;
            const bool in0 = inxy && lz >= s.bz0 && lz <= s.bz1;
            const bool in1 = inxy && lz + 4 >= s.bz0 && lz + 4 <= s.bz1;
            if (in0 || in1) {
                const float dx = fx - s.ux, dy = fy - s.uy;
                const float exy = dx * (s.k00 * dx + s.k01 * dy) + s.k11 * dy * dy;
                const float lin = s.k02 * dx + s.k12 * dy;
                const float dz0 = fz0 - s.uz, dz1 = fz1 - s.uz;
                const float e0 = exy + dz0 * (lin + s.k22 * dz0);
                const float e1 = exy + dz1 * (lin + s.k22 * dz1);
                if (in0) acc0 += s.rho * __builtin_amdgcn_exp2f(e0);
                if (in1) acc1 += s.rho * __builtin_amdgcn_exp2f(e1);
            }
        }
        __syncthreads();
    }
    if (store_xy && vz0 < g.nz) V[vz0 * plane + vy * g.nx + vx] = acc0;
    if (store_xy && vz1 < g.nz) V[vz1 * plane + vy * g.nx + vx] = acc1;
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
    voxelize_tiles<<<dim3((unsigned)w.tiles), dim3(256), 0, st>>>(
        w.rec, w.val[which], w.tile_begin, w.hdr, w.cap, dev_grid(grid), Tx, Ty, volume);
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
