// Adaptive density control (Alg. 2): clone, split and prune Gaussians from
// their averaged position-gradient norms.
//
//   avg_g = acc_g / iters (acc_g: sum of ||dL/dmu_g|| since the last pass),
//   sigma_g = largest scale.
//   clone: avg >= tau and sigma <= theta, at most n_max - n of them, largest
//          avg first (ties: lower index); original and copy carry half the
//          density; the copy's Adam moments start at zero.
//   split: avg >= tau and sigma > theta, within the room left after cloning,
//          same rule; the original becomes two Gaussians at mu + R diag(s) z_k
//          (caller-supplied standard normals z_k), scales s / 2^(1/3), same
//          density and rotation, zero Adam moments.
//   prune: neither cloned nor split, and avg <= tau_prune (near-zero
//          gradient), density <= 0, or sigma > the size limit.
//   Output: old Gaussians in index order, each emitting 0, 1 or 2 entries.
// Decisions are taken in binary32 (avg by a correctly rounded division).
//
// Selection under the cap is a radix select on the binary32 bit patterns of
// avg (non-negative, so their order is the order of the values): one
// work-group bisects the 32 key bits for the k-th largest key T; keys above T
// are taken, and the first ties at T in index order fill the rest.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

constexpr int kT = 256;

struct DensifyCfg {
    int iters;
    float tau, tau_prune, theta, sigma_max;
    int64_t n_max;
};

// flags: bit 0 clone candidate, bit 1 split candidate, bit 2 prune unless chosen
__global__ __launch_bounds__(kT) void classify(const float *__restrict__ scale, const float *__restrict__ density,
                                               const float *__restrict__ acc, int64_t n, DensifyCfg c,
                                               uint32_t *__restrict__ key, uint32_t *__restrict__ flags,
                                               uint32_t *__restrict__ cand_clone, uint32_t *__restrict__ cand_split) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n) return;
    const float avg = (float)((double)acc[g] / (double)c.iters);
    const float sigma = fmaxf(fmaxf(scale[3 * g], scale[3 * g + 1]), scale[3 * g + 2]);
    const bool hot = avg >= c.tau;
    const bool cc = hot && sigma <= c.theta, cs = hot && sigma > c.theta;
    const bool pr = avg <= c.tau_prune || !(density[g] > 0.0f) || sigma > c.sigma_max;
    key[g] = __float_as_uint(fmaxf(avg, 0.0f));
    flags[g] = (cc ? 1u : 0u) | (cs ? 2u : 0u) | (pr ? 4u : 0u);
    cand_clone[g] = cc ? 1u : 0u;
    cand_split[g] = cs ? 1u : 0u;
}

// sel[0] = T, sel[1] = take-all flag, sel[2] = ties to take, sel[3] = k (number to choose)
// cand: candidate flags (non-zero = candidate); count = number of candidates;
// room = n_max - (n + extra[0]) where extra (may be null) is a device count.
__global__ __launch_bounds__(kT) void radix_select(const uint32_t *__restrict__ key, const uint32_t *__restrict__ cand,
                                                   int64_t n, const uint32_t *__restrict__ count, int64_t n_max,
                                                   int64_t n_now, const uint32_t *__restrict__ extra,
                                                   uint32_t *__restrict__ sel) {
    __shared__ uint32_t sh[kT];
    __shared__ uint32_t T_s;
    const int64_t free_slots = n_max - n_now - (extra ? (int64_t)*extra : 0);
    const int64_t room = free_slots > 0 ? free_slots : 0;
    const uint32_t C = *count;
    const uint32_t k = (uint32_t)(room < (int64_t)C ? room : (int64_t)C);
    if (C <= k) {
        if (threadIdx.x == 0) {
            sel[0] = 0u;
            sel[1] = 1u;
            sel[2] = 0u;
            sel[3] = k;
        }
        return;
    }
    if (threadIdx.x == 0) T_s = 0u;
    __syncthreads();
    // largest T with #{cand, key >= T} >= k; k == 0 selects nothing (T = max, no ties)
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t trial = T_s | (1u << bit);
        uint32_t cnt = 0;
        for (int64_t g = threadIdx.x; g < n; g += kT) cnt += (cand[g] && key[g] >= trial) ? 1u : 0u;
        sh[threadIdx.x] = cnt;
        __syncthreads();
        for (int o = kT / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0 && sh[0] >= k && k > 0) T_s = trial;
        __syncthreads();
    }
    const uint32_t T = T_s;
    uint32_t gt = 0;
    for (int64_t g = threadIdx.x; g < n; g += kT) gt += (cand[g] && key[g] > T) ? 1u : 0u;
    sh[threadIdx.x] = gt;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sel[0] = T;
        sel[1] = 0u;
        sel[2] = k == 0 ? 0u : k - sh[0];
        sel[3] = k;
    }
}

__global__ __launch_bounds__(kT) void tie_flags(const uint32_t *__restrict__ key, const uint32_t *__restrict__ cand,
                                                int64_t n, const uint32_t *__restrict__ sel, uint32_t *__restrict__ tie) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n) return;
    tie[g] = (!sel[1] && cand[g] && key[g] == sel[0]) ? 1u : 0u;
}

// chosen[g] = 1 if candidate g is selected
__global__ __launch_bounds__(kT) void choose(const uint32_t *__restrict__ key, const uint32_t *__restrict__ cand,
                                             int64_t n, const uint32_t *__restrict__ sel,
                                             const uint32_t *__restrict__ tie_rank, uint32_t *__restrict__ chosen) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n) return;
    bool c = false;
    if (cand[g]) {
        if (sel[1]) c = true;
        else if (sel[3] > 0) c = key[g] > sel[0] || (key[g] == sel[0] && tie_rank[g] < sel[2]);
    }
    chosen[g] = c ? 1u : 0u;
}

// emitted entries per old Gaussian
__global__ __launch_bounds__(kT) void emit_counts(const uint32_t *__restrict__ flags,
                                                  const uint32_t *__restrict__ clone_sel,
                                                  const uint32_t *__restrict__ split_sel, int64_t n,
                                                  uint32_t *__restrict__ cnt, uint32_t *__restrict__ pruned) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n) return;
    const bool cl = clone_sel[g], sp = split_sel[g];
    const bool pr = !cl && !sp && (flags[g] & 4u);
    cnt[g] = pr ? 0u : ((cl || sp) ? 2u : 1u);
    pruned[g] = pr ? 1u : 0u;
}

__device__ __forceinline__ void rot_of(const float *q, float R[9]) {
    const float n = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__global__ __launch_bounds__(kT) void emit(dgr_gaussians src, dgr_gaussians dst, int64_t n,
                                           const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ off,
                                           const uint32_t *__restrict__ clone_sel,
                                           const uint32_t *__restrict__ split_sel,
                                           const float *__restrict__ normals) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n || cnt[g] == 0) return;
    const int64_t o = off[g];
    if (split_sel[g]) {
        float R[9];
        rot_of(src.quat + 4 * g, R);
        const float inv = 0.79370052598409979f;  // 2^(-1/3)
        for (int k = 0; k < 2; ++k) {
            const int64_t d = o + k;
            const float *z = normals + (g * 2 + k) * 3;
            const float a0 = src.scale[3 * g] * z[0], a1 = src.scale[3 * g + 1] * z[1], a2 = src.scale[3 * g + 2] * z[2];
            for (int i = 0; i < 3; ++i) {
                dst.mu[3 * d + i] = src.mu[3 * g + i] + (R[3 * i] * a0 + R[3 * i + 1] * a1 + R[3 * i + 2] * a2);
                dst.scale[3 * d + i] = src.scale[3 * g + i] * inv;
                dst.m_mu[3 * d + i] = dst.v_mu[3 * d + i] = 0.0f;
                dst.m_scale[3 * d + i] = dst.v_scale[3 * d + i] = 0.0f;
            }
            for (int i = 0; i < 4; ++i) {
                dst.quat[4 * d + i] = src.quat[4 * g + i];
                dst.m_quat[4 * d + i] = dst.v_quat[4 * d + i] = 0.0f;
            }
            dst.density[d] = src.density[g];
            dst.m_density[d] = dst.v_density[d] = 0.0f;
        }
        return;
    }
    const bool cl = clone_sel[g];
    for (int k = 0; k < (cl ? 2 : 1); ++k) {
        const int64_t d = o + k;
        const bool fresh = k == 1;
        for (int i = 0; i < 3; ++i) {
            dst.mu[3 * d + i] = src.mu[3 * g + i];
            dst.scale[3 * d + i] = src.scale[3 * g + i];
            dst.m_mu[3 * d + i] = fresh ? 0.0f : src.m_mu[3 * g + i];
            dst.v_mu[3 * d + i] = fresh ? 0.0f : src.v_mu[3 * g + i];
            dst.m_scale[3 * d + i] = fresh ? 0.0f : src.m_scale[3 * g + i];
            dst.v_scale[3 * d + i] = fresh ? 0.0f : src.v_scale[3 * g + i];
        }
        for (int i = 0; i < 4; ++i) {
            dst.quat[4 * d + i] = src.quat[4 * g + i];
            dst.m_quat[4 * d + i] = fresh ? 0.0f : src.m_quat[4 * g + i];
            dst.v_quat[4 * d + i] = fresh ? 0.0f : src.v_quat[4 * g + i];
        }
        dst.density[d] = cl ? src.density[g] * 0.5f : src.density[g];
        dst.m_density[d] = fresh ? 0.0f : src.m_density[g];
        dst.v_density[d] = fresh ? 0.0f : src.v_density[g];
    }
}

__global__ __launch_bounds__(kT) void grad_norm_acc(const float *__restrict__ dmu, int64_t n, float *__restrict__ acc) {
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= n) return;
    const float a = dmu[3 * g], b = dmu[3 * g + 1], c = dmu[3 * g + 2];
    acc[g] += sqrtf(a * a + b * b + c * c);
}

unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kT - 1) / kT); }

struct DWs {
    uint32_t *key, *flags, *cand_c, *cand_s, *tie, *rank, *sel_c, *sel_s, *cnt, *off, *pruned, *blk;
    uint32_t *tot;   // [0] clone candidates, [1] split candidates, [2] ties, [3] chosen clones,
                     // [4] chosen splits, [5] new n, [6] pruned
    uint32_t *sel;   // [0..3] clone selection, [4..7] split selection
    size_t bytes;
};

DWs carve_densify(void *base, int64_t n) {
    DWs w;
    Carver c(base);
    const int64_t nn = std::max<int64_t>(n, 1);
    w.key = c.take<uint32_t>(nn);
    w.flags = c.take<uint32_t>(nn);
    w.cand_c = c.take<uint32_t>(nn);
    w.cand_s = c.take<uint32_t>(nn);
    w.tie = c.take<uint32_t>(nn);
    w.rank = c.take<uint32_t>(nn);
    w.sel_c = c.take<uint32_t>(nn);
    w.sel_s = c.take<uint32_t>(nn);
    w.cnt = c.take<uint32_t>(nn);
    w.off = c.take<uint32_t>(nn);
    w.pruned = c.take<uint32_t>(nn);
    w.blk = c.take<uint32_t>(scan_f64_blocks(nn));
    w.tot = c.take<uint32_t>(8);
    w.sel = c.take<uint32_t>(8);
    w.bytes = c.off;
    return w;
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" dgr_status dgr_accumulate_grad_norm(const float *dmu, int64_t n, float *acc, void *stream) {
    DGR_CHECK(n >= 0, "n must be >= 0");
    if (n == 0) return DGR_OK;
    DGR_CHECK(dmu && acc, "null pointer argument");
    grad_norm_acc<<<nblk(n), kT, 0, as_stream(stream)>>>(dmu, n, acc);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}

extern "C" size_t dgr_densify_workspace(int64_t n) {
    if (n < 0) return 0;
    return carve_densify(nullptr, n).bytes;
}

extern "C" dgr_status dgr_densify(const dgr_gaussians *src, int64_t n, const float *acc, const float *normals,
                                  const dgr_grid *grid, const dgr_densify_params *p, const dgr_gaussians *dst,
                                  int64_t *n_out, int64_t counts[3], void *ws, size_t ws_bytes, void *stream) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    DGR_CHECK(src && dst && p && n_out && counts && ws, "null pointer argument");
    DGR_CHECK(n >= 1 && n < (int64_t(1) << 31), "n out of range");
    DGR_CHECK(acc && normals, "null accumulator or normals");
    DGR_CHECK(p->n_max >= n && p->n_max < (int64_t(1) << 31), "n_max must be in [n, 2^31)");
    DGR_CHECK(p->iters >= 1, "iters must be >= 1");
    DGR_CHECK(std::isfinite(p->tau) && std::isfinite(p->tau_prune) && std::isfinite(p->theta) && p->size_vox > 0.0f,
              "bad densification thresholds");
    const float *sp[12] = {src->mu, src->scale, src->quat, src->density, src->m_mu, src->m_scale, src->m_quat,
                           src->m_density, src->v_mu, src->v_scale, src->v_quat, src->v_density};
    const float *dp[12] = {dst->mu, dst->scale, dst->quat, dst->density, dst->m_mu, dst->m_scale, dst->m_quat,
                           dst->m_density, dst->v_mu, dst->v_scale, dst->v_quat, dst->v_density};
    for (int i = 0; i < 12; ++i) DGR_CHECK(sp[i] && dp[i], "null parameter or moment array");
    if (ws_bytes < dgr_densify_workspace(n)) return fail(DGR_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = as_stream(stream);
    DWs w = carve_densify(ws, n);
    DensifyCfg c;
    c.iters = p->iters;
    c.tau = p->tau;
    c.tau_prune = p->tau_prune;
    c.theta = p->theta;
    const float min_inv = std::min(grid->inv_h[0], std::min(grid->inv_h[1], grid->inv_h[2]));
    c.sigma_max = (3.0f * p->size_vox) / min_inv;  // binary32, as the oracle
    c.n_max = p->n_max;
    classify<<<nblk(n), kT, 0, st>>>(src->scale, src->density, acc, n, c, w.key, w.flags, w.cand_c, w.cand_s);
    DGR_LAUNCH_CHECK();
    // clones
    {
        if ((s = exclusive_scan_u32(w.cand_c, w.rank, n, w.blk, w.tot + 0, st)) != DGR_OK) return s;
        radix_select<<<1, kT, 0, st>>>(w.key, w.cand_c, n, w.tot + 0, p->n_max, n, nullptr, w.sel);
        DGR_LAUNCH_CHECK();
        tie_flags<<<nblk(n), kT, 0, st>>>(w.key, w.cand_c, n, w.sel, w.tie);
        DGR_LAUNCH_CHECK();
        if ((s = exclusive_scan_u32(w.tie, w.rank, n, w.blk, w.tot + 2, st)) != DGR_OK) return s;
        choose<<<nblk(n), kT, 0, st>>>(w.key, w.cand_c, n, w.sel, w.rank, w.sel_c);
        DGR_LAUNCH_CHECK();
        if ((s = exclusive_scan_u32(w.sel_c, w.rank, n, w.blk, w.tot + 3, st)) != DGR_OK) return s;
        // splits, in the room left after the clones
        if ((s = exclusive_scan_u32(w.cand_s, w.rank, n, w.blk, w.tot + 1, st)) != DGR_OK) return s;
        radix_select<<<1, kT, 0, st>>>(w.key, w.cand_s, n, w.tot + 1, p->n_max, n, w.tot + 3, w.sel + 4);
        DGR_LAUNCH_CHECK();
        tie_flags<<<nblk(n), kT, 0, st>>>(w.key, w.cand_s, n, w.sel + 4, w.tie);
        DGR_LAUNCH_CHECK();
        if ((s = exclusive_scan_u32(w.tie, w.rank, n, w.blk, w.tot + 2, st)) != DGR_OK) return s;
        choose<<<nblk(n), kT, 0, st>>>(w.key, w.cand_s, n, w.sel + 4, w.rank, w.sel_s);
        DGR_LAUNCH_CHECK();
        if ((s = exclusive_scan_u32(w.sel_s, w.rank, n, w.blk, w.tot + 4, st)) != DGR_OK) return s;
    }
    emit_counts<<<nblk(n), kT, 0, st>>>(w.flags, w.sel_c, w.sel_s, n, w.cnt, w.pruned);
    DGR_LAUNCH_CHECK();
    if ((s = exclusive_scan_u32(w.cnt, w.off, n, w.blk, w.tot + 5, st)) != DGR_OK) return s;
    if ((s = exclusive_scan_u32(w.pruned, w.rank, n, w.blk, w.tot + 6, st)) != DGR_OK) return s;
    emit<<<nblk(n), kT, 0, st>>>(*src, *dst, n, w.cnt, w.off, w.sel_c, w.sel_s, normals);
    DGR_LAUNCH_CHECK();
    uint32_t h[8];
    DGR_TRY_HIP(hipMemcpyAsync(h, w.tot, sizeof(h), hipMemcpyDeviceToHost, st));
    DGR_TRY_HIP(hipStreamSynchronize(st));
    *n_out = (int64_t)h[5];
    counts[0] = h[3];
    counts[1] = h[4];
    counts[2] = h[6];
    return DGR_OK;
}
