// Backward of the voxelization: gradient of a loss with respect to each
// Gaussian's mean, scale, rotation quaternion and density, given dL/dV.
//
// The paper differentiates through the aligned evaluation of each Gaussian on
// its floored box (sec. 4.1, Discretize and Align: gradients reach mu through
// the residual).  Written out, with w = dL/dV, d = p - mu and G the truncated
// Gaussian:
//   M0 = sum w G,  m1 = sum w G d,  M2 = sum w G d d^T   (over the box)
//   drho = M0,  dmu = rho Q m1,  dQ = -rho/2 M2,
//   Q = R diag(s^-2) R^T:  ds_j = -2 s_j^-3 (R^T dQ R)_jj,  dR = 2 dQ R diag(s^-2),
//   dq = (I - q_hat q_hat^T) (dR : dR/dq_hat) / |q|.
// One wavefront owns one Gaussian: its lanes stride the box (x fastest, so
// reads of dL/dV are row-coalesced), accumulate the ten moments in registers
// and reduce them across the wavefront (DPP); lane 0 stores them in the
// Gaussian's record slot.  A second kernel applies the chain rule in binary64
// with one thread per Gaussian, so the serial binary64 work no longer holds a
// whole wavefront.  No atomics; the result is deterministic.
#include <mutex>

#include "internal.h"

namespace dgr {
namespace {

// Sum over the 64 lanes of a wave (all lanes active), wave-uniform: DPP
// exchanges within each row of 16 lanes (lane ^ 1, lane ^ 2, then the mirrored
// lane of the half row and of the row), then the four row sums through
// readlane.  No LDS traffic, unlike a shuffle.
__device__ __forceinline__ float row_xchg(float v, int c) {
    const int b = __float_as_int(v);
    switch (c) {  // the control must be a constant
        case 0: return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
        case 1: return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
        case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x141, 0xF, 0xF, false));  // row_half_mirror
        default: return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x140, 0xF, 0xF, false)); // row_mirror
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v += row_xchg(v, c);
    const int b = __float_as_int(v);
    return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) + __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
           (__int_as_float(__builtin_amdgcn_readlane(b, 32)) + __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

// The ten moments of one Gaussian and its density (44 bytes, inside the
// 64-byte slot of its record).
struct GaussMoments {
    float m[10];  // M0, m1 (x, y, z), M2 (xx, yy, zz, xy, xz, yz), voxel units
    float rho;
};
static_assert(sizeof(GaussMoments) <= sizeof(GaussRec), "moments must fit the record slot");

__global__ __launch_bounds__(256) void voxelize_grad(GaussRec *__restrict__ rec, int64_t n,
                                                     const float *__restrict__ dV, DevGrid g) {
    const int64_t gi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (gi >= n) return;
    const GaussRec r = rec[gi];
    const int x0 = box_lo(r.box[0]), x1 = box_hi(r.box[0]);
    const int y0 = box_lo(r.box[1]), y1 = box_hi(r.box[1]);
    const int z0 = box_lo(r.box[2]), z1 = box_hi(r.box[2]);
    float M0 = 0.f, m1x = 0.f, m1y = 0.f, m1z = 0.f;
    float Mxx = 0.f, Myy = 0.f, Mzz = 0.f, Mxy = 0.f, Mxz = 0.f, Myz = 0.f;
    if (x0 <= x1 && y0 <= y1 && z0 <= z1) {
        const int bx = x1 - x0 + 1, by = y1 - y0 + 1, bz = z1 - z0 + 1;
        const int64_t N = (int64_t)bx * by * bz;
        // lane's first voxel and the (x, y, z) advance of a 64-voxel stride
        int x = lane % bx, y = (lane / bx) % by, z = lane / (bx * by);
        const int q = 64 / bx, sx = 64 % bx, sy = q % by, sz = q / by;
        // offsets from the floored anchor; residual subtracted in binary32
        const int ox = x0 - r.ui[0], oy = y0 - r.ui[1], oz = z0 - r.ui[2];
        const int64_t plane = (int64_t)g.nx * g.ny;
        for (int64_t i = lane; i < N; i += 64) {
            const float w = dV[(int64_t)(z0 + z) * plane + (int64_t)(y0 + y) * g.nx + (x0 + x)];
            const float dx = (float)(ox + x) - r.uf[0];
            const float dy = (float)(oy + y) - r.uf[1];
            const float dz = (float)(oz + z) - r.uf[2];
            const float e = dx * (r.k00 * dx + r.k01 * dy + r.k02 * dz) + dy * (r.k11 * dy + r.k12 * dz) +
                            r.k22 * dz * dz;
            const float wg = w * __builtin_amdgcn_exp2f(e);
            const float tx = wg * dx, ty = wg * dy, tz = wg * dz;
            M0 += wg;
            m1x += tx; m1y += ty; m1z += tz;
            Mxx = fmaf(tx, dx, Mxx); Myy = fmaf(ty, dy, Myy); Mzz = fmaf(tz, dz, Mzz);
            Mxy = fmaf(tx, dy, Mxy); Mxz = fmaf(tx, dz, Mxz); Myz = fmaf(ty, dz, Myz);
            x += sx; y += sy; z += sz;
            if (x >= bx) { x -= bx; ++y; }
            if (y >= by) { y -= by; ++z; }
        }
    }
    M0 = wave_sum(M0);
    m1x = wave_sum(m1x); m1y = wave_sum(m1y); m1z = wave_sum(m1z);
    Mxx = wave_sum(Mxx); Myy = wave_sum(Myy); Mzz = wave_sum(Mzz);
    Mxy = wave_sum(Mxy); Mxz = wave_sum(Mxz); Myz = wave_sum(Myz);
    // The ten moments replace the Gaussian's record, in its own 64-byte slot
    // (its wave has read it; no other wave reads that slot); chain_rule turns
    // them into gradients with one lane per Gaussian.
    if (lane == 0) {
        GaussMoments mo;
        mo.m[0] = M0; mo.m[1] = m1x; mo.m[2] = m1y; mo.m[3] = m1z;
        mo.m[4] = Mxx; mo.m[5] = Myy; mo.m[6] = Mzz; mo.m[7] = Mxy; mo.m[8] = Mxz; mo.m[9] = Myz;
        mo.rho = r.rho;
        *reinterpret_cast<GaussMoments *>(rec + gi) = mo;
    }
}

// Chain rule in binary64, world units, one thread per Gaussian, from the
// moments voxelize_grad left in the record slots.
__global__ __launch_bounds__(256) void chain_rule(const GaussRec *__restrict__ rec, int64_t n, DevGrid g,
                                                  const float *__restrict__ scale, const float *__restrict__ quat,
                                                  float *__restrict__ dmu, float *__restrict__ dscale,
                                                  float *__restrict__ dquat, float *__restrict__ ddensity) {
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gi >= n) return;
    const GaussMoments mo = *reinterpret_cast<const GaussMoments *>(rec + gi);
    const float M0 = mo.m[0], m1x = mo.m[1], m1y = mo.m[2], m1z = mo.m[3];
    const float Mxx = mo.m[4], Myy = mo.m[5], Mzz = mo.m[6], Mxy = mo.m[7], Mxz = mo.m[8], Myz = mo.m[9];
    const double ih[3] = {g.inv_h[0], g.inv_h[1], g.inv_h[2]};
    const double m1[3] = {m1x / ih[0], m1y / ih[1], m1z / ih[2]};
    double M2[3][3];
    M2[0][0] = Mxx / (ih[0] * ih[0]);
    M2[1][1] = Myy / (ih[1] * ih[1]);
    M2[2][2] = Mzz / (ih[2] * ih[2]);
    M2[0][1] = M2[1][0] = Mxy / (ih[0] * ih[1]);
    M2[0][2] = M2[2][0] = Mxz / (ih[0] * ih[2]);
    M2[1][2] = M2[2][1] = Myz / (ih[1] * ih[2]);
    const double s[3] = {scale[3 * gi], scale[3 * gi + 1], scale[3 * gi + 2]};
    double w = quat[4 * gi], x = quat[4 * gi + 1], y = quat[4 * gi + 2], z = quat[4 * gi + 3];
    const double qn = sqrt(w * w + x * x + y * y + z * z);
    double R[3][3];
    if (qn == 0.0) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) R[a][b] = (a == b) ? 1.0 : 0.0;
    } else {
        w /= qn; x /= qn; y /= qn; z /= qn;
        R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
        R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
        R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
    }
    double lam[3];
    for (int j = 0; j < 3; ++j) lam[j] = 1.0 / (s[j] * s[j]);
    double Q[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Q[a][b] = R[a][0] * R[b][0] * lam[0] + R[a][1] * R[b][1] * lam[1] + R[a][2] * R[b][2] * lam[2];
    const double rho = mo.rho;
    ddensity[gi] = M0;
    for (int a = 0; a < 3; ++a)
        dmu[3 * gi + a] = (float)(rho * (Q[a][0] * m1[0] + Q[a][1] * m1[1] + Q[a][2] * m1[2]));
    double dQ[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dQ[a][b] = -0.5 * rho * M2[a][b];
    double dQR[3][3];  // dQ R
    for (int a = 0; a < 3; ++a)
        for (int j = 0; j < 3; ++j) dQR[a][j] = dQ[a][0] * R[0][j] + dQ[a][1] * R[1][j] + dQ[a][2] * R[2][j];
    for (int j = 0; j < 3; ++j) {
        const double dl = R[0][j] * dQR[0][j] + R[1][j] * dQR[1][j] + R[2][j] * dQR[2][j];
        dscale[3 * gi + j] = (float)(dl * (-2.0 / (s[j] * s[j] * s[j])));
    }
    if (qn == 0.0) {
        for (int c = 0; c < 4; ++c) dquat[4 * gi + c] = 0.0f;
        return;
    }
    double dR[3][3];
    for (int a = 0; a < 3; ++a)
        for (int j = 0; j < 3; ++j) dR[a][j] = 2.0 * dQR[a][j] * lam[j];
    // dR : dR/dq_hat for q_hat = (w, x, y, z)
    double gw = 2 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    double gx = 2 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2 * x * dR[1][1] - w * dR[1][2] +
                     z * dR[2][0] + w * dR[2][1] - 2 * x * dR[2][2]);
    double gy = 2 * (-2 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                     w * dR[2][0] + z * dR[2][1] - 2 * y * dR[2][2]);
    double gz = 2 * (-2 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2 * z * dR[1][1] +
                     y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
    const double proj = w * gw + x * gx + y * gy + z * gz;
    dquat[4 * gi + 0] = (float)((gw - w * proj) / qn);
    dquat[4 * gi + 1] = (float)((gx - x * proj) / qn);
    dquat[4 * gi + 2] = (float)((gy - y * proj) / qn);
    dquat[4 * gi + 3] = (float)((gz - z * proj) / qn);
}

}  // namespace

// Fixed device array holding the per-Gaussian records of the allocation-free
// entry point.  Host code never passes its name to a kernel (in host code it
// names a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, and is kept in static_rec_ptr.
constexpr int64_t kStaticGaussians = int64_t(1) << 19;  // 524,288 records, 32 MiB
static __device__ __align__(256) GaussRec scratch[kStaticGaussians];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
GaussRec *g_static_rec[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
dgr_status static_rec_ptr(GaussRec **out) {
    int dev = -1;
    DGR_TRY_HIP(hipGetDevice(&dev));
    DGR_CHECK(dev >= 0 && dev < kMaxDevices, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_rec[dev] == nullptr) {
        void *p = nullptr;
        DGR_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        DGR_CHECK(p != nullptr, "no device address for the fixed record array");
        g_static_rec[dev] = static_cast<GaussRec *>(p);
    }
    *out = g_static_rec[dev];
    return DGR_OK;
}

dgr_status check_backward_args(const float *mu, const float *scale, const float *quat, const float *density,
                               int64_t n, const dgr_grid *grid, const dgr_trunc *trunc, const float *dvolume,
                               float *dmu, float *dscale, float *dquat, float *ddensity) {
    dgr_status s;
    if ((s = check_grid(grid)) != DGR_OK) return s;
    if ((s = check_trunc(trunc)) != DGR_OK) return s;
    DGR_CHECK(n >= 0 && n < (int64_t(1) << 31), "n = %lld out of range", (long long)n);
    if (n == 0) return DGR_OK;
    DGR_CHECK(mu && scale && quat && density && dvolume, "null input pointer");
    DGR_CHECK(dmu && dscale && dquat && ddensity, "null output pointer");
    return DGR_OK;
}

dgr_status launch_backward(const float *mu, const float *scale, const float *quat, const float *density,
                           int64_t n, const dgr_grid *grid, const dgr_trunc *trunc, const float *dvolume,
                           float *dmu, float *dscale, float *dquat, float *ddensity, GaussRec *rec,
                           hipStream_t st) {
    dgr_status s;
    if ((s = launch_prep(mu, scale, quat, density, n, grid, trunc, rec, nullptr, nullptr, st)) != DGR_OK)
        return s;
    voxelize_grad<<<dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st>>>(rec, n, dvolume, dev_grid(grid));
    DGR_LAUNCH_CHECK();
    chain_rule<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(rec, n, dev_grid(grid), scale, quat, dmu,
                                                                        dscale, dquat, ddensity);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" size_t dgr_voxelize_backward_workspace(int64_t n) {
    if (n < 0) return 0;
    return align_up(sizeof(GaussRec) * (size_t)(n > 0 ? n : 1));
}

extern "C" dgr_status dgr_voxelize_backward(const float *mu, const float *scale, const float *quat,
                                            const float *density, int64_t n, const dgr_grid *grid,
                                            const dgr_trunc *trunc, const float *dvolume, float *dmu,
                                            float *dscale, float *dquat, float *ddensity, void *ws,
                                            size_t ws_bytes, void *stream) {
    dgr_status s = check_backward_args(mu, scale, quat, density, n, grid, trunc, dvolume, dmu, dscale, dquat,
                                       ddensity);
    if (s != DGR_OK || n == 0) return s;
    DGR_CHECK(ws != nullptr, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(DGR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < dgr_voxelize_backward_workspace(n))
        return fail(DGR_ERR_WORKSPACE, "workspace holds %zu bytes, backward needs %zu", ws_bytes,
                    dgr_voxelize_backward_workspace(n));
    return launch_backward(mu, scale, quat, density, n, grid, trunc, dvolume, dmu, dscale, dquat, ddensity,
                           static_cast<GaussRec *>(ws), as_stream(stream));
}

extern "C" int64_t dgr_voxelize_backward_noalloc_max(void) { return kStaticGaussians; }

extern "C" dgr_status dgr_voxelize_backward_noalloc(const float *mu, const float *scale, const float *quat,
                                                    const float *density, int64_t n, const dgr_grid *grid,
                                                    const dgr_trunc *trunc, const float *dvolume, float *dmu,
                                                    float *dscale, float *dquat, float *ddensity,
                                                    void *stream) {
    dgr_status s = check_backward_args(mu, scale, quat, density, n, grid, trunc, dvolume, dmu, dscale, dquat,
                                       ddensity);
    if (s != DGR_OK || n == 0) return s;
    DGR_CHECK(n <= kStaticGaussians,
              "n = %lld exceeds the %lld Gaussians the allocation-free backward holds",
              (long long)n, (long long)kStaticGaussians);
    GaussRec *rec = nullptr;
    if ((s = static_rec_ptr(&rec)) != DGR_OK) return s;
    return launch_backward(mu, scale, quat, density, n, grid, trunc, dvolume, dmu, dscale, dquat, ddensity,
                           rec, as_stream(stream));
}
