// Adam update (sec. 5.1, Implementation Details: the optimiser), elementwise and
// bandwidth-bound: one read of param/grad/m/v and one write of param/m/v.  The
// updated parameter is clamped from below (a projected step: scales stay
// positive and densities non-negative, the paper's I in R+).
#include <cmath>

#include "internal.h"

namespace dgr {
namespace {

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t n, float lr, float b1, float b2, float eps,
                                                   float inv_c1, float inv_sqrt_c2, float lower) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] = fmaxf(p[i] - lr * (mi * inv_c1) / (sqrtf(vi) * inv_sqrt_c2 + eps), lower);
    }
}

}  // namespace
}  // namespace dgr

using namespace dgr;

extern "C" dgr_status dgr_adam(float *param, const float *grad, float *m, float *v, int64_t n,
                               float lr, float b1, float b2, float eps, int64_t step, float lower,
                               void *stream) {
    DGR_CHECK(n >= 0, "n must be >= 0");
    if (n == 0) return DGR_OK;
    DGR_CHECK(param && grad && m && v, "null pointer argument");
    DGR_CHECK(step >= 1, "step must be >= 1");
    DGR_CHECK(std::isfinite(lr) && b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f && eps >= 0.0f,
              "bad Adam hyper-parameters");
    DGR_CHECK(!std::isnan(lower), "lower bound is NaN (use -inf for none)");
    const double c1 = 1.0 - std::pow((double)b1, (double)step);
    const double c2 = 1.0 - std::pow((double)b2, (double)step);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    adam_kernel<<<dim3(blocks), dim3(256), 0, as_stream(stream)>>>(
        param, grad, m, v, n, lr, b1, b2, eps, (float)(1.0 / c1), (float)(1.0 / std::sqrt(c2)), lower);
    DGR_LAUNCH_CHECK();
    return DGR_OK;
}
