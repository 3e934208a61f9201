// Time-step control of a transient run (Sec. 3.3, eq. dt_spec): the largest
// temperature change over a step, reduced on the device, and the rule that
// turns it into the next step or a rejection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "te_internal.h"

namespace te {
namespace {

constexpr int kBlk = 256;
constexpr int kMaxBlocks = 1024;

// NaN-propagating maximum: a NaN anywhere makes the result NaN
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

// per workgroup: max |a - b| over a grid-stride share of the entries
__global__ void __launch_bounds__(kBlk) k_absdiff_max(const double *__restrict__ a, const double *__restrict__ b,
                                                      int64_t n, double *__restrict__ part) {
    __shared__ double s[kBlk / 64];
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlk + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlk)
        m = nanmax(m, fabs(a[i] - b[i]));
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = s[0];
        for (int w = 1; w < kBlk / 64; ++w) t = nanmax(t, s[w]);
        part[blockIdx.x] = t;
    }
}

int timestep_impl(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max, double eps,
                  double *dt_next, int32_t *accept, double *max_change, hipStream_t s) {
    TE_REQUIRE(dt_next && accept, TE_EINVAL, "NULL output");
    TE_REQUIRE(n >= 0 && (n == 0 || (T_new && T_old)), TE_EINVAL, "bad temperature arrays");
    TE_REQUIRE(dt > 0.0 && dT_max > 0.0 && eps > 0.0 && eps <= 1.0, TE_EINVAL,
               "need dt > 0, dT_max > 0 and 0 < eps <= 1");
    double dT = 0.0;
    if (n > 0) {
        const int nb = (int)std::min<int64_t>(kMaxBlocks, (n + kBlk - 1) / kBlk);
        DBuf<double> part(nb);
        hipLaunchKernelGGL(k_absdiff_max, dim3(nb), dim3(kBlk), 0, s, T_new, T_old, n, part.p);
        TE_CHECK_HIP(hipGetLastError());
        std::vector<double> h(nb);
        TE_CHECK_HIP(hipMemcpyAsync(h.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        for (double v : h) dT = (v > dT || std::isnan(v)) ? v : dT;
    }
    TE_REQUIRE(!std::isnan(dT), TE_ENAN, "NaN in a temperature field");
    if (max_change) *max_change = dT;
    if (dT > dT_max) {
        *accept = 0;
        *dt_next = 0.5 * dt;
    } else {
        *accept = 1;
        *dt_next = dT == 0.0 ? 2.0 * dt : eps * dT_max / dT * dt;
    }
    return TE_OK;
}

}  // namespace
}  // namespace te

extern "C" int te_timestep(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max, double eps,
                           double *dt_next, int32_t *accept, double *max_change, hipStream_t stream) {
    return te::guarded([&] { return te::timestep_impl(T_new, T_old, n, dt, dT_max, eps, dt_next, accept, max_change,
                                                      stream); });
}
