// Time-step control of a transient run (Sec. 3.3, eq. dt_spec): the largest
// temperature change over a step, reduced on the device, and the rule that
// turns it into the next step or a rejection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
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

// ---- the same control without allocation --------------------------------
// Scratch of te_timestep_noalloc: the partial maxima of k_absdiff_max and the
// final maximum.  One copy per GPU, held until the process ends.  Host code
// never passes `scratch` itself to a kernel (on the host it only names the
// symbol); it uses the device address that hipGetSymbolAddress returns.
constexpr int kScratchDoubles = kMaxBlocks + 64;  // 1024 partials, result at [kMaxBlocks]
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of the current GPU's scratch, looked up once per device
double *scratch_on_current_device() {
    int dev = -1;
    TE_CHECK_HIP(hipGetDevice(&dev));
    TE_REQUIRE(dev >= 0 && dev < kMaxDevices, TE_EINVAL, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        TE_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        TE_REQUIRE(p != nullptr, TE_EHIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

// one workgroup: out = NaN-propagating max of part[0..nb)
__global__ void __launch_bounds__(kBlk) k_max_partials(const double *__restrict__ part, int nb,
                                                       double *__restrict__ out) {
    __shared__ double s[kBlk / 64];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlk) m = nanmax(m, part[i]);
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = s[0];
        for (int w = 1; w < kBlk / 64; ++w) t = nanmax(t, s[w]);
        *out = t;
    }
}

int timestep_noalloc_impl(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max,
                          double eps, double *dt_next, int32_t *accept, double *max_change, hipStream_t s) {
    TE_REQUIRE(dt_next && accept, TE_EINVAL, "NULL output");
    TE_REQUIRE(n >= 0 && (n == 0 || (T_new && T_old)), TE_EINVAL, "bad temperature arrays");
    TE_REQUIRE(dt > 0.0 && dT_max > 0.0 && eps > 0.0 && eps <= 1.0, TE_EINVAL,
               "need dt > 0, dT_max > 0 and 0 < eps <= 1");
    double *sc = scratch_on_current_device();
    double dT = 0.0;
    if (n > 0) {
        // the grid-stride reduction folds any n into at most kMaxBlocks partials
        const int nb = (int)std::min<int64_t>(kMaxBlocks, (n + kBlk - 1) / kBlk);
        TE_REQUIRE(nb >= 1 && nb <= kMaxBlocks && kMaxBlocks < kScratchDoubles, TE_EINVAL,
                   "%d partials exceed the scratch of %d", nb, kMaxBlocks);
        hipLaunchKernelGGL(k_absdiff_max, dim3(nb), dim3(kBlk), 0, s, T_new, T_old, n, sc);
        TE_CHECK_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(kBlk), 0, s, sc, nb, sc + kMaxBlocks);
        TE_CHECK_HIP(hipGetLastError());
        TE_CHECK_HIP(hipMemcpyAsync(&dT, sc + kMaxBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
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

extern "C" int te_timestep_noalloc(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max,
                                   double eps, double *dt_next, int32_t *accept, double *max_change,
                                   hipStream_t stream) {
    return te::guarded([&] {
        return te::timestep_noalloc_impl(T_new, T_old, n, dt, dT_max, eps, dt_next, accept, max_change, stream);
    });
}

extern "C" int te_timestep(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max, double eps,
                           double *dt_next, int32_t *accept, double *max_change, hipStream_t stream) {
    return te::guarded([&] { return te::timestep_impl(T_new, T_old, n, dt, dT_max, eps, dt_next, accept, max_change,
                                                      stream); });
}
