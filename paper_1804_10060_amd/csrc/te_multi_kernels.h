// Multi-mesh solve: many independent hierarchies advanced together, each
// phase of the CG iteration one persistent launch over a queue of
// (mesh, level, row-tile) work, one iteration captured in a HIP graph.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "te_dev.h"

namespace te {

// Waves per workgroup of the grouped sparse products: one, so a tile is one
// slice (lane-per-row items) or one row (one-wave-per-row items).
constexpr int GW = 1;
constexpr int GBLK = GW * WAVE;

template <typename T, class Epi>
struct GItem {
    SellView<T> sv;
    RowView<T> rv;
    const T *x;
    Epi epi;
    int32_t mesh;
    int32_t fmt;
};

template <int BR, int BC, typename T, class Epi>
__global__ void __launch_bounds__(GBLK) k_group(const GItem<T, Epi> *__restrict__ items,
                                                const int64_t *__restrict__ tile0, int nitems,
                                                const int32_t *__restrict__ active, double *__restrict__ partials) {
    __shared__ double lds[GW];
    __shared__ T wb[GBLK];
    const int64_t ntiles = tile0[nitems];
    const int64_t nb = gridDim.x, lb = xcd_logical_block(blockIdx.x, nb);
    const int64_t t_lo = ntiles * lb / nb, t_hi = ntiles * (lb + 1) / nb;
    const int lane = threadIdx.x & (WAVE - 1);
    int it = 0;
    {
        int lo = 0, hi = nitems;  // last item with tile0 <= t_lo
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tile0[mid] <= t_lo) lo = mid;
            else hi = mid;
        }
        it = lo;
    }
    for (int64_t t = t_lo; t < t_hi; ++t) {
        while (it + 1 < nitems && tile0[it + 1] <= t) ++it;
        const GItem<T, Epi> &G = items[it];
        const int64_t unit = (t - tile0[it]) * GW + threadIdx.x / WAVE;
        double red = 0.0;
        if (active == nullptr || active[G.mesh]) {
            if (G.fmt == FMT_SELL) {
                // the operator values are read once per product: non-temporal loads
                if (unit < G.sv.nslices) sell1_body<BR, BC, T, T, T, Epi, true>(G.sv, G.x, G.epi, unit, lane, red);
            } else {
                if (unit < G.rv.nrows)
                    roww_body<BR, BC, T, T, T, Epi>(G.rv, G.x, G.epi, unit, lane, red,
                                                    wb + (threadIdx.x / WAVE) * WAVE);
            }
        }
        if (Epi::kReduce) {
            double s = block_sum(red, lds);
            if (threadIdx.x == 0) partials[t] = s;
        }
    }
}

// Vector phases of the multi-mesh CG (float64, one item per mesh and level).
struct VItem {
    double *a;          // u (update), r (dots), p (p-update), d (jacobi)
    double *b;          // r (update)
    double *c;          // r_old (update/flexible dots) or null
    const double *x;    // p (update), z (dots, p-update), g (jacobi)
    const double *y;    // q (update), dinv (jacobi)
    double s;           // 1/theta (jacobi)
    int64_t n;
    int32_t mesh;
};
constexpr int VTILE = BLK * 4;
enum { VOP_UPDATE = 0, VOP_DOTRZ = 1, VOP_PUPDATE = 2, VOP_JACOBI = 3, VOP_DOTSELF = 4 };

template <int OP>
__global__ void __launch_bounds__(BLK) k_group_vec(const VItem *__restrict__ items, const int64_t *__restrict__ tile0,
                                                   int nitems, const int32_t *__restrict__ active,
                                                   const double *__restrict__ coef, double *__restrict__ partials) {
    __shared__ double lds[2 * WPB];
    const int64_t ntiles = tile0[nitems];
    const int64_t nb = gridDim.x, lb = xcd_logical_block(blockIdx.x, nb);
    const int64_t t_lo = ntiles * lb / nb, t_hi = ntiles * (lb + 1) / nb;
    int it = 0;
    {
        int lo = 0, hi = nitems;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tile0[mid] <= t_lo) lo = mid;
            else hi = mid;
        }
        it = lo;
    }
    for (int64_t t = t_lo; t < t_hi; ++t) {
        while (it + 1 < nitems && tile0[it + 1] <= t) ++it;
        const VItem &V = items[it];
        const bool on = active == nullptr || active[V.mesh];
        const int64_t base = (t - tile0[it]) * VTILE;
        const int64_t hi = min(V.n, base + VTILE);
        double r1 = 0.0, r2 = 0.0;
        if (on) {
            const double cf = coef ? coef[V.mesh] : 0.0;
            for (int64_t i = base + threadIdx.x; i < hi; i += BLK) {
                if (OP == VOP_UPDATE) {          // u += a p; r_old = r; r -= a q; |r|^2
                    V.a[i] += cf * V.x[i];
                    double rv = V.b[i];
                    if (V.c) V.c[i] = rv;
                    rv -= cf * V.y[i];
                    V.b[i] = rv;
                    r1 += rv * rv;
                } else if (OP == VOP_DOTRZ) {    // (r,z), (z, r - r_old)
                    const double rv = V.a[i], zv = V.x[i];
                    r1 += rv * zv;
                    if (V.c) r2 += zv * (rv - V.c[i]);
                } else if (OP == VOP_PUPDATE) {  // p = z + beta p
                    V.a[i] = V.x[i] + cf * V.a[i];
                } else if (OP == VOP_JACOBI) {   // d = D^-1 g / theta
                    V.a[i] = V.y[i] * V.x[i] * V.s;
                } else {                          // |x|^2
                    r1 += V.x[i] * V.x[i];
                }
            }
        }
        if (OP == VOP_UPDATE || OP == VOP_DOTSELF) {
            double s = block_sum(r1, lds);
            if (threadIdx.x == 0) partials[t] = s;
        } else if (OP == VOP_DOTRZ) {
            double s1 = block_sum(r1, lds);
            double s2 = block_sum(r2, lds + WPB);
            if (threadIdx.x == 0) {
                partials[2 * t] = s1;
                partials[2 * t + 1] = s2;
            }
        }
    }
}

// per-item sums of tile partials, out[mesh * nv + v]: one wave per (item, v),
// lane l adds tiles l, l+64, ... in order, then a fixed shuffle tree
__global__ void __launch_bounds__(WAVE) k_group_reduce(const double *__restrict__ partials,
                                                       const int64_t *__restrict__ tile0,
                                                       const int32_t *__restrict__ mesh_of, int nv,
                                                       double *__restrict__ out) {
    const int i = blockIdx.x, v = blockIdx.y, lane = threadIdx.x;
    double s = 0.0;
    for (int64_t t = tile0[i] + lane; t < tile0[i + 1]; t += WAVE) s += partials[t * nv + v];
    s = wave_sum(s);
    if (lane == 0) out[mesh_of[i] * nv + v] = s;
}

// dense coarse solves of several meshes: y = Ainv x, one wave per row
struct DItem {
    const double *Ainv;
    const double *x;
    double *y;
    int64_t n;
    int32_t mesh;
};
__global__ void __launch_bounds__(BLK) k_group_dense(const DItem *__restrict__ items, const int64_t *__restrict__ tile0,
                                                     int nitems, const int32_t *__restrict__ active) {
    const int64_t ntiles = tile0[nitems];
    const int64_t nb = gridDim.x, lb = xcd_logical_block(blockIdx.x, nb);
    const int64_t t_lo = ntiles * lb / nb, t_hi = ntiles * (lb + 1) / nb;
    const int lane = threadIdx.x & (WAVE - 1);
    int it = 0;
    for (int64_t t = t_lo; t < t_hi; ++t) {
        while (it + 1 < nitems && tile0[it + 1] <= t) ++it;
        const DItem &D = items[it];
        if (active && !active[D.mesh]) continue;
        const int64_t row = (t - tile0[it]) * WPB + threadIdx.x / WAVE;
        if (row >= D.n) continue;
        const double *a = D.Ainv + row * D.n;
        double s = 0.0;
        for (int64_t j = lane; j < D.n; j += WAVE) s += a[j] * D.x[j];
        s = wave_sum(s);
        if (lane == 0) D.y[row] = s;
    }
}

// ---- multi-mesh CG scalars (thread per mesh) -------------------------------
struct MultiScal {
    double *rz, *pq, *alpha, *beta, *rr, *bb, *tol2;
    int32_t *active, *cand, *flag, *iters;
};
__global__ void k_multi_alpha(MultiScal S, const double *__restrict__ pq, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double a = 0.0;
    if (S.active[m]) {
        const double v = pq[m];
        S.pq[m] = v;
        if (!(v > 0.0)) {
            S.flag[m] = (v != v) ? 3 : 1;
            S.active[m] = 0;
        } else {
            a = S.rz[m] / v;
        }
        S.iters[m] += 1;
    }
    S.alpha[m] = a;
}
// recurrence residual; converged meshes stop and wait for the host's true check
__global__ void k_multi_rr(MultiScal S, const double *__restrict__ rr, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n || !S.active[m]) return;
    const double v = rr[m];
    S.rr[m] = v;
    if (v != v) {
        S.flag[m] = 3;
        S.active[m] = 0;
    } else if (v <= S.tol2[m] * S.bb[m]) {
        S.active[m] = 0;
        S.cand[m] = 1;
    }
}
__global__ void k_multi_beta(MultiScal S, const int32_t *__restrict__ mask, const double *__restrict__ rzf, int n,
                             int flexible) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double b = 0.0;
    if (mask[m]) {
        const double rzn = rzf[2 * m], fl = rzf[2 * m + 1];
        if (!(rzn > 0.0)) {
            S.flag[m] = (rzn != rzn) ? 3 : 2;
        } else {
            b = flexible ? fl / S.rz[m] : rzn / S.rz[m];
            S.rz[m] = rzn;
        }
    }
    S.beta[m] = b;
}

// ---- launchers -------------------------------------------------------------
constexpr int GROUP_GRID = 2048;

// Workgroups of a kernel resident on the whole device at once (the grid of a
// persistent launch); queried once per kernel.
template <class K>
int64_t resident_groups(K kernel, int threads) {
    int dev = 0, ncu = 0, per_cu = 0;
    TE_CHECK_HIP(hipGetDevice(&dev));
    TE_CHECK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    TE_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
    return std::max<int64_t>(1, (int64_t)ncu * std::max(per_cu, 1));
}

template <int BR, int BC, class Epi>
void group_launch(const void *items, const int64_t *tile0, int nitems, int64_t ntiles, const int32_t *active,
                  double *partials, hipStream_t s, int gmult = 1) {
    if (nitems == 0 || ntiles == 0) return;
    static const int64_t cap = resident_groups(k_group<BR, BC, double, Epi>, GBLK);
    const unsigned g = (unsigned)std::min<int64_t>(ntiles, cap * gmult);
    hipLaunchKernelGGL((k_group<BR, BC, double, Epi>), dim3(g), dim3(GBLK), 0, s,
                       (const GItem<double, Epi> *)items, tile0, nitems, active, partials);
    TE_CHECK_HIP(hipGetLastError());
}

template <int OP>
void group_vec_launch(const VItem *items, const int64_t *tile0, int nitems, int64_t ntiles, const int32_t *active,
                      const double *coef, double *partials, hipStream_t s, int gmult = 1) {
    if (nitems == 0 || ntiles == 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(ntiles, (int64_t)GROUP_GRID * gmult);
    hipLaunchKernelGGL(k_group_vec<OP>, dim3(g), dim3(BLK), 0, s, items, tile0, nitems, active, coef, partials);
    TE_CHECK_HIP(hipGetLastError());
}

}  // namespace te
