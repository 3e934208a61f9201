// Device-side building blocks shared by the sparse kernels: launch shape,
// the XCD-contiguous block order, deterministic reductions, the two operator
// layouts (SELL-64 lane-per-row and one-wave-per-row) with their row bodies,
// and the fused epilogues.
#pragma once

#include <hip/hip_runtime.h>

#include "te_internal.h"

namespace te {

constexpr int WAVE = 64;
constexpr int BLK = 256;   // 4 waves per workgroup
constexpr int WPB = BLK / WAVE;

// Consecutive logical blocks on one XCD: dispatch is round-robin over the 8
// XCDs, so physical block b runs on XCD b % 8.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nb) {
    int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, WAVE);
    return v;
}

// Block-wide deterministic sum of one value per thread; result valid in
// thread 0.  lds must hold blockDim.x / 64 doubles (at most 16).
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) t += lds[i];
    __syncthreads();
    return t;
}

// value loads of the streamed operator: optionally non-temporal, so the
// single-use matrix stream does not displace the reused x vector in the caches
template <bool NT, typename T>
__device__ __forceinline__ T ld_val(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Stores of the epilogue outputs: non-temporal.  Measured on the 12M-DOF disc
// against plain stores: A p 1.652 -> 1.633 ms, pre-smoothing 1.738 -> 1.719,
// residual 1.599 -> 1.569, post-smoothing step 1.659 -> 1.637 (the
// single-RHS Chebyshev start keeps plain stores, see EpiChebInit); on the
// 64-column products of the 2M-DOF disc 1-3 % faster (Chebyshev start
// included).  The multi-RHS outputs of y = A x (EpiSet) stay plain.
template <typename T>
__device__ __forceinline__ void st_out(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// Sparse-product kernel skeletons
// ---------------------------------------------------------------------------
template <typename VT>
struct SellView {
    const int32_t *__restrict__ slice_off;
    const int32_t *__restrict__ col;
    const int32_t *__restrict__ rowlen;
    const VT *__restrict__ val;
    const int32_t *__restrict__ rowmap;  // nullptr => identity
    int64_t nrows;
    int64_t nslices;
};

template <typename VT>
inline SellView<VT> view(const Sell &S, const VT *val) {
    return SellView<VT>{S.slice_off.p, S.col.p, S.rowlen.p, val, S.rowmap.p, S.nrows, S.nslices};
}

// Single right-hand side: lane = block row.  Epi::apply(row_out, acc, red)
// consumes the BR accumulated entries and may add to `red` (block-reduced
// into partials[logical block] when Epi::kReduce).
// The BR*BC values of one lane's block at slot k (layout of sell_val_off):
// 16-byte loads for the groups, single loads for the remainder.
template <int BR, int BC, typename VT, bool NT>
__device__ __forceinline__ void sell1_block(const VT *__restrict__ vp, int k, int lane, VT *v) {
    constexpr int E = BR * BC, VW = sell_vw<VT>(), G = E / VW;
    typedef VT vec_t __attribute__((ext_vector_type(VW)));
    const VT *vk = vp + (int64_t)k * (E * WAVE);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const vec_t *q = reinterpret_cast<const vec_t *>(vk + (int64_t)(g * WAVE + lane) * VW);
        vec_t t;
        if constexpr (NT) t = __builtin_nontemporal_load(q);
        else t = *q;
#pragma unroll
        for (int u = 0; u < VW; ++u) v[g * VW + u] = t[u];
    }
#pragma unroll
    for (int e = G * VW; e < E; ++e) v[e] = ld_val<NT>(&vk[(int64_t)G * VW * WAVE + (e - G * VW) * WAVE + lane]);
}

template <int BR, int BC, typename VT, typename XT, typename AT, bool NT>
__device__ __forceinline__ void sell1_entry_c(int64_t c, const VT *__restrict__ vp, int k, int lane,
                                              const XT *__restrict__ x, AT *acc) {
    AT xv[BC];
#pragma unroll
    for (int j = 0; j < BC; ++j) xv[j] = AT(x[c * BC + j]);
    VT v[BR * BC];
    sell1_block<BR, BC, VT, NT>(vp, k, lane, v);
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) acc[i] += AT(v[i * BC + j]) * xv[j];
}

template <int BR, int BC, typename VT, typename XT, typename AT, bool NT>
__device__ __forceinline__ void sell1_entry(const int32_t *__restrict__ cp, const VT *__restrict__ vp, int k,
                                            int lane, const XT *__restrict__ x, AT *acc) {
    sell1_entry_c<BR, BC, VT, XT, AT, NT>(cp[(int64_t)k * WAVE], vp, k, lane, x, acc);
}

// One slice, lane = row.  Rows of a slice are sorted by descending length,
// so lane 63 holds the shortest: entries below that length are taken by all
// lanes without a mask, two at a time (loads of both issued together), and
// only the ragged tail is masked per lane.
template <int BR, int BC, typename VT, typename XT, typename AT, class Epi, bool NT = false>
__device__ __forceinline__ void sell1_body(const SellView<VT> &A, const XT *__restrict__ x, const Epi &epi,
                                           int64_t slice, int lane, double &red) {
    const int64_t row = slice * WAVE + lane;
    const int off = A.slice_off[slice];
    const int w = A.slice_off[slice + 1] - off;
    const int len = A.rowlen[row];
    const int kmin = __builtin_amdgcn_readlane(len, WAVE - 1);
    const bool real = row < A.nrows;
    const int64_t out = real ? (A.rowmap ? (int64_t)A.rowmap[row] : row) : 0;
    typename Epi::template Pre<BR> pre{};
    if (real) pre = epi.template load<BR>(out);
    AT acc[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) acc[i] = AT(0);
    const int32_t *cp = A.col + (int64_t)off * WAVE + lane;
    const VT *vp = A.val + (int64_t)off * (BR * BC * WAVE);
    int k = 0;
    for (; k + 1 < kmin; k += 2) {
        sell1_entry<BR, BC, VT, XT, AT, NT>(cp, vp, k, lane, x, acc);
        sell1_entry<BR, BC, VT, XT, AT, NT>(cp, vp, k + 1, lane, x, acc);
    }
    for (; k < w; ++k)
        if (k < len) sell1_entry<BR, BC, VT, XT, AT, NT>(cp, vp, k, lane, x, acc);
    if (real) epi.template apply<BR>(out, acc, red, pre);
}

// One wave per stored row (format 1).  Lane = (block slot, row of the block):
// with NB = 64 / BR slots, a wave consumes NB consecutive blocks per step,
// i.e. one contiguous run of NB*BR*BC values, each lane reading the BC
// contiguous values of one block row.  The partial sums go through the
// wave's 64-entry LDS buffer; lane q < BR adds the NB slots of row q in slot
// order and runs the epilogue for that entry.
template <typename VT>
struct RowView {
    const int64_t *__restrict__ rptr;
    const int32_t *__restrict__ col;
    const VT *__restrict__ val;
    const int32_t *__restrict__ rowmap;
    int64_t nrows;
    const int64_t *__restrict__ lptr;  // symmetric storage: blocks below the diagonal (else null)
    const int32_t *__restrict__ lcol;
    const int32_t *__restrict__ lidx;
};

template <typename VT>
inline RowView<VT> rview(const Sell &S, const VT *val) {
    return RowView<VT>{S.rptr.p, S.col.p, val, S.rowmap.p, S.nrows, S.lptr.p, S.lcol.p, S.lidx.p};
}

// LDS written by some lanes of a wave and read by others: order the two
// inside the wave (no workgroup barrier; waves of a group are independent)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entries per batch of the row-wave product: a slot's U entries are loaded
// together (values and x), the columns of the next batch one batch ahead.
// Two entries per batch measured 2 % faster in the restriction (6x3
// blocks); for 6x6 blocks two per batch measured 4 % slower than one.
template <int BC>
constexpr int roww_batch() {
    return BC <= 3 ? 2 : 1;
}

// Lane `src`'s value of v (cross-lane permute through the LDS crossbar; no
// memory access, no barrier).
__device__ __forceinline__ double lane_bperm(int src, double v) {
    const int a = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bperm(int src, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// XB (BC <= BR): the first BC lanes of a slot load one x entry each of the
// block column and pass them round by lane_bperm, instead of every lane
// loading all BC (the same values, so the same result bit for bit).
template <int BR, int BC, typename VT, typename XT, typename AT, class Epi, bool NT = false, bool XB = false>
__device__ __forceinline__ void roww_body(const RowView<VT> &A, const XT *__restrict__ x, const Epi &epi, int64_t row,
                                          int lane, double &red, AT *__restrict__ wbuf) {
    static_assert(!XB || BC <= BR, "x exchange needs BC <= BR");
    constexpr int NB = WAVE / BR, U = roww_batch<BC>();
    const int slot = lane / BR, i = lane % BR;
    AT acc = AT(0);
    if (slot < NB) {
        const int64_t hi = A.rptr[row + 1];
        const int64_t k0 = A.rptr[row] + slot;
        // an entry past the row reads the slot's first entry and is not added
        int64_t cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t ku = k0 + u * NB;
            cc[u] = ku < hi ? A.col[ku] : 0;
        }
        for (int64_t k = k0; k < hi; k += U * NB) {
            int64_t cn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t ku = k + (U + u) * NB;
                cn[u] = ku < hi ? A.col[ku] : 0;
            }
            VT vv[U][BC];
            XT xx[U][BC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t ku = k + u * NB;
                const VT *v = A.val + (ku < hi ? ku : k) * (BR * BC) + i * BC;
#pragma unroll
                for (int j = 0; j < BC; ++j) vv[u][j] = ld_val<NT>(&v[j]);
                if constexpr (XB) {
                    const XT xi = i < BC ? x[cc[u] * BC + i] : XT(0);
#pragma unroll
                    for (int j = 0; j < BC; ++j) xx[u][j] = lane_bperm(slot * BR + j, xi);
                } else {
#pragma unroll
                    for (int j = 0; j < BC; ++j) xx[u][j] = x[cc[u] * BC + j];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k + u * NB < hi)
#pragma unroll
                    for (int j = 0; j < BC; ++j) acc += AT(vv[u][j]) * AT(xx[u][j]);
#pragma unroll
            for (int u = 0; u < U; ++u) cc[u] = cn[u];
        }
        if constexpr (BR == BC) {
            if (A.lptr) {
                // row i of a block below the diagonal = column i of its stored
                // mirror; the (column, mirror) pairs of the next batch are
                // loaded one batch ahead
                const int64_t lhi = A.lptr[row + 1];
                const int64_t q0 = A.lptr[row] + slot;
                int64_t lc[U], li[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t qu = q0 + u * NB;
                    lc[u] = qu < lhi ? A.lcol[qu] : 0;
                    li[u] = qu < lhi ? A.lidx[qu] : 0;
                }
                for (int64_t q = q0; q < lhi; q += U * NB) {
                    int64_t nc[U], ni[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t qu = q + (U + u) * NB;
                        nc[u] = qu < lhi ? A.lcol[qu] : 0;
                        ni[u] = qu < lhi ? A.lidx[qu] : 0;
                    }
                    VT vv[U][BC];
                    XT xx[U][BC];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const VT *v = A.val + li[u] * (BR * BC) + i;
#pragma unroll
                        for (int j = 0; j < BC; ++j) vv[u][j] = v[j * BC];
                        if constexpr (XB) {
                            const XT xi = i < BC ? x[lc[u] * BC + i] : XT(0);
#pragma unroll
                            for (int j = 0; j < BC; ++j) xx[u][j] = lane_bperm(slot * BR + j, xi);
                        } else {
#pragma unroll
                            for (int j = 0; j < BC; ++j) xx[u][j] = x[lc[u] * BC + j];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (q + u * NB < lhi)
#pragma unroll
                            for (int j = 0; j < BC; ++j) acc += AT(vv[u][j]) * AT(xx[u][j]);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        lc[u] = nc[u];
                        li[u] = ni[u];
                    }
                }
            }
        }
    }
    wbuf[lane] = acc;
    wave_lds_sync();
    if (lane < BR) {
        AT t[1] = {AT(0)};
#pragma unroll
        for (int sl = 0; sl < NB; ++sl) t[0] += wbuf[sl * BR + lane];
        const int64_t out = A.rowmap ? (int64_t)A.rowmap[row] : row;
        epi.template apply<1>(out * BR + lane, t, red);
    }
    wave_lds_sync();  // the next row's writes after these reads
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
// Each epilogue reads its per-row vector inputs with load<BR>(row) and
// finishes the row with apply<BR>(row, acc, red, pre).  The lane-per-row
// product issues load before its entry loop, so those reads are in flight
// while the operator streams instead of after it; apply(row, acc, red) does
// both at the end.  Inputs that are only streamed are read non-temporally.
template <typename T>
struct EpiSet {  // y = A x
    static constexpr bool kReduce = false;
    T *y;
    template <int BR>
    struct Pre {};
    template <int BR>
    __device__ Pre<BR> load(int64_t) const {
        return {};
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &, const Pre<BR> &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) y[r * BR + i] = T(acc[i]);
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red) const {
        apply<BR>(r, acc, red, load<BR>(r));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t r, int j, int m, AT *acc, double &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) y[(r * BR + i) * m + j] = T(acc[i]);
    }
};

template <typename T>
struct EpiAdd {  // y += A x
    static constexpr bool kReduce = false;
    T *y;
    // y is read after the entry loop: reading it early measured slower in the
    // prolongation (3x6 blocks)
    template <int BR>
    struct Pre {};
    template <int BR>
    __device__ Pre<BR> load(int64_t) const {
        return {};
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &, const Pre<BR> &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) y[r * BR + i] = T(AT(y[r * BR + i]) + acc[i]);
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red) const {
        apply<BR>(r, acc, red, load<BR>(r));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t r, int j, int m, AT *acc, double &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = (r * BR + i) * m + j;
            st_out(&y[q], T(AT(y[q]) + acc[i]));
        }
    }
};

template <typename T, bool NORM>
struct EpiResid {  // y = g - A x  (optionally red += y^2)
    static constexpr bool kReduce = NORM;
    const T *g;
    T *y;
    template <int BR>
    struct Pre {
        T g[BR];
    };
    template <int BR>
    __device__ Pre<BR> load(int64_t r) const {
        Pre<BR> p;
#pragma unroll
        for (int i = 0; i < BR; ++i) p.g[i] = ld_val<true>(&g[r * BR + i]);
        return p;
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red, const Pre<BR> &p) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            AT v = AT(p.g[i]) - acc[i];
            st_out(&y[r * BR + i], T(v));
            if (NORM) red += double(v) * double(v);
        }
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red) const {
        apply<BR>(r, acc, red, load<BR>(r));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t r, int j, int m, AT *acc, double &red) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = (r * BR + i) * m + j;
            AT v = AT(g[q]) - acc[i];
            st_out(&y[q], T(v));
            if (NORM) red += double(v) * double(v);
        }
    }
};

struct EpiDot {  // q = A p, red += p.q   (float64 outer CG)
    static constexpr bool kReduce = true;
    const double *p;
    double *q;
    template <int BR>
    struct Pre {
        double p[BR];
    };
    template <int BR>
    __device__ Pre<BR> load(int64_t r) const {
        Pre<BR> v;
#pragma unroll
        for (int i = 0; i < BR; ++i) v.p[i] = p[r * BR + i];
        return v;
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red, const Pre<BR> &v) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            st_out(&q[r * BR + i], double(acc[i]));
            red += v.p[i] * double(acc[i]);
        }
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t r, AT *acc, double &red) const {
        apply<BR>(r, acc, red, load<BR>(r));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t r, int j, int m, AT *acc, double &red) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t k = (r * BR + i) * m + j;
            st_out(&q[k], double(acc[i]));
            red += p[k] * double(acc[i]);
        }
    }
};

// Post-smoothing start: r = g - A x, d = D^-1 r / theta.
template <typename T>
struct EpiChebInit {
    static constexpr bool kReduce = false;
    const T *g;
    const T *dinv;
    T *r;
    T *d;
    T inv_theta;
    template <int BR>
    struct Pre {
        T g[BR], v[BR];
    };
    template <int BR>
    __device__ Pre<BR> load(int64_t row) const {
        Pre<BR> p;
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            p.g[i] = ld_val<true>(&g[row * BR + i]);
            p.v[i] = ld_val<true>(&dinv[row * BR + i]);
        }
        return p;
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t row, AT *acc, double &, const Pre<BR> &p) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = row * BR + i;
            T rv = T(AT(p.g[i]) - acc[i]);
            // plain stores here: with either output non-temporal this product
            // measured 1.836 instead of 1.770 ms on the 12M-DOF disc
            r[q] = rv;
            d[q] = p.v[i] * rv * inv_theta;
        }
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t row, AT *acc, double &red) const {
        apply<BR>(row, acc, red, load<BR>(row));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t row, int j, int m, AT *acc, double &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = (row * BR + i) * m + j;
            T rv = T(AT(g[q]) - acc[i]);
            st_out(&r[q], rv);
            st_out(&d[q], T(dinv[row * BR + i] * rv * inv_theta));
        }
    }
};

// One Chebyshev step on the product acc = A d:
//   r' = r - A d;  d' = c1 d + c2 D^-1 r';  x (+)= d  [+ d' on the last step]
// `d` is the gathered vector of the product (own row read here); d' goes to a
// different buffer.  XZERO: x starts from zero (pre-smoothing).
template <typename T, bool LAST, bool XZERO>
struct EpiChebStep {
    static constexpr bool kReduce = false;
    const T *rin;
    const T *d;
    const T *dinv;
    T *rout;
    T *dout;
    T *x;
    T c1, c2;
    template <int BR>
    struct Pre {
        T r[BR], d[BR], v[BR], x[BR];
    };
    template <int BR>
    __device__ Pre<BR> load(int64_t row) const {
        Pre<BR> p;
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            const int64_t q = row * BR + i;
            p.r[i] = ld_val<true>(&rin[q]);
            p.d[i] = d[q];
            p.v[i] = ld_val<true>(&dinv[q]);
            p.x[i] = XZERO ? T(0) : ld_val<true>(&x[q]);
        }
        return p;
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t row, AT *acc, double &, const Pre<BR> &p) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = row * BR + i;
            T rn = T(AT(p.r[i]) - acc[i]);
            T dv = p.d[i];
            T dn = c1 * dv + c2 * (p.v[i] * rn);
            T xv = p.x[i];
            if (LAST) {
                st_out(&x[q], T(xv + dv + dn));
            } else {
                st_out(&rout[q], rn);
                st_out(&dout[q], dn);
                st_out(&x[q], T(xv + dv));
            }
        }
    }
    template <int BR, typename AT>
    __device__ void apply(int64_t row, AT *acc, double &red) const {
        apply<BR>(row, acc, red, load<BR>(row));
    }
    template <int BR, typename AT>
    __device__ void apply_m(int64_t row, int j, int m, AT *acc, double &) const {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            int64_t q = (row * BR + i) * m + j;
            T rn = T(AT(rin[q]) - acc[i]);
            T dv = d[q];
            T dn = c1 * dv + c2 * (dinv[row * BR + i] * rn);
            T xv = XZERO ? T(0) : x[q];
            if (LAST) {
                st_out(&x[q], T(xv + dv + dn));
            } else {
                st_out(&rout[q], rn);
                st_out(&dout[q], dn);
                st_out(&x[q], T(xv + dv));
            }
        }
    }
};

}  // namespace te
