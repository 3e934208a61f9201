// Device-side products of the smoothed-aggregation setup (Sec. 2.1.3):
// strength of connection, the smoothed prolongator P = (I - w D^-1 A) P_tent,
// the product A P, the transpose R = P^T and the Galerkin product R (A P),
// all on block compressed rows, and the packing of an operator into the
// solver layouts, the MIS-2 aggregation and the per-aggregate QR of the
// tentative prolongator.  Only the greedy aggregation (an option, sequential
// by definition) and the merge of a rank-deficient aggregate into a
// neighbour stay on the host.
//
// Sparse products take two passes.  Symbolic: one wave per output row puts
// the candidate columns into an open-addressing hash set in LDS, counts them,
// and (second call) writes them sorted by rank.  Numeric: one wave per output
// row maps column -> slot through the same kind of LDS table; lane e owns
// entry e of every output block, and the contributions are added in the order
// of A's row, then B's row.  Every output value is thus summed by one lane in
// a fixed order: the result does not depend on the launch or on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "te_amg.h"
#include "te_setup_gpu.h"

namespace te {

namespace {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

template <int TB>
__device__ __forceinline__ uint32_t hslot(int32_t c) {
    return ((uint32_t)c * 2654435761u) >> (32 - ilog2(TB));
}

// Insert c into the set (tab: TB slots, -1 = empty).  New keys are appended
// to lst.  Returns false when the table is full.
template <int TB>
__device__ __forceinline__ bool set_insert(int32_t *tab, int32_t *lst, int32_t *num, int32_t c) {
    uint32_t h = hslot<TB>(c);
    for (int probe = 0; probe < TB; ++probe) {
        const int32_t old = atomicCAS(&tab[h], -1, c);
        if (old == -1) {
            const int32_t at = atomicAdd(num, 1);
            if (at < TB) lst[at] = c;
            return true;
        }
        if (old == c) return true;
        h = (h + 1) & (TB - 1);
    }
    return false;
}

// flag bits: 1 row set overflowed the table, 2 pattern/count mismatch,
//            4 row longer than the numeric table, 8 column missing from the pattern
template <int TB, bool AGG>
__global__ void __launch_bounds__(64) k_sym(int64_t n, const int64_t *__restrict__ aptr,
                                            const int32_t *__restrict__ acol, const int64_t *__restrict__ bptr,
                                            const int32_t *__restrict__ bcol, const int32_t *__restrict__ agg,
                                            int32_t *__restrict__ cnt, const int64_t *__restrict__ cptr,
                                            int32_t *__restrict__ ccol, int32_t *__restrict__ flag) {
    __shared__ int32_t tab[TB];
    __shared__ int32_t lst[TB];
    __shared__ int32_t num;
    __shared__ int64_t s_b0[64];
    __shared__ int32_t s_pre[64];
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        for (int t = lane; t < TB; t += 64) tab[t] = -1;
        if (lane == 0) num = 0;
        __syncthreads();
        bool ok = true;
        if (AGG) {
            // columns of P's row i: the aggregates of the nodes of A's row i
            for (int64_t ka = aptr[i] + lane; ka < aptr[i + 1]; ka += 64) {
                const int32_t c = agg[acol[ka]];
                if (c >= 0) ok = set_insert<TB>(tab, lst, &num, c) && ok;
            }
        } else {
            // the B rows of (up to) 64 entries of A's row at a time, taken as
            // one concatenated list: their starts and the prefix sums of their
            // lengths in LDS, every lane one entry of the list
            const int64_t a1 = aptr[i + 1];
            for (int64_t kc = aptr[i]; kc < a1; kc += 64) {
                const int na = (int)((a1 - kc) < 64 ? (a1 - kc) : 64);
                int64_t b0 = 0;
                int len = 0;
                if (lane < na) {
                    const int32_t j = acol[kc + lane];
                    b0 = bptr[j];
                    len = (int)(bptr[j + 1] - b0);
                }
                int pre = len;   // inclusive prefix sum over the lanes
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(pre, o, 64);
                    if (lane >= o) pre += t;
                }
                const int total = __shfl(pre, 63, 64);
                s_b0[lane] = b0;
                s_pre[lane] = pre;
                __syncthreads();
                for (int f = lane; f < total; f += 64) {
                    int lo = 0, hi = na - 1;   // the entry whose list part holds f
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= f) lo = mid + 1;
                        else hi = mid;
                    }
                    const int start = lo > 0 ? s_pre[lo - 1] : 0;
                    ok = set_insert<TB>(tab, lst, &num, bcol[s_b0[lo] + (f - start)]) && ok;
                }
                __syncthreads();   // s_b0 / s_pre are refilled for the next entries
            }
        }
        if (!ok) atomicOr(flag, 1);
        __syncthreads();
        const int m = min(num, TB);
        if (cptr == nullptr) {
            if (lane == 0) cnt[i] = m;
        } else {
            const int64_t c0 = cptr[i];
            if (cptr[i + 1] - c0 != (int64_t)m) {
                if (lane == 0) atomicOr(flag, 2);
            } else {
                for (int x = lane; x < m; x += 64) {
                    const int32_t key = lst[x];
                    int r = 0;
                    for (int y = 0; y < m; ++y) r += lst[y] < key ? 1 : 0;
                    ccol[c0 + r] = key;
                }
            }
        }
        __syncthreads();
    }
}

// first position in the sorted columns col[0, m) that is >= c
__device__ __forceinline__ int lower_bound_col(const int32_t *__restrict__ col, int m, int64_t c) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Numeric pass.  For each block k_a of A's row, the lanes first look up the
// output slots of the whole B row k_a points to (lane l: entry l), then walk
// that B row in order, the slot passed by a lane shuffle.  LACC: the row's
// output blocks are accumulated in dynamic LDS (mcap blocks), else in place.
// UP (a product known to be symmetric): only the blocks on and above the
// diagonal are formed (contributions to columns left of the row are
// skipped); k_mirror_lower fills the others from them afterwards.
template <int BR, int BK, int BC, int TB, bool LACC, bool UP = false>
__global__ void __launch_bounds__(64) k_num(int64_t n, const int64_t *__restrict__ aptr,
                                            const int32_t *__restrict__ acol, const double *__restrict__ aval,
                                            const int64_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                                            const double *__restrict__ bval, const int64_t *__restrict__ cptr,
                                            const int32_t *__restrict__ ccol, double *__restrict__ cval,
                                            int32_t *__restrict__ flag, int mcap) {
    constexpr int BB = BR * BC;
    static_assert(BB <= 64, "output block larger than a wave");
    __shared__ int32_t key[TB];
    __shared__ int32_t slot[TB];
    __shared__ int64_t s_b0[64], s_b1[64];
    extern __shared__ double s_acc[];  // LACC: [mcap][BB]
    const int lane = threadIdx.x;
    const bool on = lane < BB;
    const int p = on ? lane / BC : 0, q = on ? lane % BC : 0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t cs = cptr[i];
        const int mf = (int)(cptr[i + 1] - cs);
        // UP: the row's slots are its columns >= i, a suffix of the sorted row
        const int u0 = UP ? lower_bound_col(ccol + cs, mf, i) : 0;
        const int64_t c0 = cs + u0;
        const int m = mf - u0;
        if (2 * m > TB || (LACC && m > mcap)) {  // uniform over the block
            if (lane == 0) atomicOr(flag, 4);
            continue;
        }
        for (int t = lane; t < TB; t += 64) key[t] = -1;
        __syncthreads();
        for (int x = lane; x < m; x += 64) {
            const int32_t c = ccol[c0 + x];
            uint32_t h = hslot<TB>(c);
            for (int probe = 0; probe < TB; ++probe) {
                if (atomicCAS(&key[h], -1, c) == -1) {
                    slot[h] = x;
                    break;
                }
                h = (h + 1) & (TB - 1);
            }
        }
        double *acc = LACC ? s_acc : cval + c0 * BB;
        for (int64_t t = lane; t < (int64_t)m * BB; t += 64) acc[t] = 0.0;
        __syncthreads();
        const int64_t a0 = aptr[i], a1 = aptr[i + 1];
        for (int64_t kc = a0; kc < a1; kc += 64) {
            // B-row bounds of the next (up to) 64 blocks of A's row, fetched by the lanes at once
            const int na = (int)((a1 - kc) < 64 ? (a1 - kc) : 64);
            if (lane < na) {
                const int32_t jj = acol[kc + lane];
                s_b0[lane] = bptr[jj];
                s_b1[lane] = bptr[jj + 1];
            }
            __syncthreads();
            for (int ua = 0; ua < na; ++ua) {
                const int64_t ka = kc + ua;
                double ar[BK];
                const double *a = aval + ka * (BR * BK) + p * BK;
#pragma unroll
                for (int r = 0; r < BK; ++r) ar[r] = on ? a[r] : 0.0;
                const int64_t b0 = s_b0[ua], b1 = s_b1[ua];
                for (int64_t kb0 = b0; kb0 < b1; kb0 += 64) {
                    const int nb = (int)((b1 - kb0) < 64 ? (b1 - kb0) : 64);
                    int my = -1;
                    if (lane < nb) {
                        const int32_t c = bcol[kb0 + lane];
                        if (UP && (int64_t)c < i) {
                            my = -2;   // left of the diagonal: not formed
                        } else {
                            uint32_t h = hslot<TB>(c);
                            int probe = 0;
                            while (probe < TB && key[h] != c) {
                                h = (h + 1) & (TB - 1);
                                ++probe;
                            }
                            my = probe < TB ? slot[h] : -1;
                        }
                    }
                    if (__any(lane < nb && my == -1)) {
                        if (lane == 0) atomicOr(flag, 8);
                        continue;
                    }
                    if constexpr (LACC && BB == 1) {
                        // scalar blocks: every lane updates its own entry's slot
                        // (the slots of one B row are distinct), each slot still
                        // receiving its updates in A-row order
                        if (lane < nb && my >= 0) {
                            const double t1 = __dmul_rn(aval[ka], bval[kb0 + lane]);
                            acc[my] = __dadd_rn(acc[my], t1);
                        }
                        continue;
                    } else if constexpr (LACC && 2 * BB <= 64) {
                        // G groups of BB lanes take G entries of the B row at once
                        // (distinct slots); per output element the products and
                        // the accumulation run in the same order as with one group
                        constexpr int G = 64 / BB, UG = (8 + G - 1) / G;
                        const int g = lane / BB, e = lane - (lane / BB) * BB;
                        const bool gon = g < G;
                        const int gp = gon ? e / BC : 0, gq = gon ? e % BC : 0;
                        double ag[BK];
                        const double *a2 = aval + ka * (BR * BK) + gp * BK;
#pragma unroll
                        for (int r = 0; r < BK; ++r) ag[r] = gon ? a2[r] : 0.0;
                        for (int ub = 0; ub < nb; ub += G * UG) {
                            int sl[UG];
                            double t[UG], old[UG];
                            bool ok[UG];
#pragma unroll
                            for (int uu = 0; uu < UG; ++uu) {
                                const int u = ub + uu * G + g;
                                const int uc = u < nb ? u : nb - 1;
                                sl[uu] = __shfl(my, uc);
                                ok[uu] = gon && u < nb && sl[uu] >= 0;
                                t[uu] = 0.0;
                                if (ok[uu]) {
                                    const double *b = bval + (kb0 + uc) * (BK * BC) + gq;
#pragma unroll
                                    for (int r = 0; r < BK; ++r) t[uu] += ag[r] * b[r * BC];
                                }
                            }
#pragma unroll
                            for (int uu = 0; uu < UG; ++uu)
                                if (ok[uu]) old[uu] = acc[sl[uu] * BB + e];
#pragma unroll
                            for (int uu = 0; uu < UG; ++uu)
                                if (ok[uu]) acc[sl[uu] * BB + e] = old[uu] + t[uu];
                        }
                        continue;
                    }
                    // the slots of one B row are distinct: batches of UB updates
                    // load their accumulators together, then store them
                    constexpr int UB = 8;
                    for (int ub = 0; ub < nb; ub += UB) {
                        int sl[UB];
                        double t[UB], old[UB];
#pragma unroll
                        for (int uu = 0; uu < UB; ++uu) {
                            const int u = ub + uu < nb ? ub + uu : nb - 1;
                            sl[uu] = __shfl(my, u);
                            t[uu] = 0.0;
                            if (on && ub + uu < nb && sl[uu] >= 0) {
                                const double *b = bval + (kb0 + u) * (BK * BC) + q;
#pragma unroll
                                for (int r = 0; r < BK; ++r) t[uu] += ar[r] * b[r * BC];
                            }
                        }
                        if (on) {
#pragma unroll
                            for (int uu = 0; uu < UB; ++uu)
                                if (ub + uu < nb && sl[uu] >= 0) old[uu] = acc[sl[uu] * BB + lane];
#pragma unroll
                            for (int uu = 0; uu < UB; ++uu)
                                if (ub + uu < nb && sl[uu] >= 0) acc[sl[uu] * BB + lane] = old[uu] + t[uu];
                        }
                    }
                }
            }
            __syncthreads();  // s_b0 / s_b1 are refilled for the next 64 blocks
        }
        __syncthreads();
        if (LACC)
            for (int64_t t = lane; t < (int64_t)m * BB; t += 64) cval[c0 * BB + t] = s_acc[t];
        __syncthreads();
    }
}

// ---- strength of connection and diagonal -----------------------------------------
__global__ void k_fro(int64_t nnzb, int bb, const double *__restrict__ val, double *__restrict__ fro) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnzb; k += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int e = 0; e < bb; ++e) {
            const double v = val[k * bb + e];
            acc = __dadd_rn(acc, __dmul_rn(v, v));
        }
        fro[k] = __dsqrt_rn(acc);
    }
}
__global__ void k_diag_fro(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ fro, double *__restrict__ dn) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] == i) d = fro[k];
        dn[i] = d;
    }
}
__global__ void k_strength(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ dn, double *__restrict__ s /* in: fro, out: strength */) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            s[k] = (j == i) ? 0.0 : __ddiv_rn(s[k], __dsqrt_rn(__dmul_rn(dn[i], dn[j])));
        }
}
__global__ void k_diag_points(int64_t n, int b, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                              const double *__restrict__ val, double *__restrict__ d) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int p = 0; p < b; ++p) d[i * b + p] = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] == i)
                for (int p = 0; p < b; ++p) d[i * b + p] = val[k * b * b + p * b + p];
    }
}

// ---- smoothed prolongator, numeric ---------------------------------------------------
// P_iJ = [agg i = J] Q_i - w D_i^-1 sum_{j in row i, agg j = J} A_ij Q_j   (BS x 6 blocks);
// one thread per row, terms in the order of A's row, the tentative part last
template <int BS>
__global__ void k_p_numeric(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const int32_t *__restrict__ agg,
                            const double *__restrict__ Q, const double *__restrict__ d, double omega,
                            const int64_t *__restrict__ pptr, const int32_t *__restrict__ pcol,
                            double *__restrict__ pval, int32_t *__restrict__ flag) {
    constexpr int K = 6;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = pptr[i], p1 = pptr[i + 1];
        for (int64_t e = p0 * BS * K; e < p1 * BS * K; ++e) pval[e] = 0.0;
        auto find = [&](int32_t a) -> int64_t {
            int64_t lo = p0, hi = p1;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (pcol[mid] < a) lo = mid + 1;
                else hi = mid;
            }
            return (lo < p1 && pcol[lo] == a) ? lo : -1;
        };
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            const int32_t a = agg[j];
            if (a < 0) continue;
            const int64_t at = find(a);
            if (at < 0) {
                atomicOr(flag, 8);
                continue;
            }
            double *o = pval + at * BS * K;
            const double *av = val + k * BS * BS;
            const double *qv = Q + (int64_t)j * BS * K;
            for (int pp = 0; pp < BS; ++pp) {
                const double f = omega / d[i * BS + pp];
                for (int r = 0; r < BS; ++r) {
                    const double ar = av[pp * BS + r];
                    if (ar == 0.0) continue;
                    for (int c = 0; c < K; ++c) o[pp * K + c] -= f * ar * qv[r * K + c];
                }
            }
        }
        const int32_t ai = agg[i];
        if (ai >= 0) {
            const int64_t at = find(ai);
            if (at < 0) {
                atomicOr(flag, 8);
                continue;
            }
            double *o = pval + at * BS * K;
            const double *qv = Q + i * BS * K;
            for (int e = 0; e < BS * K; ++e) o[e] += qv[e];
        }
    }
}

// The same with one wave per row: lane (p, c) owns entry (p, c) of every
// block of the row and accumulates in LDS, in the same order as above (A's row,
// then the rows of the block, the tentative part last).  Dynamic LDS: mcap
// blocks of BS x 6 values, then mcap column indices.
template <int BS>
__global__ void __launch_bounds__(64) k_p_wave(int64_t n, const int64_t *__restrict__ ptr,
                                               const int32_t *__restrict__ col, const double *__restrict__ val,
                                               const int32_t *__restrict__ agg, const double *__restrict__ Q,
                                               const double *__restrict__ d, double omega,
                                               const int64_t *__restrict__ pptr, const int32_t *__restrict__ pcol,
                                               double *__restrict__ pval, int32_t *__restrict__ flag, int mcap) {
    constexpr int K = 6, BB = BS * K;
    static_assert(BB <= 64, "block larger than a wave");
    extern __shared__ double s_dyn[];
    double *s_acc = s_dyn;
    int32_t *s_pc = reinterpret_cast<int32_t *>(s_dyn + (size_t)mcap * BB);
    const int lane = threadIdx.x;
    const bool on = lane < BB;
    const int p = on ? lane / K : 0, c = on ? lane % K : 0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t p0 = pptr[i];
        const int m = (int)(pptr[i + 1] - p0);
        if (m > mcap) {  // uniform; cannot happen with mcap = the longest row
            if (lane == 0) atomicOr(flag, 4);
            continue;
        }
        for (int t = lane; t < m * BB; t += 64) s_acc[t] = 0.0;
        for (int t = lane; t < m; t += 64) s_pc[t] = pcol[p0 + t];
        __syncthreads();
        auto find = [&](int32_t a) -> int {
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_pc[mid] < a) lo = mid + 1;
                else hi = mid;
            }
            return (lo < m && s_pc[lo] == a) ? lo : -1;
        };
        const double f = on ? omega / d[i * BS + p] : 0.0;
        // the row's entries 64 at a time: every lane looks up one entry's
        // column, aggregate and output slot at once; then the entries are
        // applied in order, the block values and Q rows of U entries loaded
        // before any of them is added (the updates of one slot keep their order)
        const int64_t k1 = ptr[i + 1];
        for (int64_t kc = ptr[i]; kc < k1; kc += 64) {
            const int cnt = (int)((k1 - kc) < 64 ? (k1 - kc) : 64);
            int jl = 0, atl = -1;
            if (lane < cnt) {
                jl = col[kc + lane];
                const int32_t a = agg[jl];
                if (a >= 0) {
                    atl = find(a);
                    if (atl < 0) {
                        atomicOr(flag, 8);
                        atl = -2;
                    }
                }
            }
            constexpr int U = 4;
            for (int u0 = 0; u0 < cnt; u0 += U) {
                double ar[U][BS], qr[U][BS];
                int at[U];
#pragma unroll
                for (int t = 0; t < U; ++t) {
                    const int u = u0 + t < cnt ? u0 + t : cnt - 1;
                    at[t] = u0 + t < cnt ? __shfl(atl, u) : -1;
                    const int32_t j = __shfl(jl, u);
                    const double *av = val + (kc + u) * BS * BS + p * BS;
                    const double *qv = Q + (int64_t)j * BS * K + c;
#pragma unroll
                    for (int r = 0; r < BS; ++r) {
                        ar[t][r] = on ? av[r] : 0.0;
                        qr[t][r] = on ? qv[r * K] : 0.0;
                    }
                }
#pragma unroll
                for (int t = 0; t < U; ++t) {
                    if (at[t] < 0 || !on) continue;
                    double o = s_acc[at[t] * BB + lane];
                    for (int r = 0; r < BS; ++r) {
                        if (ar[t][r] == 0.0) continue;
                        o -= f * ar[t][r] * qr[t][r];
                    }
                    s_acc[at[t] * BB + lane] = o;
                }
            }
        }
        const int32_t ai = agg[i];
        if (ai >= 0) {
            const int at = find(ai);
            if (at < 0) {
                if (lane == 0) atomicOr(flag, 8);
            } else if (on) {
                s_acc[at * BB + lane] += Q[i * BS * K + lane];
            }
        }
        __syncthreads();
        for (int t = lane; t < m * BB; t += 64) pval[p0 * BB + t] = s_acc[t];
        __syncthreads();
    }
}

// ---- transpose --------------------------------------------------------------------------
__global__ void k_t_count(int64_t nnzb, const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnzb; k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[k]], 1);
}
// every stored block k of A goes to a free place of its column's segment;
// the segments are then sorted by k, i.e. by row of A
__global__ void k_t_place(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const int64_t *__restrict__ tptr, int32_t *__restrict__ fill, int64_t *__restrict__ src,
                          int32_t *__restrict__ row) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t c = col[k];
            const int32_t at = atomicAdd(&fill[c], 1);
            src[tptr[c] + at] = k;
            row[k] = (int32_t)i;
        }
}
// Segment r of src (the blocks of column r, placed in arbitrary order) in
// ascending order: one wave per segment, each element's rank is the number of
// smaller elements (the values are distinct block indices).  Segments longer
// than TSEG are ranked from global memory.
constexpr int TSEG = 1024;
__global__ void __launch_bounds__(64) k_t_rank(int64_t n, const int64_t *__restrict__ tptr,
                                               const int64_t *__restrict__ src, int64_t *__restrict__ dst) {
    __shared__ int64_t sv[TSEG];
    const int lane = threadIdx.x;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const int64_t lo = tptr[r];
        const int L = (int)(tptr[r + 1] - lo);
        const bool in_lds = L <= TSEG;
        const int64_t *v = in_lds ? sv : src + lo;
        if (in_lds)
            for (int t = lane; t < L; t += 64) sv[t] = src[lo + t];
        __syncthreads();
        for (int t = lane; t < L; t += 64) {
            const int64_t x = v[t];
            int rank = 0;
            for (int y = 0; y < L; ++y) rank += v[y] < x ? 1 : 0;
            dst[lo + rank] = x;
        }
        __syncthreads();
    }
}
template <int BR, int BC>
__global__ void k_t_fill(int64_t tn, const int64_t *__restrict__ src, const int32_t *__restrict__ row,
                         const double *__restrict__ val, int32_t *__restrict__ tcol, double *__restrict__ tval) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tn; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = src[t];
        tcol[t] = row[k];
        for (int p = 0; p < BR; ++p)
            for (int q = 0; q < BC; ++q) tval[t * BR * BC + q * BR + p] = val[k * BR * BC + p * BC + q];
    }
}

// ---- packing into the solver layouts ----------------------------------------------------
// SELL-64: storage position r (slice r/64, lane r%64) holds row order[r]
// BB > 0: the block size fixed at compile time, so a block's loads are all
// issued before its stores; BB = 0 takes it from bb
template <int BB>
__global__ void k_pack_sell(int64_t nr, int bb_rt, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const int32_t *__restrict__ order,
                            const int32_t *__restrict__ colmap, const int32_t *__restrict__ slice_off,
                            int64_t nslices, int32_t *__restrict__ scol, double *__restrict__ sval,
                            float *__restrict__ sval32) {
    const int bb = BB > 0 ? BB : bb_rt;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nslices * 64;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = r / 64, l = r % 64;
        const int64_t o0 = slice_off[sl], w = slice_off[sl + 1] - o0;
        const bool real = r < nr;
        const int64_t o = real ? order[r] : 0;
        const int64_t s0 = real ? ptr[o] : 0;
        const int64_t len = real ? ptr[o + 1] - s0 : 0;
        int32_t last = 0;
        for (int64_t k = 0; k < w; ++k) {
            if (k < len) last = colmap[col[s0 + k]];
            scol[(o0 + k) * 64 + l] = last;
            const int64_t e0 = (o0 + k) * bb * 64;
            if constexpr (BB > 0) {
                double v[BB];
#pragma unroll
                for (int x = 0; x < BB; ++x) v[x] = k < len ? val[(s0 + k) * BB + x] : 0.0;
#pragma unroll
                for (int x = 0; x < BB; ++x) {
                    sval[e0 + sell_val_off<sell_vw<double>()>(x, BB, (int)l)] = v[x];
                    if (sval32) sval32[e0 + sell_val_off<sell_vw<float>()>(x, BB, (int)l)] = (float)v[x];
                }
            } else {
                for (int x = 0; x < bb; ++x) {
                    const double v = k < len ? val[(s0 + k) * bb + x] : 0.0;
                    sval[e0 + sell_val_off<sell_vw<double>()>(x, bb, (int)l)] = v;
                    if (sval32) sval32[e0 + sell_val_off<sell_vw<float>()>(x, bb, (int)l)] = (float)v;
                }
            }
        }
    }
}
// one wave per row: storage row r holds row order[r], blocks contiguous
__global__ void __launch_bounds__(64) k_pack_rows(int64_t nr, int bb, const int64_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const int32_t *__restrict__ order, const int32_t *__restrict__ colmap,
                                                  const int64_t *__restrict__ rptr, int32_t *__restrict__ rcol,
                                                  double *__restrict__ rval, float *__restrict__ rval32) {
    const int lane = threadIdx.x;
    for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
        const int64_t o = order[r];
        const int64_t s0 = ptr[o], len = ptr[o + 1] - s0, d0 = rptr[r];
        for (int64_t k = lane; k < len; k += 64) rcol[d0 + k] = colmap[col[s0 + k]];
        for (int64_t t = lane; t < len * bb; t += 64) {
            const double v = val[s0 * bb + t];
            rval[d0 * bb + t] = v;
            if (rval32) rval32[d0 * bb + t] = (float)v;
        }
    }
}

// symmetric storage: upper slot u takes block src[u] of the natural matrix
__global__ void k_pack_upper(int64_t nup, int bb, const int64_t *__restrict__ src, const double *__restrict__ val,
                             double *__restrict__ rval, float *__restrict__ rval32) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nup * bb; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / bb, x = t % bb;
        const double v = val[src[u] * bb + x];
        rval[t] = v;
        if (rval32) rval32[t] = (float)v;
    }
}

// ---- dense inverse of the coarsest operator ----------------------------------------------
// Symmetric sweep operator on pivot j (Goodnight 1979): with d = a_jj,
//   a_jj <- -1/d,  a_ij <- a_ij/d,  a_jk <- a_jk/d,  a_ik <- a_ik - a_ij a_jk/d  (i, k != j);
// after sweeping every pivot the matrix holds -A^-1.  On a symmetric positive
// definite matrix each pivot is a Schur complement entry, hence positive;
// a pivot <= 0 (or NaN) is reported.  Reads `in`, writes `out` (ping-pong).
__global__ void k_sweep(int n, int j, const double *__restrict__ in, double *__restrict__ out,
                        int32_t *__restrict__ bad) {
    const double d = in[(int64_t)j * n + j];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double ajk = in[(int64_t)j * n + k];
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        const int64_t t = (int64_t)i * n + k;
        double v;
        if (i == j && k == j) {
            v = -1.0 / d;
            if (!(d > 0.0)) *bad = 1;
        } else if (i == j || k == j) {
            v = in[t] / d;
        } else {
            v = in[t] - in[(int64_t)i * n + j] * ajk / d;
        }
        out[t] = v;
    }
}
__global__ void k_negate(int64_t nn, const double *__restrict__ in, double *__restrict__ out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = -in[t];
}

inline unsigned grid_for(int64_t n, int b = 256) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + b - 1) / b, 1 << 16));
}
inline unsigned wave_grid(int64_t rows) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 1 << 17)); }

int32_t read_flag(const DBuf<int32_t> &f, hipStream_t s) {
    int32_t h = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&h, f.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return h;
}

// counts -> row pointer (host scan); returns the largest count
int64_t counts_to_ptr(const DBuf<int32_t> &cnt, int64_t n, DBuf<int64_t> &ptr, int64_t &total, hipStream_t s) {
    std::vector<int32_t> h;
    download(h, cnt.p, (size_t)n, s);
    std::vector<int64_t> p(n + 1, 0);
    int64_t mx = 0;
    for (int64_t i = 0; i < n; ++i) {
        p[i + 1] = p[i] + h[i];
        mx = std::max<int64_t>(mx, h[i]);
    }
    total = p[n];
    upload(ptr, p, s);
    return mx;
}

// The blocks left of the diagonal of a symmetric product, from their mirrors
// formed by the numeric pass with UP: C_ij = C_ji^T, C_ji found by bisection
// in row j (columns ascending).  One wave per row; flag bit 16 if a mirror is
// missing (the pattern is not symmetric).
template <int BS>
__global__ void __launch_bounds__(64) k_mirror_lower(int64_t n, const int64_t *__restrict__ cptr,
                                                     const int32_t *__restrict__ ccol, double *__restrict__ cval,
                                                     int32_t *__restrict__ flag) {
    constexpr int BB = BS * BS;
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t c0 = cptr[i];
        const int u0 = lower_bound_col(ccol + c0, (int)(cptr[i + 1] - c0), i);
        for (int x = lane; x < u0; x += 64) {
            const int64_t j = ccol[c0 + x];
            const int64_t r0 = cptr[j];
            const int mj = (int)(cptr[j + 1] - r0);
            const int y = lower_bound_col(ccol + r0, mj, i);
            if (y >= mj || ccol[r0 + y] != i) {
                atomicOr(flag, 16);
                continue;
            }
            const double *src = cval + (r0 + y) * BB;
            double *dst = cval + (c0 + x) * BB;
#pragma unroll
            for (int a = 0; a < BS; ++a)
#pragma unroll
                for (int b = 0; b < BS; ++b) dst[a * BS + b] = src[b * BS + a];
        }
    }
}

// the longest row part on and right of the diagonal (atomic maximum)
__global__ void k_upper_max(int64_t n, const int64_t *__restrict__ cptr, const int32_t *__restrict__ ccol,
                            int32_t *__restrict__ mx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c0 = cptr[i];
        const int m = (int)(cptr[i + 1] - c0);
        atomicMax(mx, m - lower_bound_col(ccol + c0, m, i));
    }
}

template <bool AGG>
void launch_sym(int tb, const DBsr &A, const int64_t *bptr, const int32_t *bcol, const int32_t *agg, int32_t *cnt,
                const int64_t *cptr, int32_t *ccol, int32_t *flag, hipStream_t s) {
    const dim3 g(wave_grid(A.nr)), b(64);
#define TE_SYM(TBV)                                                                                                  \
    case TBV:                                                                                                        \
        hipLaunchKernelGGL((k_sym<TBV, AGG>), g, b, 0, s, A.nr, A.ptr, A.col, bptr, bcol, agg, cnt, cptr, ccol, flag); \
        break;
    switch (tb) {
        TE_SYM(64)
        TE_SYM(128)
        TE_SYM(256)
        TE_SYM(512)
        TE_SYM(1024)
        TE_SYM(2048)
        TE_SYM(4096)
        default: TE_REQUIRE(false, TE_EINVAL, "bad table size %d", tb);
    }
#undef TE_SYM
    TE_CHECK_HIP(hipGetLastError());
}

// smallest table with load factor <= 1/2 for rows of `cols` blocks
int table_for(int64_t cols) {
    int tb = 64;
    while (tb < 2 * cols && tb < 4096) tb *= 2;
    return tb;
}

// symbolic product into C's own row pointer and columns; returns the longest row
template <bool AGG>
int64_t symbolic(const DBsr &A, const int64_t *bptr, const int32_t *bcol, const int32_t *agg, int first_tb, DBsr &C,
                 hipStream_t s) {
    const int64_t n = A.nr;
    DBuf<int32_t> cnt(std::max<int64_t>(n, 1)), flag(1);
    int tb = first_tb;
    for (;;) {
        TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
        launch_sym<AGG>(tb, A, bptr, bcol, agg, cnt.p, nullptr, nullptr, flag.p, s);
        if (read_flag(flag, s) == 0) break;
        TE_REQUIRE(tb < 4096, TE_ENOMEM, "sparse product row with more than 4096 blocks");
        tb = std::min(4096, tb * 4);
    }
    const int64_t mx = counts_to_ptr(cnt, n, C.ptr_own, C.nnzb, s);
    C.col_own.alloc(std::max<int64_t>(C.nnzb, 1));
    C.bind();
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    launch_sym<AGG>(table_for(mx), A, bptr, bcol, agg, nullptr, C.ptr, C.col_own.p, flag.p, s);
    TE_REQUIRE(read_flag(flag, s) == 0, TE_EHIP, "sparse product pattern pass disagrees with its count pass");
    return mx;
}

template <int BR, int BK, int BC, bool UP = false>
void launch_num(int tb, int64_t mx, const DBsr &A, const DBsr &B, DBsr &C, int32_t *flag, hipStream_t s) {
    const dim3 g(wave_grid(A.nr)), b(64);
    // LDS accumulation while a row's blocks fit in 32 KB (several waves per CU)
    const size_t lds = (size_t)std::max<int64_t>(mx, 1) * BR * BC * sizeof(double);
    const bool lacc = lds <= ((size_t)32 << 10);
    const int mcap = (int)std::max<int64_t>(mx, 1);
#define TE_NUM(TBV)                                                                                                \
    case TBV:                                                                                                      \
        if (lacc)                                                                                                  \
            hipLaunchKernelGGL((k_num<BR, BK, BC, TBV, true, UP>), g, b, lds, s, A.nr, A.ptr, A.col, A.val, B.ptr, \
                               B.col, B.val, C.ptr, C.col, C.val_own.p, flag, mcap);                               \
        else                                                                                                       \
            hipLaunchKernelGGL((k_num<BR, BK, BC, TBV, false, UP>), g, b, 0, s, A.nr, A.ptr, A.col, A.val, B.ptr,  \
                               B.col, B.val, C.ptr, C.col, C.val_own.p, flag, mcap);                               \
        break;
    switch (tb) {
        TE_NUM(64)
        TE_NUM(128)
        TE_NUM(256)
        TE_NUM(512)
        TE_NUM(1024)
        TE_NUM(2048)
        TE_NUM(4096)
        default: TE_REQUIRE(false, TE_EINVAL, "bad table size %d", tb);
    }
#undef TE_NUM
    TE_CHECK_HIP(hipGetLastError());
}

}  // namespace

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
void dev_strength(const DBsr &A, DBuf<double> &s, hipStream_t st) {
    TE_REQUIRE(A.br == A.bc, TE_EINVAL, "strength of a non-square block matrix");
    s.alloc(std::max<int64_t>(A.nnzb, 1));
    DBuf<double> dn(std::max<int64_t>(A.nr, 1));
    hipLaunchKernelGGL(k_fro, dim3(grid_for(A.nnzb)), dim3(256), 0, st, A.nnzb, A.br * A.bc, A.val, s.p);
    hipLaunchKernelGGL(k_diag_fro, dim3(grid_for(A.nr)), dim3(256), 0, st, A.nr, A.ptr, A.col, s.p, dn.p);
    hipLaunchKernelGGL(k_strength, dim3(grid_for(A.nr)), dim3(256), 0, st, A.nr, A.ptr, A.col, dn.p, s.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_CHECK_HIP(hipStreamSynchronize(st));
}

void dev_diag(const DBsr &A, DBuf<double> &d, hipStream_t st) {
    TE_REQUIRE(A.br == A.bc, TE_EINVAL, "diagonal of a non-square block matrix");
    d.alloc((size_t)std::max<int64_t>(A.nr, 1) * A.br);
    hipLaunchKernelGGL(k_diag_points, dim3(grid_for(A.nr)), dim3(256), 0, st, A.nr, A.br, A.ptr, A.col, A.val, d.p);
    TE_CHECK_HIP(hipGetLastError());
}

void dev_smoothed_p(const DBsr &A, const DBuf<int32_t> &agg, int64_t nagg, const DBuf<double> &Q,
                    const DBuf<double> &d, double omega, DBsr &P, hipStream_t s) {
    TE_REQUIRE(A.br == 3 || A.br == 6, TE_EINVAL, "unsupported block size %d", A.br);
    P.release();
    P.br = A.br;
    P.bc = 6;
    P.nr = A.nr;
    P.nc = nagg;
    const int64_t mx = symbolic<true>(A, nullptr, nullptr, agg.p, 64, P, s);
    P.val_own.alloc(std::max<int64_t>(P.nnzb * P.br * P.bc, 1));
    P.bind();
    DBuf<int32_t> flag(1);
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    const size_t lds = (size_t)std::max<int64_t>(mx, 1) * (P.br * 6 * sizeof(double) + sizeof(int32_t));
    if (lds <= (size_t)48 << 10) {
        const int mcap = (int)std::max<int64_t>(mx, 1);
        if (A.br == 3)
            hipLaunchKernelGGL(k_p_wave<3>, dim3(wave_grid(A.nr)), dim3(64), lds, s, A.nr, A.ptr, A.col, A.val, agg.p,
                               Q.p, d.p, omega, P.ptr, P.col, P.val_own.p, flag.p, mcap);
        else
            hipLaunchKernelGGL(k_p_wave<6>, dim3(wave_grid(A.nr)), dim3(64), lds, s, A.nr, A.ptr, A.col, A.val, agg.p,
                               Q.p, d.p, omega, P.ptr, P.col, P.val_own.p, flag.p, mcap);
    } else if (A.br == 3)
        hipLaunchKernelGGL(k_p_numeric<3>, dim3(grid_for(A.nr)), dim3(256), 0, s, A.nr, A.ptr, A.col, A.val, agg.p,
                           Q.p, d.p, omega, P.ptr, P.col, P.val_own.p, flag.p);
    else
        hipLaunchKernelGGL(k_p_numeric<6>, dim3(grid_for(A.nr)), dim3(256), 0, s, A.nr, A.ptr, A.col, A.val, agg.p,
                           Q.p, d.p, omega, P.ptr, P.col, P.val_own.p, flag.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_REQUIRE(read_flag(flag, s) == 0, TE_EHIP, "prolongator pattern misses a column");
}

void dev_mult(const DBsr &A, const DBsr &B, DBsr &C, hipStream_t s, bool symmetric) {
    TE_REQUIRE(A.bc == B.br && A.nc == B.nr, TE_EINVAL, "product shape mismatch");
    C.release();
    C.br = A.br;
    C.bc = B.bc;
    C.nr = A.nr;
    C.nc = B.nc;
    int64_t mx = symbolic<false>(A, B.ptr, B.col, nullptr, C.br == 3 ? 128 : 512, C, s);
    C.val_own.alloc(std::max<int64_t>(C.nnzb * C.br * C.bc, 1));
    C.bind();
    const int tb = table_for(mx);
    TE_REQUIRE(2 * mx <= tb, TE_ENOMEM, "sparse product row with %lld blocks is too long", (long long)mx);
    DBuf<int32_t> flag(1);
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    const int key = A.br * 100 + A.bc * 10 + B.bc;
    // a symmetric product of 6x6 blocks: the upper blocks, then their mirrors
    const bool up = symmetric && C.br == C.bc && C.nr == C.nc && (key == 636 || key == 666);
    if (up) {
        TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_upper_max, dim3(grid_for(C.nr)), dim3(256), 0, s, C.nr, C.ptr, C.col, flag.p);
        TE_CHECK_HIP(hipGetLastError());
        mx = std::max<int32_t>(read_flag(flag, s), 1);   // the longest upper row part
        TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    }
    if (key == 111) launch_num<1, 1, 1>(tb, mx, A, B, C, flag.p, s);
    else if (key == 336) launch_num<3, 3, 6>(tb, mx, A, B, C, flag.p, s);
    else if (key == 636) up ? launch_num<6, 3, 6, true>(tb, mx, A, B, C, flag.p, s)
                            : launch_num<6, 3, 6>(tb, mx, A, B, C, flag.p, s);
    else if (key == 666) up ? launch_num<6, 6, 6, true>(tb, mx, A, B, C, flag.p, s)
                            : launch_num<6, 6, 6>(tb, mx, A, B, C, flag.p, s);
    else TE_REQUIRE(false, TE_EINVAL, "unsupported product block shapes %dx%d * %dx%d", A.br, A.bc, B.br, B.bc);
    if (up) {
        hipLaunchKernelGGL((k_mirror_lower<6>), dim3(wave_grid(C.nr)), dim3(64), 0, s, C.nr, C.ptr, C.col,
                           C.val_own.p, flag.p);
        TE_CHECK_HIP(hipGetLastError());
    }
    TE_REQUIRE(read_flag(flag, s) == 0, TE_EHIP, "sparse product numeric pass found an inconsistent pattern");
}

void dev_transpose(const DBsr &A, DBsr &T, hipStream_t s) {
    T.release();
    T.br = A.bc;
    T.bc = A.br;
    T.nr = A.nc;
    T.nc = A.nr;
    const int64_t nt = std::max<int64_t>(T.nr, 1);
    DBuf<int32_t> cnt(nt), fill(nt), row(std::max<int64_t>(A.nnzb, 1));
    TE_CHECK_HIP(hipMemsetAsync(cnt.p, 0, nt * sizeof(int32_t), s));
    TE_CHECK_HIP(hipMemsetAsync(fill.p, 0, nt * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_t_count, dim3(grid_for(A.nnzb)), dim3(256), 0, s, A.nnzb, A.col, cnt.p);
    TE_CHECK_HIP(hipGetLastError());
    counts_to_ptr(cnt, T.nr, T.ptr_own, T.nnzb, s);
    TE_REQUIRE(T.nnzb == A.nnzb, TE_EINVAL, "transpose: column index out of range");
    DBuf<int64_t> src(std::max<int64_t>(A.nnzb, 1));
    T.col_own.alloc(std::max<int64_t>(T.nnzb, 1));
    T.val_own.alloc(std::max<int64_t>(T.nnzb * T.br * T.bc, 1));
    T.bind();
    hipLaunchKernelGGL(k_t_place, dim3(grid_for(A.nr)), dim3(256), 0, s, A.nr, A.ptr, A.col, T.ptr, fill.p, src.p,
                       row.p);
    DBuf<int64_t> srt(std::max<int64_t>(A.nnzb, 1));
    hipLaunchKernelGGL(k_t_rank, dim3(wave_grid(T.nr)), dim3(64), 0, s, T.nr, T.ptr, src.p, srt.p);
    if (A.br == 1 && A.bc == 1)
        hipLaunchKernelGGL((k_t_fill<1, 1>), dim3(grid_for(T.nnzb)), dim3(256), 0, s, T.nnzb, srt.p, row.p, A.val,
                           T.col_own.p, T.val_own.p);
    else if (A.br == 3 && A.bc == 6)
        hipLaunchKernelGGL((k_t_fill<3, 6>), dim3(grid_for(T.nnzb)), dim3(256), 0, s, T.nnzb, srt.p, row.p, A.val,
                           T.col_own.p, T.val_own.p);
    else if (A.br == 6 && A.bc == 6)
        hipLaunchKernelGGL((k_t_fill<6, 6>), dim3(grid_for(T.nnzb)), dim3(256), 0, s, T.nnzb, srt.p, row.p, A.val,
                           T.col_own.p, T.val_own.p);
    else
        TE_REQUIRE(false, TE_EINVAL, "unsupported transpose block shape %dx%d", A.br, A.bc);
    TE_CHECK_HIP(hipGetLastError());
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

// Symmetric one-wave-per-row layout of a square M (storage row r holds row
// row_order[r], storage column cs = col_map[c]): blocks with cs >= r stay,
// each block with cs < r becomes a reference to its mirror.  Returns false
// (and leaves S alone) when the pattern is not symmetric.
// ---- upper-triangle storage of a symmetric block operator --------------------
// Storage row r holds natural row o = order[r]; its entry (o, j) is an upper
// entry when the storage column map[j] is >= r, otherwise a lower one, which
// the products read transposed from its mirror (j, o).  One thread per row;
// an entry whose column is out of range is skipped by both fill passes (the
// row then writes fewer entries than counted) and flags the pattern as bad.
__global__ void k_sym_count(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ order, const int32_t *__restrict__ map,
                            int32_t *__restrict__ ucnt, int32_t *__restrict__ lcnt, int32_t *__restrict__ bad) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = order[r];
        int32_t u = 0;
        for (int64_t k = ptr[o]; k < ptr[o + 1]; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) {
                *bad = 1;
                continue;
            }
            u += map[j] >= r ? 1 : 0;
        }
        ucnt[r] = u;
        lcnt[r] = (int32_t)(ptr[o + 1] - ptr[o]) - u;
    }
}

// upper entries: storage column, source entry, and each source entry's
// position in the upper list (upos stays -1 for the lower ones)
__global__ void k_sym_upper(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ order, const int32_t *__restrict__ map,
                            const int64_t *__restrict__ rptr, int32_t *__restrict__ ucol, int64_t *__restrict__ usrc,
                            int32_t *__restrict__ upos) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = order[r];
        int64_t u = rptr[r];
        for (int64_t k = ptr[o]; k < ptr[o + 1]; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) continue;
            const int32_t cs = map[j];
            if (cs >= r) {
                upos[k] = (int32_t)u;
                usrc[u] = k;
                ucol[u] = cs;
                ++u;
            }
        }
    }
}

// lower entries: storage column and the upper-list position of the mirror
// block, found by bisection in the mirror's row (columns ascending)
__global__ void k_sym_lower(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ order, const int32_t *__restrict__ map,
                            const int64_t *__restrict__ lptr, const int32_t *__restrict__ upos,
                            int32_t *__restrict__ lcol, int32_t *__restrict__ lidx, int32_t *__restrict__ bad) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = order[r];
        int64_t l = lptr[r];
        for (int64_t k = ptr[o]; k < ptr[o + 1]; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) continue;
            const int32_t cs = map[j];
            if (cs >= r) continue;
            int64_t lo = ptr[j], hi = ptr[j + 1];
            const int64_t end = hi;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < o) lo = mid + 1;
                else hi = mid;
            }
            int32_t up = (lo < end && col[lo] == o) ? upos[lo] : -1;
            if (up < 0) {
                *bad = 1;
                up = 0;
            }
            lcol[l] = cs;
            lidx[l] = up;
            ++l;
        }
    }
}

// Upper-triangle packing on the device; false (nothing kept) when M is not
// square in one numbering, a mirror block is missing (an unsymmetric pattern,
// or columns not ascending within a row) or the upper part has 2^31 blocks.
static bool pack_rows_sym(Sell &S, const DBsr &M, const std::vector<int64_t> &hptr,
                          const std::vector<int32_t> &row_order, const std::vector<int32_t> &col_map, bool fp32,
                          hipStream_t s) {
    const int64_t n = M.nr;
    if (M.nr != M.nc || M.br != M.bc || (int64_t)hptr.size() != n + 1 || hptr[n] != M.nnzb ||
        (int64_t)row_order.size() != n || (int64_t)col_map.size() != n)
        return false;
    for (int64_t r = 0; r < n; ++r) {
        const int32_t o = row_order[r];
        if (o < 0 || o >= n || col_map[o] != r) return false;  // rows and columns in the same numbering
    }
    DBuf<int32_t> dorder, dmap, ucnt(std::max<int64_t>(n, 1)), lcnt(std::max<int64_t>(n, 1)), bad(1);
    upload(dorder, row_order, s);
    upload(dmap, col_map, s);
    TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    const unsigned g = grid_for(n);
    hipLaunchKernelGGL(k_sym_count, dim3(g), dim3(256), 0, s, n, M.ptr, M.col, dorder.p, dmap.p, ucnt.p, lcnt.p,
                       bad.p);
    TE_CHECK_HIP(hipGetLastError());
    if (read_flag(bad, s) != 0) return false;
    DBuf<int64_t> rptr, lptr;
    int64_t nup = 0, nlow = 0;
    counts_to_ptr(ucnt, n, rptr, nup, s);
    counts_to_ptr(lcnt, n, lptr, nlow, s);
    if (nup >= INT32_MAX) return false;
    DBuf<int32_t> ucol(std::max<int64_t>(nup, 1)), upos(std::max<int64_t>(M.nnzb, 1));
    DBuf<int32_t> lcol(std::max<int64_t>(nlow, 1)), lidx(std::max<int64_t>(nlow, 1));
    DBuf<int64_t> usrc(std::max<int64_t>(nup, 1));
    TE_CHECK_HIP(hipMemsetAsync(upos.p, 0xFF, (size_t)std::max<int64_t>(M.nnzb, 1) * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_sym_upper, dim3(g), dim3(256), 0, s, n, M.ptr, M.col, dorder.p, dmap.p, rptr.p, ucol.p,
                       usrc.p, upos.p);
    TE_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sym_lower, dim3(g), dim3(256), 0, s, n, M.ptr, M.col, dorder.p, dmap.p, lptr.p, upos.p,
                       lcol.p, lidx.p, bad.p);
    TE_CHECK_HIP(hipGetLastError());
    if (read_flag(bad, s) != 0) return false;
    const int bb = M.br * M.bc;
    S.format = FMT_ROWWAVE;
    S.br = M.br;
    S.bc = M.bc;
    S.nrows = n;
    S.ncols = n;
    S.nnzb = nup;
    S.nslices = 0;
    S.padded = nup;
    S.rptr = std::move(rptr);
    S.col = std::move(ucol);
    S.lptr = std::move(lptr);
    S.lcol = std::move(lcol);  // one entry at least, also without lower blocks
    S.lidx = std::move(lidx);
    S.val.alloc(std::max<int64_t>(nup * bb, 1));
    if (fp32) S.val32.alloc(std::max<int64_t>(nup * bb, 1));
    else S.val32.release();
    hipLaunchKernelGGL(k_pack_upper, dim3(grid_for(nup * bb)), dim3(256), 0, s, nup, bb, usrc.p, M.val, S.val.p,
                       fp32 ? S.val32.p : nullptr);
    TE_CHECK_HIP(hipGetLastError());
    S.slice_off.release();
    S.rowlen.release();
    S.rowmap.release();
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return true;
}

void dev_pack(Sell &S, const DBsr &M, const std::vector<int64_t> &hptr, const std::vector<int32_t> &row_order,
              const std::vector<int32_t> &col_map, const std::vector<int32_t> *out_map, bool fp32, hipStream_t s,
              int format, bool sym) {
    S.lptr.release();
    S.lcol.release();
    S.lidx.release();
    if (sym && format == FMT_ROWWAVE && !out_map && pack_rows_sym(S, M, hptr, row_order, col_map, fp32, s))
        return;
    TE_REQUIRE((int64_t)hptr.size() == M.nr + 1 && (int64_t)row_order.size() == M.nr &&
                   (int64_t)col_map.size() == M.nc && hptr[M.nr] == M.nnzb,
               TE_EINVAL, "pack: inconsistent sizes");
    const int bb = M.br * M.bc;
    DBuf<int32_t> dorder, dmap;
    upload(dorder, row_order, s);
    upload(dmap, col_map, s);
    S.format = format;
    S.br = M.br;
    S.bc = M.bc;
    S.nrows = M.nr;
    S.ncols = M.nc;
    S.nnzb = M.nnzb;
    if (format == FMT_ROWWAVE) {
        S.nslices = 0;
        S.padded = M.nnzb;
        std::vector<int64_t> rptr(M.nr + 1, 0);
        for (int64_t r = 0; r < M.nr; ++r) rptr[r + 1] = rptr[r] + (hptr[row_order[r] + 1] - hptr[row_order[r]]);
        upload(S.rptr, rptr, s);
        S.col.alloc(std::max<int64_t>(M.nnzb, 1));
        S.val.alloc(std::max<int64_t>(M.nnzb * bb, 1));
        if (fp32) S.val32.alloc(std::max<int64_t>(M.nnzb * bb, 1));
        else S.val32.release();
        hipLaunchKernelGGL(k_pack_rows, dim3(wave_grid(M.nr)), dim3(64), 0, s, M.nr, bb, M.ptr, M.col, M.val,
                           dorder.p, dmap.p, S.rptr.p, S.col.p, S.val.p, fp32 ? S.val32.p : nullptr);
        S.slice_off.release();
        S.rowlen.release();
    } else {
        S.rptr.release();
        S.nslices = (M.nr + SELL_C - 1) / SELL_C;
        std::vector<int32_t> off(S.nslices + 1, 0), rowlen(S.nslices * SELL_C, 0);
        std::vector<int64_t> width(S.nslices);
        parallel_for(S.nslices, [&](int64_t lo, int64_t hi, int) {
            for (int64_t sl = lo; sl < hi; ++sl) {
                int64_t w = 0;
                for (int l = 0; l < SELL_C; ++l) {
                    const int64_t r = sl * SELL_C + l;
                    if (r >= M.nr) break;
                    const int64_t len = hptr[row_order[r] + 1] - hptr[row_order[r]];
                    rowlen[r] = (int32_t)len;
                    w = std::max(w, len);
                }
                width[sl] = w;
            }
        });
        for (int64_t sl = 0; sl < S.nslices; ++sl) {
            TE_REQUIRE((int64_t)off[sl] + width[sl] < INT32_MAX, TE_EINVAL, "matrix too large for the SELL offsets");
            off[sl + 1] = off[sl] + (int32_t)width[sl];
        }
        S.padded = (int64_t)off[S.nslices] * SELL_C;
        upload(S.slice_off, off, s);
        upload(S.rowlen, rowlen, s);
        S.col.alloc(std::max<int64_t>(S.padded, 1));
        S.val.alloc(std::max<int64_t>(S.padded * bb, 1));
        if (fp32) S.val32.alloc(std::max<int64_t>(S.padded * bb, 1));
        else S.val32.release();
        auto kern = bb == 9 ? k_pack_sell<9> : bb == 18 ? k_pack_sell<18> : k_pack_sell<0>;
        hipLaunchKernelGGL(kern, dim3(grid_for(S.nslices * 64)), dim3(256), 0, s, M.nr, bb, M.ptr, M.col, M.val,
                           dorder.p, dmap.p, S.slice_off.p, S.nslices, S.col.p, S.val.p, fp32 ? S.val32.p : nullptr);
    }
    TE_CHECK_HIP(hipGetLastError());
    if (out_map) {
        std::vector<int32_t> rm(format == FMT_ROWWAVE ? M.nr : S.nslices * SELL_C, -1);
        parallel_for(M.nr, [&](int64_t lo, int64_t hi, int) {
            for (int64_t r = lo; r < hi; ++r) rm[r] = (*out_map)[row_order[r]];
        });
        upload(S.rowmap, rm, s);
    } else {
        S.rowmap.release();
    }
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

void dev_dense_inverse_spd(const std::vector<double> &M, int n, DBuf<double> &inv, hipStream_t s) {
    const int64_t nn = (int64_t)n * n;
    TE_REQUIRE((int64_t)M.size() == nn && n > 0, TE_EINVAL, "dense inverse: bad size");
    DBuf<double> a, b;
    upload(a, M, s);
    b.alloc(nn);
    DBuf<int32_t> bad(1);
    TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    const unsigned g = grid_for(nn);
    const dim3 gs((n + 255) / 256, std::min(n, 4096));
    for (int j = 0; j < n; ++j) {
        hipLaunchKernelGGL(k_sweep, gs, dim3(256), 0, s, n, j, a.p, b.p, bad.p);
        std::swap(a.p, b.p);
    }
    TE_CHECK_HIP(hipGetLastError());
    TE_REQUIRE(read_flag(bad, s) == 0, TE_ECHOL, "coarse factor: a pivot of the coarsest operator is not positive");
    inv.alloc(nn);
    hipLaunchKernelGGL(k_negate, dim3(g), dim3(256), 0, s, nn, a.p, inv.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Parallel (MIS-2) aggregation
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kKeyState = int64_t(1) << 61;  // key* = state * 2^61 + prio * 2^30 + i
constexpr int8_t kOut = 0, kUndecided = 1, kIn = 2;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 (Steele, Lea & Flood 2014)
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// flag[k] = 1 for block k = (i, j), i != j, with s_ij >= theta, and for its
// mirror (j, i) (binary search in the sorted row j).
__global__ void k_strong_sym(int64_t nr, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const double *__restrict__ s, double theta, uint8_t *__restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            if (j == i || !(s[k] >= theta)) continue;
            flag[k] = 1;
            int64_t lo = ptr[j], hi = ptr[j + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            if (lo < ptr[j + 1] && col[lo] == i) flag[lo] = 1;
        }
}

// pk[i] = prio(i) * 2^30 + i; state = undecided if row i has a strong block
__global__ void k_mis_init(int64_t nr, const int64_t *__restrict__ ptr, const uint8_t *__restrict__ flag,
                           uint64_t seed, int64_t *__restrict__ pk, int8_t *__restrict__ state) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        pk[i] = (int64_t)(mix64(seed ^ (uint64_t)i) >> 33) * (int64_t(1) << 30) + i;
        bool has = false;
        for (int64_t k = ptr[i]; k < ptr[i + 1] && !has; ++k) has = flag[k] != 0;
        state[i] = has ? kUndecided : kOut;
    }
}

// out[i] = max(own, max over strong neighbours j of val(j)), val from the
// current state and keys (first pass) or from the previous pass's output
template <bool FIRST>
__global__ void k_mis_max(int64_t nr, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const uint8_t *__restrict__ flag, const int8_t *__restrict__ state,
                          const int64_t *__restrict__ pk, const int64_t *__restrict__ in, int64_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = FIRST ? state[i] * kKeyState + pk[i] : in[i];
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (!flag[k]) continue;
            const int32_t j = col[k];
            const int64_t v = FIRST ? state[j] * kKeyState + pk[j] : in[j];
            m = v > m ? v : m;
        }
        out[i] = m;
    }
}

// undecided i joins if the distance-2 maximum is its own key*, is excluded if
// that maximum belongs to a member; counts the nodes still undecided
__global__ void k_mis_step(int64_t nr, const int64_t *__restrict__ pk, const int64_t *__restrict__ m2,
                           int8_t *__restrict__ state, int32_t *__restrict__ left) {
    int32_t c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        if (state[i] != kUndecided) continue;
        const int64_t own = kUndecided * kKeyState + pk[i];
        if (m2[i] == own) state[i] = kIn;
        else if (m2[i] / kKeyState == kIn) state[i] = kOut;
        else ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(left, c);
}

// phase 1: a root's id, or the id of the (unique) root among the strong
// neighbours, else -1
__global__ void k_agg_phase1(int64_t nr, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const uint8_t *__restrict__ flag, const int8_t *__restrict__ state,
                             const int32_t *__restrict__ rid, int32_t *__restrict__ agg1) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = -1;
        if (state[i] == kIn) a = rid[i];
        else
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
                if (flag[k] && state[col[k]] == kIn) {
                    a = rid[col[k]];
                    break;
                }
        agg1[i] = a;
    }
}

// phase 2 over the phase-1 snapshot agg1, neighbours in stored order
__global__ void k_agg_phase2(int64_t nr, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const uint8_t *__restrict__ flag, const double *__restrict__ s, double tie_rtol,
                             const int32_t *__restrict__ agg1, int32_t *__restrict__ agg, int32_t *__restrict__ orphan) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t ba = agg1[i];
        if (ba < 0) {
            bool has = false;
            double bs = -1.0;
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
                if (!flag[k]) continue;
                has = true;
                const int32_t a = agg1[col[k]];
                if (a < 0) continue;
                const double sv = s[k];
                if (ba < 0 || sv > bs * (1.0 + tie_rtol)) {
                    bs = sv;
                    ba = a;
                } else if (sv >= bs * (1.0 - tie_rtol) && a < ba) {
                    bs = sv;
                    ba = a;
                }
            }
            if (has && ba < 0) atomicMax(orphan, 1);
        }
        agg[i] = ba;
    }
}
}  // namespace

namespace {
__global__ void k_rbm(const double *__restrict__ X, const uint8_t *__restrict__ mask, int64_t n, double cx, double cy,
                      double cz, double *__restrict__ B) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = X[i * 3] - cx, y = X[i * 3 + 1] - cy, z = X[i * 3 + 2] - cz;
        const double b[18] = {1, 0, 0, -y, 0, z,    // row x
                              0, 1, 0, x, -z, 0,    // row y
                              0, 0, 1, 0, y, -x};   // row z
        for (int p = 0; p < 3; ++p) {
            const bool fixed = mask && mask[i * 3 + p];
            for (int q = 0; q < 6; ++q) B[(i * 3 + p) * 6 + q] = fixed ? 0.0 : b[p * 6 + q];
        }
    }
}

constexpr int kTentK = 6;
constexpr int kTentMaxRows = 640;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per aggregate: its m = bs * |J| rows of B in LDS (W, column-major
// with leading dimension ld), Householder vectors in V.  The same steps as a
// textbook thin QR: for each column j the reflector v = w - alpha e_j with
// alpha = -sign(w_j) |w|, beta = 2 / v.v, applied to columns j..5; then
// Q = H_0 ... H_5 [I; 0], and the signs flipped so that diag(R) > 0.
__global__ void __launch_bounds__(64) k_tent_qr(const int64_t *__restrict__ off, const int32_t *__restrict__ mem,
                                                const double *__restrict__ B, int bs, int ld, double rank_rtol,
                                                double *__restrict__ Q, double *__restrict__ Bc,
                                                int32_t *__restrict__ bad) {
    extern __shared__ double sh[];
    constexpr int K = kTentK;
    double *W = sh, *V = sh + K * ld;
    const int x = blockIdx.x, lane = threadIdx.x;
    const int64_t o0 = off[x];
    const int m = (int)(off[x + 1] - o0) * bs;
    if (m < K || m > ld) {  // uniform over the wave
        if (lane == 0) atomicOr(bad, 1);
        return;
    }
    for (int i = lane; i < m; i += 64) {
        const int64_t node = mem[o0 + i / bs];
        const int p = i % bs;
        for (int c = 0; c < K; ++c) W[c * ld + i] = B[(node * bs + p) * K + c];
    }
    __syncthreads();
    double beta[K];
    for (int j = 0; j < K; ++j) {
        double t = 0.0;
        for (int i = j + lane; i < m; i += 64) t += W[j * ld + i] * W[j * ld + i];
        const double nrm = sqrt(wave_sum(t));
        const double alpha = W[j * ld + j] >= 0 ? -nrm : nrm;
        for (int i = lane; i < m; i += 64) V[j * ld + i] = (i >= j) ? W[j * ld + i] - (i == j ? alpha : 0.0) : 0.0;
        __syncthreads();
        t = 0.0;
        for (int i = j + lane; i < m; i += 64) t += V[j * ld + i] * V[j * ld + i];
        const double vn = wave_sum(t);
        beta[j] = vn > 0 ? 2.0 / vn : 0.0;
        for (int c = j; c < K; ++c) {
            t = 0.0;
            for (int i = j + lane; i < m; i += 64) t += V[j * ld + i] * W[c * ld + i];
            const double f = wave_sum(t) * beta[j];
            __syncthreads();
            for (int i = j + lane; i < m; i += 64) W[c * ld + i] -= f * V[j * ld + i];
            __syncthreads();
        }
    }
    double R[K][K];
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) R[r][c] = (c >= r) ? W[c * ld + r] : 0.0;
    __syncthreads();
    for (int c = 0; c < K; ++c) {
        for (int i = lane; i < m; i += 64) W[c * ld + i] = (i == c) ? 1.0 : 0.0;
        __syncthreads();
        for (int j = K - 1; j >= 0; --j) {
            double t = 0.0;
            for (int i = j + lane; i < m; i += 64) t += V[j * ld + i] * W[c * ld + i];
            const double f = wave_sum(t) * beta[j];
            __syncthreads();
            for (int i = j + lane; i < m; i += 64) W[c * ld + i] -= f * V[j * ld + i];
            __syncthreads();
        }
    }
    double mx = 0.0, mn = INFINITY, sg[K];
    for (int r = 0; r < K; ++r) {
        sg[r] = R[r][r] < 0 ? -1.0 : 1.0;
        mx = fmax(mx, fabs(R[r][r]));
        mn = fmin(mn, fabs(R[r][r]));
    }
    if (!(mx > 0 && mn >= rank_rtol * mx)) {
        if (lane == 0) atomicOr(bad, 1);
        return;
    }
    for (int i = lane; i < m; i += 64) {
        const int64_t node = mem[o0 + i / bs];
        const int p = i % bs;
        for (int c = 0; c < K; ++c) Q[(node * bs + p) * K + c] = sg[c] * W[c * ld + i];
    }
    if (lane < K * K) {
        const int r = lane / K, c = lane % K;
        Bc[(int64_t)x * K * K + lane] = sg[r] * R[r][c];
    }
}

// sum over stored blocks of mix64(row * 2^32 + column), per row the row
// length mixed in as well; wave sums then one 64-bit atomic per wave
__global__ void k_pattern_hash(const int64_t *__restrict__ ptr, const int32_t *__restrict__ col, int64_t n,
                               unsigned long long *__restrict__ out) {
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        h += mix64(0xC0FFEEull ^ ((uint64_t)i << 32) ^ (uint64_t)(ptr[i + 1] - ptr[i]));
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) h += mix64(((uint64_t)i << 32) | (uint32_t)col[k]);
    }
    for (int o = 32; o > 0; o >>= 1) h += __shfl_down(h, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, h);
}
}  // namespace

namespace {
__global__ void k_filter_count(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                               const uint8_t *__restrict__ flag, int64_t *__restrict__ cnt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        bool diag = false;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            diag = diag || col[k] == i;
            c += (flag[k] || col[k] == i) ? 1 : 0;
        }
        cnt[i] = diag ? c : -1;
    }
}

template <int BB>
__global__ void k_filter_copy(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                              const double *__restrict__ val, const uint8_t *__restrict__ flag,
                              const int64_t *__restrict__ fptr, int32_t *__restrict__ fcol, double *__restrict__ fval) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d[BB];
        int64_t kd = -1;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] == i) kd = k;
        if (kd < 0) continue;  // rejected on the host before the launch
        for (int e = 0; e < BB; ++e) d[e] = val[kd * BB + e];
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (!flag[k] && col[k] != i)
                for (int e = 0; e < BB; ++e) d[e] += val[k * BB + e];
        int64_t o = fptr[i];
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (col[k] == i) {
                fcol[o] = (int32_t)i;
                for (int e = 0; e < BB; ++e) fval[o * BB + e] = d[e];
                ++o;
            } else if (flag[k]) {
                fcol[o] = col[k];
                for (int e = 0; e < BB; ++e) fval[o * BB + e] = val[k * BB + e];
                ++o;
            }
        }
    }
}
}  // namespace

void dev_filtered(const DBsr &A, const DBuf<double> &s, double theta, DBsr &F, hipStream_t st) {
    TE_REQUIRE(A.nr == A.nc && A.br == A.bc && (A.br == 3 || A.br == 6), TE_EINVAL, "filtered operator: block %dx%d",
               A.br, A.bc);
    const int64_t n = A.nr;
    DBuf<uint8_t> flag(std::max<int64_t>(A.nnzb, 1));
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, std::max<int64_t>(A.nnzb, 1), st));
    hipLaunchKernelGGL(k_strong_sym, dim3(grid_for(n)), dim3(256), 0, st, n, A.ptr, A.col, s.p, theta, flag.p);
    DBuf<int64_t> cnt(std::max<int64_t>(n, 1));
    hipLaunchKernelGGL(k_filter_count, dim3(grid_for(n)), dim3(256), 0, st, n, A.ptr, A.col, flag.p, cnt.p);
    TE_CHECK_HIP(hipGetLastError());
    std::vector<int64_t> c;
    download(c, cnt.p, (size_t)n, st);
    std::vector<int64_t> fp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        TE_REQUIRE(c[i] >= 1, TE_EINVAL, "filtered operator: block row %lld has no diagonal block", (long long)i);
        fp[i + 1] = fp[i] + c[i];
    }
    F.release();
    F.br = F.bc = A.br;
    F.nr = F.nc = n;
    F.nnzb = fp[n];
    upload(F.ptr_own, fp, st);
    F.col_own.alloc(std::max<int64_t>(F.nnzb, 1));
    F.val_own.alloc(std::max<int64_t>(F.nnzb * A.br * A.bc, 1));
    F.bind();
    if (A.br == 3)
        hipLaunchKernelGGL(k_filter_copy<9>, dim3(grid_for(n)), dim3(256), 0, st, n, A.ptr, A.col, A.val, flag.p,
                           F.ptr, F.col_own.p, F.val_own.p);
    else
        hipLaunchKernelGGL(k_filter_copy<36>, dim3(grid_for(n)), dim3(256), 0, st, n, A.ptr, A.col, A.val, flag.p,
                           F.ptr, F.col_own.p, F.val_own.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_CHECK_HIP(hipStreamSynchronize(st));
}

namespace {
// per workgroup: the sums of the three coordinates over a grid-stride share
// of the nodes
__global__ void __launch_bounds__(256) k_coord_sum(const double *__restrict__ X, int64_t n, double *__restrict__ part) {
    __shared__ double sh[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int q = 0; q < 3; ++q) a[q] += X[i * 3 + q];
    for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}
}  // namespace

void dev_centroid(const double *coords, int64_t n, double c[3], hipStream_t st) {
    c[0] = c[1] = c[2] = 0.0;
    if (n <= 0) return;
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    DBuf<double> part((size_t)nb * 3);
    hipLaunchKernelGGL(k_coord_sum, dim3(nb), dim3(256), 0, st, coords, n, part.p);
    TE_CHECK_HIP(hipGetLastError());
    std::vector<double> h;
    download(h, part.p, (size_t)nb * 3, st);
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 3; ++q) c[q] += h[(size_t)b * 3 + q];
    for (int q = 0; q < 3; ++q) c[q] /= (double)n;
}

void dev_rigid_body_modes(const double *coords, const uint8_t *mask, int64_t n, const double c[3], DBuf<double> &B,
                          hipStream_t st) {
    B.alloc(std::max<int64_t>(n * 18, 1));
    hipLaunchKernelGGL(k_rbm, dim3(grid_for(n)), dim3(256), 0, st, coords, mask, n, c[0], c[1], c[2], B.p);
    TE_CHECK_HIP(hipGetLastError());
}

bool dev_tentative(const std::vector<int64_t> &off, const std::vector<int32_t> &mem, const DBuf<double> &B,
                   int64_t n, int bs, double rank_rtol, DBuf<double> &Q, DBuf<double> &Bc, hipStream_t st) {
    const int64_t na = (int64_t)off.size() - 1;
    if (na <= 0) return false;
    int64_t mmax = 0;
    for (int64_t x = 0; x < na; ++x) mmax = std::max<int64_t>(mmax, (off[x + 1] - off[x]) * bs);
    if (mmax > kTentMaxRows || mmax < kTentK) return false;
    const int ld = (int)mmax;
    DBuf<int64_t> doff;
    DBuf<int32_t> dmem, bad(1);
    upload(doff, off, st);
    upload(dmem, mem, st);
    Q.alloc(std::max<int64_t>(n * bs * kTentK, 1));
    Bc.alloc(na * kTentK * kTentK);
    TE_CHECK_HIP(hipMemsetAsync(Q.p, 0, Q.bytes(), st));
    TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), st));
    const size_t lds = (size_t)2 * kTentK * ld * sizeof(double);
    hipLaunchKernelGGL(k_tent_qr, dim3((unsigned)na), dim3(64), lds, st, doff.p, dmem.p, B.p, bs, ld, rank_rtol, Q.p,
                       Bc.p, bad.p);
    TE_CHECK_HIP(hipGetLastError());
    return read_flag(bad, st) == 0;
}

namespace {
__global__ void k_check_pattern(const int64_t *__restrict__ ptr, const int32_t *__restrict__ col, int64_t n,
                                unsigned long long *__restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // columns in range, strictly ascending (the strength symmetrisation
        // binary-searches mirror rows), and a diagonal block present
        bool ok = true, diag = false;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t c = col[k];
            ok = ok && c >= 0 && c < n && (k == ptr[i] || c > col[k - 1]);
            diag = diag || c == i;
        }
        if (!ok || !diag) atomicMin(bad, (unsigned long long)i);
    }
}
}  // namespace

namespace {
__global__ void k_diag_store(const double *__restrict__ dnat, const int32_t *__restrict__ perm, int64_t n, int bs,
                             double *__restrict__ d, double *__restrict__ dinv, float *__restrict__ dinv32,
                             unsigned long long *__restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = perm[i];
        for (int p = 0; p < bs; ++p) {
            const double v = dnat[o * bs + p];
            if (!(v > 0)) atomicMin(bad, (unsigned long long)o);
            d[i * bs + p] = v;
            dinv[i * bs + p] = 1.0 / v;
            if (dinv32) dinv32[i * bs + p] = (float)(1.0 / v);
        }
    }
}
__global__ void k_rsqrt(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 1.0 / sqrt(x[i]);
}
}  // namespace

int64_t dev_diag_store(const double *dnat, const int32_t *perm, int64_t n, int bs, double *d, double *dinv,
                       float *dinv32, hipStream_t st) {
    DBuf<unsigned long long> b(1);
    TE_CHECK_HIP(hipMemsetAsync(b.p, 0xFF, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_diag_store, dim3(grid_for(n)), dim3(256), 0, st, dnat, perm, n, bs, d, dinv, dinv32, b.p);
    TE_CHECK_HIP(hipGetLastError());
    unsigned long long h = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&h, b.p, sizeof(h), hipMemcpyDeviceToHost, st));
    TE_CHECK_HIP(hipStreamSynchronize(st));
    return h == ~0ull ? -1 : (int64_t)h;
}

void dev_rsqrt(const double *x, double *y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_rsqrt, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
    TE_CHECK_HIP(hipGetLastError());
}

int64_t dev_check_pattern(const int64_t *ptr, const int32_t *col, int64_t n, hipStream_t st) {
    DBuf<unsigned long long> d(1);
    TE_CHECK_HIP(hipMemsetAsync(d.p, 0xFF, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_check_pattern, dim3(grid_for(n)), dim3(256), 0, st, ptr, col, n, d.p);
    TE_CHECK_HIP(hipGetLastError());
    unsigned long long h = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&h, d.p, sizeof(h), hipMemcpyDeviceToHost, st));
    TE_CHECK_HIP(hipStreamSynchronize(st));
    return h == ~0ull ? -1 : (int64_t)h;
}

uint64_t dev_pattern_hash(const int64_t *ptr, const int32_t *col, int64_t n, hipStream_t st) {
    DBuf<unsigned long long> d(1);
    TE_CHECK_HIP(hipMemsetAsync(d.p, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_pattern_hash, dim3(grid_for(n)), dim3(256), 0, st, ptr, col, n, d.p);
    TE_CHECK_HIP(hipGetLastError());
    unsigned long long h = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&h, d.p, sizeof(h), hipMemcpyDeviceToHost, st));
    TE_CHECK_HIP(hipStreamSynchronize(st));
    return (uint64_t)h;
}

int64_t dev_aggregate_mis2(const DBsr &A, const DBuf<double> &s, double theta, uint64_t seed, double tie_rtol,
                           std::vector<int32_t> &agg, hipStream_t st) {
    TE_REQUIRE(A.nr == A.nc && A.nr < (int64_t(1) << 30), TE_EINVAL, "parallel aggregation: %lld rows",
               (long long)A.nr);
    const int64_t n = A.nr;
    agg.assign(n, -1);
    if (n == 0) return 0;
    const unsigned g = grid_for(n);
    DBuf<uint8_t> flag(std::max<int64_t>(A.nnzb, 1));
    DBuf<int8_t> state(n);
    DBuf<int64_t> pk(n), m1(n), m2(n);
    DBuf<int32_t> left(1), rid(n), agg1(n), dagg(n), orphan(1);
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, std::max<int64_t>(A.nnzb, 1), st));
    TE_CHECK_HIP(hipMemsetAsync(orphan.p, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_strong_sym, dim3(g), dim3(256), 0, st, n, A.ptr, A.col, s.p, theta, flag.p);
    hipLaunchKernelGGL(k_mis_init, dim3(g), dim3(256), 0, st, n, A.ptr, flag.p, seed, pk.p, state.p);
    TE_CHECK_HIP(hipGetLastError());
    // every round selects at least the undecided node of largest key, so at
    // most n rounds; in practice a few tens
    for (int64_t round = 0;; ++round) {
        TE_REQUIRE(round <= n, TE_EINVAL, "parallel aggregation did not finish");
        TE_CHECK_HIP(hipMemsetAsync(left.p, 0, sizeof(int32_t), st));
        hipLaunchKernelGGL((k_mis_max<true>), dim3(g), dim3(256), 0, st, n, A.ptr, A.col, flag.p, state.p, pk.p,
                           nullptr, m1.p);
        hipLaunchKernelGGL((k_mis_max<false>), dim3(g), dim3(256), 0, st, n, A.ptr, A.col, flag.p, state.p, pk.p,
                           m1.p, m2.p);
        hipLaunchKernelGGL(k_mis_step, dim3(g), dim3(256), 0, st, n, pk.p, m2.p, state.p, left.p);
        TE_CHECK_HIP(hipGetLastError());
        if (read_flag(left, st) == 0) break;
    }
    // aggregate ids by ascending root
    std::vector<int8_t> hs;
    download(hs, state.p, (size_t)n, st);
    std::vector<int32_t> hr(n, -1);
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i)
        if (hs[i] == kIn) hr[i] = (int32_t)na++;
    upload(rid, hr, st);
    hipLaunchKernelGGL(k_agg_phase1, dim3(g), dim3(256), 0, st, n, A.ptr, A.col, flag.p, state.p, rid.p, agg1.p);
    hipLaunchKernelGGL(k_agg_phase2, dim3(g), dim3(256), 0, st, n, A.ptr, A.col, flag.p, s.p, tie_rtol, agg1.p,
                       dagg.p, orphan.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_REQUIRE(read_flag(orphan, st) == 0, TE_EINVAL, "aggregation: a node has no aggregated strong neighbour");
    download(agg, dagg.p, (size_t)n, st);
    return na;
}

void dev_pattern_to_host(const DBsr &M, HBsr &H, hipStream_t s) {
    H.br = M.br;
    H.bc = M.bc;
    H.nr = M.nr;
    H.nc = M.nc;
    download(H.ptr, M.ptr, (size_t)M.nr + 1, s);
    download(H.col, M.col, (size_t)M.nnzb, s);
    H.val.clear();
}

void dev_to_host(const DBsr &M, HBsr &H, hipStream_t s) {
    dev_pattern_to_host(M, H, s);
    download(H.val, M.val, (size_t)M.nnzb * M.br * M.bc, s);
}

}  // namespace te
