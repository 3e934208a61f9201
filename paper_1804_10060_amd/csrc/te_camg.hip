// The thermal solve on the device: classical AMG (the paper's thermal
// preconditioner is a classical AMG with a hybrid Gauss-Seidel smoother,
// Sec. 5.1), preconditioned CG for its corrections (Sec. 2.1.2), and
// Newton's method on the heat equation of eq. wf_thermal (Sec. 3.2).
//
// Setup per level (scalar compressed rows, natural numbering):
//   k_strength   one thread per row: strong entries -a_ij >= theta max(-a_ik)
//   k_infl       |S_j^T| by integer atomics (exact, order-free)
//   k_sym        an entry is a strong neighbour if either direction is strong
//                (mirror found by binary search in the sorted mirror row)
//   k_pmis_*     PMIS rounds with fixed keys (|S_i^T|, splitmix64 bits, i):
//                local maxima among undecided strong neighbours become C,
//                undecided points depending on a new C point become F; the
//                host reads the undecided count after each round
//   k_p_count/fill  direct interpolation, one thread per row, entries in
//                the row's column order
//   A_c = R (A P) with the device sparse products of the smoothed-aggregation
//   setup (1x1 blocks), R = P^T; the coarsest level as an explicit inverse.
// Solve: the l1 hybrid Gauss-Seidel sweep is two kernels, the entries
// outside each row's block in parallel (a product with that part of A,
// Jacobi across blocks) and eight blocks per wave running their rows in
// order (k_hgs8, Gauss-Seidel inside), the two parts split at setup.
// Products RG lanes per row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "te_dev.h"
#include "te_thermal.h"

namespace te {
namespace {

constexpr int TB = 256;
constexpr int MAX_BLOCK = 256;
constexpr int8_t PT_F = 0, PT_U = 1, PT_C = 2;

unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TB - 1) / TB, 1 << 20)); }

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // one step of splitmix64 (Steele, Lea & Flood 2014) on input x
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// v summed over the eight lanes of each eighth of the wave, the result in
// all eight: DPP quad permutations [1,0,3,2] and [2,3,0,1], then the
// half-row mirror (lane i of the eight takes lane 7 - i, in the other quad).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double sum8(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    return v;
}

// Scalar products, RG lanes per row (coalesced loads of the row's entries,
// the partial sums of a row's lanes added by DPP steps inside the group):
//   mode 0: y = A x; 1: y = g - A x; 2: y += A x
// A lane takes its entries CU at a time: the columns and values of all CU
// are loaded, then their x, then the products are added in entry order, so
// a row of up to RG * CU entries costs two dependent loads instead of two
// per entry (absent entries read the row's first entry and add zero).
// Measured on the 4M-node disc: 8 x 4 best (4 x 8 and 16 x 2 slower).
constexpr int RG = 8, CU = 4;

__device__ __forceinline__ double sum_rg(double v) {
    static_assert(RG == 4 || RG == 8 || RG == 16, "row group of 4, 8 or 16 lanes");
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    if (RG >= 8) v += dpp_mov<0x141>(v);
    if (RG == 16) v += dpp_mov<0x140>(v);
    return v;
}

__global__ void __launch_bounds__(TB) k_csr(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                            const double *__restrict__ val, const double *__restrict__ x, double *y,
                                            const double *g, int mode) {
    const int sub = threadIdx.x % RG;
    const int64_t stride = (int64_t)gridDim.x * (TB / RG);
    // the lanes of a row share its loop trips, and sum_rg mixes only them
    for (int64_t i = blockIdx.x * (int64_t)(TB / RG) + threadIdx.x / RG; i < n; i += stride) {
        const int64_t lo = ptr[i], hi = ptr[i + 1];
        double t = 0.0;
        for (int64_t k0 = lo + sub; k0 < hi; k0 += RG * CU) {
            int c[CU];
            double v[CU], xv[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const int64_t k = k0 + u * RG;
                const int64_t kk = k < hi ? k : lo;
                c[u] = col[kk];
                v[u] = k < hi ? val[kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CU; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < CU; ++u) t += v[u] * xv[u];
        }
        t = sum_rg(t);
        if (sub == 0) {
            if (mode == 0) y[i] = t;
            else if (mode == 2) y[i] += t;
            else y[i] = g[i] - t;
        }
    }
}

// the largest value over a row group of RG lanes (exact in any order)
__device__ __forceinline__ double max_rg(double v) {
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    if (RG >= 8) v = fmax(v, dpp_mov<0x141>(v));
    if (RG == 16) v = fmax(v, dpp_mov<0x140>(v));
    return v;
}

// Ruge-Stueben strength, RG lanes per row (coalesced entry loads)
__global__ void __launch_bounds__(TB) k_strength(int64_t n, const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 double theta, uint8_t *__restrict__ S) {
    const int sub = threadIdx.x % RG;
    const int64_t stride = (int64_t)gridDim.x * (TB / RG);
    for (int64_t i = blockIdx.x * (int64_t)(TB / RG) + threadIdx.x / RG; i < n; i += stride) {
        const int64_t lo = ptr[i], hi = ptr[i + 1];
        double m = -INFINITY;
        for (int64_t k = lo + sub; k < hi; k += RG)
            if (col[k] != i) m = fmax(m, -val[k]);
        m = max_rg(m);
        for (int64_t k = lo + sub; k < hi; k += RG) S[k] = (col[k] != i && m > 0.0 && -val[k] >= theta * m) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(TB) k_infl(int64_t n, const int64_t *__restrict__ ptr,
                                             const int32_t *__restrict__ col, const uint8_t *__restrict__ S,
                                             int32_t *__restrict__ cnt) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (S[k]) atomicAdd(&cnt[col[k]], 1);
}

// Gs[k] = S[k] or S[mirror of k]; a missing mirror (pattern not symmetric)
// raises flag.  RG lanes per row.
__global__ void __launch_bounds__(TB) k_sym(int64_t n, const int64_t *__restrict__ ptr,
                                            const int32_t *__restrict__ col, const uint8_t *__restrict__ S,
                                            uint8_t *__restrict__ Gs, int32_t *__restrict__ flag) {
    const int sub = threadIdx.x % RG;
    const int64_t stride = (int64_t)gridDim.x * (TB / RG);
    for (int64_t i = blockIdx.x * (int64_t)(TB / RG) + threadIdx.x / RG; i < n; i += stride)
        for (int64_t k = ptr[i] + sub; k < ptr[i + 1]; k += RG) {
            const int32_t j = col[k];
            int64_t lo = ptr[j], hi = ptr[j + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            const bool found = lo < ptr[j + 1] && col[lo] == i;
            if (!found) *flag = 1;
            Gs[k] = (S[k] || (found && S[lo])) ? 1 : 0;
        }
}

__global__ void __launch_bounds__(TB) k_keys(int64_t n, const int32_t *__restrict__ cnt, uint64_t seed,
                                             uint64_t *__restrict__ key, int8_t *__restrict__ state) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        key[i] = ((uint64_t)cnt[i] << 40) | (mix64(seed ^ (uint64_t)i) >> 24);
        state[i] = cnt[i] > 0 ? PT_U : PT_F;
    }
}

__global__ void __launch_bounds__(TB) k_pmis_sel(int64_t n, const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col, const uint8_t *__restrict__ Gs,
                                                 const uint64_t *__restrict__ key, const int8_t *__restrict__ state,
                                                 uint8_t *__restrict__ newc) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        if (state[i] != PT_U) {
            newc[i] = 0;
            continue;
        }
        const uint64_t ki = key[i];
        bool beaten = false;
        for (int64_t k = ptr[i]; k < ptr[i + 1] && !beaten; ++k) {
            if (!Gs[k]) continue;
            const int32_t j = col[k];
            if (state[j] == PT_U && (key[j] > ki || (key[j] == ki && j > i))) beaten = true;
        }
        newc[i] = beaten ? 0 : 1;
    }
}

__global__ void __launch_bounds__(TB) k_pmis_apply(int64_t n, const int64_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const uint8_t *__restrict__ S,
                                                   const uint8_t *__restrict__ newc, int8_t *__restrict__ state,
                                                   int32_t *__restrict__ left) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        if (state[i] != PT_U) continue;
        if (newc[i]) {
            state[i] = PT_C;
            continue;
        }
        bool dep = false;
        for (int64_t k = ptr[i]; k < ptr[i + 1] && !dep; ++k) dep = S[k] && newc[col[k]];
        if (dep) state[i] = PT_F;
        else atomicAdd(left, 1);
    }
}

__global__ void __launch_bounds__(TB) k_p_count(int64_t n, const int64_t *__restrict__ ptr,
                                                const int32_t *__restrict__ col, const uint8_t *__restrict__ S,
                                                const int8_t *__restrict__ state, int32_t *__restrict__ cnt) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        if (state[i] == PT_C) {
            cnt[i] = 1;
            continue;
        }
        int c = 0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) c += (S[k] && state[col[k]] == PT_C) ? 1 : 0;
        cnt[i] = c;
    }
}

// direct interpolation: w_ij = -(alpha or beta) a_ij / a_ii over the strong C
// neighbours, alpha (beta) the ratio of the negative (positive) off-diagonal
// sums over all neighbours and over those C neighbours; without a positive C
// entry the positive entries go to the diagonal
__global__ void __launch_bounds__(TB) k_p_fill(int64_t n, const int64_t *__restrict__ ptr,
                                               const int32_t *__restrict__ col, const double *__restrict__ val,
                                               const uint8_t *__restrict__ S, const int8_t *__restrict__ state,
                                               const int32_t *__restrict__ cidx, const int64_t *__restrict__ pptr,
                                               int32_t *__restrict__ pcol, double *__restrict__ pval) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        int64_t o = pptr[i];
        if (state[i] == PT_C) {
            pcol[o] = cidx[i];
            pval[o] = 1.0;
            continue;
        }
        if (pptr[i + 1] == o) continue;
        double diag = 0.0, sn = 0.0, spp = 0.0, cn = 0.0, cp = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            const double a = val[k];
            if (j == i) {
                diag += a;
                continue;
            }
            if (a < 0.0) sn += a;
            else spp += a;
            if (S[k] && state[j] == PT_C) {
                if (a < 0.0) cn += a;
                else cp += a;
            }
        }
        if (cp == 0.0) diag += spp;
        const double alpha = cn != 0.0 ? sn / cn : 0.0, beta = cp != 0.0 ? spp / cp : 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            if (j == i || !S[k] || state[j] != PT_C) continue;
            const double a = val[k];
            pcol[o] = cidx[j];
            pval[o] = -(a < 0.0 ? alpha : beta) * a / diag;
            ++o;
        }
    }
}

// d_i = a_ii + sum over columns outside row i's block of |a_ij|
__global__ void __launch_bounds__(TB) k_dl1(int64_t n, const int64_t *__restrict__ ptr,
                                            const int32_t *__restrict__ col, const double *__restrict__ val, int B,
                                            double *__restrict__ d, int32_t *__restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        double di = 0.0, l1 = 0.0;
        const int64_t bi = i / B;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (col[k] == i) di += val[k];
            else if (col[k] / B != bi) l1 += fabs(val[k]);
        }
        d[i] = di + l1;
        if (!(di + l1 > 0.0)) *bad = 1;
    }
}

// The smoother's split of a level matrix into the entries inside each
// row's block of B consecutive rows (local column as one byte, B <= 256)
// and the entries outside it, with 1/d of the l1 diagonal: counts, then fill.
__global__ void __launch_bounds__(TB) k_split_count(int64_t n, const int64_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col, int B, int32_t *__restrict__ cin,
                                                    int32_t *__restrict__ cout) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const int64_t bi = i / B;
        int a = 0, o = 0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (col[k] / B == bi) ++a;
            else ++o;
        }
        cin[i] = a;
        cout[i] = o;
    }
}

__global__ void __launch_bounds__(TB) k_split_fill(int64_t n, const int64_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                                   int B, const double *__restrict__ dl1,
                                                   const int64_t *__restrict__ pin, uint8_t *__restrict__ lin,
                                                   double *__restrict__ vin, const int64_t *__restrict__ pout,
                                                   int32_t *__restrict__ cout, double *__restrict__ vout,
                                                   double *__restrict__ idl) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const int64_t bi = i / B;
        int64_t a = pin[i], o = pout[i];
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t c = col[k];
            if (c / B == bi) {
                lin[a] = (uint8_t)(c - bi * B);
                vin[a++] = val[k];
            } else {
                cout[o] = c;
                vout[o++] = val[k];
            }
        }
        idl[i] = 1.0 / dl1[i];
    }
}

// One l1 hybrid Gauss-Seidel sweep, eight blocks of B rows per wave: the
// eight lanes of block g run its rows in order (ascending or descending),
// each row's in-block entries eight at a time, the products summed across
// the eight lanes by sum8; the block's x and row offsets sit in LDS.  The
// row chain (LDS read, FMA, three DPP steps, LDS write) is far shorter than
// a memory latency, so the entries, o and 1/d of the next D rows are kept in
// flight in a ring of registers: row t's slot is refilled with row t + D as
// soon as row t starts.  Everything in the row loop is predicated rather
// than branched (loads of an absent entry read entry 0 and are zeroed, rows
// past the block write a spare LDS slot), so the compiler can leave the
// ring's loads outstanding across rows.  o holds g - (entries outside the
// block) x_in, or g when x_in is NULL (x_in = 0).  x_out may be x_in: a
// block reads only its own rows of x_in.  PF: entries per lane held per row
// (8 PF per row, chosen per level from its longest in-block row; TAIL: rows
// may be longer, the rest is read in the chain).  REC: each in-block entry
// comes as one 16-byte record (value, local column), one load instead of
// two, so that a ring of several long rows stays within the hardware's count
// of outstanding loads per wave (63).
template <int PF, int D, bool TAIL, bool REC>
__global__ void __launch_bounds__(64) k_hgs8(int64_t n, int B, const int64_t *__restrict__ pin,
                                             const uint8_t *__restrict__ lin, const double *__restrict__ vin,
                                             const int4 *__restrict__ rin, const double *__restrict__ idl,
                                             const double *__restrict__ o, const double *x_in, double *x_out,
                                             int forward) {
    extern __shared__ double xs[];   // [8][B + 1] x (spare last slot), then [8][B + 1] int row offsets
    const int lane = threadIdx.x, g = lane >> 3, l = lane & 7;
    const int64_t b0 = ((int64_t)blockIdx.x * 8 + g) * B;
    const int nb = b0 < n ? (int)min<int64_t>(B, n - b0) : 0;
    double *xb = xs + g * (B + 1);
    // the block's row pointers, relative to its first entry
    int *pb = reinterpret_cast<int *>(xs + 8 * (B + 1)) + g * (B + 1);
    const int64_t e0 = nb > 0 ? pin[b0] : 0;
    for (int r = l; r < nb; r += 8) xb[r] = x_in ? x_in[b0 + r] : 0.0;
    for (int r = l; r <= nb; r += 8) pb[r] = (int)(pin[b0 + r] - e0);
    __syncthreads();
    // a slot holds the raw loads of one row and the mask of its present
    // entries; nothing is computed from the loaded values until the row runs
    struct Slot {
        int64_t lo, hi;
        double v[PF], o, id;
        int c[PF];
        unsigned msk;
    };
    Slot sl[D];
    auto fetch = [&](Slot &q, int t) {
        const bool ok = t < nb;
        const int r = ok ? (forward ? t : nb - 1 - t) : 0;
        const int64_t row = ok ? b0 + r : 0;
        const int64_t lo = e0 + pb[r], hi1 = e0 + pb[r + 1];   // r + 1 <= B: inside the LDS table
        q.lo = lo;
        q.hi = ok ? hi1 : lo;
        q.msk = 0u;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int64_t k = lo + l + 8 * u;
            const bool in = k < q.hi;
            const int64_t kk = in ? k : 0;   // an absent entry reads entry 0, masked at use
            if (REC) {
                const int4 rec = rin[kk];
                q.c[u] = rec.z;
                q.v[u] = __hiloint2double(rec.y, rec.x);
            } else {
                q.c[u] = (int)lin[kk];
                q.v[u] = vin[kk];
            }
            q.msk |= (in ? 1u : 0u) << u;
        }
        q.o = o[row];   // rows past the block update the spare slot only
        q.id = idl[row];
    };
#pragma unroll
    for (int d = 0; d < D; ++d) fetch(sl[d], d);
    for (int t0 = 0; t0 < B; t0 += D) {   // the same trip count in every eighth
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int t = t0 + d;
            const Slot cur = sl[d];
            fetch(sl[d], t + D);
            if (t < B) {   // uniform
                double sum = 0.0;
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const double p = cur.v[u] * xb[cur.c[u]];
                    sum += (cur.msk >> u) & 1u ? p : 0.0;
                }
                if (TAIL)
                    for (int64_t k = cur.lo + l + 8 * PF; k < cur.hi; k += 8) sum += vin[k] * xb[lin[k]];
                sum = sum8(sum);
                // every lane of the eighth holds the same sum: all write the
                // row's new value; steps past the block write the spare slot
                const int r = t < nb ? (forward ? t : nb - 1 - t) : B;
                xb[r] = xb[r] + (cur.o - sum) * cur.id;
                __syncthreads();
            }
        }
    }
    for (int r = l; r < nb; r += 8) x_out[b0 + r] = xb[r];
}

__global__ void __launch_bounds__(TB) k_xpby(double *__restrict__ p, const double *__restrict__ z, double beta,
                                             int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(TB) k_neg(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) y[i] = -x[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct CLv {
    int64_t n = 0;
    DBsr A, P, R;                 // 1x1 blocks
    DBuf<double> dl1;
    // smoother split of A: entries inside the row's block (local column, one
    // byte) and outside it, and 1 / l1 diagonal
    DBuf<int64_t> pin, pout;
    DBuf<uint8_t> lin;
    DBuf<int32_t> cout;
    DBuf<double> vin, vout, idl;
    DBuf<int4> rin;               // in-block entries as 16-byte records (levels with long rows)
    int max_in = 0;               // longest in-block row
    DBuf<int8_t> state;
    DBuf<double> g, x, s, o, t;   // work vectors
};

}  // namespace te

struct camg_handle {
    camg_options opt{};
    std::vector<te::CLv> L;
    te::DBuf<double> Ainv;
    int nc = 0;
    te::DBuf<double> r, z, p, q, t, part, red;  // CG workspace (level-0 size)
    double setup_ms = 0.0;
};

namespace te {
namespace {

unsigned grid_rows(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TB / RG - 1) / (TB / RG), 1 << 20));
}

void csr_apply(const DBsr &A, const double *x, double *y, const double *g, int mode, hipStream_t s) {
    if (A.nr == 0) return;
    hipLaunchKernelGGL(k_csr, dim3(grid_rows(A.nr)), dim3(TB), 0, s, A.nr, A.ptr, A.col, A.val, x, y, g, mode);
    TE_CHECK_HIP(hipGetLastError());
}

double dev_norm(camg_handle *h, const double *a, const double *b, int64_t n, hipStream_t s) {
    dot_partials(a, b, n, 1, h->part.p, s);
    reduce_partials(h->part.p, dot_nblocks(n), 1, h->red.p, s);
    double v = 0.0;
    TE_CHECK_HIP(hipMemcpyAsync(&v, h->red.p, sizeof(double), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return v;
}

int32_t read_i32(const DBuf<int32_t> &d, hipStream_t s) {
    int32_t v = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&v, d.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return v;
}

// one l1 hybrid Gauss-Seidel sweep for A z = g from z = x_in (NULL: zero)
void sweep(camg_handle *h, CLv &L, const double *g, const double *x_in, double *x_out, bool forward, hipStream_t s) {
    const int B = h->opt.block;
    const double *o = g;
    if (x_in) {
        // o = g - (entries outside the blocks) x_in
        hipLaunchKernelGGL(k_csr, dim3(grid_rows(L.n)), dim3(TB), 0, s, L.n, L.pout.p, L.cout.p, L.vout.p, x_in,
                           L.o.p, g, 1);
        o = L.o.p;
    }
    const int64_t nblk = (L.n + B - 1) / B;
    const unsigned grid = (unsigned)((nblk + 7) / 8);
    auto go = [&](auto kern) {
        const size_t lds = (size_t)8 * (B + 1) * (sizeof(double) + sizeof(int));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, s, L.n, B, L.pin.p, L.lin.p, L.vin.p, L.rin.p, L.idl.p, o,
                           x_in, x_out, forward ? 1 : 0);
    };
    // a level of fewer waves than SIMDs has no other waves to hide the loads
    // behind: a deeper ring there (more registers, one wave per SIMD anyway).  The ring's depth is capped by the hardware's count of
    // outstanding loads per wave (63): a row issues PF + 2 loads per lane
    // with records (levels whose rows exceed 24 in-block entries), 2 PF + 2
    // with the byte columns and values apart.
    const bool deep = grid < 1024;
    if (L.max_in <= 24) deep ? go(k_hgs8<3, 8, false, false>) : go(k_hgs8<3, 4, false, false>);
    else if (L.max_in <= 64) deep ? go(k_hgs8<8, 6, false, true>) : go(k_hgs8<8, 4, false, true>);
    else if (L.max_in <= 128) go(k_hgs8<16, 3, false, true>);
    else go(k_hgs8<16, 3, true, true>);
    TE_CHECK_HIP(hipGetLastError());
}

void vcycle(camg_handle *h, size_t l, const double *g, double *x, hipStream_t s) {
    if (l + 1 == h->L.size()) {
        dense_mv<double>(h->Ainv.p, g, x, h->nc, 1, s);
        return;
    }
    CLv &L = h->L[l];
    CLv &N = h->L[l + 1];
    sweep(h, L, g, nullptr, x, true, s);
    csr_apply(L.A, x, L.s.p, g, 1, s);
    csr_apply(L.R, L.s.p, N.g.p, nullptr, 0, s);
    vcycle(h, l + 1, N.g.p, N.x.p, s);
    csr_apply(L.P, N.x.p, x, nullptr, 2, s);
    sweep(h, L, g, x, x, false, s);
}

void copy_csr(const te_csr *A, DBsr &M, hipStream_t s) {
    M.release();
    M.br = M.bc = 1;
    M.nr = M.nc = A->n_rows;
    M.nnzb = A->nnz;
    M.ptr_own.alloc(A->n_rows + 1);
    M.col_own.alloc(std::max<int64_t>(A->nnz, 1));
    M.val_own.alloc(std::max<int64_t>(A->nnz, 1));
    M.bind();
    TE_CHECK_HIP(hipMemcpyAsync(M.ptr_own.p, A->row_ptr, (A->n_rows + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (A->nnz) {
        TE_CHECK_HIP(hipMemcpyAsync(M.col_own.p, A->col_idx, A->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        TE_CHECK_HIP(hipMemcpyAsync(M.val_own.p, A->val, A->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
}

void check_csr(const te_csr *A) {
    TE_REQUIRE(A && A->row_ptr && A->col_idx && A->val, TE_EINVAL, "matrix or its arrays are NULL");
    TE_REQUIRE(A->n_rows > 0 && A->n_rows < (int64_t)INT32_MAX && A->nnz >= A->n_rows, TE_EINVAL,
               "bad matrix size (%lld rows, %lld entries)", (long long)A->n_rows, (long long)A->nnz);
}

// explicit inverse by Gauss-Jordan with partial pivoting (host, small n)
bool host_inverse(std::vector<double> M, int n, std::vector<double> &inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)piv * n + c])) piv = r;
        if (!(std::fabs(M[(size_t)piv * n + c]) > 0.0)) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(M[(size_t)c * n + k], M[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        const double d = M[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            M[(size_t)c * n + k] /= d;
            inv[(size_t)c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = M[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                M[(size_t)r * n + k] -= f * M[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return true;
}

// the records of the in-block entries: {value low word, value high word, local column, 0}
__global__ void __launch_bounds__(TB) k_split_rec(int64_t m, const uint8_t *__restrict__ lin,
                                                  const double *__restrict__ vin, int4 *__restrict__ rin) {
    for (int64_t a = blockIdx.x * (int64_t)TB + threadIdx.x; a < m; a += (int64_t)gridDim.x * TB)
        rin[a] = make_int4(__double2loint(vin[a]), __double2hiint(vin[a]), (int)lin[a], 0);
}

void split_level(CLv &L, int B, hipStream_t s) {
    const int64_t n = L.n;
    DBuf<int32_t> ci(n), co(n);
    hipLaunchKernelGGL(k_split_count, dim3(grid1(n)), dim3(TB), 0, s, n, L.A.ptr, L.A.col, B, ci.p, co.p);
    TE_CHECK_HIP(hipGetLastError());
    std::vector<int32_t> hi_, ho_;
    download(hi_, ci.p, (size_t)n, s);
    download(ho_, co.p, (size_t)n, s);
    std::vector<int64_t> pi(n + 1, 0), po(n + 1, 0);
    L.max_in = 0;
    for (int64_t i = 0; i < n; ++i) {
        pi[i + 1] = pi[i] + hi_[i];
        po[i + 1] = po[i] + ho_[i];
        L.max_in = std::max(L.max_in, hi_[i]);
    }
    upload(L.pin, pi, s);
    upload(L.pout, po, s);
    L.lin.alloc(std::max<int64_t>(pi[n], 1));
    L.vin.alloc(std::max<int64_t>(pi[n], 1));
    L.cout.alloc(std::max<int64_t>(po[n], 1));
    L.vout.alloc(std::max<int64_t>(po[n], 1));
    L.idl.alloc(n);
    hipLaunchKernelGGL(k_split_fill, dim3(grid1(n)), dim3(TB), 0, s, n, L.A.ptr, L.A.col, L.A.val, B, L.dl1.p,
                       L.pin.p, L.lin.p, L.vin.p, L.pout.p, L.cout.p, L.vout.p, L.idl.p);
    TE_CHECK_HIP(hipGetLastError());
    if (L.max_in > 24 && pi[n] > 0) {   // the sweeps of this level read records
        L.rin.alloc(pi[n]);
        hipLaunchKernelGGL(k_split_rec, dim3(grid1(pi[n])), dim3(TB), 0, s, pi[n], L.lin.p, L.vin.p, L.rin.p);
        TE_CHECK_HIP(hipGetLastError());
    }
}

void alloc_work(CLv &L) {
    L.g.alloc(std::max<int64_t>(L.n, 1));
    L.x.alloc(std::max<int64_t>(L.n, 1));
    L.s.alloc(std::max<int64_t>(L.n, 1));
    L.o.alloc(std::max<int64_t>(L.n, 1));
    L.t.alloc(std::max<int64_t>(L.n, 1));
}

// the C/F splitting and interpolation of level l; false if nothing coarsens
bool coarsen(camg_handle *h, size_t l, hipStream_t s) {
    CLv &L = h->L[l];
    const DBsr &A = L.A;
    const int64_t n = L.n;
    const unsigned g = grid1(n);
    DBuf<uint8_t> S(std::max<int64_t>(A.nnzb, 1)), Gs(std::max<int64_t>(A.nnzb, 1)), newc(n);
    DBuf<int32_t> cnt(n), flag(1), left(1);
    DBuf<uint64_t> key(n);
    L.state.alloc(n);
    hipLaunchKernelGGL(k_strength, dim3(grid_rows(n)), dim3(TB), 0, s, n, A.ptr, A.col, A.val, h->opt.theta, S.p);
    TE_CHECK_HIP(hipMemsetAsync(cnt.p, 0, n * sizeof(int32_t), s));
    TE_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_infl, dim3(g), dim3(TB), 0, s, n, A.ptr, A.col, S.p, cnt.p);
    hipLaunchKernelGGL(k_sym, dim3(grid_rows(n)), dim3(TB), 0, s, n, A.ptr, A.col, S.p, Gs.p, flag.p);
    hipLaunchKernelGGL(k_keys, dim3(g), dim3(TB), 0, s, n, cnt.p, (uint64_t)(0xC1A5 + l), key.p, L.state.p);
    TE_CHECK_HIP(hipGetLastError());
    TE_REQUIRE(read_i32(flag, s) == 0, TE_EINVAL, "classical AMG needs a symmetric pattern (level %d)", (int)l);
    // every round makes the undecided point of largest key C, so at most n rounds
    for (int64_t round = 0; round < n; ++round) {
        TE_CHECK_HIP(hipMemsetAsync(left.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_pmis_sel, dim3(g), dim3(TB), 0, s, n, A.ptr, A.col, Gs.p, key.p, L.state.p, newc.p);
        hipLaunchKernelGGL(k_pmis_apply, dim3(g), dim3(TB), 0, s, n, A.ptr, A.col, S.p, newc.p, L.state.p, left.p);
        TE_CHECK_HIP(hipGetLastError());
        if (read_i32(left, s) == 0) break;
    }
    std::vector<int8_t> st;
    download(st, L.state.p, (size_t)n, s);
    std::vector<int32_t> cidx(n, -1);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i)
        if (st[i] == PT_C) cidx[i] = nc++;
    if (nc == 0 || (double)nc > h->opt.max_coarse_ratio * (double)n) return false;
    DBuf<int32_t> dcidx;
    upload(dcidx, cidx, s);
    hipLaunchKernelGGL(k_p_count, dim3(g), dim3(TB), 0, s, n, A.ptr, A.col, S.p, L.state.p, cnt.p);
    TE_CHECK_HIP(hipGetLastError());
    std::vector<int32_t> hc;
    download(hc, cnt.p, (size_t)n, s);
    std::vector<int64_t> pp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) pp[i + 1] = pp[i] + hc[i];
    DBsr &P = L.P;
    P.release();
    P.br = P.bc = 1;
    P.nr = n;
    P.nc = nc;
    P.nnzb = pp[n];
    upload(P.ptr_own, pp, s);
    P.col_own.alloc(std::max<int64_t>(P.nnzb, 1));
    P.val_own.alloc(std::max<int64_t>(P.nnzb, 1));
    P.bind();
    hipLaunchKernelGGL(k_p_fill, dim3(g), dim3(TB), 0, s, n, A.ptr, A.col, A.val, S.p, L.state.p, dcidx.p, P.ptr,
                       P.col_own.p, P.val_own.p);
    TE_CHECK_HIP(hipGetLastError());
    dev_transpose(P, L.R, s);
    DBsr AP;
    dev_mult(A, P, AP, s);
    h->L.emplace_back();
    CLv &N = h->L.back();  // L may have moved: use h->L[l] below
    dev_mult(h->L[l].R, AP, N.A, s);
    N.n = nc;
    return true;
}

int setup_impl(const te_csr *A, const camg_options *o, camg_handle **out, hipStream_t s) {
    TE_REQUIRE(out, TE_EINVAL, "out is NULL");
    check_csr(A);
    auto t0 = std::chrono::steady_clock::now();
    camg_handle *h = new camg_handle;
    try {
        camg_options_default(&h->opt);
        if (o) h->opt = *o;
        TE_REQUIRE(h->opt.block >= 1 && h->opt.block <= MAX_BLOCK, TE_EINVAL, "block must be in 1..%d", MAX_BLOCK);
        TE_REQUIRE(h->opt.max_levels >= 1 && h->opt.max_levels <= 16 && h->opt.coarse_max >= 1, TE_EINVAL,
                   "bad level limits");
        TE_REQUIRE(h->opt.theta > 0.0 && h->opt.theta < 1.0, TE_EINVAL, "theta must be in (0, 1)");
        {
            const int64_t i = dev_check_pattern(A->row_ptr, A->col_idx, A->n_rows, s);
            TE_REQUIRE(i < 0, TE_EINVAL,
                       "row %lld has a column out of range or out of ascending order, or no diagonal", (long long)i);
        }
        h->L.reserve(16);
        h->L.emplace_back();
        h->L[0].n = A->n_rows;
        copy_csr(A, h->L[0].A, s);
        for (size_t l = 0;; ++l) {
            const int64_t n = h->L[l].n;
            if (n <= h->opt.coarse_max || (int)l + 1 >= h->opt.max_levels) break;
            if (!coarsen(h, l, s)) break;
        }
        // coarsest level: explicit inverse
        CLv &C = h->L.back();
        C.P.release();
        C.R.release();
        TE_REQUIRE(C.n <= 8192, TE_ENOMEM, "coarsest level of %lld rows is too large for a dense inverse",
                   (long long)C.n);
        HBsr hc;
        dev_to_host(C.A, hc, s);
        const int nc = (int)C.n;
        std::vector<double> dense((size_t)nc * nc, 0.0), inv;
        for (int64_t i = 0; i < nc; ++i)
            for (int64_t k = hc.ptr[i]; k < hc.ptr[i + 1]; ++k) dense[(size_t)i * nc + hc.col[k]] += hc.val[k];
        TE_REQUIRE(host_inverse(dense, nc, inv), TE_ECHOL, "the coarsest level (%d rows) is singular", nc);
        upload(h->Ainv, inv, s);
        h->nc = nc;
        for (size_t l = 0; l < h->L.size(); ++l) {
            CLv &L = h->L[l];
            alloc_work(L);
            if (l + 1 < h->L.size()) {
                DBuf<int32_t> bad(1);
                TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
                L.dl1.alloc(L.n);
                hipLaunchKernelGGL(k_dl1, dim3(grid1(L.n)), dim3(TB), 0, s, L.n, L.A.ptr, L.A.col, L.A.val,
                                   h->opt.block, L.dl1.p, bad.p);
                TE_CHECK_HIP(hipGetLastError());
                TE_REQUIRE(read_i32(bad, s) == 0, TE_EINVAL, "level %d has a row with a non-positive l1 diagonal",
                           (int)l);
                split_level(L, h->opt.block, s);
            }
        }
        const int64_t n0 = h->L[0].n;
        h->r.alloc(n0);
        h->z.alloc(n0);
        h->p.alloc(n0);
        h->q.alloc(n0);
        h->t.alloc(n0);
        h->part.alloc((size_t)dot_nblocks(n0) + 1024);
        h->red.alloc(4);
        TE_CHECK_HIP(hipStreamSynchronize(s));
    } catch (...) {
        delete h;
        throw;
    }
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return TE_OK;
}

// PCG (Saad Alg. 9.1) on A with the V-cycle; stop as amg_pcg_solve
int pcg_impl(camg_handle *h, const te_csr *A, const double *b, double *x, double rtol, int maxit, int32_t *iters,
             double *relres, hipStream_t s) {
    TE_REQUIRE(h && b && x, TE_EINVAL, "NULL argument");
    check_csr(A);
    const int64_t n = h->L[0].n;
    TE_REQUIRE(A->n_rows == n, TE_EINVAL, "matrix has %lld rows, the hierarchy %lld", (long long)A->n_rows,
               (long long)n);
    TE_REQUIRE(rtol > 0.0 && maxit >= 0, TE_EINVAL, "need rtol > 0 and maxit >= 0");
    DBsr Av;  // view of the caller's matrix
    Av.br = Av.bc = 1;
    Av.nr = Av.nc = n;
    Av.nnzb = A->nnz;
    Av.ptr = A->row_ptr;
    Av.col = A->col_idx;
    Av.val = A->val;
    const unsigned g = grid1(n);
    auto done = [&](int it, double rel, int code) {
        if (iters) *iters = it;
        if (relres) *relres = rel;
        return code;
    };
    const double bn = std::sqrt(dev_norm(h, b, b, n, s));
    TE_REQUIRE(std::isfinite(bn), TE_ENAN, "NaN or Inf in the right-hand side");
    if (bn == 0.0) {
        TE_CHECK_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        return done(0, 0.0, TE_OK);
    }
    csr_apply(Av, x, h->r.p, b, 1, s);
    double rn = std::sqrt(dev_norm(h, h->r.p, h->r.p, n, s)) / bn;
    TE_REQUIRE(std::isfinite(rn), TE_ENAN, "NaN or Inf in the residual");
    if (rn <= rtol) return done(0, rn, TE_OK);
    vcycle(h, 0, h->r.p, h->z.p, s);
    double rz = dev_norm(h, h->r.p, h->z.p, n, s);
    TE_REQUIRE(rz > 0.0, TE_EINDEF, "CG breakdown: (r, z) <= 0");
    TE_CHECK_HIP(hipMemcpyAsync(h->p.p, h->z.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int replaced = 0;
    for (int it = 0; it < maxit;) {
        csr_apply(Av, h->p.p, h->q.p, nullptr, 0, s);
        const double pq = dev_norm(h, h->p.p, h->q.p, n, s);
        TE_REQUIRE(pq > 0.0, TE_EINDEF, "CG breakdown: (p, Ap) <= 0");
        const double alpha = rz / pq;
        axpy<double>(x, h->p.p, alpha, n, s);
        axpy<double>(h->r.p, h->q.p, -alpha, n, s);
        ++it;
        rn = std::sqrt(dev_norm(h, h->r.p, h->r.p, n, s)) / bn;
        TE_REQUIRE(std::isfinite(rn), TE_ENAN, "NaN or Inf in the residual");
        if (rn <= rtol) {
            csr_apply(Av, x, h->t.p, b, 1, s);
            const double rt = std::sqrt(dev_norm(h, h->t.p, h->t.p, n, s)) / bn;
            if (rt <= rtol) return done(it, rt, TE_OK);
            if (replaced >= 3) return done(it, rt, TE_ENOTCONV);
            ++replaced;
            TE_CHECK_HIP(hipMemcpyAsync(h->r.p, h->t.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        vcycle(h, 0, h->r.p, h->z.p, s);
        const double rz_new = dev_norm(h, h->r.p, h->z.p, n, s);
        TE_REQUIRE(rz_new > 0.0, TE_EINDEF, "CG breakdown: (r, z) <= 0");
        hipLaunchKernelGGL(k_xpby, dim3(g), dim3(TB), 0, s, h->p.p, h->z.p, rz_new / rz, n);
        TE_CHECK_HIP(hipGetLastError());
        rz = rz_new;
    }
    csr_apply(Av, x, h->t.p, b, 1, s);
    const double rt = std::sqrt(dev_norm(h, h->t.p, h->t.p, n, s)) / bn;
    return done(maxit, rt, TE_ENOTCONV);
}

}  // namespace
}  // namespace te

struct thermal_solver {
    te::ThermalAsm ta;
    te::DBuf<double> Jval, F, rhs, d, part, red;
    camg_handle *amg = nullptr;
    int base_iters = -1;
    bool stale = true;
    ~thermal_solver() {
        if (amg) delete amg;
    }
};

using namespace te;

extern "C" void camg_options_default(camg_options *o) {
    if (!o) return;
    o->theta = 0.25;
    o->coarse_max = 500;
    o->max_levels = 10;
    o->max_coarse_ratio = 0.9;
    o->block = 128;
}

extern "C" void newton_options_default(newton_options *o) {
    if (!o) return;
    o->rtol = 1e-9;
    o->atol = 1e-8;
    o->lin_rtol = 1e-8;
    o->maxit = 25;
    o->lin_maxit = 500;
    o->rebuild_factor = 1.5;
    camg_options_default(&o->amg);
}

extern "C" int camg_setup(const te_csr *A, const camg_options *opt, camg_handle **out, hipStream_t stream) {
    return guarded([&] { return setup_impl(A, opt, out, stream); });
}

extern "C" int camg_destroy(camg_handle *h) {
    delete h;
    return TE_OK;
}

extern "C" int camg_get_info(const camg_handle *h, camg_info *info) {
    return guarded([&]() -> int {
        TE_REQUIRE(h && info, TE_EINVAL, "NULL argument");
        *info = camg_info{};
        info->n_levels = (int32_t)h->L.size();
        for (size_t l = 0; l < h->L.size() && l < 16; ++l) {
            info->n_rows[l] = h->L[l].n;
            info->nnz[l] = h->L[l].A.nnzb;
            info->p_nnz[l] = h->L[l].P.nnzb;
        }
        info->setup_ms = h->setup_ms;
        return TE_OK;
    });
}

extern "C" int camg_get_splitting(const camg_handle *h, int32_t level, int8_t *state_host) {
    return guarded([&]() -> int {
        TE_REQUIRE(h && state_host, TE_EINVAL, "NULL argument");
        TE_REQUIRE(level >= 0 && level + 1 < (int)h->L.size(), TE_EINVAL, "level %d has no splitting", level);
        const CLv &L = h->L[level];
        TE_CHECK_HIP(hipMemcpy(state_host, L.state.p, L.n, hipMemcpyDeviceToHost));
        return TE_OK;
    });
}

extern "C" int camg_get_level_matrix(const camg_handle *h, int32_t level, int32_t which, int64_t *n_rows_out,
                                     int64_t *nnz_out, int64_t *row_ptr, int32_t *col, double *val) {
    return guarded([&]() -> int {
        TE_REQUIRE(h, TE_EINVAL, "NULL handle");
        TE_REQUIRE(level >= 0 && level < (int)h->L.size(), TE_EINVAL, "level %d out of range", level);
        TE_REQUIRE(which >= 0 && which <= 2, TE_EINVAL, "which must be 0, 1 or 2");
        TE_REQUIRE(which == 0 || level + 1 < (int)h->L.size(), TE_EINVAL, "the coarsest level has no P or R");
        const CLv &L = h->L[level];
        const DBsr &M = which == 0 ? L.A : (which == 1 ? L.P : L.R);
        if (n_rows_out) *n_rows_out = M.nr;
        if (nnz_out) *nnz_out = M.nnzb;
        if (row_ptr) TE_CHECK_HIP(hipMemcpy(row_ptr, M.ptr, (M.nr + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (col && M.nnzb) TE_CHECK_HIP(hipMemcpy(col, M.col, M.nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (val && M.nnzb) TE_CHECK_HIP(hipMemcpy(val, M.val, M.nnzb * sizeof(double), hipMemcpyDeviceToHost));
        return TE_OK;
    });
}

extern "C" int camg_apply(camg_handle *h, int32_t level, int32_t op, const double *x, double *y,
                          hipStream_t stream) {
    return guarded([&]() -> int {
        TE_REQUIRE(h && x && y, TE_EINVAL, "NULL argument");
        TE_REQUIRE(level >= 0 && level < (int)h->L.size(), TE_EINVAL, "level %d out of range", level);
        const bool last = level + 1 == (int)h->L.size();
        CLv &L = h->L[level];
        switch (op) {
            case TE_CAMG_A: csr_apply(L.A, x, y, nullptr, 0, stream); break;
            case TE_CAMG_P:
                TE_REQUIRE(!last, TE_EINVAL, "the coarsest level has no P");
                csr_apply(L.P, x, y, nullptr, 0, stream);
                break;
            case TE_CAMG_R:
                TE_REQUIRE(!last, TE_EINVAL, "the coarsest level has no R");
                csr_apply(L.R, x, y, nullptr, 0, stream);
                break;
            case TE_CAMG_VCYCLE: vcycle(h, (size_t)level, x, y, stream); break;
            case TE_CAMG_SWEEP_FWD:
            case TE_CAMG_SWEEP_BWD:
                TE_REQUIRE(!last, TE_EINVAL, "the coarsest level has no smoother");
                sweep(h, L, x, y, L.t.p, op == TE_CAMG_SWEEP_FWD, stream);
                TE_CHECK_HIP(hipMemcpyAsync(y, L.t.p, L.n * sizeof(double), hipMemcpyDeviceToDevice, stream));
                break;
            default: TE_REQUIRE(false, TE_EINVAL, "unknown operation %d", op);
        }
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

extern "C" int camg_pcg_solve(camg_handle *h, const te_csr *A, const double *b, double *x, double rtol,
                              int32_t maxit, int32_t *iters, double *relres, hipStream_t stream) {
    return guarded([&] { return pcg_impl(h, A, b, x, rtol, maxit, iters, relres, stream); });
}

extern "C" int fe_assemble_thermal(const te_mesh *mesh, const te_thermal_tables *tab, const int32_t *cell_material,
                                   const te_robin *robin, const double *T, const double *T_old, double dt, te_csr *J,
                                   double *F, hipStream_t stream) {
    return guarded([&]() -> int {
        TE_REQUIRE(T && F && J && J->row_ptr && J->col_idx && J->val, TE_EINVAL, "NULL array argument");
        TE_REQUIRE(mesh && J->n_rows == mesh->n_nodes, TE_EINVAL, "J.n_rows != n_nodes");
        TE_REQUIRE(T_old == nullptr || dt > 0.0, TE_EINVAL, "a transient step needs dt > 0");
        ThermalAsm ta;
        thermal_asm_init(ta, mesh, tab, cell_material, robin, stream);
        TE_REQUIRE(ta.nnz == J->nnz, TE_EINVAL, "J.nnz (%lld) != the mesh's pattern (%lld)", (long long)J->nnz,
                   (long long)ta.nnz);
        TE_CHECK_HIP(hipMemcpyAsync(J->row_ptr, ta.ptr.p, (ta.n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                                    stream));
        TE_CHECK_HIP(hipMemcpyAsync(J->col_idx, ta.col.p, ta.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
        thermal_asm_run(ta, T, T_old, dt, J->val, F, stream);
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

extern "C" int thermal_create(const te_mesh *mesh, const te_thermal_tables *tab, const int32_t *cell_material,
                              const te_robin *robin, thermal_solver **out, hipStream_t stream) {
    return guarded([&]() -> int {
        TE_REQUIRE(out, TE_EINVAL, "out is NULL");
        thermal_solver *ts = new thermal_solver;
        try {
            thermal_asm_init(ts->ta, mesh, tab, cell_material, robin, stream);
            ts->Jval.alloc(std::max<int64_t>(ts->ta.nnz, 1));
            ts->F.alloc(ts->ta.n);
            ts->rhs.alloc(ts->ta.n);
            ts->d.alloc(ts->ta.n);
            ts->part.alloc((size_t)dot_nblocks(ts->ta.n) + 1024);
            ts->red.alloc(4);
            TE_CHECK_HIP(hipStreamSynchronize(stream));
        } catch (...) {
            delete ts;
            throw;
        }
        *out = ts;
        return TE_OK;
    });
}

extern "C" int thermal_set_exterior(thermal_solver *ts, const double *T_bc, hipStream_t stream) {
    return guarded([&]() -> int {
        TE_REQUIRE(ts, TE_EINVAL, "NULL solver");
        if (ts->ta.n_faces == 0) return TE_OK;
        TE_REQUIRE(T_bc, TE_EINVAL, "T_bc is NULL");
        TE_CHECK_HIP(hipMemcpyAsync(ts->ta.T_bc.p, T_bc, ts->ta.n_faces * sizeof(double), hipMemcpyDeviceToDevice,
                                    stream));
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

extern "C" int thermal_reset_preconditioner(thermal_solver *ts) {
    return guarded([&]() -> int {
        TE_REQUIRE(ts, TE_EINVAL, "NULL solver");
        delete ts->amg;
        ts->amg = nullptr;
        ts->base_iters = -1;
        ts->stale = true;
        return TE_OK;
    });
}

extern "C" int thermal_newton(thermal_solver *ts, double *T, const double *T_old, double dt,
                              const newton_options *opt, newton_report *rep, hipStream_t stream) {
    return guarded([&]() -> int {
        TE_REQUIRE(ts && T, TE_EINVAL, "NULL argument");
        TE_REQUIRE(T_old == nullptr || dt > 0.0, TE_EINVAL, "a transient step needs dt > 0");
        newton_options o;
        newton_options_default(&o);
        if (opt) o = *opt;
        TE_REQUIRE(o.rtol > 0.0 && o.atol >= 0.0 && o.lin_rtol > 0.0 && o.maxit >= 0 && o.maxit <= 32 && o.lin_maxit >= 1 &&
                       o.rebuild_factor >= 1.0,
                   TE_EINVAL, "bad Newton options");
        auto t0 = std::chrono::steady_clock::now();
        newton_report r{};
        const ThermalAsm &ta = ts->ta;
        const int64_t n = ta.n;
        te_csr J{n, ta.nnz, ta.ptr.p, ta.col.p, ts->Jval.p};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        struct Ev {
            hipEvent_t *a, *b;
            ~Ev() {
                if (*a) (void)hipEventDestroy(*a);
                if (*b) (void)hipEventDestroy(*b);
            }
        } ev{&e0, &e1};
        TE_CHECK_HIP(hipEventCreate(&e0));
        TE_CHECK_HIP(hipEventCreate(&e1));
        auto timed = [&](double &acc, auto &&f) {
            TE_CHECK_HIP(hipEventRecord(e0, stream));
            f();
            TE_CHECK_HIP(hipEventRecord(e1, stream));
            TE_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            acc += ms;
        };
        int code = TE_OK;
        double f0 = 0.0;
        for (int k = 0;; ++k) {
            timed(r.assembly_ms, [&] { thermal_asm_run(ta, T, T_old, dt, ts->Jval.p, ts->F.p, stream); });
            double fsq = 0.0;
            dot_partials(ts->F.p, ts->F.p, n, 1, ts->part.p, stream);
            reduce_partials(ts->part.p, dot_nblocks(n), 1, ts->red.p, stream);
            TE_CHECK_HIP(hipMemcpyAsync(&fsq, ts->red.p, sizeof(double), hipMemcpyDeviceToHost, stream));
            TE_CHECK_HIP(hipStreamSynchronize(stream));
            const double f = std::sqrt(fsq);
            TE_REQUIRE(std::isfinite(f), TE_ENAN, "NaN or Inf in the thermal residual");
            if (k == 0) f0 = f;
            r.res_hist[k] = f;
            r.res = f;
            if (f <= std::max(o.rtol * f0, o.atol) || f0 == 0.0) {
                r.converged = 1;
                break;
            }
            if (k == o.maxit) {
                code = TE_ENOTCONV;
                break;
            }
            if (!ts->amg || ts->stale) {
                delete ts->amg;
                ts->amg = nullptr;
                timed(r.setup_ms, [&] { setup_impl(&J, &o.amg, &ts->amg, stream); });
                ts->base_iters = -1;
                ts->stale = false;
                ++r.rebuilds;
            }
            hipLaunchKernelGGL(k_neg, dim3(grid1(n)), dim3(TB), 0, stream, ts->F.p, ts->rhs.p, n);
            TE_CHECK_HIP(hipGetLastError());
            TE_CHECK_HIP(hipMemsetAsync(ts->d.p, 0, n * sizeof(double), stream));
            int32_t it = 0;
            double rel = 0.0;
            int c = TE_OK;
            timed(r.solve_ms, [&] { c = pcg_impl(ts->amg, &J, ts->rhs.p, ts->d.p, o.lin_rtol, o.lin_maxit, &it, &rel,
                                                 stream); });
            if (c == TE_ENOTCONV) code = TE_ENOTCONV;
            r.lin_iters[k] = it;
            r.lin_iters_total += it;
            if (ts->base_iters < 0) ts->base_iters = it;
            else if ((double)it > o.rebuild_factor * (double)ts->base_iters) ts->stale = true;
            axpy<double>(T, ts->d.p, 1.0, n, stream);
            r.iters = k + 1;
        }
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        r.res0 = f0;
        r.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rep) *rep = r;
        return code;
    });
}

extern "C" int thermal_destroy(thermal_solver *ts) {
    delete ts;
    return TE_OK;
}
