// Kernels of block conjugate gradients over the columns of a multi-RHS solve
// (O'Leary 1980; the driver is in te_solve.cpp).  Block vectors are the
// solve's [rows][m] arrays (right-hand sides fastest, m <= 64); small matrices
// are 64 x 64 row-major with zero padding.
//
// The three kernels are tall-skinny dense contractions done with plain
// float64 vector FMAs (no matrix cores), register-tiled like a GEMM:
//
//   k_gram      C_t = L_t^T R_t for up to three pairs of block vectors in one
//               pass over the rows, one wave per pair.  The workgroup stages
//               32 block rows of each distinct block vector in LDS (coalesced
//               loads); lane (a, b) accumulates the 8 x 8 tile
//               C[8a..8a+7][8b..8b+7] from them (64 FMAs per 16 LDS values).
//               One partial per workgroup, summed in workgroup order
//               (k_gram_sum1/2: deterministic).
//   k_block_xr  X += P alpha, R -= Q alpha, plus per-column partial sums of
//               R^2.  A wave computes 32 block rows x 64 columns: lane (a, b)
//               the 4 x 8 tile of rows 4a.. and columns 8b..; the row entries
//               come from global memory four at a time (the next four loaded
//               while the current ones are used), alpha from LDS.
//   k_block_p   P <- Z T1 + P T2 in place, organised as k_block_xr (a wave
//               reads its 32 rows of Z and P whole before it writes them).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "te_dev.h"

namespace te {
namespace {

constexpr int GM = 64;      // largest block size
constexpr int GBLKS = 1024; // workgroups of the Gram pass
constexpr int GSPLIT = 16;  // first-stage slices of the Gram partial sum
constexpr int GT = 32;      // block rows per LDS stage of the Gram pass
constexpr int UBLK = 256;   // threads of the update kernels (4 waves)
constexpr int TRW = 32;     // block rows per wave in the updates
constexpr int KB = 4;       // row entries per load batch in the updates

struct GramArgs {
    const double *mat[3];   // distinct block vectors [rows][m]
    int nmat;
    int li[3], ri[3];       // pair t: mat[li[t]]^T mat[ri[t]]
    int npair;
    int64_t rows;
    int m;
    double *partials;       // [GBLKS][npair][GM][GM]
};

// blockDim = 64 * npair: wave p computes pair p over the workgroup's rows.
__global__ void __launch_bounds__(192) k_gram(GramArgs g) {
    __shared__ double tile[3][GT][GM];
    const int lane = threadIdx.x & (WAVE - 1), p = threadIdx.x / WAVE;
    const int ta = (lane >> 3) * 8, tb = (lane & 7) * 8;
    const int m = g.m, nmat = g.nmat;
    const int lm = g.li[p], rm = g.ri[p];
    double acc[8][8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[q][t] = 0.0;
    const int64_t chunk = (g.rows + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(g.rows, lo + chunk);
    for (int64_t r0 = lo; r0 < hi; r0 += GT) {
        const int nr = (int)min<int64_t>(GT, hi - r0);
        // stage rows r0 .. r0+nr-1 of every distinct block vector (zero beyond
        // m and nr); the rows are contiguous in memory
        for (int t = 0; t < nmat; ++t) {
            const double *__restrict__ src = g.mat[t] + r0 * m;
            for (int e = threadIdx.x; e < GT * GM; e += blockDim.x) {
                const int rr = e / GM, c = e % GM;
                tile[t][rr][c] = (rr < nr && c < m) ? src[rr * m + c] : 0.0;
            }
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            double l[8], r[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                l[q] = tile[lm][rr][ta + q];
                r[q] = tile[rm][rr][tb + q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int t = 0; t < 8; ++t) acc[q][t] = fma(l[q], r[t], acc[q][t]);
        }
        __syncthreads();
    }
    double *out = g.partials + ((int64_t)blockIdx.x * g.npair + p) * GM * GM;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < 8; ++t) out[(ta + q) * GM + tb + t] = acc[q][t];
}

// Partial sums over the GBLKS workgroups in a fixed order: slice y of the
// workgroups into out2[y], then the GSPLIT slices in order.
__global__ void __launch_bounds__(256) k_gram_sum1(const double *__restrict__ partials, int64_t n,
                                                   double *__restrict__ out2) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    constexpr int per = GBLKS / GSPLIT;
    double s = 0.0;
#pragma unroll 8
    for (int b = blockIdx.y * per; b < (int)(blockIdx.y + 1) * per; ++b) s += partials[(int64_t)b * n + e];
    out2[(int64_t)blockIdx.y * n + e] = s;
}
__global__ void __launch_bounds__(256) k_gram_sum2(const double *__restrict__ out2, int64_t n,
                                                   double *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
#pragma unroll
    for (int y = 0; y < GSPLIT; ++y) s += out2[(int64_t)y * n + e];
    out[e] = s;
}

// acc[u][t] (+)= sum_k A[row0 + ra + u][k] C[k][cb + t] for the lane's 4 x 8
// tile; A's entries four at a time with the next four in flight.
__device__ __forceinline__ void tile_times(const double *__restrict__ A, int64_t row0, int ra, int cb, int64_t rows,
                                           int m, const double *C, double (&acc)[4][8]) {
    double cur[4][KB], nxt[4][KB];
    auto load = [&](double (&dst)[4][KB], int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + ra + u;
#pragma unroll
            for (int q = 0; q < KB; ++q) dst[u][q] = (row < rows && k0 + q < m) ? A[row * m + k0 + q] : 0.0;
        }
    };
    load(cur, 0);
    for (int k0 = 0; k0 < m; k0 += KB) {
        if (k0 + KB < m) load(nxt, k0 + KB);
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            double c[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) c[t] = C[(k0 + q) * GM + cb + t];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < 8; ++t) acc[u][t] = fma(cur[u][q], c[t], acc[u][t]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < KB; ++q) cur[u][q] = nxt[u][q];
    }
}

// X += P alpha, R -= Q alpha; a wave takes TRW rows, lane (a, b) rows
// 4a..4a+3 and columns 8b..8b+7 of them.
__global__ void __launch_bounds__(UBLK) k_block_xr(int64_t rows, int m, const double *__restrict__ alpha,
                                                   const double *__restrict__ P, const double *__restrict__ Q,
                                                   double *__restrict__ X, double *__restrict__ R,
                                                   double *__restrict__ partials) {
    __shared__ double s_a[GM * GM];
    __shared__ double s_col[UBLK / WAVE][8][GM];
    for (int e = threadIdx.x; e < GM * GM; e += blockDim.x) s_a[e] = alpha[e];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int ra = (lane >> 3) * 4, cb = (lane & 7) * 8;
    double rr[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) rr[t] = 0.0;
    const int64_t step = (int64_t)gridDim.x * (UBLK / WAVE) * TRW;
    for (int64_t row0 = ((int64_t)blockIdx.x * (UBLK / WAVE) + w) * TRW; row0 < rows; row0 += step) {
        double acc[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[u][t] = 0.0;
        tile_times(P, row0, ra, cb, rows, m, s_a, acc);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + ra + u;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (row < rows && cb + t < m) X[row * m + cb + t] += acc[u][t];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[u][t] = 0.0;
        tile_times(Q, row0, ra, cb, rows, m, s_a, acc);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + ra + u;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (row < rows && cb + t < m) {
                    const double r = R[row * m + cb + t] - acc[u][t];
                    R[row * m + cb + t] = r;
                    rr[t] += r * r;
                }
        }
    }
    // per-column partial of this workgroup: (wave, row group) in order
#pragma unroll
    for (int t = 0; t < 8; ++t) s_col[w][lane >> 3][cb + t] = rr[t];
    __syncthreads();
    if ((int)threadIdx.x < m) {
        double tot = 0.0;
        for (int v = 0; v < UBLK / WAVE; ++v)
            for (int gq = 0; gq < 8; ++gq) tot += s_col[v][gq][threadIdx.x];
        partials[(int64_t)blockIdx.x * m + threadIdx.x] = tot;
    }
}

// P <- Z T1 + P T2 in place; tiles as in k_block_xr.
__global__ void __launch_bounds__(UBLK) k_block_p(int64_t rows, int m, const double *__restrict__ T1,
                                                  const double *__restrict__ T2, const double *__restrict__ Z,
                                                  double *P) {
    __shared__ double s_1[GM * GM], s_2[GM * GM];
    for (int e = threadIdx.x; e < GM * GM; e += blockDim.x) {
        s_1[e] = T1[e];
        s_2[e] = T2[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int ra = (lane >> 3) * 4, cb = (lane & 7) * 8;
    const int64_t step = (int64_t)gridDim.x * (UBLK / WAVE) * TRW;
    for (int64_t row0 = ((int64_t)blockIdx.x * (UBLK / WAVE) + w) * TRW; row0 < rows; row0 += step) {
        double acc[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[u][t] = 0.0;
        tile_times(Z, row0, ra, cb, rows, m, s_1, acc);
        tile_times(P, row0, ra, cb, rows, m, s_2, acc);
        // the wave's rows of P are read whole by every lane before any lane
        // writes: wait for the whole wave here
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = row0 + ra + u;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (row < rows && cb + t < m) P[row * m + cb + t] = acc[u][t];
        }
    }
}

inline unsigned update_grid(int64_t rows) {
    const int64_t per = (int64_t)(UBLK / WAVE) * TRW;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + per - 1) / per, 2048));
}

}  // namespace

int block_gram_nblocks() { return GBLKS + GSPLIT; }
int block_xr_nblocks(int64_t rows) { return (int)update_grid(rows); }

void block_gram(const double *const *mats, int nmat, const int *li, const int *ri, int npair, int64_t rows, int m,
                double *partials, double *out, hipStream_t s) {
    TE_REQUIRE(nmat >= 1 && nmat <= 3 && npair >= 1 && npair <= 3 && m >= 1 && m <= GM, TE_EINVAL,
               "block Gram: bad arguments");
    for (int p = 0; p < npair; ++p)
        TE_REQUIRE(li[p] >= 0 && li[p] < nmat && ri[p] >= 0 && ri[p] < nmat, TE_EINVAL, "block Gram: bad pair");
    GramArgs g{};
    for (int i = 0; i < nmat; ++i) g.mat[i] = mats[i];
    g.nmat = nmat;
    for (int p = 0; p < npair; ++p) {
        g.li[p] = li[p];
        g.ri[p] = ri[p];
    }
    g.npair = npair;
    g.rows = rows;
    g.m = m;
    g.partials = partials;
    hipLaunchKernelGGL(k_gram, dim3(GBLKS), dim3(64 * npair), 0, s, g);
    const int64_t n = (int64_t)npair * GM * GM;
    double *out2 = partials + (int64_t)GBLKS * n;
    const unsigned gx = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_gram_sum1, dim3(gx, GSPLIT), dim3(256), 0, s, partials, n, out2);
    hipLaunchKernelGGL(k_gram_sum2, dim3(gx), dim3(256), 0, s, out2, n, out);
    TE_CHECK_HIP(hipGetLastError());
}

void block_xr(int64_t rows, int m, const double *alpha, const double *P, const double *Q, double *X, double *R,
              double *partials, hipStream_t s) {
    TE_REQUIRE(m >= 1 && m <= GM, TE_EINVAL, "block update: m = %d", m);
    hipLaunchKernelGGL(k_block_xr, dim3(update_grid(rows)), dim3(UBLK), 0, s, rows, m, alpha, P, Q, X, R, partials);
    TE_CHECK_HIP(hipGetLastError());
}

void block_p(int64_t rows, int m, const double *T1, const double *T2, const double *Z, double *P, hipStream_t s) {
    TE_REQUIRE(m >= 1 && m <= GM, TE_EINVAL, "block update: m = %d", m);
    hipLaunchKernelGGL(k_block_p, dim3(update_grid(rows)), dim3(UBLK), 0, s, rows, m, T1, T2, Z, P);
    TE_CHECK_HIP(hipGetLastError());
}

}  // namespace te
