// Kernels of block conjugate gradients over the columns of a multi-RHS solve
// (O'Leary 1980; the driver is in te_solve.cpp).  Block vectors are the
// solve's [rows][m] arrays (right-hand sides fastest, m <= 64); small matrices
// are 64 x 64 row-major with zero padding.
//
// All three are tall-skinny dense contractions and run on the float64 matrix
// cores (v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16); lane i holds
// A[i%16][i/16] and B[i/16][i%16], and D[i/16 + 4q][i%16] in register q).
//
//   k_gram      C_t = L_t^T R_t for up to three pairs of block vectors in one
//               pass over the rows.  A = 16 columns of L over 4 rows and
//               B = 16 columns of R over the same 4 rows are both plain
//               4-row x 16-column loads; two waves per pair each hold 8 of the
//               16 output tiles.  One partial per workgroup, summed in
//               workgroup order (k_gram_sum1/2: deterministic).
//   k_block_xr  X += P alpha, R -= Q alpha; one wave per 16 rows, alpha in
//               LDS, plus per-column partial sums of R^2.
//   k_block_p   P <- Z T1 + P T2 in place (a wave reads all of its 16 rows
//               before it writes them); T1, T2 in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "te_dev.h"

namespace te {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GM = 64;      // largest block size
constexpr int GBLKS = 512;  // workgroups of the Gram pass
constexpr int GSPLIT = 16;  // first-stage slices of the Gram partial sum
constexpr int GU = 4;       // 4-row steps per load batch in the Gram pass
constexpr int UBLK = 512;   // threads of the update kernels (8 waves)

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct GramArgs {
    const double *mat[3];   // distinct block vectors [rows][m]
    int nmat;
    int li[3], ri[3];       // pair t: mat[li[t]]^T mat[ri[t]]
    int npair;
    int64_t rows;
    int m;
    double *partials;       // [GBLKS][npair][GM][GM]
};

// blockDim = 128 * npair: wave w takes pair w / 2 and output row tiles
// 2 (w % 2), 2 (w % 2) + 1 against all four column tiles.
__global__ void __launch_bounds__(384) k_gram(GramArgs g) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int p = w >> 1, jt0 = (w & 1) * 2;
    const int kr = lane >> 4, kc = lane & 15;
    const int m = g.m;
    const double *__restrict__ L = g.mat[g.li[p]];
    const double *__restrict__ R = g.mat[g.ri[p]];
    const bool tj[2] = {jt0 * 16 < m, (jt0 + 1) * 16 < m};
    d4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[t][c] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t step = 4 * GU;
    const int64_t chunk = ((g.rows + gridDim.x - 1) / gridDim.x + step - 1) / step * step;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(g.rows, lo + chunk);
    // fragments of one batch of GU 4-row steps; the next batch is loaded
    // while the current one goes through the matrix cores
    double a[GU][2], b[GU][4];
    auto load = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int64_t row = r0 + 4 * u + kr;
            const bool ok = row < hi;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int col = (jt0 + t) * 16 + kc;
                a[u][t] = (ok && col < m) ? L[row * m + col] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = c * 16 + kc;
                b[u][c] = (ok && col < m) ? R[row * m + col] : 0.0;
            }
        }
    };
    if (lo < hi) load(lo);
    for (int64_t r0 = lo; r0 < hi; r0 += step) {
        double ca[GU][2], cb[GU][4];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
#pragma unroll
            for (int t = 0; t < 2; ++t) ca[u][t] = a[u][t];
#pragma unroll
            for (int c = 0; c < 4; ++c) cb[u][c] = b[u][c];
        }
        if (r0 + step < hi) load(r0 + step);
#pragma unroll
        for (int u = 0; u < GU; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (tj[t] && c * 16 < m) acc[t][c] = mfma(ca[u][t], cb[u][c], acc[t][c]);
    }
    double *out = g.partials + ((int64_t)blockIdx.x * g.npair + p) * GM * GM;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) out[((jt0 + t) * 16 + kr + 4 * q) * GM + c * 16 + kc] = acc[t][c][q];
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

// X += P alpha, R -= Q alpha.  Wave tile: 16 rows x m columns; A fragments
// are P (or Q) at rows r0 + i%16, columns 4s + i/16; B fragments alpha rows
// 4s + i/16, columns 16c + i%16 from LDS.
__global__ void __launch_bounds__(UBLK) k_block_xr(int64_t rows, int m, const double *__restrict__ alpha,
                                                   const double *__restrict__ P, const double *__restrict__ Q,
                                                   double *__restrict__ X, double *__restrict__ R,
                                                   double *__restrict__ partials) {
    __shared__ double s_a[GM * GM];
    __shared__ double s_col[UBLK / WAVE][4][GM];
    for (int e = threadIdx.x; e < GM * GM; e += blockDim.x) s_a[e] = alpha[e];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int kr = lane >> 4, kc = lane & 15;
    const int nk = (m + 3) / 4, nc = (m + 15) / 16;
    double rr[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = ((int64_t)blockIdx.x * nw + w) * 16; r0 < rows; r0 += (int64_t)gridDim.x * nw * 16) {
        // all fragments of the 16 rows first (loads in flight together)
        const int64_t ra = r0 + kc;
        double pa[GM / 4], qa[GM / 4];
#pragma unroll
        for (int s = 0; s < GM / 4; ++s) {
            const int k = 4 * s + kr;
            const bool ok = ra < rows && k < m;
            pa[s] = ok ? P[ra * m + k] : 0.0;
            qa[s] = ok ? Q[ra * m + k] : 0.0;
        }
        // one 16-column tile at a time: its X and R entries are loaded before
        // its matrix-core steps, which then cover their latency
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= nc) break;
            const int col = c * 16 + kc;
            double xo[4], ro[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = r0 + kr + 4 * q;
                const bool ok = row < rows && col < m;
                xo[q] = ok ? X[row * m + col] : 0.0;
                ro[q] = ok ? R[row * m + col] : 0.0;
            }
            d4 dx = d4{0.0, 0.0, 0.0, 0.0}, dr = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < GM / 4; ++s) {
                if (s >= nk) break;
                const double bv = s_a[(4 * s + kr) * GM + col];
                dx = mfma(pa[s], bv, dx);
                dr = mfma(qa[s], bv, dr);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = r0 + kr + 4 * q;
                if (col < m && row < rows) {
                    X[row * m + col] = xo[q] + dx[q];
                    const double r = ro[q] - dr[q];
                    R[row * m + col] = r;
                    rr[c] += r * r;
                }
            }
        }
    }
    // per-column partial of this workgroup: (wave, row group) in order
#pragma unroll
    for (int c = 0; c < 4; ++c) s_col[w][kr][c * 16 + kc] = rr[c];
    __syncthreads();
    if ((int)threadIdx.x < m) {
        double t = 0.0;
        for (int v = 0; v < nw; ++v)
            for (int g = 0; g < 4; ++g) t += s_col[v][g][threadIdx.x];
        partials[(int64_t)blockIdx.x * m + threadIdx.x] = t;
    }
}

// P <- Z T1 + P T2 in place.
__global__ void __launch_bounds__(UBLK) k_block_p(int64_t rows, int m, const double *__restrict__ T1,
                                                  const double *__restrict__ T2, const double *__restrict__ Z,
                                                  double *P) {
    __shared__ double s_1[GM * GM], s_2[GM * GM];
    for (int e = threadIdx.x; e < GM * GM; e += blockDim.x) {
        s_1[e] = T1[e];
        s_2[e] = T2[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int kr = lane >> 4, kc = lane & 15;
    const int nk = (m + 3) / 4, nc = (m + 15) / 16;
    for (int64_t r0 = ((int64_t)blockIdx.x * nw + w) * 16; r0 < rows; r0 += (int64_t)gridDim.x * nw * 16) {
        d4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
        const int64_t ra = r0 + kc;
        double za[GM / 4], pa[GM / 4];
#pragma unroll
        for (int s = 0; s < GM / 4; ++s) {
            const int k = 4 * s + kr;
            const bool ok = ra < rows && k < m;
            za[s] = ok ? Z[ra * m + k] : 0.0;
            pa[s] = ok ? P[ra * m + k] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < GM / 4; ++s) {
            if (s >= nk) break;
            const int k = 4 * s + kr;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nc) {
                    acc[c] = mfma(za[s], s_1[k * GM + c * 16 + kc], acc[c]);
                    acc[c] = mfma(pa[s], s_2[k * GM + c * 16 + kc], acc[c]);
                }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = c * 16 + kc;
            if (c >= nc || col >= m) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = r0 + kr + 4 * q;
                if (row < rows) P[row * m + col] = acc[c][q];
            }
        }
    }
}

inline unsigned update_grid(int64_t rows) {
    const int64_t per = 16 * (UBLK / WAVE);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + per - 1) / per, 768));
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
    hipLaunchKernelGGL(k_gram, dim3(GBLKS), dim3(128 * npair), 0, s, g);
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
