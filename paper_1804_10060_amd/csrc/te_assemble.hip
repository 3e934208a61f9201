// Finite-element assembly of the thermoelastic system (weak form wf_elastic,
// Sec. 3.1) into 3x3-block compressed rows, and Dirichlet elimination; and
// the residual and Newton Jacobian of the heat equation (weak form
// wf_thermal) in scalar compressed rows.
//
// Gather formulation, nothing is scattered: the stiffness rows of a node are
// built by one wave that walks the cells containing the node (ascending cell
// id, so the summation order is fixed and the result deterministic): the
// element blocks of a chunk of cells go through LDS and each lane adds them
// to the row blocks it owns, which are written once.  The load vector takes
// one thread per node.  Element integrals:
//   stiffness  P1: constant gradients (one-point exact); P2: degree-2
//              integrand, 4-point rule (a,b,b,b), a = (5+3 sqrt5)/20,
//              b = (5-sqrt5)/20, weights 1/4 (exact for degree 2);
//   thermal    P1: centroid rule (degree 1 exact); P2: degree-3 integrand,
//              5-point rule with barycentric points (1/4,...) weight -4/5 and
//              the permutations of (1/2,1/6,1/6,1/6) weight 9/20 (exact for
//              degree 3);
//   body force consistent mass: P1 |K|(1+delta_ac)/20; P2 the closed-form
//              10-node mass matrix (|K|/420: 6/1 vertex-vertex, -4/-6
//              vertex-edge, 32/16/8 edge-edge).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>

#include "te_internal.h"
#include "te_thermal.h"

namespace te {

constexpr int ABLK = 64;
constexpr int PCAP = 192;  // maximum distinct neighbours of one node

__constant__ int c_edge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// ---------------------------------------------------------------------------
// node -> (cell, local index) incidence
// ---------------------------------------------------------------------------
__global__ void k_check_cells(const int32_t *__restrict__ cells, int64_t n_entries, int64_t n_nodes,
                              int32_t *__restrict__ bad) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_entries; t += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = cells[t];
        if (v < 0 || v >= n_nodes) *bad = 1;
    }
}

__global__ void k_inc_count(const int32_t *__restrict__ cells, int64_t n_entries, int32_t *__restrict__ cnt) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_entries; t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[cells[t]], 1);
}

__global__ void k_inc_fill(const int32_t *__restrict__ cells, int64_t n_entries, const int64_t *__restrict__ start,
                           int32_t *__restrict__ fill, int64_t *__restrict__ inc) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_entries; t += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = cells[t];
        int32_t k = atomicAdd(&fill[v], 1);
        inc[start[v] + k] = t;  // t = cell * npe + local
    }
}

// per node: sort its incidence entries ascending (insertion sort, short lists)
__global__ void k_inc_sort(const int64_t *__restrict__ start, int64_t *__restrict__ inc, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = start[i], hi = start[i + 1];
        for (int64_t a = lo + 1; a < hi; ++a) {
            int64_t v = inc[a];
            int64_t b = a - 1;
            while (b >= lo && inc[b] > v) {
                inc[b + 1] = inc[b];
                --b;
            }
            inc[b + 1] = v;
        }
    }
}

// Exclusive scan of int32 counts into int64 offsets (out[0] = 0, out[n] = total),
// three phases with fixed-size blocks.
__global__ void k_scan_block(const int32_t *__restrict__ in, int64_t *__restrict__ out, int64_t n,
                             int64_t *__restrict__ block_sums) {
    __shared__ int64_t s[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    int64_t i = base + threadIdx.x;
    s[threadIdx.x] = (i < n) ? (int64_t)in[i] : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t v = (threadIdx.x >= (unsigned)o) ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < n) out[i + 1] = s[threadIdx.x];  // inclusive -> shifted
    if (threadIdx.x == 1023) block_sums[blockIdx.x] = s[1023];
}
__global__ void k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ block_off) {
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) out[i + 1] += block_off[blockIdx.x];
    if (i == 0) out[0] = 0;
}

static void scan_counts(const int32_t *cnt, int64_t *out, int64_t n, hipStream_t s) {
    int64_t nb = (n + 1023) / 1024;
    DBuf<int64_t> bs(std::max<int64_t>(nb, 1));
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(1024), 0, s, cnt, out, n, bs.p);
        TE_CHECK_HIP(hipGetLastError());
    }
    std::vector<int64_t> h;
    download(h, bs.p, (size_t)nb, s);
    std::vector<int64_t> off(nb, 0);
    for (int64_t b = 1; b < nb; ++b) off[b] = off[b - 1] + h[b - 1];
    DBuf<int64_t> doff;
    upload(doff, off, s);
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(1024), 0, s, out, n, doff.p);
        TE_CHECK_HIP(hipGetLastError());
    } else {
        TE_CHECK_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    }
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

static void build_incidence(const te_mesh *m, int npe, Incidence &I, hipStream_t s) {
    const int64_t n = m->n_nodes, ne = m->n_cells * (int64_t)npe;
    DBuf<int32_t> bad(1);
    TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    unsigned g = (unsigned)std::min<int64_t>((ne + 255) / 256 + 1, 1 << 20);
    hipLaunchKernelGGL(k_check_cells, dim3(g), dim3(256), 0, s, m->cells, ne, n, bad.p);
    TE_CHECK_HIP(hipGetLastError());
    int32_t hb = 0;
    TE_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    TE_REQUIRE(hb == 0, TE_EINVAL, "cells reference a node index outside [0, n_nodes)");
    DBuf<int32_t> cnt(n);
    TE_CHECK_HIP(hipMemsetAsync(cnt.p, 0, n * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_inc_count, dim3(g), dim3(256), 0, s, m->cells, ne, cnt.p);
    TE_CHECK_HIP(hipGetLastError());
    I.start.alloc(n + 1);
    scan_counts(cnt.p, I.start.p, n, s);
    TE_CHECK_HIP(hipMemsetAsync(cnt.p, 0, n * sizeof(int32_t), s));
    I.inc.alloc(std::max<int64_t>(ne, 1));
    hipLaunchKernelGGL(k_inc_fill, dim3(g), dim3(256), 0, s, m->cells, ne, I.start.p, cnt.p, I.inc.p);
    TE_CHECK_HIP(hipGetLastError());
    unsigned gn = (unsigned)std::min<int64_t>((n + 255) / 256 + 1, 1 << 20);
    hipLaunchKernelGGL(k_inc_sort, dim3(gn), dim3(256), 0, s, I.start.p, I.inc.p, n);
    TE_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// sparsity pattern
// ---------------------------------------------------------------------------
// Sorted distinct neighbours of node i in an LDS list (thread-private slice).
// mode 0: write count to cnt[i]; mode 1: write the list to col[row_ptr[i]..].
__global__ void __launch_bounds__(ABLK) k_pattern(const int32_t *__restrict__ cells, int npe,
                                                  const int64_t *__restrict__ start, const int64_t *__restrict__ inc,
                                                  int64_t n, int mode, int32_t *__restrict__ cnt,
                                                  const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                  int32_t *__restrict__ overflow) {
    __shared__ int32_t lst[ABLK * PCAP];
    int64_t i = (int64_t)blockIdx.x * ABLK + threadIdx.x;
    if (i >= n) return;
    int32_t *L = lst + threadIdx.x;  // strided by ABLK to spread banks
    int len = 0;
    bool over = false;
    for (int64_t e = start[i]; e < start[i + 1] && !over; ++e) {
        const int64_t cell = inc[e] / npe;
        for (int b = 0; b < npe; ++b) {
            int32_t v = cells[cell * npe + b];
            // binary search for v in L[0..len)
            int lo = 0, hi = len;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (L[mid * ABLK] < v) lo = mid + 1;
                else hi = mid;
            }
            if (lo < len && L[lo * ABLK] == v) continue;
            if (len == PCAP) {
                over = true;
                break;
            }
            for (int k = len; k > lo; --k) L[k * ABLK] = L[(k - 1) * ABLK];
            L[lo * ABLK] = v;
            ++len;
        }
    }
    if (over) {
        *overflow = 1;
        return;
    }
    if (mode == 0) {
        cnt[i] = len;
    } else {
        // row_ptr comes from the caller: never write past its row
        if (row_ptr[i + 1] - row_ptr[i] != len) {
            *overflow = 2;
            return;
        }
        int32_t *o = col + row_ptr[i];
        for (int k = 0; k < len; ++k) o[k] = L[k * ABLK];
    }
}

// ---------------------------------------------------------------------------
// element integrals
// ---------------------------------------------------------------------------
struct Geo {
    double G[4][3];  // gradient of barycentric coordinate k
    double vol;
};

__device__ __forceinline__ Geo cell_geo(const double *__restrict__ X, const int32_t *__restrict__ cv) {
    double x0[3], J[3][3];
    for (int c = 0; c < 3; ++c) x0[c] = X[(int64_t)cv[0] * 3 + c];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) J[c][k] = X[(int64_t)cv[k + 1] * 3 + c] - x0[c];  // columns = edges
    // inverse via cofactors: rows of J^-1 are the gradients of l1..l3
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double id = 1.0 / det;
    Geo g;
    g.G[1][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    g.G[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    g.G[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    g.G[2][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    g.G[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    g.G[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    g.G[3][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    g.G[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    g.G[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    for (int c = 0; c < 3; ++c) g.G[0][c] = -(g.G[1][c] + g.G[2][c] + g.G[3][c]);
    g.vol = fabs(det) / 6.0;
    return g;
}

// Element tables are indexed by runtime node numbers; to keep them out of
// private (scratch) memory, the barycentric values are selected from
// registers and the gradients are read from LDS (G: [4][3] row-major).
__device__ __forceinline__ double sel4(double v0, double v1, double v2, double v3, int k) {
    return k == 0 ? v0 : (k == 1 ? v1 : (k == 2 ? v2 : v3));
}

// gradient of the P2 basis function a at the barycentric point (l0..l3)
__device__ __forceinline__ void p2_grad(int a, double l0, double l1, double l2, double l3, const double *G,
                                        double out[3]) {
    if (a < 4) {
        const double s = 4.0 * sel4(l0, l1, l2, l3, a) - 1.0;
        for (int c = 0; c < 3; ++c) out[c] = s * G[a * 3 + c];
    } else {
        const int i = c_edge[a - 4][0], j = c_edge[a - 4][1];
        const double li = sel4(l0, l1, l2, l3, i), lj = sel4(l0, l1, l2, l3, j);
        for (int c = 0; c < 3; ++c) out[c] = 4.0 * (lj * G[i * 3 + c] + li * G[j * 3 + c]);
    }
}

__device__ __forceinline__ double p2_val(int a, double l0, double l1, double l2, double l3) {
    if (a < 4) {
        const double la = sel4(l0, l1, l2, l3, a);
        return la * (2.0 * la - 1.0);
    }
    return 4.0 * sel4(l0, l1, l2, l3, c_edge[a - 4][0]) * sel4(l0, l1, l2, l3, c_edge[a - 4][1]);
}

// closed-form P2 mass matrix times 420/|K|
__device__ __forceinline__ double p2_mass420(int a, int c) {
    if (a < 4 && c < 4) return a == c ? 6.0 : 1.0;
    if (a >= 4 && c >= 4) {
        if (a == c) return 32.0;
        int i0 = c_edge[a - 4][0], i1 = c_edge[a - 4][1], j0 = c_edge[c - 4][0], j1 = c_edge[c - 4][1];
        bool share = (i0 == j0) || (i0 == j1) || (i1 == j0) || (i1 == j1);
        return share ? 16.0 : 8.0;
    }
    int v = a < 4 ? a : c, e = a < 4 ? c : a;
    bool contains = (c_edge[e - 4][0] == v) || (c_edge[e - 4][1] == v);
    return contains ? -4.0 : -6.0;
}

struct AsmArgs {
    const double *X;
    const int32_t *cells;
    int npe;
    const int64_t *start;
    const int64_t *inc;
    int64_t n;
    double lam, mu, calpha, T_ref;
    const double *coef;  // per cell (lam, mu, (3 lam + 2 mu) alpha) [C][3], or null: the scalars above
    const double *T;   // [nrhs][N]
    const double *f;   // [nrhs][N][3] or null
    const int64_t *row_ptr;
    const int32_t *col;
    double *val;       // stiffness values (k_stiff)
    double *b;         // [N][3][nrhs]
    int nrhs;
};

// Load of node i for right-hand side j (thermal strain and body force).
template <int DEG>
__global__ void __launch_bounds__(ABLK) k_assemble(AsmArgs A, int j) {
    const int64_t i = (int64_t)blockIdx.x * ABLK + threadIdx.x;
    if (i >= A.n) return;
    constexpr int NPE = DEG == 1 ? 4 : 10;
    const double *T = A.T + (int64_t)j * A.n;
    const double *f = A.f ? A.f + (int64_t)j * A.n * 3 : nullptr;
    __shared__ double s_g[ABLK][12];
    double *G = s_g[threadIdx.x];  // this thread's gradients, addressable without scratch
    double bi[3] = {0.0, 0.0, 0.0};
    for (int64_t e = A.start[i]; e < A.start[i + 1]; ++e) {
        const int64_t cell = A.inc[e] / NPE;
        const int a = (int)(A.inc[e] % NPE);
        const int32_t *cv = A.cells + cell * NPE;
        const Geo g = cell_geo(A.X, cv);
        const double calpha = A.coef ? A.coef[cell * 3 + 2] : A.calpha;
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) G[k * 3 + c] = g.G[k][c];
        double dT[NPE];
        for (int c = 0; c < NPE; ++c) dT[c] = T[cv[c]] - A.T_ref;
        if (DEG == 1) {
            // thermal: (3 lam + 2 mu) alpha |K| mean(dT) grad l_a
            double mT = 0.25 * (dT[0] + dT[1] + dT[2] + dT[3]);
            for (int c = 0; c < 3; ++c) bi[c] += calpha * g.vol * mT * G[a * 3 + c];
            if (f)
                for (int c = 0; c < 4; ++c) {
                    double m = g.vol * (c == a ? 2.0 : 1.0) / 20.0;
                    for (int k = 0; k < 3; ++k) bi[k] += m * f[(int64_t)cv[c] * 3 + k];
                }
        } else {
            // thermal load, degree-3 exact 5-point rule
            {
                const double w5[5] = {-0.8, 0.45, 0.45, 0.45, 0.45};
                for (int qp = 0; qp < 5; ++qp) {
                    // (1/4,1/4,1/4,1/4), then the permutations of (1/2,1/6,1/6,1/6)
                    const double l0 = qp == 0 ? 0.25 : (qp == 1 ? 0.5 : 1.0 / 6.0);
                    const double l1 = qp == 0 ? 0.25 : (qp == 2 ? 0.5 : 1.0 / 6.0);
                    const double l2 = qp == 0 ? 0.25 : (qp == 3 ? 0.5 : 1.0 / 6.0);
                    const double l3 = qp == 0 ? 0.25 : (qp == 4 ? 0.5 : 1.0 / 6.0);
                    double Tq = 0.0;
#pragma unroll
                    for (int c = 0; c < 10; ++c) Tq += dT[c] * p2_val(c, l0, l1, l2, l3);
                    double gr[3];
                    p2_grad(a, l0, l1, l2, l3, G, gr);
                    for (int c = 0; c < 3; ++c) bi[c] += calpha * w5[qp] * g.vol * Tq * gr[c];
                }
            }
            if (f)
                for (int c = 0; c < 10; ++c) {
                    double m = g.vol * p2_mass420(a, c) / 420.0;
                    for (int k = 0; k < 3; ++k) bi[k] += m * f[(int64_t)cv[c] * 3 + k];
                }
        }
    }
    for (int c = 0; c < 3; ++c) A.b[(i * 3 + c) * A.nrhs + j] = bi[c];
}

// Stiffness rows, one wave per node row.  The row's incident cells are taken
// in chunks of SCH: lanes compute the chunk's cell geometries, then the
// element blocks K_e[a][b] of all (cell, b) pairs with the position of block
// b in the row; lane q owns blocks q, q + 64, q + 128 of the row (at most
// PCAP) and adds the chunk's blocks to them in cell order.
constexpr int SCH = 16;

template <int DEG>
__global__ void __launch_bounds__(64) k_stiff(AsmArgs A) {
    constexpr int NPE = DEG == 1 ? 4 : 10;
    static_assert(NPE % 2 == 0, "cell entries are read in pairs");
    __shared__ double s_geo[SCH][15];  // gradients of the 4 barycentric coordinates, volume, lam, mu
    __shared__ int32_t s_cv[SCH][NPE];
    __shared__ int32_t s_a[SCH];
    __shared__ double s_k[SCH * NPE][9];
    __shared__ __align__(8) int32_t s_pos[SCH * NPE];  // NPE is even: a cell's entries read as int2
    __shared__ int32_t s_col[PCAP];                    // the row's columns, searched in LDS
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < A.n; i += gridDim.x) {
        const int64_t r0 = A.row_ptr[i], r1 = A.row_ptr[i + 1];
        const int len = (int)(r1 - r0);
        for (int t = lane; t < len; t += 64) s_col[t] = A.col[r0 + t];
        double acc[3][9];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[q][k] = 0.0;
        const int64_t e0 = A.start[i], e1 = A.start[i + 1];
        for (int64_t cb = e0; cb < e1; cb += SCH) {
            const int nc = (int)((e1 - cb) < SCH ? (e1 - cb) : SCH);
            if (lane < nc) {
                const int64_t ent = A.inc[cb + lane];
                const int32_t *cv = A.cells + (ent / NPE) * NPE;
                s_a[lane] = (int)(ent % NPE);
                for (int b = 0; b < NPE; ++b) s_cv[lane][b] = cv[b];
                const Geo g = cell_geo(A.X, cv);
                for (int k = 0; k < 4; ++k)
                    for (int c = 0; c < 3; ++c) s_geo[lane][k * 3 + c] = g.G[k][c];
                s_geo[lane][12] = g.vol;
                s_geo[lane][13] = A.coef ? A.coef[(ent / NPE) * 3] : A.lam;
                s_geo[lane][14] = A.coef ? A.coef[(ent / NPE) * 3 + 1] : A.mu;
            }
            __syncthreads();
            for (int t = lane; t < nc * NPE; t += 64) {
                const int c = t / NPE, bb = t % NPE, a = s_a[c];
                const double *G = s_geo[c];
                const double vol = s_geo[c][12], lam = s_geo[c][13], mu = s_geo[c][14];
                double K[9];
                if (DEG == 1) {
                    const double *ga = G + a * 3, *gb = G + bb * 3;
                    const double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q)
                            K[p * 3 + q] =
                                vol * (lam * ga[p] * gb[q] + mu * ga[q] * gb[p] + (p == q ? mu * dot : 0.0));
                } else {
                    // degree-2 integrand: 4-point rule (a,b,b,b), weights |K|/4
                    const double qa = 0.5854101966249685, qb = 0.1381966011250105;
                    for (int k = 0; k < 9; ++k) K[k] = 0.0;
                    for (int qp = 0; qp < 4; ++qp) {
                        const double l0 = qp == 0 ? qa : qb, l1 = qp == 1 ? qa : qb, l2 = qp == 2 ? qa : qb,
                                     l3 = qp == 3 ? qa : qb;
                        double ga[3], gb[3];
                        p2_grad(a, l0, l1, l2, l3, G, ga);
                        p2_grad(bb, l0, l1, l2, l3, G, gb);
                        const double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q)
                                K[p * 3 + q] += lam * ga[p] * gb[q] + mu * ga[q] * gb[p] + (p == q ? mu * dot : 0.0);
                    }
                    const double w = 0.25 * vol;
                    for (int k = 0; k < 9; ++k) K[k] *= w;
                }
                const int32_t v = s_cv[c][bb];
                int lo = 0, hi = len;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_col[mid] < v) lo = mid + 1;
                    else hi = mid;
                }
                s_pos[t] = (lo < len && s_col[lo] == v) ? lo : -1;  // -1 unreachable with a matching pattern
                for (int k = 0; k < 9; ++k) s_k[t][k] = K[k];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int blk = lane + 64 * q;
                if (blk < len)
                    for (int c = 0; c < nc; ++c) {  // cells ascending; a cell meets a block at most once
                        const int2 *pp = reinterpret_cast<const int2 *>(&s_pos[c * NPE]);
                        int hit = -1;
#pragma unroll
                        for (int h = 0; h < NPE / 2; ++h) {
                            const int2 v = pp[h];
                            hit = v.x == blk ? 2 * h : hit;
                            hit = v.y == blk ? 2 * h + 1 : hit;
                        }
                        if (hit >= 0)
#pragma unroll
                            for (int k = 0; k < 9; ++k) acc[q][k] += s_k[c * NPE + hit][k];
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int blk = lane + 64 * q;
            if (blk < len)
#pragma unroll
                for (int k = 0; k < 9; ++k) A.val[(r0 + blk) * 9 + k] = acc[q][k];
        }
    }
}

// Dirichlet elimination, one thread per row.  Lifting with the unconstrained
// values first, then rows/columns of constrained DOFs zeroed, unit diagonal,
// b_D = u_D.
__global__ void k_dirichlet(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                            double *__restrict__ val, double *__restrict__ b, const uint8_t *__restrict__ mask,
                            const double *__restrict__ ubc) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bool mi[3] = {mask[i * 3] != 0, mask[i * 3 + 1] != 0, mask[i * 3 + 2] != 0};
        double bi[3] = {b[i * 3], b[i * 3 + 1], b[i * 3 + 2]};
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int64_t J = col[k];
            double *blk = val + k * 9;
            for (int q = 0; q < 3; ++q) {
                if (!mask[J * 3 + q]) continue;
                double u = ubc ? ubc[J * 3 + q] : 0.0;
                for (int p = 0; p < 3; ++p) bi[p] -= blk[p * 3 + q] * u;
            }
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    if (mi[p] || mask[J * 3 + q]) blk[p * 3 + q] = (J == i && p == q) ? 1.0 : 0.0;
        }
        for (int p = 0; p < 3; ++p) b[i * 3 + p] = mi[p] ? (ubc ? ubc[i * 3 + p] : 0.0) : bi[p];
    }
}

// load-only variant: constrained entries set to zero (u_bc = 0, no lifting needed)
__global__ void k_zero_masked(int64_t n, int nrhs, double *__restrict__ b, const uint8_t *__restrict__ mask) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * 3 * nrhs; t += (int64_t)gridDim.x * blockDim.x)
        if (mask[t / nrhs]) b[t] = 0.0;
}

// ---------------------------------------------------------------------------
// Temperature-dependent materials and boundary pressure
// ---------------------------------------------------------------------------
// Value of one table (n samples at temperatures Tt, ascending) at Tm: linear
// between samples, constant beyond the ends.
__device__ __forceinline__ double table_at(const double *Tt, const double *v, int n, double Tm) {
    if (n == 1 || Tm <= Tt[0]) return v[0];
    if (Tm >= Tt[n - 1]) return v[n - 1];
    int k = 0;
    while (k + 2 < n && Tm >= Tt[k + 1]) ++k;
    const double slope = (v[k + 1] - v[k]) / (Tt[k + 1] - Tt[k]);
    return slope * (Tm - Tt[k]) + v[k];
}

// Per cell: mean of T_h over the cell (P1: vertex average; P2: -1/20 of each
// vertex value plus 1/5 of each edge value, the exact cell integrals of the
// basis), the material's E, nu, alpha there, and (lam, mu, (3 lam + 2 mu) alpha).
// tab = [T | E | nu | alpha], each [nmat][npts].
template <int DEG>
__global__ void k_cell_coef(int64_t nc, const int32_t *__restrict__ cells, const double *__restrict__ T,
                            const int32_t *__restrict__ cmat, int nmat, int npts, const double *__restrict__ tab,
                            double *__restrict__ coef, int32_t *__restrict__ bad) {
    constexpr int NPE = DEG == 1 ? 4 : 10;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t *cv = cells + c * NPE;
        double Tm;
        if (DEG == 1) {
            Tm = 0.25 * (T[cv[0]] + T[cv[1]] + T[cv[2]] + T[cv[3]]);
        } else {
            double sv = 0.0, se = 0.0;
            for (int k = 0; k < 4; ++k) sv += T[cv[k]];
            for (int k = 4; k < 10; ++k) se += T[cv[k]];
            Tm = -0.05 * sv + 0.2 * se;
        }
        int m = cmat[c];
        if (m < 0 || m >= nmat) {
            *bad = 1;
            m = 0;
        }
        const int64_t so = (int64_t)nmat * npts, mo = (int64_t)m * npts;
        const double *Tt = tab + mo;
        const double E = table_at(Tt, tab + so + mo, npts, Tm);
        const double nu = table_at(Tt, tab + 2 * so + mo, npts, Tm);
        const double al = table_at(Tt, tab + 3 * so + mo, npts, Tm);
        const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double mu = E / (2.0 * (1.0 + nu));
        coef[c * 3] = lam;
        coef[c * 3 + 1] = mu;
        coef[c * 3 + 2] = (3.0 * lam + 2.0 * mu) * al;
    }
}

// Pressure load, one thread per node: b_i += p_f |F| w_a n_f over the node's
// (face, local node) entries in face order (w_a = 1/3 for P1 nodes and P2
// edge nodes; P2 vertices have none).
__global__ void k_pressure(int64_t n, const int64_t *__restrict__ ptr, const int64_t *__restrict__ ent, int npf,
                           const int32_t *__restrict__ faces, const double *__restrict__ p,
                           const double *__restrict__ X, double *__restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (ptr[i] == ptr[i + 1]) continue;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
            const int64_t f = ent[e] / npf;
            const int32_t *fv = faces + f * npf;
            double x0[3], d1[3], d2[3];
            for (int k = 0; k < 3; ++k) {
                x0[k] = X[(int64_t)fv[0] * 3 + k];
                d1[k] = X[(int64_t)fv[1] * 3 + k] - x0[k];
                d2[k] = X[(int64_t)fv[2] * 3 + k] - x0[k];
            }
            const double nv[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2],
                                  d1[0] * d2[1] - d1[1] * d2[0]};
            // p |F| / 3 * n = p * |nv| / 2 / 3 * nv / |nv| = p nv / 6
            const double s = p[f] / 6.0;
            for (int k = 0; k < 3; ++k) acc[k] += s * nv[k];
        }
        for (int k = 0; k < 3; ++k) b[i * 3 + k] += acc[k];
    }
}

// ---------------------------------------------------------------------------
// heat equation (eq. wf_thermal): residual and Newton Jacobian
// ---------------------------------------------------------------------------
// F_i = sum over cells of kappa_c (K_c T)_i + rho c_c / dt (M_c (T - T_old))_i
//     + sum over heat-transfer faces of h_f ((M_f T)_i - T_bc,f int_f phi_i),
// kappa_c and c_c the cell's material tables at the cell mean Tbar_c of T_h
// (weights w: P1 1/4; P2 -1/20 vertices, 1/5 edges); J = dF/dT adds the
// rank-one terms kappa'(Tbar) (K_c T) w^T and rho c'(Tbar)/dt (M_c dT) w^T.
struct ThArgs {
    const double *X;
    const int32_t *cells;
    int64_t n;
    const int64_t *start, *inc;
    const int32_t *cmat;
    const double *tab;  // [3][nm][np]
    int nm, np;
    const double *rho;
    const int64_t *fptr, *fent;
    const int32_t *faces;
    const double *h, *Tbc;
    const double *T, *Told;
    double inv_dt;      // 0: steady
    const int64_t *ptr;
    const int32_t *col;
    double *J, *F;
};

// piecewise-linear table, constant beyond its ends: value at x and the slope
// of the segment [T_k, T_k+1) holding x (0 outside)
__device__ __forceinline__ void table_eval(const double *Tt, const double *v, int np, double x, double &val,
                                           double &slope) {
    int k = -1;
    for (int j = 0; j < np; ++j)
        if (Tt[j] <= x) k = j;
    if (k < 0) {
        val = v[0];
        slope = 0.0;
    } else if (k >= np - 1) {
        val = v[np - 1];
        slope = 0.0;
    } else {
        slope = (v[k + 1] - v[k]) / (Tt[k + 1] - Tt[k]);
        val = slope * (x - Tt[k]) + v[k];
    }
}

__device__ __forceinline__ int64_t row_pos(const int32_t *__restrict__ col, int64_t r0, int64_t r1, int32_t c) {
    int64_t lo = r0, hi = r1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// P2 triangle mass matrix times 180/|F| (vertices, then edges 01, 02, 12)
__device__ __forceinline__ double p2_face_mass180(int a, int b) {
    if (a < 3 && b < 3) return a == b ? 6.0 : -1.0;
    if (a >= 3 && b >= 3) return a == b ? 32.0 : 16.0;
    const int v = a < 3 ? a : b, e = a < 3 ? b : a;
    // edge 3 = (0,1), 4 = (0,2), 5 = (1,2): the vertex opposite is 2, 1, 0
    return (5 - e) == v ? -4.0 : 0.0;
}

template <int DEG>
__global__ void __launch_bounds__(ABLK) k_thermal(ThArgs A) {
    const int64_t i = (int64_t)blockIdx.x * ABLK + threadIdx.x;
    if (i >= A.n) return;
    constexpr int NPE = DEG == 1 ? 4 : 10;
    constexpr int NPF = DEG == 1 ? 3 : 6;
    __shared__ double s_g[ABLK][12];
    double *G = s_g[threadIdx.x];
    const int64_t r0 = A.ptr[i], r1 = A.ptr[i + 1];
    for (int64_t k = r0; k < r1; ++k) A.J[k] = 0.0;
    double Fi = 0.0;
    for (int64_t e = A.start[i]; e < A.start[i + 1]; ++e) {
        const int64_t cell = A.inc[e] / NPE;
        const int a = (int)(A.inc[e] % NPE);
        const int32_t *cv = A.cells + cell * NPE;
        const Geo g = cell_geo(A.X, cv);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) G[k * 3 + c] = g.G[k][c];
        double Tc[NPE], w[NPE];
        double Tbar = 0.0;
        for (int c = 0; c < NPE; ++c) {
            Tc[c] = A.T[cv[c]];
            w[c] = DEG == 1 ? 0.25 : (c < 4 ? -0.05 : 0.2);
            Tbar += w[c] * Tc[c];
        }
        const int m = A.cmat[cell];
        double kap, dkap, cvv = 0.0, dcv = 0.0;
        table_eval(A.tab + (int64_t)m * A.np, A.tab + (int64_t)(A.nm + m) * A.np, A.np, Tbar, kap, dkap);
        if (A.inv_dt > 0.0)
            table_eval(A.tab + (int64_t)m * A.np, A.tab + (int64_t)(2 * A.nm + m) * A.np, A.np, Tbar, cvv, dcv);
        // row a of the reference stiffness int grad phi_a . grad phi_b and mass
        double Kab[NPE], Mab[NPE];
        if (DEG == 1) {
            for (int b = 0; b < NPE; ++b) {
                Kab[b] = g.vol * (G[a * 3] * G[b * 3] + G[a * 3 + 1] * G[b * 3 + 1] + G[a * 3 + 2] * G[b * 3 + 2]);
                Mab[b] = g.vol * (a == b ? 2.0 : 1.0) / 20.0;
            }
        } else {
            for (int b = 0; b < NPE; ++b) Kab[b] = 0.0;
            const double qa = 0.5854101966249685, qb = 0.1381966011250105;
            for (int q = 0; q < 4; ++q) {
                const double l0 = q == 0 ? qa : qb, l1 = q == 1 ? qa : qb, l2 = q == 2 ? qa : qb,
                             l3 = q == 3 ? qa : qb;
                double ga[3];
                p2_grad(a, l0, l1, l2, l3, G, ga);
                for (int b = 0; b < NPE; ++b) {
                    double gb[3];
                    p2_grad(b, l0, l1, l2, l3, G, gb);
                    Kab[b] += 0.25 * g.vol * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
                }
            }
            for (int b = 0; b < NPE; ++b) Mab[b] = g.vol * p2_mass420(a, b) / 420.0;
        }
        double KT = 0.0, MdT = 0.0;
        for (int b = 0; b < NPE; ++b) KT += Kab[b] * Tc[b];
        Fi += kap * KT;
        const double rc = A.inv_dt > 0.0 ? A.rho[m] * A.inv_dt : 0.0;
        if (A.inv_dt > 0.0) {
            for (int b = 0; b < NPE; ++b) MdT += Mab[b] * (Tc[b] - A.Told[cv[b]]);
            Fi += rc * cvv * MdT;
        }
        for (int b = 0; b < NPE; ++b) {
            double v = kap * Kab[b] + dkap * w[b] * KT;
            if (A.inv_dt > 0.0) v += rc * (cvv * Mab[b] + dcv * w[b] * MdT);
            A.J[row_pos(A.col, r0, r1, cv[b])] += v;
        }
    }
    if (A.fptr) {
        for (int64_t e = A.fptr[i]; e < A.fptr[i + 1]; ++e) {
            const int64_t f = A.fent[e] / NPF;
            const int a = (int)(A.fent[e] % NPF);
            const int32_t *fv = A.faces + f * NPF;
            double d1[3], d2[3];
            for (int k = 0; k < 3; ++k) {
                const double x0 = A.X[(int64_t)fv[0] * 3 + k];
                d1[k] = A.X[(int64_t)fv[1] * 3 + k] - x0;
                d2[k] = A.X[(int64_t)fv[2] * 3 + k] - x0;
            }
            const double nx = d1[1] * d2[2] - d1[2] * d2[1], ny = d1[2] * d2[0] - d1[0] * d2[2],
                         nz = d1[0] * d2[1] - d1[1] * d2[0];
            const double area = 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
            const double hf = A.h[f];
            double MT = 0.0;
            for (int b = 0; b < NPF; ++b) {
                const double mf = DEG == 1 ? area * (a == b ? 2.0 : 1.0) / 12.0 : area * p2_face_mass180(a, b) / 180.0;
                MT += mf * A.T[fv[b]];
                A.J[row_pos(A.col, r0, r1, fv[b])] += hf * mf;
            }
            const double fint = DEG == 1 ? area / 3.0 : (a < 3 ? 0.0 : area / 3.0);
            Fi += hf * (MT - A.Tbc[f] * fint);
        }
    }
    A.F[i] = Fi;
}

static void pattern_impl(const te_mesh *m, Incidence &I, int64_t *row_ptr, int32_t *col, hipStream_t s);

void thermal_asm_init(ThermalAsm &ta, const te_mesh *m, const te_thermal_tables *tab, const int32_t *cell_material,
                      const te_robin *robin, hipStream_t s) {
    TE_REQUIRE(m && tab && cell_material, TE_EINVAL, "NULL argument");
    TE_REQUIRE(m->degree == 1 || m->degree == 2, TE_EINVAL, "degree must be 1 or 2 (got %d)", m->degree);
    TE_REQUIRE(m->n_nodes > 0 && m->n_cells > 0 && m->coords && m->cells, TE_EINVAL, "empty mesh");
    TE_REQUIRE(m->n_nodes < (int64_t)INT32_MAX, TE_EINVAL, "too many nodes for 32-bit indices");
    const int nm = tab->n_materials, np = tab->n_points;
    TE_REQUIRE(nm >= 1 && np >= 1 && tab->T && tab->kappa && tab->cv && tab->rho, TE_EINVAL,
               "thermal tables are empty or NULL");
    std::vector<double> h((size_t)3 * nm * np);
    const size_t so = (size_t)nm * np;
    for (int mm = 0; mm < nm; ++mm) {
        TE_REQUIRE(tab->rho[mm] > 0.0, TE_EINVAL, "material %d: density must be positive", mm);
        for (int k = 0; k < np; ++k) {
            const size_t q = (size_t)mm * np + k;
            TE_REQUIRE(k == 0 || tab->T[q] > tab->T[q - 1], TE_EINVAL, "material %d: temperatures not ascending", mm);
            TE_REQUIRE(tab->kappa[q] > 0.0 && tab->cv[q] > 0.0, TE_EINVAL,
                       "material %d: conductivity and specific heat must be positive", mm);
            h[q] = tab->T[q];
            h[so + q] = tab->kappa[q];
            h[2 * so + q] = tab->cv[q];
        }
    }
    ta.n = m->n_nodes;
    ta.nc = m->n_cells;
    ta.degree = m->degree;
    ta.npe = m->degree == 1 ? 4 : 10;
    ta.npf = m->degree == 1 ? 3 : 6;
    ta.nm = nm;
    ta.np = np;
    upload(ta.tab, h, s);
    upload(ta.rho, std::vector<double>(tab->rho, tab->rho + nm), s);
    ta.coords.alloc(ta.n * 3);
    ta.cells.alloc(ta.nc * ta.npe);
    ta.cell_material.alloc(ta.nc);
    TE_CHECK_HIP(hipMemcpyAsync(ta.coords.p, m->coords, ta.n * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    TE_CHECK_HIP(hipMemcpyAsync(ta.cells.p, m->cells, ta.nc * ta.npe * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    TE_CHECK_HIP(hipMemcpyAsync(ta.cell_material.p, cell_material, ta.nc * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    te_mesh mc{ta.n, ta.nc, ta.degree, ta.coords.p, ta.cells.p};
    build_incidence(&mc, ta.npe, ta.I, s);  // rejects node ids outside the mesh
    {
        std::vector<int32_t> cm;
        download(cm, ta.cell_material.p, (size_t)ta.nc, s);
        for (int32_t v : cm) TE_REQUIRE(v >= 0 && v < nm, TE_EINVAL, "a cell material id is outside 0..%d", nm - 1);
    }
    ta.n_faces = robin ? robin->n_faces : 0;
    TE_REQUIRE(ta.n_faces >= 0, TE_EINVAL, "negative face count");
    if (ta.n_faces > 0) {
        TE_REQUIRE(robin->faces && robin->h && robin->T_bc, TE_EINVAL, "heat-transfer face arrays are NULL");
        const int npf = ta.npf;
        std::vector<int32_t> fh;
        download(fh, robin->faces, (size_t)ta.n_faces * npf, s);
        std::vector<double> hh, tb;
        download(hh, robin->h, (size_t)ta.n_faces, s);
        download(tb, robin->T_bc, (size_t)ta.n_faces, s);
        for (double v : hh) TE_REQUIRE(v >= 0.0, TE_EINVAL, "heat-transfer coefficients must be >= 0");
        std::vector<int64_t> cnt(ta.n + 1, 0);
        for (int64_t q = 0; q < (int64_t)fh.size(); ++q) {
            TE_REQUIRE(fh[q] >= 0 && fh[q] < ta.n, TE_EINVAL, "face %lld has a node outside the mesh",
                       (long long)(q / npf));
            ++cnt[fh[q] + 1];
        }
        for (int64_t i = 0; i < ta.n; ++i) cnt[i + 1] += cnt[i];
        std::vector<int64_t> ent(cnt[ta.n]), fill(cnt.begin(), cnt.end() - 1);
        for (int64_t q = 0; q < (int64_t)fh.size(); ++q) ent[fill[fh[q]]++] = q;
        upload(ta.fptr, cnt, s);
        upload(ta.fent, ent, s);
        upload(ta.faces, fh, s);
        upload(ta.h, hh, s);
        upload(ta.T_bc, tb, s);
    }
    ta.ptr.alloc(ta.n + 1);
    pattern_impl(&mc, ta.I, ta.ptr.p, nullptr, s);
    TE_CHECK_HIP(hipMemcpyAsync(&ta.nnz, ta.ptr.p + ta.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    ta.col.alloc(std::max<int64_t>(ta.nnz, 1));
    pattern_impl(&mc, ta.I, ta.ptr.p, ta.col.p, s);
}

void thermal_asm_run(const ThermalAsm &ta, const double *T, const double *T_old, double dt, double *Jval, double *F,
                     hipStream_t s) {
    const bool transient = T_old != nullptr && dt > 0.0;
    ThArgs a{ta.coords.p, ta.cells.p, ta.n, ta.I.start.p, ta.I.inc.p, ta.cell_material.p, ta.tab.p, ta.nm, ta.np,
             ta.rho.p, ta.n_faces > 0 ? ta.fptr.p : nullptr, ta.fent.p, ta.faces.p, ta.h.p, ta.T_bc.p, T,
             transient ? T_old : nullptr, transient ? 1.0 / dt : 0.0, ta.ptr.p, ta.col.p, Jval, F};
    const unsigned g = (unsigned)((ta.n + ABLK - 1) / ABLK);
    if (ta.degree == 1) hipLaunchKernelGGL(k_thermal<1>, dim3(g), dim3(ABLK), 0, s, a);
    else hipLaunchKernelGGL(k_thermal<2>, dim3(g), dim3(ABLK), 0, s, a);
    TE_CHECK_HIP(hipGetLastError());
}

static void check_mesh(const te_mesh *m) {
    TE_REQUIRE(m, TE_EINVAL, "mesh is NULL");
    TE_REQUIRE(m->degree == 1 || m->degree == 2, TE_EINVAL, "degree must be 1 or 2 (got %d)", m->degree);
    TE_REQUIRE(m->n_nodes > 0 && m->n_cells > 0, TE_EINVAL, "empty mesh");
    TE_REQUIRE(m->n_nodes < (int64_t)INT32_MAX, TE_EINVAL, "too many nodes for 32-bit indices");
    TE_REQUIRE(m->coords && m->cells, TE_EINVAL, "mesh arrays are NULL");
}

static void pattern_impl(const te_mesh *m, Incidence &I, int64_t *row_ptr, int32_t *col, hipStream_t s) {
    const int npe = m->degree == 1 ? 4 : 10;
    const int64_t n = m->n_nodes;
    DBuf<int32_t> ovf(1);
    TE_CHECK_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int32_t), s));
    unsigned g = (unsigned)((n + ABLK - 1) / ABLK);
    if (!col) {
        DBuf<int32_t> cnt(n);
        hipLaunchKernelGGL(k_pattern, dim3(g), dim3(ABLK), 0, s, m->cells, npe, I.start.p, I.inc.p, n, 0, cnt.p,
                           nullptr, nullptr, ovf.p);
        TE_CHECK_HIP(hipGetLastError());
        int32_t h = 0;
        TE_CHECK_HIP(hipMemcpyAsync(&h, ovf.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        TE_REQUIRE(h == 0, TE_EINVAL, "a node couples to more than %d nodes", PCAP);
        scan_counts(cnt.p, row_ptr, n, s);
    } else {
        hipLaunchKernelGGL(k_pattern, dim3(g), dim3(ABLK), 0, s, m->cells, npe, I.start.p, I.inc.p, n, 1, nullptr,
                           row_ptr, col, ovf.p);
        TE_CHECK_HIP(hipGetLastError());
        int32_t h = 0;
        TE_CHECK_HIP(hipMemcpyAsync(&h, ovf.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        TE_REQUIRE(h == 0, TE_EINVAL, h == 1 ? "a node couples to more than 192 nodes"
                                             : "row_ptr does not match this mesh's sparsity pattern");
    }
}

}  // namespace te

using namespace te;

extern "C" int fe_assemble_pattern(const te_mesh *mesh, int64_t *row_ptr, int64_t *nnzb_out, hipStream_t stream) {
    return guarded([&]() -> int {
        check_mesh(mesh);
        TE_REQUIRE(row_ptr && nnzb_out, TE_EINVAL, "row_ptr / nnzb_out is NULL");
        Incidence I;
        build_incidence(mesh, mesh->degree == 1 ? 4 : 10, I, stream);
        pattern_impl(mesh, I, row_ptr, nullptr, stream);
        TE_CHECK_HIP(hipMemcpyAsync(nnzb_out, row_ptr + mesh->n_nodes, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

static void material_consts(const te_material *mat, double &lam, double &mu, double &calpha) {
    TE_REQUIRE(mat, TE_EINVAL, "material is NULL");
    TE_REQUIRE(mat->E > 0 && mat->nu > -1.0 && mat->nu < 0.5, TE_EINVAL, "invalid E / nu");
    lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
    mu = mat->E / (2.0 * (1.0 + mat->nu));
    calpha = (3.0 * lam + 2.0 * mu) * mat->alpha;
}

extern "C" int fe_assemble_thermoelastic(const te_mesh *mesh, const te_material *mat, const double *T,
                                         const double *f, const uint8_t *dir_mask, const double *u_bc, te_bsr *A,
                                         double *b, hipStream_t stream) {
    return guarded([&]() -> int {
        check_mesh(mesh);
        TE_REQUIRE(T && b && A && A->row_ptr && A->col_idx && A->val, TE_EINVAL, "NULL array argument");
        TE_REQUIRE(A->n_brows == mesh->n_nodes, TE_EINVAL, "A.n_brows != n_nodes");
        double lam, mu, calpha;
        material_consts(mat, lam, mu, calpha);
        const int npe = mesh->degree == 1 ? 4 : 10;
        Incidence I;
        build_incidence(mesh, npe, I, stream);
        int64_t nnzb = 0;
        TE_CHECK_HIP(hipMemcpyAsync(&nnzb, A->row_ptr + mesh->n_nodes, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        TE_REQUIRE(nnzb == A->nnzb, TE_EINVAL, "A.nnzb (%lld) != row_ptr[N] (%lld)", (long long)A->nnzb,
                   (long long)nnzb);
        pattern_impl(mesh, I, A->row_ptr, A->col_idx, stream);
        AsmArgs a{mesh->coords, mesh->cells, npe, I.start.p, I.inc.p, mesh->n_nodes, lam, mu, calpha, mat->T_ref,
                  nullptr, T, f, A->row_ptr, A->col_idx, A->val, b, 1};
        const unsigned gs = (unsigned)std::min<int64_t>(mesh->n_nodes, 1 << 18);
        if (mesh->degree == 1) hipLaunchKernelGGL(k_stiff<1>, dim3(gs), dim3(64), 0, stream, a);
        else hipLaunchKernelGGL(k_stiff<2>, dim3(gs), dim3(64), 0, stream, a);
        TE_CHECK_HIP(hipGetLastError());
        unsigned g = (unsigned)((mesh->n_nodes + ABLK - 1) / ABLK);
        if (mesh->degree == 1) hipLaunchKernelGGL(k_assemble<1>, dim3(g), dim3(ABLK), 0, stream, a, 0);
        else hipLaunchKernelGGL(k_assemble<2>, dim3(g), dim3(ABLK), 0, stream, a, 0);
        TE_CHECK_HIP(hipGetLastError());
        if (dir_mask) {
            unsigned gd = (unsigned)std::min<int64_t>((mesh->n_nodes + 255) / 256, 1 << 20);
            hipLaunchKernelGGL(k_dirichlet, dim3(gd), dim3(256), 0, stream, mesh->n_nodes, A->row_ptr, A->col_idx,
                               A->val, b, dir_mask, u_bc);
            TE_CHECK_HIP(hipGetLastError());
        }
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

extern "C" int fe_assemble_load(const te_mesh *mesh, const te_material *mat, const double *T, const double *f,
                                const uint8_t *dir_mask, int32_t nrhs, double *b, hipStream_t stream) {
    return guarded([&]() -> int {
        check_mesh(mesh);
        TE_REQUIRE(T && b, TE_EINVAL, "NULL array argument");
        TE_REQUIRE(nrhs >= 1 && nrhs <= 64, TE_EINVAL, "nrhs must be in 1..64");
        double lam, mu, calpha;
        material_consts(mat, lam, mu, calpha);
        const int npe = mesh->degree == 1 ? 4 : 10;
        Incidence I;
        build_incidence(mesh, npe, I, stream);
        AsmArgs a{mesh->coords, mesh->cells, npe, I.start.p, I.inc.p, mesh->n_nodes, lam, mu, calpha, mat->T_ref,
                  nullptr, T, f, nullptr, nullptr, nullptr, b, nrhs};
        unsigned g = (unsigned)((mesh->n_nodes + ABLK - 1) / ABLK);
        for (int j = 0; j < nrhs; ++j) {
            if (mesh->degree == 1) hipLaunchKernelGGL(k_assemble<1>, dim3(g), dim3(ABLK), 0, stream, a, j);
            else hipLaunchKernelGGL(k_assemble<2>, dim3(g), dim3(ABLK), 0, stream, a, j);
            TE_CHECK_HIP(hipGetLastError());
        }
        if (dir_mask) {
            unsigned gd = (unsigned)std::min<int64_t>((mesh->n_nodes * 3 * nrhs + 255) / 256, 1 << 20);
            hipLaunchKernelGGL(k_zero_masked, dim3(gd), dim3(256), 0, stream, mesh->n_nodes, nrhs, b, dir_mask);
            TE_CHECK_HIP(hipGetLastError());
        }
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}

extern "C" int fe_assemble_thermoelastic_materials(const te_mesh *mesh, const te_material_tables *mat,
                                                   const int32_t *cell_material, const double *T, const double *f,
                                                   const te_pressure *pressure, const uint8_t *dir_mask,
                                                   const double *u_bc, te_bsr *A, double *b, hipStream_t stream) {
    return guarded([&]() -> int {
        check_mesh(mesh);
        TE_REQUIRE(mat && cell_material && T && b && A && A->row_ptr && A->col_idx && A->val, TE_EINVAL,
                   "NULL argument");
        TE_REQUIRE(A->n_brows == mesh->n_nodes, TE_EINVAL, "A.n_brows != n_nodes");
        const int nm = mat->n_materials, np = mat->n_points;
        TE_REQUIRE(nm >= 1 && np >= 1 && mat->T && mat->E && mat->nu && mat->alpha, TE_EINVAL,
                   "material tables are empty or NULL");
        std::vector<double> tab((size_t)4 * nm * np);
        for (int m = 0; m < nm; ++m)
            for (int k = 0; k < np; ++k) {
                const size_t q = (size_t)m * np + k, so = (size_t)nm * np;
                const double Tk = mat->T[q], E = mat->E[q], nu = mat->nu[q];
                TE_REQUIRE(k == 0 || Tk > mat->T[q - 1], TE_EINVAL, "material %d: temperatures not ascending", m);
                TE_REQUIRE(E > 0 && nu > -1.0 && nu < 0.5, TE_EINVAL, "material %d: invalid E / nu at sample %d", m, k);
                tab[q] = Tk;
                tab[so + q] = E;
                tab[2 * so + q] = nu;
                tab[3 * so + q] = mat->alpha[q];
            }
        const int npe = mesh->degree == 1 ? 4 : 10;
        const int64_t nc = mesh->n_cells, n = mesh->n_nodes;
        // node -> cell incidence first: it rejects node ids outside the mesh
        // before any kernel reads through them
        Incidence I;
        build_incidence(mesh, npe, I, stream);
        DBuf<double> dtab, coef(nc * 3);
        upload(dtab, tab, stream);
        DBuf<int32_t> bad(1);
        TE_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), stream));
        const unsigned gc = (unsigned)std::min<int64_t>((nc + 255) / 256, 1 << 20);
        if (mesh->degree == 1)
            hipLaunchKernelGGL(k_cell_coef<1>, dim3(gc), dim3(256), 0, stream, nc, mesh->cells, T, cell_material, nm,
                               np, dtab.p, coef.p, bad.p);
        else
            hipLaunchKernelGGL(k_cell_coef<2>, dim3(gc), dim3(256), 0, stream, nc, mesh->cells, T, cell_material, nm,
                               np, dtab.p, coef.p, bad.p);
        TE_CHECK_HIP(hipGetLastError());
        int32_t hb = 0;
        TE_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        int64_t nnzb = 0;
        TE_CHECK_HIP(hipMemcpyAsync(&nnzb, A->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        TE_REQUIRE(hb == 0, TE_EINVAL, "a cell material id is outside 0..%d", nm - 1);
        TE_REQUIRE(nnzb == A->nnzb, TE_EINVAL, "A.nnzb (%lld) != row_ptr[N] (%lld)", (long long)A->nnzb,
                   (long long)nnzb);
        // node -> (face, local node) entries of the pressure faces, in face order
        const bool has_p = pressure && pressure->n_faces > 0;
        DBuf<int64_t> pptr, pent;
        const int npf = mesh->degree == 1 ? 3 : 6;
        if (has_p) {
            TE_REQUIRE(pressure->faces && pressure->p, TE_EINVAL, "pressure faces / values are NULL");
            std::vector<int32_t> fh;
            download(fh, pressure->faces, (size_t)pressure->n_faces * npf, stream);
            std::vector<int64_t> cnt(n + 1, 0);
            const int a0 = mesh->degree == 1 ? 0 : 3;  // P2 vertices carry no pressure load
            for (int64_t q = 0; q < (int64_t)fh.size(); ++q) {
                TE_REQUIRE(fh[q] >= 0 && fh[q] < n, TE_EINVAL, "pressure face %lld has a node outside the mesh",
                           (long long)(q / npf));
                if (q % npf >= a0) ++cnt[fh[q] + 1];
            }
            for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
            std::vector<int64_t> ent(cnt[n]), fill(cnt.begin(), cnt.end() - 1);
            for (int64_t q = 0; q < (int64_t)fh.size(); ++q)
                if (q % npf >= a0) ent[fill[fh[q]]++] = q;
            upload(pptr, cnt, stream);
            upload(pent, ent, stream);
        }
        pattern_impl(mesh, I, A->row_ptr, A->col_idx, stream);
        AsmArgs a{mesh->coords, mesh->cells, npe, I.start.p, I.inc.p, n, 0.0, 0.0, 0.0, mat->T_ref,
                  coef.p, T, f, A->row_ptr, A->col_idx, A->val, b, 1};
        const unsigned gs = (unsigned)std::min<int64_t>(n, 1 << 18);
        if (mesh->degree == 1) hipLaunchKernelGGL(k_stiff<1>, dim3(gs), dim3(64), 0, stream, a);
        else hipLaunchKernelGGL(k_stiff<2>, dim3(gs), dim3(64), 0, stream, a);
        TE_CHECK_HIP(hipGetLastError());
        const unsigned g = (unsigned)((n + ABLK - 1) / ABLK);
        if (mesh->degree == 1) hipLaunchKernelGGL(k_assemble<1>, dim3(g), dim3(ABLK), 0, stream, a, 0);
        else hipLaunchKernelGGL(k_assemble<2>, dim3(g), dim3(ABLK), 0, stream, a, 0);
        TE_CHECK_HIP(hipGetLastError());
        if (has_p) {
            const unsigned gp = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20);
            hipLaunchKernelGGL(k_pressure, dim3(gp), dim3(256), 0, stream, n, pptr.p, pent.p, npf, pressure->faces,
                               pressure->p, mesh->coords, b);
            TE_CHECK_HIP(hipGetLastError());
        }
        if (dir_mask) {
            const unsigned gd = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20);
            hipLaunchKernelGGL(k_dirichlet, dim3(gd), dim3(256), 0, stream, n, A->row_ptr, A->col_idx, A->val, b,
                               dir_mask, u_bc);
            TE_CHECK_HIP(hipGetLastError());
        }
        TE_CHECK_HIP(hipStreamSynchronize(stream));
        return TE_OK;
    });
}
