// Sparse and vector kernels of the PCG / V-cycle hot loop (gfx950, wave64).
//
// Every sparse product runs on the SELL-64 block layout of te_internal.h:
// one lane per block row, 64 rows per wave, entry k of all 64 lanes stored
// contiguously so each value plane is one fully coalesced 512-byte (float64)
// load per wave.  Rows inside a slice are sorted by descending length, so the
// per-lane length mask switches off whole cache lines of padding at the tail.
// The x gathers hit L2: node numbering is lexicographic, and the block index
// is remapped so that each XCD streams one contiguous range of slices and
// keeps its own L2 window of x.
//
// Multi-RHS products (nrhs > 1, vectors laid out [row][comp][rhs]) use one
// wave per block row with the right-hand sides on the lanes; the block values
// are wave-uniform and come through the scalar cache.
//
// Epilogues fuse the vector work of the Chebyshev smoother (Saad, Alg. 12.1),
// the residual of the V-cycle and the dot products of CG into the product.
// All reductions are deterministic: per-block partials in a fixed order,
// then summed in a fixed order (by one workgroup, or, for large partial
// tables, by fixed chunks and then the chunk sums).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "te_dev.h"

namespace te {
// Single right-hand side, lane per row: each wave handles `spw` consecutive
// slices, a workgroup blockDim/64 waves (both chosen by the autotuner);
// `remap` turns the XCD-contiguous block order on.
template <int BR, int BC, typename VT, typename XT, typename AT, class Epi, bool NT>
__global__ void __launch_bounds__(512) k_sell1(SellView<VT> A, const XT *__restrict__ x, Epi epi,
                                               double *__restrict__ partials, int spw, int remap) {
    __shared__ double lds[16];
    const int64_t nb = gridDim.x;
    const int64_t lb = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w0 = (lb * (blockDim.x / WAVE) + threadIdx.x / WAVE) * spw;
    double red = 0.0;
    for (int u = 0; u < spw; ++u)
        if (w0 + u < A.nslices) sell1_body<BR, BC, VT, XT, AT, Epi, NT>(A, x, epi, w0 + u, lane, red);
    if (Epi::kReduce) {
        double t = block_sum(red, lds);
        if (threadIdx.x == 0) partials[lb] = t;
    }
}

// Several right-hand sides on the SELL layout, one wave per block row with
// the right-hand sides on the lanes (at most 64); the block values are
// wave-uniform (scalar loads), the row's column indices come 64 at a time
// and are taken by readlane, and the x rows of 4 entries are loaded before
// any of them is used.  The default above 16 columns; the tuner may pick
// the row groups below instead.
template <int BR, int BC, typename VT, typename XT, typename AT, class Epi>
__global__ void __launch_bounds__(512) k_sellw(SellView<VT> A, const XT *__restrict__ x, Epi epi, int nrhs,
                                               double *__restrict__ partials, int wpb) {
    constexpr int MU = BC <= 3 ? 4 : 2;
    __shared__ double lds[8 * WAVE];
    const int64_t nb = gridDim.x;
    const int64_t lb = xcd_logical_block(blockIdx.x, nb);
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t row = (int64_t)__builtin_amdgcn_readfirstlane((int)(lb * wpb + threadIdx.x / WAVE));
    double red = 0.0;
    if (row < A.nrows) {
        const int rl = (int)(row % WAVE);
        const int off = A.slice_off[row / WAVE];
        const int len = A.rowlen[row];
        AT acc[BR];
#pragma unroll
        for (int i = 0; i < BR; ++i) acc[i] = AT(0);
        auto entry = [&](int k, const AT *xv) {
            const VT *vk = A.val + (int64_t)(off + k) * (BR * BC * WAVE);
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j)
                    acc[i] += AT(vk[sell_val_off<sell_vw<VT>()>(i * BC + j, BR * BC, rl)]) * xv[j];
        };
        for (int k0 = 0; k0 < len; k0 += WAVE) {
            const int cnt = min(WAVE, len - k0);
            const int cl = k0 + lane < len ? A.col[(int64_t)(off + k0 + lane) * WAVE + rl] : 0;
            if (lane < nrhs) {
                int u = 0;
                for (; u + MU <= cnt; u += MU) {
                    AT xv[MU][BC];
#pragma unroll
                    for (int t = 0; t < MU; ++t) {
                        const int64_t c = __builtin_amdgcn_readlane(cl, u + t);
#pragma unroll
                        for (int j = 0; j < BC; ++j) xv[t][j] = AT(x[(c * BC + j) * nrhs + lane]);
                    }
#pragma unroll
                    for (int t = 0; t < MU; ++t) entry(k0 + u + t, xv[t]);
                }
                for (; u < cnt; ++u) {
                    const int64_t c = __builtin_amdgcn_readlane(cl, u);
                    AT xv[BC];
#pragma unroll
                    for (int j = 0; j < BC; ++j) xv[j] = AT(x[(c * BC + j) * nrhs + lane]);
                    entry(k0 + u, xv);
                }
            }
        }
        if (lane < nrhs) {
            const int64_t out = A.rowmap ? (int64_t)A.rowmap[row] : row;
            epi.template apply_m<BR>(out, lane, nrhs, acc, red);
        }
    }
    if (Epi::kReduce) {
        lds[threadIdx.x] = red;
        __syncthreads();
        if (threadIdx.x < WAVE && threadIdx.x < nrhs) {
            double t = 0.0;
            for (int w = 0; w < wpb; ++w) t += lds[w * WAVE + threadIdx.x];
            partials[lb * nrhs + threadIdx.x] = t;
        }
    }
}

// Several right-hand sides on the SELL layout in row groups: R consecutive
// block rows of one slice per wave, T = 64 / R lanes per row, each lane S
// right-hand sides
// (c0 + j, c0 + j + T, ...) of the column tile c0 = blockIdx.y * T * S.  A
// lane loads its row's block values (vector loads: the R rows of a wave
// share each 16-byte value piece line) and reuses them for its S columns;
// the x rows of MU entries are loaded before any is used.  Column tiles are
// the slowest grid dimension, so the whole matrix runs for one tile before
// the next and the x rows an XCD gathers (tile width x 24 bytes per node)
// stay in its L2; the matrix is read once per tile.  The rows of a slice are
// sorted by descending length, so the first row of the wave bounds the
// entry loop; shorter rows run over their zero padding blocks (valid
// columns).  `wpb` waves per workgroup.  With split_tiles > 0 the column
// tiles are spread over the XCDs instead (see the kernel).
template <int BC, int S>
constexpr int multi_unroll() {
    return BC <= 3 && S <= 2 ? 2 : 1;
}

template <int BR, int BC, typename VT, typename XT, typename AT, class Epi, int R, int S>
__global__ void __launch_bounds__(512) k_sellm(SellView<VT> A, const XT *__restrict__ x, Epi epi, int nrhs,
                                                double *__restrict__ partials, int wpb, int split_tiles,
                                                int64_t split_chunk, int64_t nrb) {
    constexpr int T = WAVE / R, E = BR * BC, MU = multi_unroll<BC, S>();
    constexpr int VW = sell_vw<VT>(), G = E / VW;
    typedef VT vec_t __attribute__((ext_vector_type(VW)));
    __shared__ double lds[16 * WAVE];
    int64_t lb;
    int c0;
    if (split_tiles) {
        // workgroup b runs on XCD b % 8: the XCDs are split_tiles column tiles
        // times 8 / split_tiles row ranges, so the XCDs of one range stream the
        // same rows (and value lines) at the same time, each for its tile
        const int xcd = (int)(blockIdx.x & 7);
        const int64_t i = blockIdx.x >> 3;
        lb = (int64_t)(xcd / split_tiles) * split_chunk + i;
        if (i >= split_chunk || lb >= nrb) return;   // the whole workgroup
        c0 = (xcd % split_tiles) * (T * S);
    } else {
        lb = xcd_logical_block(blockIdx.x, gridDim.x);
        c0 = blockIdx.y * (T * S);
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int q = lane / T, w = threadIdx.x / WAVE;
    const int j = c0 + lane % T;      // first column of the lane
    const int64_t row0 = (lb * wpb + w) * R;
    const int64_t row = row0 + q;
    double red[S];
#pragma unroll
    for (int t = 0; t < S; ++t) red[t] = 0.0;
    if (row0 < A.nrows) {
        // rows past the end (last slice) compute on row0's entries, store nothing
        const bool live = row < A.nrows;
        const int64_t rr = live ? row : row0;
        const int rl = (int)(rr % WAVE);
        const int off = A.slice_off[rr / WAVE];
        const int lmax = __builtin_amdgcn_readfirstlane(A.rowlen[row0]);
        AT acc[S][BR];
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int i = 0; i < BR; ++i) acc[t][i] = AT(0);
        for (int k = 0; k < lmax; k += MU) {
            VT v[MU][E];
            AT xv[MU][S][BC];
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                const int kk = min(k + u, lmax - 1);   // a repeated entry is not accumulated
                const int64_t c = A.col[(int64_t)(off + kk) * WAVE + rl];
                const VT *vk = A.val + (int64_t)(off + kk) * (E * WAVE);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const vec_t t = *reinterpret_cast<const vec_t *>(vk + (int64_t)(g * WAVE + rl) * VW);
#pragma unroll
                    for (int e = 0; e < VW; ++e) v[u][g * VW + e] = t[e];
                }
#pragma unroll
                for (int e = G * VW; e < E; ++e) v[u][e] = vk[(int64_t)(G * VW) * WAVE + (e - G * VW) * WAVE + rl];
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    const int jj = j + t * T;
#pragma unroll
                    for (int b = 0; b < BC; ++b) xv[u][t][b] = jj < nrhs ? AT(x[(c * BC + b) * nrhs + jj]) : AT(0);
                }
            }
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                if (k + u >= lmax) break;
#pragma unroll
                for (int t = 0; t < S; ++t)
#pragma unroll
                    for (int i = 0; i < BR; ++i)
#pragma unroll
                        for (int b = 0; b < BC; ++b) acc[t][i] += AT(v[u][i * BC + b]) * xv[u][t][b];
            }
        }
        if (live) {
            const int64_t out = A.rowmap ? (int64_t)A.rowmap[row] : row;
#pragma unroll
            for (int t = 0; t < S; ++t)
                if (j + t * T < nrhs) epi.template apply_m<BR>(out, j + t * T, nrhs, acc[t], red[t]);
        }
    }
    if (Epi::kReduce) {
        // per column: the R rows of the wave by a fixed shuffle tree, then the
        // waves of the block in order
#pragma unroll
        for (int t = 0; t < S; ++t) {
            double v = red[t];
#pragma unroll
            for (int o = T; o < WAVE; o <<= 1) v += __shfl_xor(v, o, WAVE);
            if (q == 0) lds[w * WAVE + (j - c0) + t * T] = v;
        }
        __syncthreads();
        if (threadIdx.x < T * S && c0 + (int)threadIdx.x < nrhs) {
            double t = 0.0;
            for (int ww = 0; ww < wpb; ++ww) t += lds[ww * WAVE + threadIdx.x];
            partials[lb * nrhs + c0 + threadIdx.x] = t;
        }
    }
}

template <int BR, int BC, typename VT, typename XT, typename AT, class Epi, bool NT>
__global__ void __launch_bounds__(512) k_roww(RowView<VT> A, const XT *__restrict__ x, Epi epi,
                                              double *__restrict__ partials, int spw, int remap, int xb) {
    __shared__ double rlds[16];
    __shared__ AT wb[512];
    const int64_t nb = gridDim.x;
    const int64_t lb = remap ? xcd_logical_block(blockIdx.x, nb) : (int64_t)blockIdx.x;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t w0 = (lb * (blockDim.x / WAVE) + threadIdx.x / WAVE) * spw;
    AT *wbuf = wb + (threadIdx.x / WAVE) * WAVE;
    double red = 0.0;
    if constexpr (BC <= BR) {
        if (xb) {
            for (int u = 0; u < spw; ++u)
                if (w0 + u < A.nrows)
                    roww_body<BR, BC, VT, XT, AT, Epi, NT, true>(A, x, epi, w0 + u, lane, red, wbuf);
        } else {
            for (int u = 0; u < spw; ++u)
                if (w0 + u < A.nrows) roww_body<BR, BC, VT, XT, AT, Epi, NT>(A, x, epi, w0 + u, lane, red, wbuf);
        }
    } else {
        for (int u = 0; u < spw; ++u)
            if (w0 + u < A.nrows) roww_body<BR, BC, VT, XT, AT, Epi, NT>(A, x, epi, w0 + u, lane, red, wbuf);
    }
    if (Epi::kReduce) {
        double t = block_sum(red, rlds);
        if (threadIdx.x == 0) partials[lb] = t;
    }
}

// Format 1 with several right-hand sides: one wave per row, lane = RHS, MU
// blocks' x rows loaded before they are used (as k_sellm).
template <int BR, int BC, typename VT, typename XT, typename AT, class Epi>
__global__ void __launch_bounds__(1024) k_rowwm(RowView<VT> A, const XT *__restrict__ x, Epi epi, int nrhs,
                                                double *__restrict__ partials, int wpb) {
    constexpr int MU = BC <= 3 ? 4 : 2;
    __shared__ double lds[1024];
    const int64_t nb = gridDim.x;
    const int64_t lb = xcd_logical_block(blockIdx.x, nb);
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t row = (int64_t)__builtin_amdgcn_readfirstlane((int)(lb * wpb + threadIdx.x / WAVE));
    double red = 0.0;
    if (row < A.nrows) {
        AT acc[BR];
#pragma unroll
        for (int i = 0; i < BR; ++i) acc[i] = AT(0);
        // TR: the block is stored transposed (mirror of a lower block)
        auto block = [&](const VT *v, const AT *xv, bool tr) {
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j) acc[i] += AT(tr ? v[j * BC + i] : v[i * BC + j]) * xv[j];
        };
        // column indices 64 at a time (every lane active), taken with readlane
        const int64_t lo = A.rptr[row], hi = A.rptr[row + 1];
        for (int64_t k0 = lo; k0 < hi; k0 += WAVE) {
            const int cnt = (int)min((int64_t)WAVE, hi - k0);
            const int cl = k0 + lane < hi ? A.col[k0 + lane] : 0;
            if (lane < nrhs) {
                int u = 0;
                for (; u + MU <= cnt; u += MU) {
                    AT xv[MU][BC];
#pragma unroll
                    for (int t = 0; t < MU; ++t) {
                        const int64_t c = __builtin_amdgcn_readlane(cl, u + t);
#pragma unroll
                        for (int j = 0; j < BC; ++j) xv[t][j] = AT(x[(c * BC + j) * nrhs + lane]);
                    }
#pragma unroll
                    for (int t = 0; t < MU; ++t) block(A.val + (k0 + u + t) * (BR * BC), xv[t], false);
                }
                for (; u < cnt; ++u) {
                    const int64_t c = __builtin_amdgcn_readlane(cl, u);
                    AT xv[BC];
#pragma unroll
                    for (int j = 0; j < BC; ++j) xv[j] = AT(x[(c * BC + j) * nrhs + lane]);
                    block(A.val + (k0 + u) * (BR * BC), xv, false);
                }
            }
        }
        if constexpr (BR == BC) {
            if (A.lptr) {
                const int64_t llo = A.lptr[row], lhi = A.lptr[row + 1];
                for (int64_t q0 = llo; q0 < lhi; q0 += WAVE) {
                    const int cnt = (int)min((int64_t)WAVE, lhi - q0);
                    const int cl = q0 + lane < lhi ? A.lcol[q0 + lane] : 0;
                    const int il = q0 + lane < lhi ? A.lidx[q0 + lane] : 0;
                    if (lane < nrhs) {
                        int u = 0;
                        for (; u + MU <= cnt; u += MU) {
                            AT xv[MU][BC];
#pragma unroll
                            for (int t = 0; t < MU; ++t) {
                                const int64_t c = __builtin_amdgcn_readlane(cl, u + t);
#pragma unroll
                                for (int j = 0; j < BC; ++j) xv[t][j] = AT(x[(c * BC + j) * nrhs + lane]);
                            }
#pragma unroll
                            for (int t = 0; t < MU; ++t)
                                block(A.val + (int64_t)__builtin_amdgcn_readlane(il, u + t) * (BR * BC), xv[t], true);
                        }
                        for (; u < cnt; ++u) {
                            const int64_t c = __builtin_amdgcn_readlane(cl, u);
                            AT xv[BC];
#pragma unroll
                            for (int j = 0; j < BC; ++j) xv[j] = AT(x[(c * BC + j) * nrhs + lane]);
                            block(A.val + (int64_t)__builtin_amdgcn_readlane(il, u) * (BR * BC), xv, true);
                        }
                    }
                }
            }
        }
        if (lane < nrhs) {
            const int64_t out = A.rowmap ? (int64_t)A.rowmap[row] : row;
            epi.template apply_m<BR>(out, lane, nrhs, acc, red);
        }
    }
    if (Epi::kReduce) {
        lds[threadIdx.x] = red;
        __syncthreads();
        if (threadIdx.x < WAVE && threadIdx.x < nrhs) {
            double t = 0.0;
            for (int w = 0; w < wpb; ++w) t += lds[w * WAVE + threadIdx.x];
            partials[lb * nrhs + threadIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <typename T>
static inline const Tune &tune_of(const Sell &A) {
    return sizeof(T) == 4 ? A.tune32 : A.tune64;
}

// Block rows per wave of the SELL multi-RHS product for nrhs columns: 16
// rows (4 lanes each) for at most 4 columns, else 4 rows of 16 lanes; one
// row per wave for the lane-per-column kernel (tile 0, above 16 columns).
static inline int multi_rows(int nrhs, int mtile) {
    if (mtile == 0 && nrhs > 16) return 1;   // k_sellw
    return nrhs <= 4 ? 16 : 4;
}
// Columns per lane: the column tile (16, 32 or 64 columns per pass over the
// matrix, tuned) over the 16 lanes of a row.
static inline int multi_cols(int nrhs, int mtile) {
    if (nrhs <= 4) return 1;
    const int need = (nrhs + 15) / 16;   // 1..4
    const int s = std::min(need, mtile / 16);
    return s >= 4 ? 4 : (s >= 2 ? 2 : 1);
}

static inline int64_t sell_grid(const Sell &A, int nrhs, const Tune &t) {
    if (nrhs == 1) {
        const int64_t units = A.format == FMT_SELL ? A.nslices : A.nrows;
        const int64_t per = (int64_t)t.wpb * t.spw;
        return (units + per - 1) / per;
    }
    const int64_t per = (int64_t)t.mwpb * (A.format == FMT_SELL ? multi_rows(nrhs, t.mtile) : 1);
    return (A.nrows + per - 1) / per;
}

int sell_partials_count(const Sell &A, int nrhs) { return (int)sell_grid(A, nrhs, A.tune64); }

template <int BR, int BC, typename VT, typename XT, typename AT, class Epi>
static void launch_t(const Sell &A, const VT *val, const XT *x, const Epi &epi, int nrhs, double *partials,
                     hipStream_t s) {
    const Tune &t = tune_of<VT>(A);
    // the partial-sum tables hold one entry per 4 block rows at most; the SELL
    // multi-RHS kernel runs at most 8 waves per workgroup
    TE_REQUIRE(nrhs == 1 || t.mwpb == 4 || t.mwpb == 8 || (t.mwpb == 16 && A.format == FMT_ROWWAVE), TE_EINVAL,
               "bad waves per workgroup %d", t.mwpb);
    int64_t g = sell_grid(A, nrhs, t);
    if (g == 0) return;
    const dim3 blk(64 * (nrhs == 1 ? t.wpb : t.mwpb));
    if (nrhs == 1) {
        if (A.format == FMT_ROWWAVE) {
            if (t.nt)
                hipLaunchKernelGGL((k_roww<BR, BC, VT, XT, AT, Epi, true>), dim3((unsigned)g), blk, 0, s,
                                   rview(A, val), x, epi, partials, t.spw, t.remap, t.xb);
            else
                hipLaunchKernelGGL((k_roww<BR, BC, VT, XT, AT, Epi, false>), dim3((unsigned)g), blk, 0, s,
                                   rview(A, val), x, epi, partials, t.spw, t.remap, t.xb);
        } else {
            if (t.nt)
                hipLaunchKernelGGL((k_sell1<BR, BC, VT, XT, AT, Epi, true>), dim3((unsigned)g), blk, 0, s,
                                   view(A, val), x, epi, partials, t.spw, t.remap);
            else
                hipLaunchKernelGGL((k_sell1<BR, BC, VT, XT, AT, Epi, false>), dim3((unsigned)g), blk, 0, s,
                                   view(A, val), x, epi, partials, t.spw, t.remap);
        }
    } else if (A.format == FMT_ROWWAVE) {
        hipLaunchKernelGGL((k_rowwm<BR, BC, VT, XT, AT, Epi>), dim3((unsigned)g), blk, 0, s, rview(A, val), x, epi,
                           nrhs, partials, t.mwpb);
    } else {
        const int R = multi_rows(nrhs, t.mtile);
        if (R == 1) {
            hipLaunchKernelGGL((k_sellw<BR, BC, VT, XT, AT, Epi>), dim3((unsigned)g), blk, 0, s, view(A, val), x,
                               epi, nrhs, partials, t.mwpb);
            TE_CHECK_HIP(hipGetLastError());
            return;
        }
        const int S = multi_cols(nrhs, t.mtile);
        const int tile = (WAVE / R) * S;
        const unsigned tiles = (unsigned)((nrhs + tile - 1) / tile);
        dim3 grid((unsigned)g, tiles);
        int split = 0;
        int64_t chunk = 0;
        if (t.msplit && (tiles == 2 || tiles == 4 || tiles == 8)) {
            split = (int)tiles;
            chunk = (g + 8 / split - 1) / (8 / split);
            grid = dim3((unsigned)(8 * chunk), 1);
        }
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, blk, 0, s, view(A, val), x, epi, nrhs, partials, t.mwpb, split, chunk,
                               g);
        };
        if (R == 16) go(k_sellm<BR, BC, VT, XT, AT, Epi, 16, 1>);
        else if (S == 1) go(k_sellm<BR, BC, VT, XT, AT, Epi, 4, 1>);
        else if (S == 2) go(k_sellm<BR, BC, VT, XT, AT, Epi, 4, 2>);
        else go(k_sellm<BR, BC, VT, XT, AT, Epi, 4, 4>);
    }
    TE_CHECK_HIP(hipGetLastError());
}

template <typename T, class Epi>
static void dispatch(const Sell &A, const T *x, const Epi &epi, int nrhs, double *partials, hipStream_t s) {
    const T *val;
    if constexpr (sizeof(T) == 4) {
        TE_REQUIRE(A.val32.p, TE_EINVAL, "float32 operator copy not built");
        val = A.val32.p;
    } else {
        val = A.val.p;
    }
    const int key = A.br * 10 + A.bc;
    switch (key) {
        case 33: launch_t<3, 3, T, T, T>(A, val, x, epi, nrhs, partials, s); break;
        case 66: launch_t<6, 6, T, T, T>(A, val, x, epi, nrhs, partials, s); break;
        case 36: launch_t<3, 6, T, T, T>(A, val, x, epi, nrhs, partials, s); break;
        case 63: launch_t<6, 3, T, T, T>(A, val, x, epi, nrhs, partials, s); break;
        case 11: launch_t<1, 1, T, T, T>(A, val, x, epi, nrhs, partials, s); break;
        default: TE_REQUIRE(false, TE_EINVAL, "unsupported block shape %dx%d", A.br, A.bc);
    }
}

template <typename T>
void sell_apply(const Sell &A, const T *x, T *y, const T *g, int mode, int nrhs, hipStream_t s) {
    if (mode == 0) dispatch(A, x, EpiSet<T>{y}, nrhs, nullptr, s);
    else if (mode == 1) dispatch(A, x, EpiAdd<T>{y}, nrhs, nullptr, s);
    else dispatch(A, x, EpiResid<T, false>{g, y}, nrhs, nullptr, s);
}
template void sell_apply<double>(const Sell &, const double *, double *, const double *, int, int, hipStream_t);
template void sell_apply<float>(const Sell &, const float *, float *, const float *, int, int, hipStream_t);

void sell_resid_norm(const Sell &A, const double *x, const double *g, double *y, int nrhs, double *partials,
                     hipStream_t s) {
    dispatch(A, x, EpiResid<double, true>{g, y}, nrhs, partials, s);
}

void sell_dot(const Sell &A, const double *p, double *q, int nrhs, double *partials, hipStream_t s) {
    dispatch(A, p, EpiDot{p, q}, nrhs, partials, s);
}

template <typename T>
void cheb_init(const Sell &A, const T *x, const T *g, const T *dinv, T *r, T *d, double inv_theta, int nrhs,
               hipStream_t s) {
    dispatch(A, x, EpiChebInit<T>{g, dinv, r, d, T(inv_theta)}, nrhs, nullptr, s);
}
template void cheb_init<double>(const Sell &, const double *, const double *, const double *, double *, double *,
                                double, int, hipStream_t);
template void cheb_init<float>(const Sell &, const float *, const float *, const float *, float *, float *, double,
                               int, hipStream_t);

template <typename T>
void cheb_step(const Sell &A, const T *d, const T *rin, const T *dinv, T *rout, T *dout, T *x, double c1, double c2,
               bool last, bool xzero, int nrhs, hipStream_t s) {
    if (last && xzero)
        dispatch(A, d, EpiChebStep<T, true, true>{rin, d, dinv, rout, dout, x, T(c1), T(c2)}, nrhs, nullptr, s);
    else if (last)
        dispatch(A, d, EpiChebStep<T, true, false>{rin, d, dinv, rout, dout, x, T(c1), T(c2)}, nrhs, nullptr, s);
    else if (xzero)
        dispatch(A, d, EpiChebStep<T, false, true>{rin, d, dinv, rout, dout, x, T(c1), T(c2)}, nrhs, nullptr, s);
    else
        dispatch(A, d, EpiChebStep<T, false, false>{rin, d, dinv, rout, dout, x, T(c1), T(c2)}, nrhs, nullptr, s);
}
template void cheb_step<double>(const Sell &, const double *, const double *, const double *, double *, double *,
                                double *, double, double, bool, bool, int, hipStream_t);
template void cheb_step<float>(const Sell &, const float *, const float *, const float *, float *, float *, float *,
                               double, double, bool, bool, int, hipStream_t);

// ---------------------------------------------------------------------------
// Element-wise kernels
// ---------------------------------------------------------------------------
static inline unsigned egrid(int64_t n) {
    int64_t g = (n + BLK - 1) / BLK;
    if (g > (1 << 20)) g = 1 << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

// d = D^-1 g / theta  (pre-smoothing start, x0 = 0); rows*bs*nrhs entries
template <typename T>
__global__ void k_jacobi_scale(const T *__restrict__ g, const T *__restrict__ dinv, T *__restrict__ d, T inv_theta,
                               int64_t n, int nrhs) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
        d[i] = dinv[i / nrhs] * g[i] * inv_theta;
}
template <typename T>
void jacobi_scale(const T *g, const T *dinv, T *d, double inv_theta, int64_t n, int nrhs, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_jacobi_scale<T>, dim3(egrid(n)), dim3(BLK), 0, s, g, dinv, d, T(inv_theta), n, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}
template void jacobi_scale<double>(const double *, const double *, double *, double, int64_t, int, hipStream_t);
template void jacobi_scale<float>(const float *, const float *, float *, double, int64_t, int, hipStream_t);

template <typename T>
__global__ void k_axpy(T *__restrict__ y, const T *__restrict__ x, T a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) y[i] += a * x[i];
}
template <typename T>
void axpy(T *y, const T *x, double a, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpy<T>, dim3(egrid(n)), dim3(BLK), 0, s, y, x, T(a), n);
    TE_CHECK_HIP(hipGetLastError());
}
template void axpy<double>(double *, const double *, double, int64_t, hipStream_t);
template void axpy<float>(float *, const float *, double, int64_t, hipStream_t);

template <typename A, typename B>
__global__ void k_cast(const A *__restrict__ x, B *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) y[i] = B(x[i]);
}
void cast_f64_f32(const double *x, float *y, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_cast<double, float>), dim3(egrid(n)), dim3(BLK), 0, s, x, y, n);
    TE_CHECK_HIP(hipGetLastError());
}
void cast_f32_f64(const float *x, double *y, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_cast<float, double>), dim3(egrid(n)), dim3(BLK), 0, s, x, y, n);
    TE_CHECK_HIP(hipGetLastError());
}

// dst[i] = src[map[i]] per node (bs*nrhs contiguous values per node)
__global__ void k_perm_gather(const double *__restrict__ src, double *__restrict__ dst, const int32_t *__restrict__ map,
                              int64_t n, int per) {
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * per; t += (int64_t)gridDim.x * BLK) {
        int64_t i = t / per, k = t % per;
        dst[t] = src[(int64_t)map[i] * per + k];
    }
}
__global__ void k_perm_scatter(const double *__restrict__ src, double *__restrict__ dst,
                               const int32_t *__restrict__ map, int64_t n, int per) {
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * per; t += (int64_t)gridDim.x * BLK) {
        int64_t i = t / per, k = t % per;
        dst[(int64_t)map[i] * per + k] = src[t];
    }
}
void permute_gather(const double *src, double *dst, const int32_t *map, int64_t n_nodes, int bs, int nrhs,
                    hipStream_t s) {
    if (n_nodes == 0) return;
    hipLaunchKernelGGL(k_perm_gather, dim3(egrid(n_nodes * bs * nrhs)), dim3(BLK), 0, s, src, dst, map, n_nodes,
                       bs * nrhs);
    TE_CHECK_HIP(hipGetLastError());
}
void permute_scatter(const double *src, double *dst, const int32_t *map, int64_t n_nodes, int bs, int nrhs,
                     hipStream_t s) {
    if (n_nodes == 0) return;
    hipLaunchKernelGGL(k_perm_scatter, dim3(egrid(n_nodes * bs * nrhs)), dim3(BLK), 0, s, src, dst, map, n_nodes,
                       bs * nrhs);
    TE_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Deterministic dot products (per right-hand side column)
// ---------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 1024;

int dot_nblocks(int64_t n) {
    int64_t g = (n + BLK - 1) / BLK;
    return (int)(g < 1 ? 1 : (g > DOT_BLOCKS ? DOT_BLOCKS : g));
}

// Single column: block b sums a contiguous chunk in a fixed order.
__global__ void k_dot1(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                       double *__restrict__ partials) {
    __shared__ double lds[WPB];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double t = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += BLK) t += a[i] * b[i];
    t = block_sum(t, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Several columns (layout [rows][nrhs]): lane = column, waves over rows.
__global__ void k_dotm(const double *__restrict__ a, const double *__restrict__ b, int64_t rows, int nrhs,
                       double *__restrict__ partials) {
    __shared__ double lds[BLK];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (rows + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(rows, lo + chunk);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    double t = 0.0;
    if (lane < nrhs)
        for (int64_t i = lo + w; i < hi; i += WPB) t += a[i * nrhs + lane] * b[i * nrhs + lane];
    lds[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x < nrhs) {
        double s = 0.0;
        for (int k = 0; k < WPB; ++k) s += lds[k * WAVE + threadIdx.x];
        partials[blockIdx.x * (int64_t)nrhs + threadIdx.x] = s;
    }
}

void dot_partials(const double *a, const double *b, int64_t n, int nrhs, double *partials, hipStream_t s) {
    int64_t rows = n / nrhs;
    int nb = dot_nblocks(rows);
    if (nrhs == 1)
        hipLaunchKernelGGL(k_dot1, dim3(nb), dim3(BLK), 0, s, a, b, n, partials);
    else
        hipLaunchKernelGGL(k_dotm, dim3(nb), dim3(BLK), 0, s, a, b, rows, nrhs, partials);
    TE_CHECK_HIP(hipGetLastError());
}

// out[j] = sum_b partials[b*nrhs + j], fixed order (thread j, sequential b).
__global__ void k_reduce_partials(const double *__restrict__ partials, int nparts, int nrhs, double *__restrict__ out) {
    __shared__ double lds[BLK];
    // each column j: threads split the parts in a fixed strided way, then tree
    for (int j = 0; j < nrhs; ++j) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nparts; b += BLK) t += partials[(int64_t)b * nrhs + j];
        lds[threadIdx.x] = t;
        __syncthreads();
        for (int o = BLK / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[j] = lds[0];
        __syncthreads();
    }
}
// Many partials (one per workgroup of a sparse product): two passes.  Pass 1:
// workgroup g sums rows [g*chunk, (g+1)*chunk) of the [nparts][ncols] table,
// thread (row offset, column) with coalesced reads, then the row offsets in
// order; pass 2: one thread per column adds the G chunk sums in order.
constexpr int REDUCE_ONE_PASS = 4096;
__global__ void __launch_bounds__(BLK) k_reduce_cols1(const double *__restrict__ partials, int nparts, int ncols,
                                                      int chunk, double *__restrict__ out2) {
    __shared__ double lds[BLK];
    const int R = BLK / ncols;  // rows per pass
    const int r = threadIdx.x / ncols, c = threadIdx.x % ncols;
    const int lo = blockIdx.x * chunk, hi = min(nparts, lo + chunk);
    double t = 0.0;
    if (r < R)
        for (int b = lo + r; b < hi; b += R) t += partials[(int64_t)b * ncols + c];
    lds[threadIdx.x] = t;
    __syncthreads();
    if ((int)threadIdx.x < ncols) {
        double u = 0.0;
        for (int k = 0; k < R; ++k) u += lds[k * ncols + threadIdx.x];
        out2[(int64_t)blockIdx.x * ncols + threadIdx.x] = u;
    }
}
__global__ void __launch_bounds__(BLK) k_reduce_cols2(const double *__restrict__ out2, int G, int ncols,
                                                      double *__restrict__ out) {
    for (int c = threadIdx.x; c < ncols; c += BLK) {
        double u = 0.0;
        for (int g = 0; g < G; ++g) u += out2[(int64_t)g * ncols + c];
        out[c] = u;
    }
}
static void reduce_cols(const double *partials, int nparts, int ncols, double *out, hipStream_t s) {
    TE_REQUIRE(ncols >= 1 && ncols <= BLK, TE_EINVAL, "reduction over %d columns", ncols);
    const int G = std::min(1024, std::max(1, nparts / 64));
    const int chunk = (nparts + G - 1) / G;
    double *out2 = const_cast<double *>(partials) + (int64_t)nparts * ncols;
    hipLaunchKernelGGL(k_reduce_cols1, dim3(G), dim3(BLK), 0, s, partials, nparts, ncols, chunk, out2);
    hipLaunchKernelGGL(k_reduce_cols2, dim3(1), dim3(BLK), 0, s, out2, G, ncols, out);
    TE_CHECK_HIP(hipGetLastError());
}

void reduce_partials(const double *partials, int nparts, int nrhs, double *out, hipStream_t s) {
    if (nparts > REDUCE_ONE_PASS) {
        reduce_cols(partials, nparts, nrhs, out, s);
        return;
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(BLK), 0, s, partials, nparts, nrhs, out);
    TE_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// CG vector updates (float64), per-column scalars on the device
// ---------------------------------------------------------------------------
// u += alpha_j p; r_old = r (if keep_old); r -= alpha_j q; red_j += r^2
__global__ void k_cg_update(double *__restrict__ u, double *__restrict__ r, double *__restrict__ r_old,
                            const double *__restrict__ p, const double *__restrict__ q, const double *__restrict__ alpha,
                            int64_t rows, int nrhs, double *__restrict__ partials) {
    __shared__ double lds[BLK];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (rows + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(rows, lo + chunk);
    if (nrhs == 1) {
        const double a = alpha[0];
        double t = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += BLK) {
            u[i] += a * p[i];
            double rv = r[i];
            if (r_old) r_old[i] = rv;
            rv -= a * q[i];
            r[i] = rv;
            t += rv * rv;
        }
        t = block_sum(t, lds);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
        return;
    }
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    double t = 0.0;
    if (lane < nrhs) {
        const double a = alpha[lane];
        for (int64_t i = lo + w; i < hi; i += WPB) {
            int64_t k = i * nrhs + lane;
            u[k] += a * p[k];
            double rv = r[k];
            if (r_old) r_old[k] = rv;
            rv -= a * q[k];
            r[k] = rv;
            t += rv * rv;
        }
    }
    lds[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x < nrhs) {
        double s = 0.0;
        for (int k = 0; k < WPB; ++k) s += lds[k * WAVE + threadIdx.x];
        partials[blockIdx.x * (int64_t)nrhs + threadIdx.x] = s;
    }
}
void cg_update(double *u, double *r, double *r_old, const double *p, const double *q, const double *alpha,
               int64_t rows, int nrhs, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update, dim3(dot_nblocks(rows)), dim3(BLK), 0, s, u, r, r_old, p, q, alpha, rows, nrhs,
                       partials);
    TE_CHECK_HIP(hipGetLastError());
}

// (r, z) and, for the flexible variant, (z, r - r_old) per column
__global__ void k_dot_rz(const double *__restrict__ r, const double *__restrict__ z, const double *__restrict__ r_old,
                         int64_t rows, int nrhs, double *__restrict__ partials) {
    __shared__ double lds[2 * BLK];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (rows + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(rows, lo + chunk);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    double t = 0.0, f = 0.0;
    if (nrhs == 1) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += BLK) {
            t += r[i] * z[i];
            if (r_old) f += z[i] * (r[i] - r_old[i]);
        }
        double a = block_sum(t, lds);
        double b = block_sum(f, lds + WPB);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = a;
            partials[2 * blockIdx.x + 1] = b;
        }
        return;
    }
    if (lane < nrhs)
        for (int64_t i = lo + w; i < hi; i += WPB) {
            int64_t k = i * nrhs + lane;
            t += r[k] * z[k];
            if (r_old) f += z[k] * (r[k] - r_old[k]);
        }
    lds[threadIdx.x] = t;
    lds[BLK + threadIdx.x] = f;
    __syncthreads();
    if (threadIdx.x < nrhs) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < WPB; ++k) {
            s1 += lds[k * WAVE + threadIdx.x];
            s2 += lds[BLK + k * WAVE + threadIdx.x];
        }
        partials[(blockIdx.x * (int64_t)nrhs + threadIdx.x) * 2] = s1;
        partials[(blockIdx.x * (int64_t)nrhs + threadIdx.x) * 2 + 1] = s2;
    }
}
void dot_rz(const double *r, const double *z, const double *r_old, int64_t rows, int nrhs, double *partials,
            hipStream_t s) {
    hipLaunchKernelGGL(k_dot_rz, dim3(dot_nblocks(rows)), dim3(BLK), 0, s, r, z, r_old, rows, nrhs, partials);
    TE_CHECK_HIP(hipGetLastError());
}

// p = z + beta_j p
__global__ void k_p_update(double *__restrict__ p, const double *__restrict__ z, const double *__restrict__ beta,
                           int64_t n, int nrhs) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
        p[i] = z[i] + beta[i % nrhs] * p[i];
}
void p_update(double *p, const double *z, const double *beta, int64_t n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_p_update, dim3(egrid(n)), dim3(BLK), 0, s, p, z, beta, n, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}

// Scalar bookkeeping of the CG recurrence, one thread per column.
//   alpha: pq from partials -> alpha = active ? rz/pq : 0 ; flag if pq <= 0
//   beta:  rz_new (+ flexible term) -> beta; rz = rz_new; flag if rz_new <= 0
__global__ void k_cg_alpha(CgScalars *S, const double *__restrict__ pq_sum, int nrhs) {
    int j = threadIdx.x;
    if (j >= nrhs) return;
    double pq = pq_sum[j];
    S->pq[j] = pq;
    double a = 0.0;
    if (S->active[j]) {
        if (!(pq > 0.0)) {
            S->flag[j] = (pq != pq) ? 3 : 1;
        } else {
            a = S->rz[j] / pq;
        }
    }
    S->alpha[j] = a;
}
__global__ void k_cg_beta(CgScalars *S, const double *__restrict__ rzf, int nrhs, int flexible) {
    int j = threadIdx.x;
    if (j >= nrhs) return;
    double rzn = rzf[2 * j], fl = rzf[2 * j + 1];
    double b = 0.0;
    if (S->active[j]) {
        if (!(rzn > 0.0)) {
            S->flag[j] = (rzn != rzn) ? 3 : 2;
        } else {
            b = flexible ? fl / S->rz[j] : rzn / S->rz[j];
            S->rz[j] = rzn;
        }
    }
    S->beta[j] = b;
}
__global__ void k_cg_rz0(CgScalars *S, const double *__restrict__ rzf, int nrhs) {
    int j = threadIdx.x;
    if (j >= nrhs) return;
    double rzn = rzf[2 * j];
    if (S->active[j] && !(rzn > 0.0)) S->flag[j] = (rzn != rzn) ? 3 : 2;
    S->rz[j] = rzn;
}
// reduce interleaved (rz, flex) partial pairs
__global__ void k_reduce_pairs(const double *__restrict__ partials, int nparts, int nrhs, double *__restrict__ out) {
    __shared__ double lds[BLK];
    for (int jj = 0; jj < 2 * nrhs; ++jj) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nparts; b += BLK) t += partials[(int64_t)b * 2 * nrhs + jj];
        lds[threadIdx.x] = t;
        __syncthreads();
        for (int o = BLK / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[jj] = lds[0];
        __syncthreads();
    }
}

void cg_alpha(void *S, const double *pq_sum, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, s, (CgScalars *)S, pq_sum, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}
void cg_beta(void *S, const double *rzf, int nrhs, int flexible, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, s, (CgScalars *)S, rzf, nrhs, flexible);
    TE_CHECK_HIP(hipGetLastError());
}
void cg_rz0(void *S, const double *rzf, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_rz0, dim3(1), dim3(64), 0, s, (CgScalars *)S, rzf, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}
void reduce_pairs(const double *partials, int nparts, int nrhs, double *out, hipStream_t s) {
    if (nparts > REDUCE_ONE_PASS) {
        reduce_cols(partials, nparts, 2 * nrhs, out, s);
        return;
    }
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(BLK), 0, s, partials, nparts, nrhs, out);
    TE_CHECK_HIP(hipGetLastError());
}
size_t cg_scalars_bytes() { return sizeof(CgScalars); }

// Column select: r[:, j] = t[:, j] where sel[j] != 0
__global__ void k_copy_cols(double *__restrict__ r, const double *__restrict__ t, const int32_t *__restrict__ sel,
                            int64_t n, int nrhs) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
        if (sel[i % nrhs]) r[i] = t[i];
}
void copy_cols(double *r, const double *t, const int32_t *sel, int64_t n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_cols, dim3(egrid(n)), dim3(BLK), 0, s, r, t, sel, n, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Dense coarse solve: y = Ainv x (Ainv symmetric n x n, float64)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(BLK) k_dense_mv(const double *__restrict__ Ainv, const T *__restrict__ x,
                                                  T *__restrict__ y, int n, int nrhs) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t row = (int64_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + threadIdx.x / WAVE));
    if (row >= n) return;
    const double *a = Ainv + row * (int64_t)n;
    if (nrhs == 1) {
        double t = 0.0;
        for (int j = lane; j < n; j += WAVE) t += a[j] * double(x[j]);
        t = wave_sum(t);
        if (lane == 0) y[row] = T(t);
        return;
    }
    if (lane >= nrhs) return;
    double t = 0.0;
    for (int j = 0; j < n; ++j) t += a[j] * double(x[(int64_t)j * nrhs + lane]);
    y[row * nrhs + lane] = T(t);
}
template <typename T>
void dense_mv(const double *Ainv, const T *x, T *y, int n, int nrhs, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_dense_mv<T>, dim3((n + WPB - 1) / WPB), dim3(BLK), 0, s, Ainv, x, y, n, nrhs);
    TE_CHECK_HIP(hipGetLastError());
}
template void dense_mv<double>(const double *, const double *, double *, int, int, hipStream_t);
template void dense_mv<float>(const double *, const float *, float *, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Lanczos helpers (setup)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    // Steele, Lea & Flood 2014: one step of the generator on input x
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// v[new*bs + c] = U(splitmix64(seed ^ natural_dof)) - 0.5
__global__ void k_lanczos_start(double *__restrict__ v, const int32_t *__restrict__ perm, int64_t n, int bs,
                                uint64_t seed) {
    for (int64_t t = blockIdx.x * (int64_t)BLK + threadIdx.x; t < n * bs; t += (int64_t)gridDim.x * BLK) {
        int64_t i = t / bs, c = t % bs;
        uint64_t nat = (uint64_t)perm[i] * (uint64_t)bs + (uint64_t)c;
        uint64_t z = splitmix64(seed ^ nat);
        v[t] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
    }
}
void lanczos_start(double *v, const int32_t *perm, int64_t n, int bs, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_start, dim3(egrid(n * bs)), dim3(BLK), 0, s, v, perm, n, bs, seed);
    TE_CHECK_HIP(hipGetLastError());
}

// y = a*x + b*y element-wise, then helpers for D^{1/2} scaling
__global__ void k_scale_mul(const double *__restrict__ x, const double *__restrict__ s, double *__restrict__ y,
                            int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) y[i] = s[i] * x[i];
}
void scale_mul(const double *x, const double *sc, double *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_mul, dim3(egrid(n)), dim3(BLK), 0, s, x, sc, y, n);
    TE_CHECK_HIP(hipGetLastError());
}
// w = sc * w - beta * vprev  (in place on w)
__global__ void k_lanczos_w(double *__restrict__ w, const double *__restrict__ sc, const double *__restrict__ vprev,
                            double beta, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
        w[i] = sc[i] * w[i] - beta * vprev[i];
}
void lanczos_w(double *w, const double *sc, const double *vprev, double beta, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_w, dim3(egrid(n)), dim3(BLK), 0, s, w, sc, vprev, beta, n);
    TE_CHECK_HIP(hipGetLastError());
}
__global__ void k_scal(double *__restrict__ x, double a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) x[i] *= a;
}
void scal(double *x, double a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scal, dim3(egrid(n)), dim3(BLK), 0, s, x, a, n);
    TE_CHECK_HIP(hipGetLastError());
}

}  // namespace te

