// Block compressed-row matrices on the device and the sparse products of the
// smoothed-aggregation setup that run on them (te_setup_gpu.hip).
#pragma once

#include "te_internal.h"

namespace te {

// Natural numbering, sorted columns per row, blocks row-major [nnzb][br][bc].
// The pointers either refer to the owned buffers or, for a caller's matrix,
// to memory the library does not own.
struct DBsr {
    int br = 0, bc = 0;
    int64_t nr = 0, nc = 0, nnzb = 0;
    const int64_t *ptr = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
    DBuf<int64_t> ptr_own;
    DBuf<int32_t> col_own;
    DBuf<double> val_own;
    void bind() {
        ptr = ptr_own.p;
        col = col_own.p;
        val = val_own.p;
    }
    void release() {
        ptr_own.release();
        col_own.release();
        val_own.release();
        ptr = nullptr;
        col = nullptr;
        val = nullptr;
        nnzb = 0;
    }
};

// s[k] = |A_k|_F / sqrt(|A_ii|_F |A_jj|_F) for the off-diagonal block k = (i, j),
// 0 on the diagonal; squares and sums rounded separately (no contraction).
void dev_strength(const DBsr &A, DBuf<double> &s, hipStream_t st);

// Point diagonal of A in natural numbering: d[i*br + p] = A_ii[p][p].
void dev_diag(const DBsr &A, DBuf<double> &d, hipStream_t st);

// P = (I - omega D^-1 A) P_tent with P_tent given by the aggregate of each
// node (agg, -1 = none) and the orthonormal rows Q [n][br][6].
void dev_smoothed_p(const DBsr &A, const DBuf<int32_t> &agg, int64_t nagg, const DBuf<double> &Q,
                    const DBuf<double> &d, double omega, DBsr &P, hipStream_t s);

// C = A B with the blocks summed in the order of A's row, then B's row
// (block shapes 1x1 * 1x1, 3x3 * 3x6, 6x3 * 3x6, 6x6 * 6x6).  symmetric: C is
// known to be symmetric (a Galerkin product P^T (A P) of a symmetric A) and
// has 6x6 blocks: the blocks on and above the diagonal are formed, those below
// are their transposes (other shapes ignore the flag).
void dev_mult(const DBsr &A, const DBsr &B, DBsr &C, hipStream_t s, bool symmetric = false);

// T = A^T (blocks transposed; rows of each column in ascending order;
// block shapes 1x1, 3x6, 6x6).
void dev_transpose(const DBsr &A, DBsr &T, hipStream_t s);

// Pack M into a solver layout (SELL-64 or one wave per row).  hptr is M's
// row pointer on the host.
//   row_order[i] = row of M stored at position i (lane i%64 of slice i/64)
//   col_map[c]   = column index stored for column c of M
//   out_map      = if non-null, position i writes output row (*out_map)[row_order[i]];
//                  otherwise position i writes output row i
//   sym          = a square M in the one-wave-per-row format keeps only its
//                  blocks on and above the diagonal when its pattern is
//                  symmetric (columns ascending within each row)
void dev_pack(Sell &S, const DBsr &M, const std::vector<int64_t> &hptr, const std::vector<int32_t> &row_order,
              const std::vector<int32_t> &col_map, const std::vector<int32_t> *out_map, bool fp32, hipStream_t s,
              int format, bool sym = false);

// inv = M^-1 for a symmetric positive definite n x n matrix M (host,
// row-major), computed on the device by n symmetric sweeps; TE_ECHOL if a
// pivot is not positive.
void dev_dense_inverse_spd(const std::vector<double> &M, int n, DBuf<double> &inv, hipStream_t s);

// Parallel aggregation of a level (square A with a symmetric pattern, s from
// dev_strength): the strong graph made symmetric (block k = (i, j) strong if
// s_ij or s_ji >= theta, i != j); phase-1 roots = the maximal distance-2
// independent set chosen by fixed keys (splitmix64(seed ^ i) >> 33, i) in
// parallel rounds; aggregates numbered by ascending root; phase-1 aggregate
// = root and its strong neighbours; phase 2 joins each remaining node with a
// strong neighbour to its strongest neighbour's phase-1 aggregate (relative
// ties within tie_rtol: the smaller id).  agg: host [n], -1 for isolated
// nodes; returns the number of aggregates.
int64_t dev_aggregate_mis2(const DBsr &A, const DBuf<double> &s, double theta, uint64_t seed, double tie_rtol,
                           std::vector<int32_t> &agg, hipStream_t st);

// Filtered operator for the prolongator smoothing: per block row the diagonal
// block plus every dropped block (summed in stored order) and the strong
// off-diagonal blocks unchanged; strong = s_ij or s_ji >= theta (i != j).
void dev_filtered(const DBsr &A, const DBuf<double> &s, double theta, DBsr &F, hipStream_t st);

// c = mean of the n node coordinates (device [n][3]); partial sums per
// workgroup on the device, added on the host in workgroup order
void dev_centroid(const double *coords, int64_t n, double c[3], hipStream_t st);

// Level-0 near-nullspace on the device: the six rigid-body modes about the
// point c, B [n][3][6] (translations x, y, z, then rotations about z, x, y),
// rows of constrained DOFs (mask, may be NULL) zero.
void dev_rigid_body_modes(const double *coords, const uint8_t *mask, int64_t n, const double c[3], DBuf<double> &B,
                          hipStream_t st);

// Tentative prolongator on the device: for each aggregate (members ascending,
// given by the host as off/mem), the thin Householder QR of its rows of B
// [n][bs][6] with diag(R) > 0; Q [n][bs][6] (zero rows for nodes in no
// aggregate) and Bc [na][6][6] = R.  Returns false, leaving the outputs
// unspecified, if an aggregate is rank deficient (min |R_kk| < rank_rtol
// max |R_kk|) or has more than 640 rows: the caller then takes the host path.
bool dev_tentative(const std::vector<int64_t> &off, const std::vector<int32_t> &mem, const DBuf<double> &B,
                   int64_t n, int bs, double rank_rtol, DBuf<double> &Q, DBuf<double> &Bc, hipStream_t st);

// First block row (ascending) with a column index outside [0, n) or without
// its diagonal block, or -1.
int64_t dev_check_pattern(const int64_t *ptr, const int32_t *col, int64_t n, hipStream_t st);

// Point diagonal in the storage order of a level: d[i*bs+p] = dnat[perm[i]*bs+p]
// and its reciprocals in float64 and (if dinv32) float32.  Returns the first
// natural block row with a diagonal entry that is not positive, or -1.
int64_t dev_diag_store(const double *dnat, const int32_t *perm, int64_t n, int bs, double *d, double *dinv,
                       float *dinv32, hipStream_t st);
// y = 1 / sqrt(x), n entries.
void dev_rsqrt(const double *x, double *y, int64_t n, hipStream_t st);

// Order-independent 64-bit hash of a block pattern (row pointers and columns).
uint64_t dev_pattern_hash(const int64_t *ptr, const int32_t *col, int64_t n, hipStream_t st);

// Host copies of the pattern or of the whole matrix.
void dev_pattern_to_host(const DBsr &M, HBsr &H, hipStream_t s);
void dev_to_host(const DBsr &M, HBsr &H, hipStream_t s);

}  // namespace te
