// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "te.h"

namespace te {

// ---- error handling ------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

struct Error {
    int code;
};

#define TE_CHECK_HIP(expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::te::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                            __LINE__);                                                      \
            throw ::te::Error{TE_EHIP};                                                     \
        }                                                                                   \
    } while (0)

#define TE_REQUIRE(cond, code, ...)     \
    do {                                \
        if (!(cond)) {                  \
            ::te::set_error(__VA_ARGS__); \
            throw ::te::Error{code};    \
        }                               \
    } while (0)

// Runs f() and converts library exceptions into return codes.
template <class F>
int guarded(F &&f) {
    try {
        clear_error();
        return f();
    } catch (const Error &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return TE_ENOMEM;
    }
}

// ---- device memory -------------------------------------------------------
// Owning device buffer (hipMalloc / hipFree).
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            set_error("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
            throw Error{TE_ENOMEM};
        }
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Copies between pageable host memory and the device.  Transfers of a few MB
// and more go through a process-wide pinned staging buffer in chunks (the
// DMA of one chunk overlaps the host copy of the next), which runs at the
// pinned rate instead of the pageable one.  Both return with the copy done.
void copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t s);
void copy_d2h(void *dst, const void *src, size_t bytes, hipStream_t s);

template <class T>
void upload(DBuf<T> &d, const std::vector<T> &h, hipStream_t s) {
    d.alloc(h.size());
    if (!h.empty()) copy_h2d(d.p, h.data(), h.size() * sizeof(T), s);
}

template <class T>
void download(std::vector<T> &h, const T *d, size_t n, hipStream_t s) {
    h.resize(n);
    if (n) copy_d2h(h.data(), d, n * sizeof(T), s);
    else TE_CHECK_HIP(hipStreamSynchronize(s));
}

// ---- host block-sparse matrix (natural numbering) -------------------------
struct HBsr {
    int br = 0, bc = 0;
    int64_t nr = 0, nc = 0;
    std::vector<int64_t> ptr;   // [nr+1]
    std::vector<int32_t> col;   // [nnzb]
    std::vector<double> val;    // [nnzb][br][bc]
    int64_t nnzb() const { return (int64_t)col.size(); }
};

// ---- SELL-64 block matrix on the device -----------------------------------
// Rows are grouped into slices of 64; lane l of slice s holds row s*64+l of
// the (permuted) row order.  Entry k of every lane of a slice is stored
// contiguously across lanes:
//   col[(off_s + k) * 64 + lane]
//   val[(off_s + k) * br*bc * 64 + sell_val_off<VW>(e, br*bc, lane)]   e = i*bc + j
// The E = br*bc values of a block go in groups of VW = 16 / sizeof(value)
// consecutive entries, one 16-byte piece per lane, the pieces of the 64
// lanes contiguous; the E % VW remaining entries take one plane of 64 values
// each.  A lane thus reads its block with 16-byte loads.  Padding entries
// carry a zero block and a valid column.
constexpr int SELL_C = 64;

template <int VW>
__host__ __device__ __forceinline__ constexpr int64_t sell_val_off(int e, int E, int lane) {
    return e < E / VW * VW ? ((int64_t)(e / VW) * SELL_C + lane) * VW + e % VW
                           : (int64_t)(E / VW * VW) * SELL_C + (int64_t)(e - E / VW * VW) * SELL_C + lane;
}
template <typename VT>
constexpr int sell_vw() {
    return 16 / (int)sizeof(VT);
}

// Second layout for operators whose rows are few and long (6-row blocks:
// coarse operators and the restrictions): format 1 stores the blocks of a row
// contiguously (val[k][br][bc], rptr[row]..rptr[row+1]) and one wave handles
// one row, lane = (block slot, row of the block).
constexpr int FMT_SELL = 0;
constexpr int FMT_ROWWAVE = 1;

// Launch configuration of one operator, chosen by the autotuner:
// waves per workgroup, slices (or rows) per wave, XCD-contiguous block order,
// non-temporal loads of the matrix values.
struct Tune {
    int wpb = 4, spw = 1, remap = 1, nt = 0;
    int mwpb = 4;    // several right-hand sides: waves per workgroup
    int mtile = 0;   // several right-hand sides on the SELL layout: columns per pass (0: row per wave)
    int msplit = 0;  // ... and the column tiles on different XCDs instead of passes
    int xb = 0;      // one wave per row: a slot's lanes share the block column's x entries by lane permutes
};

struct Sell {
    Tune tune64, tune32;
    int format = FMT_SELL;
    int br = 0, bc = 0;
    int64_t nrows = 0;          // block rows
    int64_t ncols = 0;          // block columns
    int64_t nslices = 0;
    int64_t nnzb = 0;           // real blocks (without padding)
    int64_t padded = 0;         // stored entries per lane-column sum (= off_end*64)
    DBuf<int32_t> slice_off;    // [nslices+1] in units of 64-wide entry columns
    DBuf<int32_t> col;          // [padded]
    DBuf<int32_t> rowlen;       // [nslices*64] entries of each row
    DBuf<double> val;           // [padded * br*bc]
    DBuf<float> val32;          // optional float32 copy
    DBuf<int32_t> rowmap;       // [nslices*64] output row of each lane, -1 = none; empty = identity
    DBuf<int64_t> rptr;         // format 1: [nrows+1] block offset of each stored row
    // Format 1, symmetric operator: rptr/col/val hold only the blocks on or
    // above the diagonal (storage numbering); the blocks below it are read
    // transposed from their mirror: row r's lower blocks are
    // lptr[r]..lptr[r+1], column lcol[k], mirror block lidx[k] of val.
    DBuf<int64_t> lptr;
    DBuf<int32_t> lcol;
    DBuf<int32_t> lidx;
    bool sym() const { return lptr.p != nullptr; }
    size_t bytes() const {
        return slice_off.bytes() + col.bytes() + rowlen.bytes() + val.bytes() + val32.bytes() + rowmap.bytes() +
               rptr.bytes() + lptr.bytes() + lcol.bytes() + lidx.bytes();
    }
};

// Row order sorted by descending length inside windows of `window` rows.
std::vector<int32_t> window_sorted_order(const std::vector<int64_t> &ptr, int64_t window);

// ---- device-side CG scalars (one entry per right-hand side) ----------------
struct CgScalars {
    double rz[64], pq[64], alpha[64], beta[64], rr[64], bb[64], tr[64];
    int32_t active[64];
    int32_t flag[64];  // 1: (p,Ap) <= 0, 2: (r,z) <= 0, 3: NaN
};

// ---- kernel launchers (te_kernels.hip) ------------------------------------
template <typename T>
void sell_apply(const Sell &A, const T *x, T *y, const T *g, int mode, int nrhs, hipStream_t s);
void sell_resid_norm(const Sell &A, const double *x, const double *g, double *y, int nrhs, double *partials,
                     hipStream_t s);
void sell_dot(const Sell &A, const double *p, double *q, int nrhs, double *partials, hipStream_t s);
int sell_partials_count(const Sell &A, int nrhs);
template <typename T>
void cheb_init(const Sell &A, const T *x, const T *g, const T *dinv, T *r, T *d, double inv_theta, int nrhs,
               hipStream_t s);
template <typename T>
void cheb_step(const Sell &A, const T *d, const T *rin, const T *dinv, T *rout, T *dout, T *x, double c1, double c2,
               bool last, bool xzero, int nrhs, hipStream_t s);
template <typename T>
void jacobi_scale(const T *g, const T *dinv, T *d, double inv_theta, int64_t n, int nrhs, hipStream_t s);
template <typename T>
void axpy(T *y, const T *x, double a, int64_t n, hipStream_t s);
void cast_f64_f32(const double *x, float *y, int64_t n, hipStream_t s);
void cast_f32_f64(const float *x, double *y, int64_t n, hipStream_t s);
void permute_gather(const double *src, double *dst, const int32_t *map, int64_t n_nodes, int bs, int nrhs,
                    hipStream_t s);  // dst[i] = src[map[i]]
void permute_scatter(const double *src, double *dst, const int32_t *map, int64_t n_nodes, int bs, int nrhs,
                     hipStream_t s);  // dst[map[i]] = src[i]
int dot_nblocks(int64_t n);
void dot_partials(const double *a, const double *b, int64_t n, int nrhs, double *partials, hipStream_t s);
// out[j] = sum over b of partials[b*nrhs + j], in a fixed order.  Above 4096
// parts the sum takes two passes whose chunk sums are written after the
// input: the buffer must then hold (nparts + min(1024, nparts/64)) * nrhs.
void reduce_partials(const double *partials, int nparts, int nrhs, double *out, hipStream_t s);

// Block CG kernels (te_block.hip); block vectors [rows][m], m <= 64, small
// matrices 64 x 64 row-major (entries beyond m or the block rank are zero).
//   block_gram: out[p] = mats[li[p]]^T mats[ri[p]] for p < npair (npair,
//     nmat <= 3); partials: block_gram_nblocks() * npair * 4096 doubles.
//   block_xr:   X += P alpha, R -= Q alpha; partials[b * m + j] = partial
//     sums of R_j^2 over block_xr_nblocks(rows) workgroups.
//   block_p:    P <- Z T1 + P T2 (in place).
int block_gram_nblocks();
int block_xr_nblocks(int64_t rows);
void block_gram(const double *const *mats, int nmat, const int *li, const int *ri, int npair, int64_t rows, int m,
                double *partials, double *out, hipStream_t s);
void block_xr(int64_t rows, int m, const double *alpha, const double *P, const double *Q, double *X, double *R,
              double *partials, hipStream_t s);
void block_p(int64_t rows, int m, const double *T1, const double *T2, const double *Z, double *P, hipStream_t s);
void reduce_pairs(const double *partials, int nparts, int nrhs, double *out, hipStream_t s);
void cg_update(double *u, double *r, double *r_old, const double *p, const double *q, const double *alpha,
               int64_t rows, int nrhs, double *partials, hipStream_t s);
void dot_rz(const double *r, const double *z, const double *r_old, int64_t rows, int nrhs, double *partials,
            hipStream_t s);
void p_update(double *p, const double *z, const double *beta, int64_t n, int nrhs, hipStream_t s);
void cg_alpha(void *S, const double *pq_sum, int nrhs, hipStream_t s);
void cg_beta(void *S, const double *rzf, int nrhs, int flexible, hipStream_t s);
void cg_rz0(void *S, const double *rzf, int nrhs, hipStream_t s);
size_t cg_scalars_bytes();
void copy_cols(double *r, const double *t, const int32_t *sel, int64_t n, int nrhs, hipStream_t s);
template <typename T>
void dense_mv(const double *Ainv, const T *x, T *y, int n, int nrhs, hipStream_t s);
void lanczos_start(double *v, const int32_t *perm, int64_t n, int bs, uint64_t seed, hipStream_t s);
void scale_mul(const double *x, const double *sc, double *y, int64_t n, hipStream_t s);
void lanczos_w(double *w, const double *sc, const double *vprev, double beta, int64_t n, hipStream_t s);
void scal(double *x, double a, int64_t n, hipStream_t s);

}  // namespace te
