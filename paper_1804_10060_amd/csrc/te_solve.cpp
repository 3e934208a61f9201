// V-cycle and (flexible) preconditioned conjugate gradients on the device.
//
// CG follows the paper's solver (Sec. 2.1.2; Sec. 5.1: CG preconditioned by
// smoothed-aggregation AMG with Chebyshev smoothing), in the form of Saad's
// Algorithm 9.1.  For the float32 V-cycle the flexible beta of Notay (2000),
// (z', r' - r)/(z, r), keeps CG convergent with a preconditioner that is not
// an exact fixed linear operator.  Every column of a multi-RHS solve keeps its
// own recurrence; the sparse products are shared.  The host reads back one
// residual norm per column and iteration to decide convergence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "te_amg.h"

namespace te {

template <typename T>
static Work<T> &work(Level &L);
template <>
Work<double> &work<double>(Level &L) {
    return L.w64;
}
template <>
Work<float> &work<float>(Level &L) {
    return L.w32;
}
template <typename T>
static const T *dinv_of(const Level &L);
template <>
const double *dinv_of<double>(const Level &L) {
    return L.dinv.p;
}
template <>
const float *dinv_of<float>(const Level &L) {
    return L.dinv32.p;
}

// Chebyshev steps after the start d0 (and r0 = rin), accumulating into x.
template <typename T>
static void cheb_chain(Level &L, const T *rin, T *x, bool xzero, int degree, int m, hipStream_t s) {
    Work<T> &W = work<T>(L);
    const T *dinv = dinv_of<T>(L);
    T *dc = W.d.p, *dn = W.d2.p;
    if (degree == 1) {
        if (xzero) TE_CHECK_HIP(hipMemcpyAsync(x, dc, (size_t)L.n * L.bs * m * sizeof(T), hipMemcpyDeviceToDevice, s));
        else axpy<T>(x, dc, 1.0, L.n * L.bs * m, s);
        return;
    }
    for (int k = 0; k + 1 < degree; ++k) {
        const bool last = (k + 2 == degree);
        cheb_step<T>(level_op<T>(L), dc, rin, dinv, W.r.p, dn, x, L.c1[k], L.c2[k], last, xzero && k == 0, m, s);
        rin = W.r.p;
        std::swap(dc, dn);
    }
}

// x = Chebyshev(g, x0 = x) (post-smoothing form, x0 arbitrary)
template <typename T>
static void smooth_from(amg_handle *h, Level &L, const T *g, T *x, int m, hipStream_t s) {
    Work<T> &W = work<T>(L);
    cheb_init<T>(level_op<T>(L), x, g, dinv_of<T>(L), W.r.p, W.d.p, 1.0 / L.theta, m, s);
    cheb_chain<T>(L, W.r.p, x, false, h->opt.cheb_degree, m, s);
}

template <typename T>
void vcycle(amg_handle *h, int l, const T *g, T *x, int m, hipStream_t s) {
    Level &L = h->L[l];
    Prof *pf = (l == 0) ? &h->prof : nullptr;
    auto B = [&](int c) { if (pf) pf->begin(c); };
    auto E = [&](int c) { if (pf) pf->end(c); };
    if (l + 1 == (int)h->L.size()) {
        B(TE_K_COARSE);
        dense_mv<T>(h->Ainv.p, g, x, h->nc, m, s);
        E(TE_K_COARSE);
        return;
    }
    Work<T> &W = work<T>(L);
    const int64_t nv = L.n * L.bs * m;
    const T *dinv = dinv_of<T>(L);
    const int deg = h->opt.cheb_degree;
    // pre-smoothing from x0 = 0: r0 = g, d0 = D^-1 g / theta
    B(TE_K_VECTOR);
    jacobi_scale<T>(g, dinv, W.d.p, 1.0 / L.theta, nv, m, s);
    E(TE_K_VECTOR);
    B(TE_K_PRE);
    cheb_chain<T>(L, g, x, true, deg, m, s);
    E(TE_K_PRE);
    // residual, restriction, coarse correction, prolongation
    B(TE_K_RESID);
    sell_apply<T>(level_op<T>(L), x, W.s.p, g, 2, m, s);
    E(TE_K_RESID);
    Level &N = h->L[l + 1];
    Work<T> &WN = work<T>(N);
    B(TE_K_RESTRICT);
    sell_apply<T>(L.R, W.s.p, WN.g.p, nullptr, 0, m, s);
    E(TE_K_RESTRICT);
    B(TE_K_COARSE);
    vcycle<T>(h, l + 1, WN.g.p, WN.x.p, m, s);
    E(TE_K_COARSE);
    B(TE_K_PROLONG);
    sell_apply<T>(L.P, WN.x.p, x, nullptr, 1, m, s);
    E(TE_K_PROLONG);
    // post-smoothing from the corrected x
    B(TE_K_POSTINIT);
    cheb_init<T>(level_op<T>(L), x, g, dinv, W.r.p, W.d.p, 1.0 / L.theta, m, s);
    E(TE_K_POSTINIT);
    B(TE_K_POST);
    cheb_chain<T>(L, W.r.p, x, false, deg, m, s);
    E(TE_K_POST);
}

// z = M^-1 r on level 0 (float64 in and out)
static void precondition_body(amg_handle *h, const double *r, double *z, int m, bool mixed, hipStream_t s) {
    Level &L0 = h->L[0];
    const int64_t nv = L0.n * 3 * m;
    if (!mixed) {
        vcycle<double>(h, 0, r, z, m, s);
        return;
    }
    h->prof.begin(TE_K_VECTOR);
    cast_f64_f32(r, L0.w32.g.p, nv, s);
    h->prof.end(TE_K_VECTOR);
    vcycle<float>(h, 0, L0.w32.g.p, L0.w32.x.p, m, s);
    h->prof.begin(TE_K_VECTOR);
    cast_f32_f64(L0.w32.x.p, z, nv, s);
    h->prof.end(TE_K_VECTOR);
}

// The preconditioner of a solve (r and z are the handle's own vectors) is a
// fixed sequence of launches: captured once per (precision, nrhs) as a HIP
// graph and replayed, which removes the host launch cost of its many small
// kernels on small meshes.  Profiled solves launch the kernels directly.
static void precondition(amg_handle *h, const double *r, double *z, int m, bool mixed, hipStream_t s) {
    if (h->prof.on) {
        precondition_body(h, r, z, m, mixed, s);
        return;
    }
    const int key = (mixed ? 1000 : 0) + m;
    hipGraphExec_t x = h->vgraphs.find(key);
    if (!x) {
        if (!h->vgraphs.cap) TE_CHECK_HIP(hipStreamCreateWithFlags(&h->vgraphs.cap, hipStreamNonBlocking));
        hipStream_t c = h->vgraphs.cap;
        hipGraph_t g = nullptr;
        TE_CHECK_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        try {
            precondition_body(h, r, z, m, mixed, c);
        } catch (...) {
            (void)hipStreamEndCapture(c, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        TE_CHECK_HIP(hipStreamEndCapture(c, &g));
        const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        TE_CHECK_HIP(e);
        h->vgraphs.g.emplace_back(key, x);
    }
    TE_CHECK_HIP(hipGraphLaunch(x, s));
}

struct HostScal {
    std::vector<double> v;
    std::vector<int32_t> f;
};

static void fetch(const double *dsum, int count, std::vector<double> &out, hipStream_t s) {
    out.resize(count);
    TE_CHECK_HIP(hipMemcpyAsync(out.data(), dsum, count * sizeof(double), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Block CG (O'Leary, Linear Algebra Appl. 29, 1980) over the columns
// ---------------------------------------------------------------------------
// One Krylov space shared by the m columns, with the search block
// orthonormalised every step and its numerically dependent directions
// dropped (the breakdown-free form of Ji and Li 2017; Dubrulle 2001):
//   R = B - A X;  Z = M^-1 R;  P = orth(Z)
//   repeat:  Q = A P;  alpha = (P^T Q)^-1 (P^T R);  X += P alpha;  R -= Q alpha
//            stop test;  Z = M^-1 R;  beta = -(P^T Q)^-1 (Q^T Z);  P = orth(Z + P beta)
// The m x m algebra runs on the host in float64.  orth uses a pivoted
// Cholesky factor of the Gram matrix (W^T W = Pi L L^T Pi^T, P = W Pi L^-T),
// dropping directions whose remaining pivot is below (1e-6)^2 of the largest
// diagonal; P^T R, P^T Q, P^T P, P^T Z, Q^T Z, Z^T Z come from two fused
// passes over the block vectors, and W^T W = Z^T Z + beta^T P^T Z +
// Z^T P beta + beta^T P^T P beta is formed from them.
namespace {
constexpr int BM = 64;

struct Small {  // 64 x 64 row-major, zero-padded
    std::vector<double> a = std::vector<double>(BM * BM, 0.0);
    double &operator()(int i, int j) { return a[(size_t)i * BM + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * BM + j]; }
};

// X = G^-1 Y for the leading r x r block of an SPD G (Cholesky); false if G
// is not positive definite there.  Y, X: r x m.
bool chol_solve(const Small &G, int r, const Small &Y, int m, Small &X) {
    std::vector<double> L((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j) {
        double d = G(j, j);
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * r + k] * L[(size_t)j * r + k];
        if (!(d > 0.0)) return false;
        L[(size_t)j * r + j] = std::sqrt(d);
        for (int i = j + 1; i < r; ++i) {
            double v = G(i, j);
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * r + k] * L[(size_t)j * r + k];
            L[(size_t)i * r + j] = v / L[(size_t)j * r + j];
        }
    }
    X = Small();
    for (int c = 0; c < m; ++c) {
        std::vector<double> y(r);
        for (int i = 0; i < r; ++i) {
            double v = Y(i, c);
            for (int k = 0; k < i; ++k) v -= L[(size_t)i * r + k] * y[k];
            y[i] = v / L[(size_t)i * r + i];
        }
        for (int i = r - 1; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < r; ++k) v -= L[(size_t)k * r + i] * X(k, c);
            X(i, c) = v / L[(size_t)i * r + i];
        }
    }
    return true;
}

// T (m x rank) with (W T)^T (W T) = I from the Gram matrix G = W^T W.
int orth_transform(const Small &G, int m, double drop_tol, Small &T) {
    Small A = G;
    std::vector<int> perm(m);
    for (int i = 0; i < m; ++i) perm[i] = i;
    double d0 = 0.0;
    for (int i = 0; i < m; ++i) d0 = std::max(d0, A(i, i));
    Small L;
    int rank = 0;
    for (int k = 0; k < m && d0 > 0.0; ++k) {
        int q = k;
        for (int i = k + 1; i < m; ++i)
            if (A(i, i) > A(q, q)) q = i;
        if (!(A(q, q) > drop_tol * drop_tol * d0)) break;
        if (q != k) {
            std::swap(perm[k], perm[q]);
            for (int j = 0; j < m; ++j) std::swap(A.a[(size_t)k * BM + j], A.a[(size_t)q * BM + j]);
            for (int i = 0; i < m; ++i) std::swap(A.a[(size_t)i * BM + k], A.a[(size_t)i * BM + q]);
            for (int j = 0; j < k; ++j) std::swap(L.a[(size_t)k * BM + j], L.a[(size_t)q * BM + j]);
        }
        const double lkk = std::sqrt(A(k, k));
        L(k, k) = lkk;
        for (int i = k + 1; i < m; ++i) L(i, k) = A(i, k) / lkk;
        for (int i = k + 1; i < m; ++i)
            for (int j = k + 1; j <= i; ++j) {
                A(i, j) -= L(i, k) * L(j, k);
                A(j, i) = A(i, j);
            }
        ++rank;
    }
    // T = Pi[:, :rank] L_r^-T: solve L_r^T Y = I (upper triangular) column by column
    T = Small();
    for (int c = 0; c < rank; ++c) {
        std::vector<double> y(rank, 0.0);
        for (int i = rank - 1; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k < rank; ++k) v -= L(k, i) * y[k];
            y[i] = v / L(i, i);
        }
        for (int i = 0; i < rank; ++i) T(perm[i], c) = y[i];
    }
    return rank;
}

Small matmul(const Small &A, const Small &B, int n, int k, int m) {  // (n x k)(k x m)
    Small C;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int l = 0; l < k; ++l) v += A(i, l) * B(l, j);
            C(i, j) = v;
        }
    return C;
}
}  // namespace

static int block_solve_impl(amg_handle *h, const double *b_nat, double *u_nat, int m, const pcg_options &o,
                            pcg_report *rep, hipStream_t s) {
    TE_REQUIRE(o.precision == TE_PREC_FP64, TE_EINVAL, "block CG runs in float64");
    const double drop_tol = 1e-6;
    Level &L0 = h->L[0];
    const int64_t n = L0.n, rows = n * 3, nv = rows * m;
    double *part = h->partials.p, *sums = h->sums.p;
    h->prof.reset(false, s);
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    TE_CHECK_HIP(hipEventCreate(&ev.a));
    TE_CHECK_HIP(hipEventCreate(&ev.b));
    TE_CHECK_HIP(hipEventRecord(ev.a, s));
    double *X = h->u.p, *R = h->r.p, *Z = h->z.p, *P = h->p.p, *Q = h->q.p, *B = h->b.p, *Tt = h->t.p;
    permute_gather(b_nat, B, L0.perm.p, n, 3, m, s);
    permute_gather(u_nat, X, L0.perm.p, n, 3, m, s);
    const int nxr = block_xr_nblocks(rows);
    {  // kept in the handle: the sizes depend on the level-0 rows and max_nrhs only
        const size_t mm = (size_t)h->opt.max_nrhs;
        if (!h->bgpart.p) h->bgpart.alloc((size_t)block_gram_nblocks() * 3 * BM * BM);
        if (!h->bgout.p) h->bgout.alloc(3 * BM * BM);
        if (!h->bsmall.p) h->bsmall.alloc(2 * BM * BM);
        if (!h->bxpart.p) h->bxpart.alloc((size_t)(nxr + 1024) * mm);
    }
    DBuf<double> &gpart = h->bgpart, &gout = h->bgout, &smalls = h->bsmall, &xpart = h->bxpart;
    std::vector<double> bb, rr, tr;
    dot_partials(B, B, nv, m, part, s);
    reduce_partials(part, dot_nblocks(rows), m, sums, s);
    fetch(sums, m, bb, s);
    auto rel_of = [&](const std::vector<double> &v, std::vector<double> &out) {
        out.resize(m);
        bool all = true;
        for (int j = 0; j < m; ++j) {
            TE_REQUIRE(std::isfinite(v[j]), TE_ENAN, "NaN in block CG column %d", j);
            out[j] = bb[j] > 0 ? std::sqrt(v[j] / bb[j]) : 0.0;
            all = all && out[j] <= o.rtol;
        }
        return all;
    };
    auto gram = [&](std::initializer_list<const double *> mats, std::initializer_list<std::pair<int, int>> pairs,
                    std::vector<Small> &res) {
        const double *mv[3];
        int li[3], ri[3], k = 0;
        for (const double *p : mats) mv[k++] = p;
        const int nmat = k;
        k = 0;
        for (auto pr : pairs) {
            li[k] = pr.first;
            ri[k] = pr.second;
            ++k;
        }
        block_gram(mv, nmat, li, ri, k, rows, m, gpart.p, gout.p, s);
        std::vector<double> hbuf;
        fetch(gout.p, k * BM * BM, hbuf, s);
        res.assign(k, Small());
        for (int p = 0; p < k; ++p) std::copy(hbuf.begin() + (size_t)p * BM * BM, hbuf.begin() + (size_t)(p + 1) * BM * BM,
                                              res[p].a.begin());
    };
    auto put_small = [&](const Small &A0, const Small &A1) {
        std::vector<double> hbuf(2 * BM * BM);
        std::copy(A0.a.begin(), A0.a.end(), hbuf.begin());
        std::copy(A1.a.begin(), A1.a.end(), hbuf.begin() + BM * BM);
        TE_CHECK_HIP(hipMemcpyAsync(smalls.p, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
    };
    // R = B - A X
    sell_resid_norm(cg_operator(h), X, B, R, m, part, s);
    reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
    fetch(sums, m, rr, s);
    std::vector<double> rel;
    bool done = rel_of(rr, rel);
    int it = 0, replaced = 0, rank = 0;
    std::vector<Small> g1, g2;
    if (!done) {
        precondition(h, R, Z, m, false, s);
        gram({Z}, {{0, 0}}, g2);
        Small T;
        rank = orth_transform(g2[0], m, drop_tol, T);
        TE_CHECK_HIP(hipMemsetAsync(P, 0, nv * sizeof(double), s));
        put_small(T, Small());
        block_p(rows, m, smalls.p, smalls.p + BM * BM, Z, P, s);
    }
    bool conv = done;
    while (!done && rank > 0 && it < o.maxit) {
        sell_apply<double>(cg_operator(h), P, Q, nullptr, 0, m, s);
        gram({P, Q, R}, {{0, 1}, {0, 2}, {0, 0}}, g1);  // P^T Q, P^T R, P^T P
        Small alpha;
        TE_REQUIRE(chol_solve(g1[0], rank, g1[1], m, alpha), TE_EINDEF, "block CG breakdown: P^T A P is not SPD");
        put_small(alpha, Small());
        block_xr(rows, m, smalls.p, P, Q, X, R, xpart.p, s);
        reduce_partials(xpart.p, nxr, m, sums, s);
        fetch(sums, m, rr, s);
        ++it;
        if (rel_of(rr, rel)) {
            sell_resid_norm(cg_operator(h), X, B, Tt, m, part, s);
            reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
            fetch(sums, m, tr, s);
            if (rel_of(tr, rel)) {
                conv = true;
                break;
            }
            if (replaced >= o.max_replace) break;
            ++replaced;
            TE_CHECK_HIP(hipMemcpyAsync(R, Tt, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        precondition(h, R, Z, m, false, s);
        gram({P, Q, Z}, {{0, 2}, {1, 2}, {2, 2}}, g2);  // P^T Z, Q^T Z, Z^T Z
        Small beta;
        TE_REQUIRE(chol_solve(g1[0], rank, g2[1], m, beta), TE_EINDEF, "block CG breakdown: P^T A P is not SPD");
        for (double &v : beta.a) v = -v;
        // W^T W with W = Z + P beta
        Small G = g2[2];
        const Small btPZ = [&] {  // beta^T (P^T Z)
            Small c;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) {
                    double v = 0.0;
                    for (int l = 0; l < rank; ++l) v += beta(l, i) * g2[0](l, j);
                    c(i, j) = v;
                }
            return c;
        }();
        const Small PPb = matmul(g1[2], beta, rank, rank, m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double v = 0.0;
                for (int l = 0; l < rank; ++l) v += beta(l, i) * PPb(l, j);
                G(i, j) += btPZ(i, j) + btPZ(j, i) + v;
            }
        Small T;
        const int nr = orth_transform(G, m, drop_tol, T);
        const Small T2 = matmul(beta, T, rank, m, nr);  // P_new = Z T + P (beta T)
        put_small(T, T2);
        block_p(rows, m, smalls.p, smalls.p + BM * BM, Z, P, s);
        rank = nr;
    }
    if (!conv) {  // final true residual of every column
        sell_resid_norm(cg_operator(h), X, B, Tt, m, part, s);
        reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
        fetch(sums, m, tr, s);
        rel_of(tr, rel);
    }
    permute_scatter(X, u_nat, L0.perm.p, n, 3, m, s);
    TE_CHECK_HIP(hipEventRecord(ev.b, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    TE_CHECK_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    bool all = true;
    for (int j = 0; j < m; ++j) {
        const bool cj = rel[j] <= o.rtol;
        all = all && cj;
        if (rep) {
            if (rep->iters) rep->iters[j] = it;
            if (rep->converged) rep->converged[j] = cj;
            if (rep->relres_true) rep->relres_true[j] = rel[j];
        }
    }
    if (rep) {
        if (rep->history)
            for (int k = 0; k <= o.maxit; ++k)
                for (int j = 0; j < m; ++j) rep->history[(size_t)k * m + j] = NAN;
        rep->max_iters = it;
        rep->time_ms = ms;
        for (int c = 0; c < TE_K_COUNT; ++c) {
            rep->kernel_ms[c] = 0.0;
            rep->kernel_launches[c] = 0;
        }
    }
    return all ? TE_OK : TE_ENOTCONV;
}

static int solve_impl(amg_handle *h, const double *b_nat, double *u_nat, int m, const pcg_options *opt_in,
                      pcg_report *rep, hipStream_t s) {
    TE_REQUIRE(h && b_nat && u_nat, TE_EINVAL, "NULL argument");
    TE_REQUIRE(m >= 1 && m <= h->opt.max_nrhs, TE_EINVAL, "nrhs %d outside 1..max_nrhs (%d)", m, h->opt.max_nrhs);
    pcg_options o;
    if (opt_in) o = *opt_in;
    else pcg_options_default(&o);
    TE_REQUIRE(o.rtol > 0 && o.maxit >= 0, TE_EINVAL, "bad rtol / maxit");
    const bool mixed = o.precision == TE_PREC_MIXED;
    TE_REQUIRE(o.precision == TE_PREC_FP64 || mixed, TE_EINVAL, "unknown precision %d", o.precision);
    TE_REQUIRE(!mixed || h->opt.build_fp32, TE_EINVAL, "mixed precision needs build_fp32 at setup");
    if (o.block && m > 1) return block_solve_impl(h, b_nat, u_nat, m, o, rep, s);
    Level &L0 = h->L[0];
    const int64_t n = L0.n, rows = n * 3, nv = rows * m;
    CgScalars *S = reinterpret_cast<CgScalars *>(h->scal.p);
    double *part = h->partials.p, *sums = h->sums.p;

    h->prof.reset(o.profile != 0, s);
    struct Events {  // released on every exit, errors included
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    TE_CHECK_HIP(hipEventCreate(&ev.a));
    TE_CHECK_HIP(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    TE_CHECK_HIP(hipEventRecord(e0, s));

    permute_gather(b_nat, h->b.p, L0.perm.p, n, 3, m, s);
    permute_gather(u_nat, h->u.p, L0.perm.p, n, 3, m, s);
    std::vector<double> bb, rr, tr;
    dot_partials(h->b.p, h->b.p, nv, m, part, s);
    reduce_partials(part, dot_nblocks(rows), m, sums, s);
    fetch(sums, m, bb, s);
    sell_resid_norm(cg_operator(h), h->u.p, h->b.p, h->r.p, m, part, s);
    reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
    fetch(sums, m, rr, s);

    std::vector<int32_t> active(64, 0), flags(64, 0), iters(m, 0), conv(m, 0), replaced(m, 0);
    std::vector<double> hist;
    if (rep && rep->history) {
        for (int k = 0; k <= o.maxit; ++k)
            for (int j = 0; j < m; ++j) rep->history[(size_t)k * m + j] = NAN;
    }
    int n_active = 0;
    std::vector<int32_t> zero_cols(64, 0);
    bool any_zero = false;
    for (int j = 0; j < m; ++j) {
        const double rel = bb[j] > 0 ? std::sqrt(rr[j] / bb[j]) : 0.0;
        if (rep && rep->history) rep->history[j] = rel;
        TE_REQUIRE(std::isfinite(rr[j]) && std::isfinite(bb[j]), TE_ENAN, "NaN/Inf in the right-hand side or guess");
        if (bb[j] == 0.0) {
            conv[j] = 1;  // u = 0 is the solution
            zero_cols[j] = 1;
            any_zero = true;
        } else if (rel <= o.rtol) {
            conv[j] = 1;
        } else {
            active[j] = 1;
            ++n_active;
        }
    }
    if (any_zero) {  // b = 0 has the solution u = 0 whatever the guess
        TE_CHECK_HIP(hipMemcpyAsync(h->colsel.p, zero_cols.data(), 64 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        TE_CHECK_HIP(hipMemsetAsync(h->t.p, 0, nv * sizeof(double), s));
        copy_cols(h->u.p, h->t.p, h->colsel.p, nv, m, s);
        TE_CHECK_HIP(hipStreamSynchronize(s));
    }
    if (n_active) {
        TE_CHECK_HIP(hipMemsetAsync(h->scal.p, 0, sizeof(CgScalars), s));
        TE_CHECK_HIP(hipMemcpyAsync(S->active, active.data(), 64 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        // zero-guess columns that are already converged stay untouched (alpha = 0)
        precondition(h, h->r.p, h->z.p, m, mixed, s);
        dot_rz(h->r.p, h->z.p, nullptr, rows, m, part, s);
        reduce_pairs(part, dot_nblocks(rows), m, sums, s);
        cg_rz0(S, sums, m, s);
        TE_CHECK_HIP(hipMemcpyAsync(h->p.p, h->z.p, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
        TE_CHECK_HIP(hipMemcpyAsync(flags.data(), S->flag, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < m; ++j)
            if (active[j] && flags[j]) {
                TE_REQUIRE(flags[j] != 3, TE_ENAN, "NaN in (r,z) of column %d", j);
                TE_REQUIRE(false, TE_EINDEF, "CG breakdown at start: (r,z) <= 0 in column %d", j);
            }
    }
    int it = 0;
    while (n_active > 0 && it < o.maxit) {
        ++it;
        h->prof.begin(TE_K_AP);
        sell_dot(cg_operator(h), h->p.p, h->q.p, m, part, s);
        h->prof.end(TE_K_AP);
        h->prof.begin(TE_K_VECTOR);
        reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
        cg_alpha(S, sums, m, s);
        cg_update(h->u.p, h->r.p, mixed ? h->r_old.p : nullptr, h->p.p, h->q.p, S->alpha, rows, m, part, s);
        reduce_partials(part, dot_nblocks(rows), m, sums, s);
        h->prof.end(TE_K_VECTOR);
        TE_CHECK_HIP(hipMemcpyAsync(flags.data(), S->flag, 64 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        fetch(sums, m, rr, s);
        std::vector<int32_t> cand(m, 0);
        bool any_cand = false;
        for (int j = 0; j < m; ++j) {
            if (!active[j]) continue;
            if (flags[j] == 3 || !std::isfinite(rr[j])) TE_REQUIRE(false, TE_ENAN, "NaN in CG column %d", j);
            if (flags[j]) TE_REQUIRE(false, TE_EINDEF, "CG breakdown in column %d at iteration %d: (p,Ap) <= 0", j, it);
            iters[j] = it;
            const double rel = std::sqrt(rr[j] / bb[j]);
            if (rep && rep->history) rep->history[(size_t)it * m + j] = rel;
            if (rel <= o.rtol) {
                cand[j] = 1;
                any_cand = true;
            }
        }
        if (any_cand) {
            sell_resid_norm(cg_operator(h), h->u.p, h->b.p, h->t.p, m, part, s);
            reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
            fetch(sums, m, tr, s);
            std::vector<int32_t> repl(64, 0);
            bool any_repl = false, changed = false;
            for (int j = 0; j < m; ++j) {
                if (!cand[j]) continue;
                const double rel = std::sqrt(tr[j] / bb[j]);
                if (rel <= o.rtol) {
                    conv[j] = 1;
                    active[j] = 0;
                    --n_active;
                    changed = true;
                } else if (replaced[j] < o.max_replace) {
                    ++replaced[j];
                    repl[j] = 1;
                    any_repl = true;
                } else {
                    active[j] = 0;
                    --n_active;
                    changed = true;
                }
            }
            if (any_repl) {
                TE_CHECK_HIP(hipMemcpyAsync(h->colsel.p, repl.data(), 64 * sizeof(int32_t), hipMemcpyHostToDevice, s));
                copy_cols(h->r.p, h->t.p, h->colsel.p, nv, m, s);
                TE_CHECK_HIP(hipStreamSynchronize(s));
            }
            if (changed)
                TE_CHECK_HIP(hipMemcpyAsync(S->active, active.data(), 64 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        if (n_active == 0) break;
        precondition(h, h->r.p, h->z.p, m, mixed, s);
        h->prof.begin(TE_K_VECTOR);
        dot_rz(h->r.p, h->z.p, mixed ? h->r_old.p : nullptr, rows, m, part, s);
        reduce_pairs(part, dot_nblocks(rows), m, sums, s);
        cg_beta(S, sums, m, mixed ? 1 : 0, s);
        p_update(h->p.p, h->z.p, S->beta, nv, m, s);
        h->prof.end(TE_K_VECTOR);
    }
    // final true residual of every column
    sell_resid_norm(cg_operator(h), h->u.p, h->b.p, h->t.p, m, part, s);
    reduce_partials(part, sell_partials_count(cg_operator(h), m), m, sums, s);
    permute_scatter(h->u.p, u_nat, L0.perm.p, n, 3, m, s);
    TE_CHECK_HIP(hipEventRecord(e1, s));
    fetch(sums, m, tr, s);
    float ms = 0.f;
    TE_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    bool all_conv = true;
    int maxit_seen = 0;
    for (int j = 0; j < m; ++j) {
        const double rel = bb[j] > 0 ? std::sqrt(tr[j] / bb[j]) : 0.0;
        if (bb[j] > 0) conv[j] = conv[j] && rel <= o.rtol;
        all_conv = all_conv && conv[j];
        maxit_seen = std::max(maxit_seen, iters[j]);
        if (rep) {
            if (rep->iters) rep->iters[j] = iters[j];
            if (rep->converged) rep->converged[j] = conv[j];
            if (rep->relres_true) rep->relres_true[j] = rel;
        }
    }
    if (rep) {
        rep->max_iters = maxit_seen;
        rep->time_ms = ms;
        for (int c = 0; c < TE_K_COUNT; ++c) {
            double t = 0.0;
            for (int i = 0; i < h->prof.used[c]; ++i) {
                float e = 0.f;
                TE_CHECK_HIP(hipEventElapsedTime(&e, h->prof.ev[c][2 * i], h->prof.ev[c][2 * i + 1]));
                t += e;
            }
            rep->kernel_ms[c] = t;
            rep->kernel_launches[c] = h->prof.used[c];
        }
    }
    h->prof.reset(false, s);
    return all_conv ? TE_OK : TE_ENOTCONV;
}

// ---------------------------------------------------------------------------
// component access for tests (natural numbering of the level)
// ---------------------------------------------------------------------------
static void to_f32(const double *x, DBuf<float> &y, int64_t n, hipStream_t s) {
    y.alloc(n);
    cast_f64_f32(x, y.p, n, s);
}

static int apply_impl(amg_handle *h, int l, int op, int prec, const double *x, double *y, hipStream_t s) {
    TE_REQUIRE(h && x && y, TE_EINVAL, "NULL argument");
    TE_REQUIRE(l >= 0 && l < (int)h->L.size(), TE_EINVAL, "bad level %d", l);
    const bool f32 = prec == TE_PREC_MIXED;
    TE_REQUIRE(!f32 || h->opt.build_fp32, TE_EINVAL, "float32 copies not built");
    h->prof.reset(false, s);
    Level &L = h->L[l];
    const int64_t nl = L.n * L.bs;
    const bool has_next = l + 1 < (int)h->L.size();
    TE_REQUIRE(op == TE_OP_A || op == TE_OP_VCYCLE || has_next, TE_EINVAL, "level %d has no transfer/smoother", l);
    Level *N = has_next ? &h->L[l + 1] : nullptr;
    const int64_t nn = N ? N->n * N->bs : 0;
    DBuf<double> xs, ys;
    switch (op) {
        case TE_OP_A:
        case TE_OP_SMOOTH:
        case TE_OP_VCYCLE: {
            xs.alloc(nl);
            ys.alloc(nl);
            permute_gather(x, xs.p, L.perm.p, L.n, L.bs, 1, s);
            if (op == TE_OP_SMOOTH) permute_gather(y, ys.p, L.perm.p, L.n, L.bs, 1, s);
            if (!f32) {
                if (op == TE_OP_A) sell_apply<double>(L.A, xs.p, ys.p, nullptr, 0, 1, s);
                else if (op == TE_OP_SMOOTH) smooth_from<double>(h, L, xs.p, ys.p, 1, s);
                else vcycle<double>(h, l, xs.p, ys.p, 1, s);
            } else {
                DBuf<float> x32, y32;
                to_f32(xs.p, x32, nl, s);
                y32.alloc(nl);
                if (op == TE_OP_SMOOTH) cast_f64_f32(ys.p, y32.p, nl, s);
                if (op == TE_OP_A) sell_apply<float>(level_op<float>(L), x32.p, y32.p, nullptr, 0, 1, s);
                else if (op == TE_OP_SMOOTH) smooth_from<float>(h, L, x32.p, y32.p, 1, s);
                else vcycle<float>(h, l, x32.p, y32.p, 1, s);
                cast_f32_f64(y32.p, ys.p, nl, s);
                TE_CHECK_HIP(hipStreamSynchronize(s));
            }
            permute_scatter(ys.p, y, L.perm.p, L.n, L.bs, 1, s);
            break;
        }
        case TE_OP_P: {
            xs.alloc(nn);
            ys.alloc(nl);
            permute_gather(x, xs.p, N->perm.p, N->n, N->bs, 1, s);
            TE_CHECK_HIP(hipMemsetAsync(ys.p, 0, nl * sizeof(double), s));
            if (!f32) {
                sell_apply<double>(L.P, xs.p, ys.p, nullptr, 1, 1, s);
            } else {
                DBuf<float> x32, y32(nl);
                to_f32(xs.p, x32, nn, s);
                TE_CHECK_HIP(hipMemsetAsync(y32.p, 0, nl * sizeof(float), s));
                sell_apply<float>(L.P, x32.p, y32.p, nullptr, 1, 1, s);
                cast_f32_f64(y32.p, ys.p, nl, s);
                TE_CHECK_HIP(hipStreamSynchronize(s));
            }
            permute_scatter(ys.p, y, L.perm.p, L.n, L.bs, 1, s);
            break;
        }
        case TE_OP_R: {
            xs.alloc(nl);
            ys.alloc(nn);
            permute_gather(x, xs.p, L.perm.p, L.n, L.bs, 1, s);
            if (!f32) {
                sell_apply<double>(L.R, xs.p, ys.p, nullptr, 0, 1, s);
            } else {
                DBuf<float> x32, y32(nn);
                to_f32(xs.p, x32, nl, s);
                sell_apply<float>(L.R, x32.p, y32.p, nullptr, 0, 1, s);
                cast_f32_f64(y32.p, ys.p, nn, s);
                TE_CHECK_HIP(hipStreamSynchronize(s));
            }
            permute_scatter(ys.p, y, N->perm.p, N->n, N->bs, 1, s);
            break;
        }
        default:
            TE_REQUIRE(false, TE_EINVAL, "unknown op %d", op);
    }
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return TE_OK;
}

// u0 <- gamma u0 with gamma = (b, u0) / (u0, A u0): the multiple of the guess
// with the lowest energy 1/2 u^T A u - b^T u, i.e. the smallest A-norm error
// along the guess; gamma = 0 (the zero guess) when the guess cannot beat zero.
static int energy_scale_impl(amg_handle *h, const double *b_nat, double *u_nat, double *gamma_out, hipStream_t s) {
    TE_REQUIRE(h && b_nat && u_nat, TE_EINVAL, "NULL argument");
    Level &L0 = h->L[0];
    const int64_t n = L0.n, nv = n * 3;
    permute_gather(b_nat, h->b.p, L0.perm.p, n, 3, 1, s);
    permute_gather(u_nat, h->t.p, L0.perm.p, n, 3, 1, s);
    sell_apply<double>(cg_operator(h), h->t.p, h->q.p, nullptr, 0, 1, s);
    double *part = h->partials.p, *sums = h->sums.p;
    dot_partials(h->b.p, h->t.p, nv, 1, part, s);
    reduce_partials(part, dot_nblocks(nv), 1, sums, s);
    dot_partials(h->t.p, h->q.p, nv, 1, part, s);
    reduce_partials(part, dot_nblocks(nv), 1, sums + 1, s);
    std::vector<double> v;
    fetch(sums, 2, v, s);
    const double bu = v[0], uau = v[1];
    TE_REQUIRE(std::isfinite(bu) && std::isfinite(uau), TE_ENAN, "NaN/Inf in the guess");
    const double gamma = (uau > 0.0 && bu > 0.0) ? bu / uau : 0.0;
    if (gamma == 0.0) TE_CHECK_HIP(hipMemsetAsync(u_nat, 0, nv * sizeof(double), s));
    else scal(u_nat, gamma, nv, s);
    TE_CHECK_HIP(hipStreamSynchronize(s));
    if (gamma_out) *gamma_out = gamma;
    return TE_OK;
}

}  // namespace te

using namespace te;

extern "C" int amg_energy_scale(amg_handle *h, const double *b, double *u0, double *gamma, hipStream_t stream) {
    return guarded([&] { return energy_scale_impl(h, b, u0, gamma, stream); });
}

extern "C" void pcg_options_default(pcg_options *o) {
    if (!o) return;
    o->rtol = 1e-8;
    o->maxit = 500;
    o->precision = TE_PREC_FP64;
    o->max_replace = 3;
    o->profile = 0;
    o->block = 0;
}

extern "C" int amg_pcg_solve(amg_handle *h, const double *b, double *u, int32_t nrhs, const pcg_options *opt,
                             pcg_report *rep, hipStream_t stream) {
    return guarded([&] { return solve_impl(h, b, u, nrhs, opt, rep, stream); });
}

extern "C" int amg_apply(amg_handle *h, int32_t level, int32_t op, int32_t precision, const double *x, double *y,
                         hipStream_t stream) {
    return guarded([&] { return apply_impl(h, level, op, precision, x, y, stream); });
}
