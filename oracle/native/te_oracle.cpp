// Oracle, large-size form: a plain C++17/OpenMP restatement of the float64
// oracle of the thermoelastic solve (assembly of eq. wf_elastic, Dirichlet
// elimination of eq. u-dbc, smoothed-aggregation AMG of Sec. 2.1.3 and 5.1,
// preconditioned CG of Sec. 2.1.2), so that an oracle solution exists at the
// size of a whole one-GPU problem (12M DOF), where the NumPy oracle cannot go.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark load this library.  It shares no code,
// header, table or constant generator with the HIP library.
//
// Style: one loop per definition, rows in parallel (OpenMP) where rows are
// independent; no blocking, no fusion, no reordering of a definition beyond
// what parallel rows need.  Dot products and norms sum fixed chunks in a fixed
// order, so results do not depend on the thread count.
//
// What is computed (each step cites the passage it follows; the readings
// where the paper is silent are the same as the NumPy oracle's):
//  * Lagrange P1/P2 basis on affine tetrahedra (Sec. 3.1), exact integrals of
//    barycentric monomials: int l0^a l1^b l2^c l3^d = a!b!c!d! 3! |K| / (a+b+c+d+3)!.
//  * K[(a,i),(b,j)] = int lam d_i phi_a d_j phi_b + mu d_j phi_a d_i phi_b
//                       + mu delta_ij grad phi_a . grad phi_b                (eq. wf_elastic)
//    b[(a,i)] = (3 lam + 2 mu) alpha int (T_h - T_ref) d_i phi_a + int f_i phi_a.
//  * Dirichlet: b -= A[:,D] u_D, rows/columns of D zeroed, unit diagonal, b_D = u_D.
//  * Near-nullspace: 3 translations and 3 rotations about the node centroid,
//    zero at constrained DOFs.
//  * Per level: strength s_IJ = |A_IJ|_F / sqrt(|A_II|_F |A_JJ|_F), theta_l =
//    theta0 2^-l; aggregation (MIS-2 roots = the sequential phase 1 visited by
//    descending fixed key, or greedy in node order), phase 2 with the 1e-9 tie
//    rule; tentative P by per-aggregate QR with diag(R) > 0 (merge of a rank
//    deficient aggregate); lambda_hat by 20 Lanczos steps on D^-1/2 A D^-1/2;
//    P = (I - 4/(3 lambda_hat) D^-1 A) P_tent; A_c = P^T (A P); stop at
//    coarse_max DOF, max_levels or a coarse share above max_coarse_ratio; dense
//    Cholesky of (A + A^T)/2 on the coarsest level.
//  * Chebyshev smoother on D^-1 A over [b/ratio, b], b = safety lambda_hat
//    (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1);
//    V-cycle with pre-smoothing from zero and post-smoothing with the same
//    polynomial; PCG (Saad Alg. 9.1) with the true-residual stop and at most
//    max_replace residual replacements, standard or flexible beta.
#include <omp.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

namespace {

using i64 = int64_t;
using i32 = int32_t;

// ---------------------------------------------------------------------------
// Barycentric polynomials and the reference integrals
// ---------------------------------------------------------------------------
struct Mono {
    std::array<int, 4> e;
    double c;
};
using Poly = std::vector<Mono>;

Poly p_mul(const Poly &p, const Poly &q) {
    Poly out;
    for (const Mono &a : p)
        for (const Mono &b : q) {
            Mono m{{a.e[0] + b.e[0], a.e[1] + b.e[1], a.e[2] + b.e[2], a.e[3] + b.e[3]}, a.c * b.c};
            bool merged = false;
            for (Mono &o : out)
                if (o.e == m.e) {
                    o.c += m.c;
                    merged = true;
                    break;
                }
            if (!merged) out.push_back(m);
        }
    return out;
}

Poly p_lam(int k, double c) {
    Mono m{{0, 0, 0, 0}, c};
    m.e[k] = 1;
    return {m};
}

// d/d l_k
Poly p_diff(const Poly &p, int k) {
    Poly out;
    for (const Mono &a : p)
        if (a.e[k] > 0) {
            Mono m = a;
            m.c *= a.e[k];
            m.e[k] -= 1;
            out.push_back(m);
        }
    return out;
}

double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// (1/|K|) int_K p dx
double p_int(const Poly &p) {
    double s = 0.0;
    for (const Mono &m : p) {
        const int d = m.e[0] + m.e[1] + m.e[2] + m.e[3];
        s += m.c * fact(m.e[0]) * fact(m.e[1]) * fact(m.e[2]) * fact(m.e[3]) * 6.0 / fact(d + 3);
    }
    return s;
}

const int EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// Lagrange basis: P1 phi_a = l_a; P2 vertices l_a (2 l_a - 1), edges 4 l_a l_b
std::vector<Poly> basis(int degree) {
    std::vector<Poly> ph;
    if (degree == 1) {
        for (int a = 0; a < 4; ++a) ph.push_back(p_lam(a, 1.0));
        return ph;
    }
    for (int a = 0; a < 4; ++a) {
        Poly v = p_mul(p_lam(a, 2.0), p_lam(a, 1.0));
        v.push_back(Mono{{0, 0, 0, 0}, 0.0});
        Poly lin = p_lam(a, -1.0);
        v.insert(v.end(), lin.begin(), lin.end());
        ph.push_back(v);
    }
    for (int e = 0; e < 6; ++e) ph.push_back(p_mul(p_lam(EDGE[e][0], 4.0), p_lam(EDGE[e][1], 1.0)));
    return ph;
}

struct Tables {
    int n = 0;                 // nodes per cell
    std::vector<double> S;     // [a][b][k][l] = int d_k phi_a d_l phi_b / |K|
    std::vector<double> W;     // [c][a][k]    = int phi_c d_k phi_a / |K|
    std::vector<double> M;     // [a][c]       = int phi_a phi_c / |K|
};

Tables make_tables(int degree) {
    Tables t;
    std::vector<Poly> ph = basis(degree);
    t.n = (int)ph.size();
    const int n = t.n;
    std::vector<std::vector<Poly>> d(n, std::vector<Poly>(4));
    for (int a = 0; a < n; ++a)
        for (int k = 0; k < 4; ++k) d[a][k] = p_diff(ph[a], k);
    t.S.assign((size_t)n * n * 16, 0.0);
    t.W.assign((size_t)n * n * 4, 0.0);
    t.M.assign((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            t.M[a * n + b] = p_int(p_mul(ph[a], ph[b]));
            for (int k = 0; k < 4; ++k) {
                t.W[((size_t)a * n + b) * 4 + k] = p_int(p_mul(ph[a], d[b][k]));
                for (int l = 0; l < 4; ++l) t.S[(((size_t)a * n + b) * 4 + k) * 4 + l] = p_int(p_mul(d[a][k], d[b][l]));
            }
        }
    return t;
}

// Cell geometry: vol = |det J| / 6 and G[k][i] = d_i l_k, J = [x1-x0, x2-x0, x3-x0]
void cell_geom(const double *X, const i32 *c, double &vol, double G[4][3]) {
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) J[r][k] = X[(i64)c[k + 1] * 3 + r] - X[(i64)c[0] * 3 + r];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    // inverse by cofactors: Jinv[k][r] = cof[r][k] / det; row k of J^-1 = grad l_{k+1}
    double cof[3][3];
    cof[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    cof[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
    cof[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    cof[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
    cof[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    cof[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
    cof[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    cof[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
    cof[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) G[k + 1][i] = cof[i][k] / det;
    for (int i = 0; i < 3; ++i) G[0][i] = -(G[1][i] + G[2][i] + G[3][i]);
    vol = std::fabs(det) / 6.0;
}

// ---------------------------------------------------------------------------
// Block compressed rows
// ---------------------------------------------------------------------------
struct Bsr {
    int br = 0, bc = 0;
    i64 nr = 0, nc = 0;
    std::vector<i64> ptr;
    std::vector<i32> col;
    std::vector<double> val;
    i64 nnzb() const { return (i64)col.size(); }
    int bsz() const { return br * bc; }
};

// y = A x (scalar vectors of nr*br and nc*bc entries)
void spmv(const Bsr &A, const double *x, double *y) {
    const int br = A.br, bc = A.bc;
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 I = 0; I < A.nr; ++I) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            const double *blk = &A.val[(size_t)k * br * bc];
            const double *xj = x + (i64)A.col[k] * bc;
            for (int i = 0; i < br; ++i)
                for (int j = 0; j < bc; ++j) acc[i] += blk[i * bc + j] * xj[j];
        }
        for (int i = 0; i < br; ++i) y[I * br + i] = acc[i];
    }
}

constexpr int NCHUNK = 512;

// sum over fixed chunks in a fixed order: independent of the thread count
template <class F>
double chunked_sum(i64 n, F f) {
    double part[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        const i64 lo = n * c / NCHUNK, hi = n * (c + 1) / NCHUNK;
        double s = 0.0;
        for (i64 i = lo; i < hi; ++i) s += f(i);
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < NCHUNK; ++c) s += part[c];
    return s;
}

double dot(const double *a, const double *b, i64 n) {
    return chunked_sum(n, [&](i64 i) { return a[i] * b[i]; });
}
double nrm2(const double *a, i64 n) { return std::sqrt(dot(a, a, n)); }

// ---------------------------------------------------------------------------
// Assembly (Sec. 2.3.3; eq. wf_elastic) and Dirichlet elimination (eq. u-dbc)
// ---------------------------------------------------------------------------
struct Problem {
    i64 n = 0;
    Bsr A;                    // Dirichlet-eliminated, 3x3 blocks
    std::vector<double> b;    // [3n]
    std::vector<uint8_t> mask;
    std::vector<double> coords;
    double t_assemble = 0.0;
};

// node -> incident (cell, local node) pairs, cells in ascending order
void incidence(i64 n, i64 nc, int npe, const i32 *cells, std::vector<i64> &start, std::vector<i64> &ent) {
    start.assign(n + 1, 0);
    for (i64 c = 0; c < nc; ++c)
        for (int a = 0; a < npe; ++a) start[cells[c * npe + a] + 1]++;
    for (i64 i = 0; i < n; ++i) start[i + 1] += start[i];
    ent.assign(start[n], 0);
    std::vector<i64> fill(start.begin(), start.end() - 1);
    for (i64 c = 0; c < nc; ++c)
        for (int a = 0; a < npe; ++a) ent[fill[cells[c * npe + a]]++] = c * npe + a;
}

Problem *assemble(i64 n, i64 nc, int degree, const double *X, const i32 *cells, double E, double nu, double alpha,
                  double T_ref, const double *T, const double *f, const uint8_t *mask, const double *u_bc) {
    auto t0 = std::chrono::steady_clock::now();
    Problem *P = new Problem;
    P->n = n;
    P->coords.assign(X, X + n * 3);
    P->mask.assign((size_t)n * 3, 0);
    if (mask) std::copy(mask, mask + n * 3, P->mask.begin());
    const int npe = degree == 1 ? 4 : 10;
    const Tables tb = make_tables(degree);
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    const double calpha = (3.0 * lam + 2.0 * mu) * alpha;
    std::vector<i64> start, ent;
    incidence(n, nc, npe, cells, start, ent);
    // pattern: I ~ J when both belong to one cell; sorted columns
    Bsr &A = P->A;
    A.br = A.bc = 3;
    A.nr = A.nc = n;
    A.ptr.assign(n + 1, 0);
    std::vector<std::vector<i32>> rows(n);
#pragma omp parallel for schedule(dynamic, 256)
    for (i64 I = 0; I < n; ++I) {
        std::vector<i32> &r = rows[I];
        for (i64 q = start[I]; q < start[I + 1]; ++q) {
            const i64 c = ent[q] / npe;
            for (int b = 0; b < npe; ++b) r.push_back(cells[c * npe + b]);
        }
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
    }
    for (i64 I = 0; I < n; ++I) A.ptr[I + 1] = A.ptr[I] + (i64)rows[I].size();
    A.col.resize(A.ptr[n]);
    A.val.assign((size_t)A.ptr[n] * 9, 0.0);
    std::vector<double> b((size_t)n * 3, 0.0);
#pragma omp parallel for schedule(dynamic, 256)
    for (i64 I = 0; I < n; ++I) {
        std::copy(rows[I].begin(), rows[I].end(), A.col.begin() + A.ptr[I]);
        std::vector<i32>().swap(rows[I]);
        const i32 *rc = &A.col[A.ptr[I]];
        const i64 rn = A.ptr[I + 1] - A.ptr[I];
        double *rv = &A.val[(size_t)A.ptr[I] * 9];
        for (i64 q = start[I]; q < start[I + 1]; ++q) {
            const i64 c = ent[q] / npe;
            const int a = (int)(ent[q] % npe);
            const i32 *cn = cells + c * npe;
            double vol, G[4][3];
            cell_geom(X, cn, vol, G);
            // block (a, b): with A1 = G^T S_ab G (3x3), the three terms of the
            // bilinear form are lam A1, mu A1^T and mu tr(A1) I
            for (int bb = 0; bb < npe; ++bb) {
                const double *S = &tb.S[((size_t)a * npe + bb) * 16];
                double A1[3][3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int k = 0; k < 4; ++k)
                            for (int l = 0; l < 4; ++l) s += S[k * 4 + l] * G[k][i] * G[l][j];
                        A1[i][j] = s;
                    }
                const double tr = A1[0][0] + A1[1][1] + A1[2][2];
                const i32 J = cn[bb];
                const i64 pos = std::lower_bound(rc, rc + rn, J) - rc;
                double *blk = rv + pos * 9;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        blk[i * 3 + j] += vol * (lam * A1[i][j] + mu * A1[j][i] + (i == j ? mu * tr : 0.0));
            }
            // load: thermal term and consistent body force
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int cc = 0; cc < npe; ++cc) {
                    const double dT = T[cn[cc]] - T_ref;
                    double w = 0.0;
                    for (int k = 0; k < 4; ++k) w += tb.W[((size_t)cc * npe + a) * 4 + k] * G[k][i];
                    s += dT * w;
                }
                double fb = 0.0;
                if (f)
                    for (int cc = 0; cc < npe; ++cc) fb += tb.M[a * npe + cc] * f[(i64)cn[cc] * 3 + i];
                b[I * 3 + i] += calpha * vol * s + vol * fb;
            }
        }
    }
    // Dirichlet elimination: lifting with the unconstrained A, then zero rows
    // and columns of constrained DOFs, unit diagonal, b_D = u_D
    std::vector<double> uD((size_t)n * 3, 0.0);
    if (u_bc)
        for (i64 d = 0; d < n * 3; ++d) uD[d] = P->mask[d] ? u_bc[d] : 0.0;
    std::vector<double> Au((size_t)n * 3, 0.0);
    spmv(A, uD.data(), Au.data());
    const uint8_t *m = P->mask.data();
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 I = 0; I < n; ++I) {
        for (int i = 0; i < 3; ++i) {
            const i64 d = I * 3 + i;
            b[d] = m[d] ? uD[d] : b[d] - Au[d];
        }
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            const i64 J = A.col[k];
            double *blk = &A.val[(size_t)k * 9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    if (m[I * 3 + i] || m[J * 3 + j]) blk[i * 3 + j] = 0.0;
            if (J == I)
                for (int i = 0; i < 3; ++i)
                    if (m[I * 3 + i]) blk[i * 3 + i] = 1.0;
        }
    }
    P->b.swap(b);
    P->t_assemble = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return P;
}

// ---------------------------------------------------------------------------
// splitmix64 (Steele, Lea & Flood 2014), from its published definition
// ---------------------------------------------------------------------------
uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Smoothed-aggregation hierarchy (Sec. 2.1.3, Sec. 5.1)
// ---------------------------------------------------------------------------
struct Opts {
    double theta0;
    i32 coarse_max, max_levels, lanczos_steps, cheb_degree;
    double cheb_ratio, cheb_safety, max_coarse_ratio;
    i32 aggregation;  // 0 greedy (node order), 1 MIS-2 (descending fixed key)
    i32 threads;
};

constexpr double TIE_RTOL = 1e-9;
constexpr double RANK_RTOL = 1e-10;
constexpr uint64_t MIS_SEED = 0xA66;

struct Level {
    Bsr A;
    int bs = 3;
    std::vector<double> D;     // point diagonal
    double lam = 0.0;
    Bsr P, R;                  // bs x 6 and 6 x bs blocks
    std::vector<i32> agg;
    // coarsest: lower Cholesky factor (dense, row-major)
    std::vector<double> L;
    i64 nd = 0;
    // smoother coefficients
    double theta = 0, delta = 0, sigma = 0;
};

struct Hier {
    Opts opt;
    std::vector<Level> lv;
    double t_setup = 0.0;
};

// strengths per stored block (0 on the diagonal); Frobenius squares summed
// in row-major order
std::vector<double> strength(const Bsr &A) {
    const int e = A.bsz();
    std::vector<double> fro(A.nnzb()), dn(A.nr, 0.0), s(A.nnzb(), 0.0);
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 I = 0; I < A.nr; ++I)
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            double acc = 0.0;
            for (int q = 0; q < e; ++q) acc = acc + A.val[(size_t)k * e + q] * A.val[(size_t)k * e + q];
            fro[k] = std::sqrt(acc);
            if (A.col[k] == I) dn[I] = fro[k];
        }
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 I = 0; I < A.nr; ++I)
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
            s[k] = A.col[k] == I ? 0.0 : fro[k] / std::sqrt(dn[I] * dn[A.col[k]]);
    return s;
}

// position of (J, I) for every stored (I, J); the pattern must be symmetric
std::vector<i64> mirror(const Bsr &A) {
    std::vector<i64> t(A.nnzb(), -1);
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 I = 0; I < A.nr; ++I)
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            const i64 J = A.col[k];
            const i32 *b0 = &A.col[A.ptr[J]], *b1 = &A.col[A.ptr[J + 1]];
            const i32 *p = std::lower_bound(b0, b1, (i32)I);
            if (p != b1 && *p == I) t[k] = A.ptr[J] + (p - b0);
        }
    return t;
}

// phase 2: each free node with strong neighbours joins the phase-1 aggregate
// (snapshot) of its strongest aggregated neighbour; relative ties within
// TIE_RTOL go to the smaller aggregate id
void attach_rest(const Bsr &A, const std::vector<uint8_t> &strong, const std::vector<double> &s, std::vector<i32> &agg) {
    const std::vector<i32> snap = agg;
    for (i64 I = 0; I < A.nr; ++I) {
        if (snap[I] >= 0) continue;
        bool has = false;
        double best_s = -1.0;
        i32 best_a = -1;
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            if (!strong[k]) continue;
            has = true;
            const i32 a = snap[A.col[k]];
            if (a < 0) continue;
            const double sj = s[k];
            if (best_a < 0 || sj > best_s * (1.0 + TIE_RTOL)) {
                best_s = sj;
                best_a = a;
            } else if (sj >= best_s * (1.0 - TIE_RTOL) && a < best_a) {
                best_s = sj;
                best_a = a;
            }
        }
        if (has) agg[I] = best_a;  // -1 only if no neighbour is aggregated (cannot happen)
    }
}

// returns n_agg; strong[k] = the strong-graph flag used for the neighbour lists
i32 aggregate(const Bsr &A, double theta, int rule, uint64_t seed, const std::vector<double> &s,
              std::vector<uint8_t> &strong, std::vector<i32> &agg) {
    const i64 n = A.nr;
    strong.assign(A.nnzb(), 0);
    agg.assign(n, -1);
    if (rule == 0) {
        for (i64 I = 0; I < n; ++I)
            for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) strong[k] = A.col[k] != I && s[k] >= theta;
    } else {
        // symmetric strong graph: strong if s_IJ >= theta or s_JI >= theta
        const std::vector<i64> t = mirror(A);
        for (i64 I = 0; I < n; ++I)
            for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
                if (t[k] < 0) return -1;  // pattern not symmetric
                strong[k] = A.col[k] != I && (s[k] >= theta || s[t[k]] >= theta);
            }
    }
    auto free_nbhd = [&](i64 I) {
        bool any = false;
        if (agg[I] >= 0) return false;
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
            if (strong[k]) {
                any = true;
                if (agg[A.col[k]] >= 0) return false;
            }
        return any;
    };
    i32 n_agg = 0;
    if (rule == 0) {
        // phase 1 in node order, ids in creation order
        for (i64 I = 0; I < n; ++I)
            if (free_nbhd(I)) {
                agg[I] = n_agg;
                for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
                    if (strong[k]) agg[A.col[k]] = n_agg;
                ++n_agg;
            }
    } else {
        // phase 1 visiting nodes by descending key (splitmix64(seed ^ I) >> 33, I)
        std::vector<i64> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::vector<uint64_t> pr(n);
        for (i64 I = 0; I < n; ++I) pr[I] = splitmix64(seed ^ (uint64_t)I) >> 33;
        std::sort(order.begin(), order.end(), [&](i64 a, i64 b) { return pr[a] != pr[b] ? pr[a] > pr[b] : a > b; });
        std::vector<i64> roots;
        for (i64 I : order)
            if (free_nbhd(I)) {
                agg[I] = 0;  // mark; numbered below
                for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
                    if (strong[k]) agg[A.col[k]] = 0;
                roots.push_back(I);
            }
        // aggregates numbered by ascending root
        std::sort(roots.begin(), roots.end());
        std::fill(agg.begin(), agg.end(), -1);
        for (i64 r : roots) {
            agg[r] = n_agg;
            for (i64 k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
                if (strong[k]) agg[A.col[k]] = n_agg;
            ++n_agg;
        }
    }
    attach_rest(A, strong, s, agg);
    return n_agg;
}

// thin Householder QR of an m x 6 matrix (m >= 6), then signs so diag(R) > 0.
// Q: m x 6, R: 6 x 6 (row-major)
void qr6(int m, const double *B, double *Q, double *R) {
    std::vector<double> a(B, B + (size_t)m * 6);
    std::vector<double> v((size_t)6 * m, 0.0);
    double beta[6];
    for (int j = 0; j < 6; ++j) {
        double nx = 0.0;
        for (int i = j; i < m; ++i) nx += a[(size_t)i * 6 + j] * a[(size_t)i * 6 + j];
        nx = std::sqrt(nx);
        double *vj = &v[(size_t)j * m];
        for (int i = 0; i < m; ++i) vj[i] = 0.0;
        if (nx == 0.0) {
            beta[j] = 0.0;
            continue;
        }
        const double x0 = a[(size_t)j * 6 + j];
        const double alpha = x0 >= 0 ? -nx : nx;
        for (int i = j; i < m; ++i) vj[i] = a[(size_t)i * 6 + j];
        vj[j] = x0 - alpha;
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += vj[i] * vj[i];
        beta[j] = vv > 0 ? 2.0 / vv : 0.0;
        for (int c = j; c < 6; ++c) {
            double t = 0.0;
            for (int i = j; i < m; ++i) t += vj[i] * a[(size_t)i * 6 + c];
            t *= beta[j];
            for (int i = j; i < m; ++i) a[(size_t)i * 6 + c] -= t * vj[i];
        }
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) R[i * 6 + j] = j >= i ? a[(size_t)i * 6 + j] : 0.0;
    // Q = H0 H1 ... H5 applied to the first six unit columns
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 6; ++j) Q[(size_t)i * 6 + j] = i == j ? 1.0 : 0.0;
    for (int j = 5; j >= 0; --j) {
        const double *vj = &v[(size_t)j * m];
        for (int c = 0; c < 6; ++c) {
            double t = 0.0;
            for (int i = j; i < m; ++i) t += vj[i] * Q[(size_t)i * 6 + c];
            t *= beta[j];
            for (int i = j; i < m; ++i) Q[(size_t)i * 6 + c] -= t * vj[i];
        }
    }
    for (int k = 0; k < 6; ++k)
        if (R[k * 6 + k] < 0) {
            for (int j = 0; j < 6; ++j) R[k * 6 + j] = -R[k * 6 + j];
            for (int i = 0; i < m; ++i) Q[(size_t)i * 6 + k] = -Q[(size_t)i * 6 + k];
        }
}

bool rank_ok(int m, const double *R) {
    if (m < 6) return false;
    double mn = INFINITY, mx = 0.0;
    for (int k = 0; k < 6; ++k) {
        mn = std::min(mn, std::fabs(R[k * 6 + k]));
        mx = std::max(mx, std::fabs(R[k * 6 + k]));
    }
    return mx > 0 && mn >= RANK_RTOL * mx;
}

// Tentative prolongator (block rows of P_tent, one bs x 6 block per aggregated
// node) and the coarse near-nullspace; a rank-deficient aggregate merges into
// the neighbour aggregate of largest summed strength (ties: smaller id).
// Returns the compact number of aggregates or -1 (rank error).
i32 tentative(const Bsr &A, int bs, const std::vector<double> &Bn, const std::vector<double> &s, std::vector<i32> &agg,
              i32 n_agg, std::vector<double> &Qn, std::vector<double> &Bc) {
    const i64 n = A.nr;
    std::vector<std::vector<i64>> mem(n_agg);
    for (i64 I = 0; I < n; ++I)
        if (agg[I] >= 0) mem[agg[I]].push_back(I);
    auto Bj_of = [&](const std::vector<i64> &nodes, std::vector<double> &M) {
        M.assign(nodes.size() * bs * 6, 0.0);
        for (size_t q = 0; q < nodes.size(); ++q)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < 6; ++c) M[(q * bs + r) * 6 + c] = Bn[((size_t)nodes[q] * bs + r) * 6 + c];
    };
    i32 a_id = 0;
    std::vector<double> M, Q, R(36);
    while (a_id < n_agg) {
        std::vector<i64> &nodes = mem[a_id];
        if (nodes.empty()) {
            ++a_id;
            continue;
        }
        const int m = (int)nodes.size() * bs;
        bool ok = false;
        if (m >= 6) {
            Bj_of(nodes, M);
            Q.assign((size_t)m * 6, 0.0);
            qr6(m, M.data(), Q.data(), R.data());
            ok = rank_ok(m, R.data());
        }
        if (ok) {
            ++a_id;
            continue;
        }
        std::map<i32, double> score;
        for (i64 I : nodes)
            for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
                if (A.col[k] == I) continue;
                const i32 t = agg[A.col[k]];
                if (t >= 0 && t != a_id) score[t] += s[k];
            }
        if (score.empty()) return -1;
        i32 best = -1;
        double bs_ = -1.0;
        for (auto &kv : score)
            if (kv.second > bs_) {  // map order: ascending id, so ties keep the smaller id
                bs_ = kv.second;
                best = kv.first;
            }
        for (i64 I : nodes) agg[I] = best;
        std::vector<i64> merged = mem[best];
        merged.insert(merged.end(), nodes.begin(), nodes.end());
        std::sort(merged.begin(), merged.end());
        mem[best] = merged;
        nodes.clear();
        a_id = best < a_id ? best : a_id + 1;
    }
    std::vector<i32> newid(n_agg, -1);
    i32 nc = 0;
    for (i32 a = 0; a < n_agg; ++a)
        if (!mem[a].empty()) newid[a] = nc++;
    for (i64 I = 0; I < n; ++I) agg[I] = agg[I] >= 0 ? newid[agg[I]] : -1;
    Qn.assign((size_t)n * bs * 6, 0.0);
    Bc.assign((size_t)nc * 36, 0.0);
    std::vector<i32> live;
    for (i32 a = 0; a < n_agg; ++a)
        if (!mem[a].empty()) live.push_back(a);
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 J = 0; J < (i64)live.size(); ++J) {
        const std::vector<i64> &nodes = mem[live[J]];
        const int m = (int)nodes.size() * bs;
        std::vector<double> Mj((size_t)m * 6), Qj((size_t)m * 6), Rj(36);
        for (size_t q = 0; q < nodes.size(); ++q)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < 6; ++c) Mj[(q * bs + r) * 6 + c] = Bn[((size_t)nodes[q] * bs + r) * 6 + c];
        qr6(m, Mj.data(), Qj.data(), Rj.data());
        for (size_t q = 0; q < nodes.size(); ++q)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < 6; ++c) Qn[((size_t)nodes[q] * bs + r) * 6 + c] = Qj[(q * bs + r) * 6 + c];
        std::copy(Rj.begin(), Rj.end(), Bc.begin() + J * 36);
    }
    return nc;
}

// largest eigenvalue of the symmetric tridiagonal (a, b) by bisection on the
// Sturm count (number of eigenvalues below x)
double tridiag_max(const std::vector<double> &a, const std::vector<double> &b) {
    const int n = (int)a.size();
    if (n == 1) return a[0];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < n; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 400 && hi - lo > 2.0 * 2.220446049250313e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (below(mid) >= n) hi = mid;  // all eigenvalues below mid
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

double lanczos_max(const Bsr &A, const std::vector<double> &D, int steps, uint64_t seed) {
    const i64 n = A.nr * A.br;
    std::vector<double> dh(n), v(n), vp(n, 0.0), w(n), t(n);
    for (i64 i = 0; i < n; ++i) dh[i] = 1.0 / std::sqrt(D[i]);
    for (i64 i = 0; i < n; ++i) v[i] = (double)(splitmix64(seed ^ (uint64_t)i) >> 11) * 0x1.0p-53 - 0.5;
    const double nv = nrm2(v.data(), n);
    for (i64 i = 0; i < n; ++i) v[i] /= nv;
    double beta_prev = 0.0;
    std::vector<double> al, be;
    for (int j = 0; j < steps; ++j) {
        for (i64 i = 0; i < n; ++i) t[i] = dh[i] * v[i];
        spmv(A, t.data(), w.data());
        for (i64 i = 0; i < n; ++i) w[i] = dh[i] * w[i] - beta_prev * vp[i];
        const double a = dot(w.data(), v.data(), n);
        for (i64 i = 0; i < n; ++i) w[i] = w[i] - a * v[i];
        const double b = nrm2(w.data(), n);
        al.push_back(a);
        if (j == steps - 1 || b <= 1e-12 * (std::fabs(a) + beta_prev)) break;
        be.push_back(b);
        for (i64 i = 0; i < n; ++i) {
            vp[i] = v[i];
            v[i] = w[i] / b;
        }
        beta_prev = b;
    }
    be.resize(al.size() - 1);
    return tridiag_max(al, be);
}

// A P for block operators (A: bs x bs, P: bs x 6): Gustavson row by row
Bsr block_product(const Bsr &A, const Bsr &B) {
    Bsr C;
    C.br = A.br;
    C.bc = B.bc;
    C.nr = A.nr;
    C.nc = B.nc;
    C.ptr.assign(A.nr + 1, 0);
    const int ar = A.br, ac = A.bc, bcc = B.bc;
    std::vector<std::vector<i32>> cols(A.nr);
#pragma omp parallel
    {
        std::vector<i32> mark(B.nc, -1);
#pragma omp for schedule(dynamic, 256)
        for (i64 I = 0; I < A.nr; ++I) {
            std::vector<i32> &c = cols[I];
            for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
                const i64 J = A.col[k];
                for (i64 q = B.ptr[J]; q < B.ptr[J + 1]; ++q)
                    if (mark[B.col[q]] != (i32)I) {
                        mark[B.col[q]] = (i32)I;
                        c.push_back(B.col[q]);
                    }
            }
            std::sort(c.begin(), c.end());
        }
    }
    for (i64 I = 0; I < A.nr; ++I) C.ptr[I + 1] = C.ptr[I] + (i64)cols[I].size();
    C.col.resize(C.ptr[A.nr]);
    C.val.assign((size_t)C.ptr[A.nr] * ar * bcc, 0.0);
#pragma omp parallel for schedule(dynamic, 256)
    for (i64 I = 0; I < A.nr; ++I) {
        std::copy(cols[I].begin(), cols[I].end(), C.col.begin() + C.ptr[I]);
        const i32 *cc = &C.col[C.ptr[I]];
        const i64 cn = C.ptr[I + 1] - C.ptr[I];
        std::vector<i32>().swap(cols[I]);
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k) {
            const i64 J = A.col[k];
            const double *a = &A.val[(size_t)k * ar * ac];
            for (i64 q = B.ptr[J]; q < B.ptr[J + 1]; ++q) {
                const i64 pos = std::lower_bound(cc, cc + cn, B.col[q]) - cc;
                double *out = &C.val[(size_t)(C.ptr[I] + pos) * ar * bcc];
                const double *bq = &B.val[(size_t)q * ac * bcc];
                for (int i = 0; i < ar; ++i)
                    for (int j = 0; j < bcc; ++j) {
                        double s = 0.0;
                        for (int l = 0; l < ac; ++l) s += a[i * ac + l] * bq[l * bcc + j];
                        out[i * bcc + j] += s;
                    }
            }
        }
    }
    return C;
}

// explicit transpose of a block operator
Bsr transpose(const Bsr &P) {
    Bsr R;
    R.br = P.bc;
    R.bc = P.br;
    R.nr = P.nc;
    R.nc = P.nr;
    R.ptr.assign(R.nr + 1, 0);
    for (i64 k = 0; k < P.nnzb(); ++k) R.ptr[P.col[k] + 1]++;
    for (i64 i = 0; i < R.nr; ++i) R.ptr[i + 1] += R.ptr[i];
    R.col.resize(P.nnzb());
    R.val.resize(P.val.size());
    std::vector<i64> fill(R.ptr.begin(), R.ptr.end() - 1);
    const int e = P.bsz();
    for (i64 I = 0; I < P.nr; ++I)
        for (i64 k = P.ptr[I]; k < P.ptr[I + 1]; ++k) {
            const i64 dst = fill[P.col[k]]++;
            R.col[dst] = (i32)I;
            for (int i = 0; i < P.br; ++i)
                for (int j = 0; j < P.bc; ++j) R.val[(size_t)dst * e + j * P.br + i] = P.val[(size_t)k * e + i * P.bc + j];
        }
    return R;
}

// dense Cholesky (lower) of (A + A^T)/2; false if a pivot is <= 0
bool dense_cholesky(const Bsr &A, std::vector<double> &L, i64 &nd) {
    nd = A.nr * A.br;
    std::vector<double> M((size_t)nd * nd, 0.0);
    const int e = A.bsz();
    for (i64 I = 0; I < A.nr; ++I)
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
            for (int i = 0; i < A.br; ++i)
                for (int j = 0; j < A.bc; ++j)
                    M[(size_t)(I * A.br + i) * nd + (i64)A.col[k] * A.bc + j] = A.val[(size_t)k * e + i * A.bc + j];
    L.assign((size_t)nd * nd, 0.0);
    for (i64 i = 0; i < nd; ++i)
        for (i64 j = 0; j <= i; ++j) L[(size_t)i * nd + j] = 0.5 * (M[(size_t)i * nd + j] + M[(size_t)j * nd + i]);
    for (i64 j = 0; j < nd; ++j) {
        double d = L[(size_t)j * nd + j];
        for (i64 k = 0; k < j; ++k) d -= L[(size_t)j * nd + k] * L[(size_t)j * nd + k];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        L[(size_t)j * nd + j] = d;
#pragma omp parallel for schedule(static)
        for (i64 i = j + 1; i < nd; ++i) {
            double s = L[(size_t)i * nd + j];
            for (i64 k = 0; k < j; ++k) s -= L[(size_t)i * nd + k] * L[(size_t)j * nd + k];
            L[(size_t)i * nd + j] = s / d;
        }
    }
    for (i64 i = 0; i < nd; ++i)
        for (i64 j = i + 1; j < nd; ++j) L[(size_t)i * nd + j] = 0.0;
    return true;
}

void cholesky_solve(const Level &c, const double *g, double *x) {
    const i64 n = c.nd;
    std::vector<double> y(n);
    for (i64 i = 0; i < n; ++i) {
        double s = g[i];
        for (i64 k = 0; k < i; ++k) s -= c.L[(size_t)i * n + k] * y[k];
        y[i] = s / c.L[(size_t)i * n + i];
    }
    for (i64 i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (i64 k = i + 1; k < n; ++k) s -= c.L[(size_t)k * n + i] * x[k];
        x[i] = s / c.L[(size_t)i * n + i];
    }
}

// rigid-body modes [N][3][6] about the node centroid, zero at constrained DOFs
std::vector<double> rigid_body_modes(const Problem &P) {
    const i64 n = P.n;
    double c[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (i64 i = 0; i < n; ++i) s += P.coords[i * 3 + d];
        c[d] = s / (double)n;
    }
    std::vector<double> B((size_t)n * 18, 0.0);
    for (i64 i = 0; i < n; ++i) {
        const double x = P.coords[i * 3] - c[0], y = P.coords[i * 3 + 1] - c[1], z = P.coords[i * 3 + 2] - c[2];
        double *b = &B[(size_t)i * 18];
        b[0 * 6 + 0] = 1.0;
        b[1 * 6 + 1] = 1.0;
        b[2 * 6 + 2] = 1.0;
        b[0 * 6 + 3] = -y;
        b[1 * 6 + 3] = x;
        b[1 * 6 + 4] = -z;
        b[2 * 6 + 4] = y;
        b[0 * 6 + 5] = z;
        b[2 * 6 + 5] = -x;
        for (int r = 0; r < 3; ++r)
            if (P.mask[i * 3 + r])
                for (int q = 0; q < 6; ++q) b[r * 6 + q] = 0.0;
    }
    return B;
}

void point_diagonal(const Bsr &A, std::vector<double> &D) {
    D.assign((size_t)A.nr * A.br, 0.0);
    for (i64 I = 0; I < A.nr; ++I)
        for (i64 k = A.ptr[I]; k < A.ptr[I + 1]; ++k)
            if (A.col[k] == I)
                for (int i = 0; i < A.br; ++i) D[I * A.br + i] = A.val[(size_t)k * A.bsz() + i * A.bc + i];
}

int setup(Hier &H, const Problem &P, const std::vector<std::vector<i32>> *given) {
    auto t0 = std::chrono::steady_clock::now();
    const Opts &o = H.opt;
    H.lv.clear();
    H.lv.emplace_back();
    H.lv[0].A = P.A;
    H.lv[0].bs = 3;
    std::vector<double> Bl = rigid_body_modes(P);
    for (int l = 0; l < o.max_levels; ++l) {
        Level &L = H.lv[l];
        point_diagonal(L.A, L.D);
        const i64 ndof = L.A.nr * L.bs;
        if (ndof <= o.coarse_max || l == o.max_levels - 1) break;
        L.lam = lanczos_max(L.A, L.D, o.lanczos_steps, 0x5EED + (uint64_t)l);
        const double theta = o.theta0 * std::pow(2.0, -l);
        const std::vector<double> s = strength(L.A);
        std::vector<uint8_t> strong;
        std::vector<i32> agg;
        i32 n_agg;
        if (given && l < (int)given->size()) {
            agg = (*given)[l];
            n_agg = 0;
            for (i32 a : agg) n_agg = std::max(n_agg, a + 1);
        } else {
            n_agg = aggregate(L.A, theta, o.aggregation, MIS_SEED + (uint64_t)l, s, strong, agg);
            if (n_agg < 0) return -2;
        }
        if (n_agg == 0) break;
        std::vector<double> Qn, Bc;
        const i32 nc = tentative(L.A, L.bs, Bl, s, agg, n_agg, Qn, Bc);
        if (nc < 0) return -6;
        // P_tent: one bs x 6 block per aggregated node
        Bsr Pt;
        Pt.br = L.bs;
        Pt.bc = 6;
        Pt.nr = L.A.nr;
        Pt.nc = nc;
        Pt.ptr.assign(Pt.nr + 1, 0);
        for (i64 I = 0; I < Pt.nr; ++I) Pt.ptr[I + 1] = Pt.ptr[I] + (agg[I] >= 0 ? 1 : 0);
        Pt.col.resize(Pt.ptr[Pt.nr]);
        Pt.val.resize((size_t)Pt.ptr[Pt.nr] * L.bs * 6);
        for (i64 I = 0; I < Pt.nr; ++I)
            if (agg[I] >= 0) {
                Pt.col[Pt.ptr[I]] = agg[I];
                std::copy(&Qn[(size_t)I * L.bs * 6], &Qn[(size_t)(I + 1) * L.bs * 6], &Pt.val[(size_t)Pt.ptr[I] * L.bs * 6]);
            }
        // P = P_tent - omega D^-1 (A P_tent), on the union pattern
        Bsr AP = block_product(L.A, Pt);
        const double omega = 4.0 / (3.0 * L.lam);
        Bsr Ps = AP;  // pattern of A P_tent contains the pattern of P_tent (diagonal blocks of A)
        const int e = L.bs * 6;
#pragma omp parallel for schedule(dynamic, 1024)
        for (i64 I = 0; I < Ps.nr; ++I) {
            for (i64 k = Ps.ptr[I]; k < Ps.ptr[I + 1]; ++k)
                for (int i = 0; i < L.bs; ++i)
                    for (int j = 0; j < 6; ++j) {
                        const size_t q = (size_t)k * e + i * 6 + j;
                        Ps.val[q] = -omega * (AP.val[q] / L.D[I * L.bs + i]);
                    }
            if (agg[I] >= 0) {
                const i64 *b0 = &Ps.ptr[I];
                const i32 *c0 = &Ps.col[*b0], *c1 = &Ps.col[Ps.ptr[I + 1]];
                const i64 pos = *b0 + (std::lower_bound(c0, c1, agg[I]) - c0);
                for (int q = 0; q < e; ++q) Ps.val[(size_t)pos * e + q] += Pt.val[(size_t)Pt.ptr[I] * e + q];
            }
        }
        AP = Bsr();
        Bsr APs = block_product(L.A, Ps);
        Bsr R = transpose(Ps);
        Bsr Ac = block_product(R, APs);
        APs = Bsr();
        if ((double)(Ac.nr * 6) > o.max_coarse_ratio * (double)ndof) break;
        L.P = std::move(Ps);
        L.R = std::move(R);
        L.agg = agg;
        H.lv.emplace_back();
        Level &N = H.lv.back();
        N.A = std::move(Ac);
        N.bs = 6;
        // coarse near-nullspace: B_c = R_J stacked [n_agg][6][6]
        Bl.swap(Bc);
    }
    Level &C = H.lv.back();
    C.P = Bsr();
    C.R = Bsr();
    if (!dense_cholesky(C.A, C.L, C.nd)) return -7;
    for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
        Level &L = H.lv[l];
        if (L.lam == 0.0) L.lam = lanczos_max(L.A, L.D, o.lanczos_steps, 0x5EED + (uint64_t)l);
        const double b = o.cheb_safety * L.lam, a = b / o.cheb_ratio;
        L.theta = 0.5 * (b + a);
        L.delta = 0.5 * (b - a);
        L.sigma = L.theta / L.delta;
    }
    H.t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

// Chebyshev on D^-1 A over [b/ratio, b] (Saad Alg. 12.1), x in/out
void chebyshev(const Level &L, int degree, const double *g, double *x) {
    const i64 n = L.A.nr * L.bs;
    std::vector<double> r(n), d(n), Ad(n);
    spmv(L.A, x, r.data());
#pragma omp parallel for
    for (i64 i = 0; i < n; ++i) {
        r[i] = g[i] - r[i];
        d[i] = (r[i] / L.D[i]) / L.theta;
    }
    double rho = 1.0 / L.sigma;
    for (int k = 0; k < degree; ++k) {
#pragma omp parallel for
        for (i64 i = 0; i < n; ++i) x[i] = x[i] + d[i];
        if (k < degree - 1) {
            spmv(L.A, d.data(), Ad.data());
            const double rho_new = 1.0 / (2.0 * L.sigma - rho);
            const double c1 = rho_new * rho, c2 = 2.0 * rho_new / L.delta;
#pragma omp parallel for
            for (i64 i = 0; i < n; ++i) {
                r[i] = r[i] - Ad[i];
                d[i] = c1 * d[i] + c2 * (r[i] / L.D[i]);
            }
            rho = rho_new;
        }
    }
}

void vcycle(const Hier &H, size_t l, const double *g, double *x) {
    const Level &L = H.lv[l];
    if (l + 1 == H.lv.size()) {
        cholesky_solve(L, g, x);
        return;
    }
    const i64 n = L.A.nr * L.bs;
    const int deg = H.opt.cheb_degree;
    std::fill(x, x + n, 0.0);
    chebyshev(L, deg, g, x);
    std::vector<double> s(n);
    spmv(L.A, x, s.data());
#pragma omp parallel for
    for (i64 i = 0; i < n; ++i) s[i] = g[i] - s[i];
    const Level &N = H.lv[l + 1];
    const i64 nn = N.A.nr * N.bs;
    std::vector<double> gc(nn), xc(nn), e(n);
    spmv(L.R, s.data(), gc.data());
    vcycle(H, l + 1, gc.data(), xc.data());
    spmv(L.P, xc.data(), e.data());
#pragma omp parallel for
    for (i64 i = 0; i < n; ++i) x[i] = x[i] + e[i];
    chebyshev(L, deg, g, x);
}

struct CgOut {
    i32 iters = 0, converged = 0, code = 0;
    double relres = 0.0;
    std::vector<double> hist;
};

// PCG (Saad Alg. 9.1) with the true-residual stop; flexible beta (Notay 2000)
// when `flexible`.  code: 0 ok, 1 maxit, -4 breakdown
CgOut pcg(const Hier &H, const double *b, double *u, double rtol, int maxit, int max_replace, bool flexible) {
    const Bsr &A = H.lv[0].A;
    const i64 n = A.nr * 3;
    CgOut out;
    const double bn = nrm2(b, n);
    std::vector<double> r(n), z(n), p(n), q(n), ro(n), t(n);
    if (bn == 0.0) {
        std::fill(u, u + n, 0.0);
        out.converged = 1;
        out.hist.push_back(0.0);
        return out;
    }
    spmv(A, u, t.data());
#pragma omp parallel for
    for (i64 i = 0; i < n; ++i) r[i] = b[i] - t[i];
    out.hist.push_back(nrm2(r.data(), n) / bn);
    if (out.hist.back() <= rtol) {
        out.converged = 1;
        out.relres = out.hist.back();
        return out;
    }
    vcycle(H, 0, r.data(), z.data());
    double rz = dot(r.data(), z.data(), n);
    if (!(rz > 0)) {
        out.code = -4;
        return out;
    }
    p = z;
    int replaced = 0, it = 0;
    while (it < maxit) {
        spmv(A, p.data(), q.data());
        const double pq = dot(p.data(), q.data(), n);
        if (!(pq > 0)) {
            out.code = -4;
            return out;
        }
        const double alpha = rz / pq;
#pragma omp parallel for
        for (i64 i = 0; i < n; ++i) {
            u[i] = u[i] + alpha * p[i];
            ro[i] = r[i];
            r[i] = r[i] - alpha * q[i];
        }
        ++it;
        const double rn = nrm2(r.data(), n) / bn;
        out.hist.push_back(rn);
        if (rn <= rtol) {
            spmv(A, u, t.data());
#pragma omp parallel for
            for (i64 i = 0; i < n; ++i) t[i] = b[i] - t[i];
            const double rtn = nrm2(t.data(), n) / bn;
            if (rtn <= rtol) {
                out.iters = it;
                out.converged = 1;
                out.relres = rtn;
                return out;
            }
            if (replaced >= max_replace) {
                out.iters = it;
                out.relres = rtn;
                out.code = 1;
                return out;
            }
            ++replaced;
            r = t;
        }
        vcycle(H, 0, r.data(), z.data());
        const double rz_new = dot(r.data(), z.data(), n);
        if (!(rz_new > 0)) {
            out.code = -4;
            return out;
        }
        double beta;
        if (flexible) {
#pragma omp parallel for
            for (i64 i = 0; i < n; ++i) t[i] = r[i] - ro[i];
            beta = dot(z.data(), t.data(), n) / rz;
        } else {
            beta = rz_new / rz;
        }
#pragma omp parallel for
        for (i64 i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    spmv(A, u, t.data());
    for (i64 i = 0; i < n; ++i) t[i] = b[i] - t[i];
    out.iters = it;
    out.relres = nrm2(t.data(), n) / bn;
    out.code = 1;
    return out;
}

void set_threads(int t) {
    if (t > 0) omp_set_num_threads(t);
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (plain pointers, host memory, called through ctypes)
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
    double theta0;
    int32_t coarse_max, max_levels, lanczos_steps, cheb_degree;
    double cheb_ratio, cheb_safety, max_coarse_ratio;
    int32_t aggregation;
    int32_t threads;
} ora_opts;

int ora_max_threads(void) { return omp_get_max_threads(); }

// Assembles the Dirichlet-eliminated system (mask, u_bc, f may be NULL).
void *ora_assemble(int64_t n, int64_t nc, int32_t degree, const double *coords, const int32_t *cells, double E,
                   double nu, double alpha, double T_ref, const double *T, const double *f, const uint8_t *mask,
                   const double *u_bc, int32_t threads) {
    set_threads(threads);
    return assemble(n, nc, degree, coords, cells, E, nu, alpha, T_ref, T, f, mask, u_bc);
}

int64_t ora_sys_nnzb(void *p) { return static_cast<Problem *>(p)->A.nnzb(); }
double ora_sys_time(void *p) { return static_cast<Problem *>(p)->t_assemble; }

void ora_sys_get(void *p, int64_t *ptr, int32_t *col, double *val, double *b) {
    const Problem *P = static_cast<Problem *>(p);
    if (ptr) std::copy(P->A.ptr.begin(), P->A.ptr.end(), ptr);
    if (col) std::copy(P->A.col.begin(), P->A.col.end(), col);
    if (val) std::copy(P->A.val.begin(), P->A.val.end(), val);
    if (b) std::copy(P->b.begin(), P->b.end(), b);
}

void ora_sys_free(void *p) { delete static_cast<Problem *>(p); }

// Builds the hierarchy; agg_given: NULL or n_given host arrays (imposed maps).
// Returns 0, or -2 (asymmetric pattern), -6 (rank), -7 (coarse pivot).
int ora_setup(void *sys, const ora_opts *o, const int32_t *const *agg_given, int32_t n_given, void **out) {
    Hier *H = new Hier;
    H->opt = Opts{o->theta0, o->coarse_max, o->max_levels, o->lanczos_steps, o->cheb_degree,
                  o->cheb_ratio, o->cheb_safety, o->max_coarse_ratio, o->aggregation, o->threads};
    set_threads(o->threads);
    const Problem *P = static_cast<Problem *>(sys);
    std::vector<std::vector<i32>> given;
    if (agg_given) {
        // level sizes follow the imposed maps: level l+1 has max(map)+1 nodes
        i64 nl = P->n;
        for (int l = 0; l < n_given; ++l) {
            given.emplace_back(agg_given[l], agg_given[l] + nl);
            i32 m = -1;
            for (i64 i = 0; i < nl; ++i) m = std::max(m, agg_given[l][i]);
            nl = m + 1;
        }
    }
    const int rc = setup(*H, *P, agg_given ? &given : nullptr);
    *out = H;
    return rc;
}

void ora_hier_free(void *h) { delete static_cast<Hier *>(h); }
int32_t ora_levels(void *h) { return (int32_t) static_cast<Hier *>(h)->lv.size(); }
double ora_setup_time(void *h) { return static_cast<Hier *>(h)->t_setup; }

// sizes of level l: block rows, stored blocks of A, block size, lambda_hat,
// stored blocks of P (0 on the coarsest)
void ora_level_info(void *h, int32_t l, int64_t *nr, int64_t *nnzb, int32_t *bs, double *lam, int64_t *p_nnzb) {
    const Level &L = static_cast<Hier *>(h)->lv[l];
    *nr = L.A.nr;
    *nnzb = L.A.nnzb();
    *bs = L.bs;
    *lam = L.lam;
    *p_nnzb = L.P.nnzb();
}

// which: 0 = A_l, 1 = P_l, 2 = R_l; any output may be NULL
void ora_level_matrix(void *h, int32_t l, int32_t which, int64_t *ptr, int32_t *col, double *val, int64_t *nnzb,
                      int64_t *nr) {
    const Level &L = static_cast<Hier *>(h)->lv[l];
    const Bsr &M = which == 0 ? L.A : which == 1 ? L.P : L.R;
    if (nnzb) *nnzb = M.nnzb();
    if (nr) *nr = M.nr;
    if (ptr) std::copy(M.ptr.begin(), M.ptr.end(), ptr);
    if (col) std::copy(M.col.begin(), M.col.end(), col);
    if (val) std::copy(M.val.begin(), M.val.end(), val);
}

void ora_level_agg(void *h, int32_t l, int32_t *agg) {
    const Level &L = static_cast<Hier *>(h)->lv[l];
    std::copy(L.agg.begin(), L.agg.end(), agg);
}

// z = M^-1 r (the V-cycle from level 0)
void ora_vcycle(void *h, const double *r, double *z) { vcycle(*static_cast<Hier *>(h), 0, r, z); }

// u: in guess, out solution.  hist: host (maxit+1) or NULL.  Returns 0, 1
// (maxit / replacements exhausted), -4 (breakdown); the solve time in *t_solve.
int ora_pcg(void *h, const double *b, double *u, double rtol, int32_t maxit, int32_t max_replace, int32_t flexible,
            int32_t *iters, double *relres, double *hist, double *t_solve) {
    auto t0 = std::chrono::steady_clock::now();
    const Hier &H = *static_cast<Hier *>(h);
    set_threads(H.opt.threads);
    CgOut o = pcg(H, b, u, rtol, maxit, max_replace, flexible != 0);
    *t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *iters = o.iters;
    *relres = o.relres;
    if (hist)
        for (size_t i = 0; i < o.hist.size() && i <= (size_t)maxit; ++i) hist[i] = o.hist[i];
    return o.code;
}

}  // extern "C"
