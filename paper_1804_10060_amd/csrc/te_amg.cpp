// Smoothed-aggregation AMG setup (Sec. 2.1.3 and 5.1 of the paper; the
// method of Vanek, Mandel & Brezina 1996 with the rigid-body near-nullspace).
//
// Host part: the greedy aggregation, the tentative prolongator by
// Householder QR per aggregate and the storage order of every level.  Device
// part (te_setup_gpu.hip and te_kernels.hip): strength of connection,
// prolongator smoothing, the products A P and P^T (A P), the transpose, the
// packing into the solver layouts, the Lanczos estimate of the largest
// eigenvalue of D^-1 A and the dense inverse of the coarsest level.  Matrix values never leave the device, except those of the
// coarsest level.
//
// Readings of what the paper leaves open (strength threshold 0.08 halved per
// level, tie handling, QR sign, 20 Lanczos steps, coarse size 3000 DOF,
// Chebyshev interval) are the library defaults of amg_options.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>

#include "te_amg.h"
#include "te_setup_gpu.h"

namespace te {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_err[1024] = "";
void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }
const char *last_error() { return g_err; }

// ---------------------------------------------------------------------------
// host <-> device copies through pinned staging
// ---------------------------------------------------------------------------
static constexpr size_t kStage = (size_t)32 << 20;  // bytes per staging half
static std::mutex g_stage_mu;
static char *g_stage = nullptr;  // 2 x kStage pinned bytes, kept until the process ends

static char *stage_buffer() {
    if (!g_stage) {
        void *p = nullptr;
        TE_CHECK_HIP(hipHostMalloc(&p, 2 * kStage, hipHostMallocDefault));
        g_stage = static_cast<char *>(p);
    }
    return g_stage;
}

void copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes < ((size_t)4 << 20)) {
        TE_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        return;
    }
    std::lock_guard<std::mutex> lock(g_stage_mu);
    char *st = stage_buffer();
    const char *in = static_cast<const char *>(src);
    char *out = static_cast<char *>(dst);
    int half = 0;
    for (size_t off = 0; off < bytes; off += kStage, half ^= 1) {
        const size_t n = std::min(kStage, bytes - off);
        char *buf = st + half * kStage;
        std::memcpy(buf, in + off, n);  // overlaps the DMA of the previous chunk (other half)
        TE_CHECK_HIP(hipStreamSynchronize(s));  // that DMA is done: its half may be refilled next
        TE_CHECK_HIP(hipMemcpyAsync(out + off, buf, n, hipMemcpyHostToDevice, s));
    }
    TE_CHECK_HIP(hipStreamSynchronize(s));
}

void copy_d2h(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes < ((size_t)4 << 20)) {
        TE_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        TE_CHECK_HIP(hipStreamSynchronize(s));
        return;
    }
    std::lock_guard<std::mutex> lock(g_stage_mu);
    char *st = stage_buffer();
    const char *in = static_cast<const char *>(src);
    char *out = static_cast<char *>(dst);
    size_t prev_off = 0, prev_n = 0;
    int half = 0;
    for (size_t off = 0; off < bytes; off += kStage, half ^= 1) {
        const size_t n = std::min(kStage, bytes - off);
        TE_CHECK_HIP(hipMemcpyAsync(st + half * kStage, in + off, n, hipMemcpyDeviceToHost, s));
        if (prev_n) std::memcpy(out + prev_off, st + (half ^ 1) * kStage, prev_n);  // overlaps this DMA
        TE_CHECK_HIP(hipStreamSynchronize(s));
        prev_off = off;
        prev_n = n;
    }
    std::memcpy(out + prev_off, st + (half ^ 1) * kStage, prev_n);
}

// ---------------------------------------------------------------------------
// threads
// ---------------------------------------------------------------------------
static int g_threads = 0;
// host_threads if set, else OMP_NUM_THREADS (the process's CPU share), else
// the hardware thread count, at most 64
static int n_threads() {
    if (g_threads > 0) return g_threads;
    if (const char *e = std::getenv("OMP_NUM_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0) return std::min(v, 64);
    }
    unsigned h = std::thread::hardware_concurrency();
    return h ? (int)std::min(h, 64u) : 4;
}
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t, int)> &fn, int64_t grain) {
    int nt = (int)std::min<int64_t>(n_threads(), std::max<int64_t>(1, n / std::max<int64_t>(grain, 1)));
    if (nt <= 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([=, &fn] { fn(lo, hi, t); });
    }
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// strength and aggregation
// ---------------------------------------------------------------------------
struct Strength {
    std::vector<double> s;  // per stored block (0 on the diagonal)
};

static const double kTieRtol = 1e-9;
static const uint64_t kMisSeed = 0xA66;  // key stream of level l: kMisSeed + l
static const double kRankRtol = 1e-10;

// agg[i] = aggregate id or -1 (isolated); returns the number of aggregates
static int64_t greedy_aggregate(const HBsr &A, const Strength &S, double theta, std::vector<int32_t> &agg) {
    const int64_t n = A.nr;
    agg.assign(n, -1);
    // strong[k]: off-diagonal block k at or above the threshold
    std::vector<uint8_t> strong(A.col.size(), 0), has_strong(n, 0);
    parallel_for(n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                if (A.col[k] != i && S.s[k] >= theta) {
                    strong[k] = 1;
                    has_strong[i] = 1;
                }
    });
    int64_t na = 0;
    // phase 1 (sequential by definition): a free node whose strong neighbours
    // are all free roots a new aggregate
    for (int64_t i = 0; i < n; ++i) {
        if (!has_strong[i] || agg[i] >= 0) continue;
        bool free = true;
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1] && free; ++k)
            if (strong[k] && agg[A.col[k]] >= 0) free = false;
        if (!free) continue;
        agg[i] = (int32_t)na;
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (strong[k]) agg[A.col[k]] = (int32_t)na;
        ++na;
    }
    // phase 2 (independent per node): remaining nodes join the phase-1
    // aggregate of their strongest strong neighbour; near-equal strengths go
    // to the smaller aggregate id
    const std::vector<int32_t> snap(agg);
    std::atomic<int64_t> orphan{-1};
    parallel_for(n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) {
            if (!has_strong[i] || snap[i] >= 0) continue;
            double bs = -1.0;
            int32_t ba = -1;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                if (!strong[k]) continue;
                const int32_t a = snap[A.col[k]];
                if (a < 0) continue;
                const double sv = S.s[k];
                if (ba < 0 || sv > bs * (1.0 + kTieRtol)) {
                    bs = sv;
                    ba = a;
                } else if (sv >= bs * (1.0 - kTieRtol) && a < ba) {
                    bs = sv;
                    ba = a;
                }
            }
            if (ba < 0) orphan.store(i);
            agg[i] = ba;
        }
    });
    TE_REQUIRE(orphan.load() < 0, TE_EINVAL, "aggregation: node %lld has no aggregated strong neighbour",
               (long long)orphan.load());
    return na;
}

// ---------------------------------------------------------------------------
// Householder QR of an m x k matrix (column-major), thin Q with diag(R) > 0
// ---------------------------------------------------------------------------
static bool qr_thin(int m, int k, std::vector<double> &M /* m x k col-major in, Q out */, double *R /* k x k */) {
    if (m < k) return false;
    std::vector<double> V((size_t)m * k, 0.0), beta(k, 0.0);
    std::vector<double> W(M);
    for (int j = 0; j < k; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += W[(size_t)j * m + i] * W[(size_t)j * m + i];
        nrm = std::sqrt(nrm);
        double x0 = W[(size_t)j * m + j];
        double alpha = x0 >= 0 ? -nrm : nrm;
        double *v = &V[(size_t)j * m];
        for (int i = j; i < m; ++i) v[i] = W[(size_t)j * m + i];
        v[j] -= alpha;
        double vn = 0.0;
        for (int i = j; i < m; ++i) vn += v[i] * v[i];
        beta[j] = vn > 0 ? 2.0 / vn : 0.0;
        for (int c = j; c < k; ++c) {
            double t = 0.0;
            for (int i = j; i < m; ++i) t += v[i] * W[(size_t)c * m + i];
            t *= beta[j];
            for (int i = j; i < m; ++i) W[(size_t)c * m + i] -= t * v[i];
        }
    }
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) R[r * k + c] = (c >= r) ? W[(size_t)c * m + r] : 0.0;
    // Q = H_0 ... H_{k-1} [I_k; 0]
    for (int c = 0; c < k; ++c) {
        double *q = &M[(size_t)c * m];
        for (int i = 0; i < m; ++i) q[i] = (i == c) ? 1.0 : 0.0;
        for (int j = k - 1; j >= 0; --j) {
            const double *v = &V[(size_t)j * m];
            double t = 0.0;
            for (int i = j; i < m; ++i) t += v[i] * q[i];
            t *= beta[j];
            for (int i = j; i < m; ++i) q[i] -= t * v[i];
        }
    }
    // positive diagonal of R
    for (int r = 0; r < k; ++r)
        if (R[r * k + r] < 0) {
            for (int c = 0; c < k; ++c) R[r * k + c] = -R[r * k + c];
            for (int i = 0; i < m; ++i) M[(size_t)r * m + i] = -M[(size_t)r * m + i];
        }
    return true;
}

static bool rank_ok(const double *R, int k) {
    double mx = 0.0, mn = INFINITY;
    for (int r = 0; r < k; ++r) {
        double v = std::fabs(R[r * k + r]);
        mx = std::max(mx, v);
        mn = std::min(mn, v);
    }
    return mx > 0 && mn >= kRankRtol * mx;
}

struct Tentative {
    int64_t nc = 0;
    std::vector<int32_t> agg;   // compact ids, -1 isolated
    std::vector<double> Q;      // [n][bs][k] (zero rows for isolated nodes)
    std::vector<double> Bc;     // [nc][k][k]
};

// Nodes of an aggregate as a 'bs*|J| x k' column-major block of B.
static void gather_B(const int32_t *nodes, size_t cnt, const std::vector<double> &B, int bs, int k,
                     std::vector<double> &M) {
    const int m = (int)cnt * bs;
    M.assign((size_t)m * k, 0.0);
    for (size_t a = 0; a < cnt; ++a)
        for (int p = 0; p < bs; ++p)
            for (int c = 0; c < k; ++c) M[(size_t)c * m + a * bs + p] = B[((size_t)nodes[a] * bs + p) * k + c];
}

// strength(): the per-block strengths, fetched only if an aggregate is rank
// deficient and has to be merged
static Tentative tentative(const HBsr &A, const std::function<const Strength &()> &strength,
                           std::vector<int32_t> agg, int64_t na, const std::vector<double> &B, int bs, int k) {
    const int64_t n = A.nr;
    // members of each aggregate, ascending (counting sort by aggregate id);
    // aggregates whose membership changes by a merge get an explicit list
    std::vector<int64_t> off(na + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        if (agg[i] >= 0) ++off[agg[i] + 1];
    for (int64_t x = 0; x < na; ++x) off[x + 1] += off[x];
    std::vector<int32_t> mem(off[na]);
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            if (agg[i] >= 0) mem[fill[agg[i]]++] = (int32_t)i;
    }
    std::vector<uint8_t> changed(na, 0);
    std::vector<std::vector<int32_t>> moved(na);  // lists of the changed aggregates
    auto members = [&](int64_t x, const int32_t *&p, size_t &cnt) {
        if (changed[x]) {
            p = moved[x].data();
            cnt = moved[x].size();
        } else {
            p = mem.data() + off[x];
            cnt = (size_t)(off[x + 1] - off[x]);
        }
    };
    Tentative T;
    T.Q.assign((size_t)n * bs * k, 0.0);
    std::vector<double> Rall((size_t)na * k * k, 0.0);
    // thin QR of an aggregate's block of B: Q rows of its nodes, R; full rank?
    auto factor = [&](int64_t x, std::vector<double> &M) {
        const int32_t *nodes;
        size_t cnt;
        members(x, nodes, cnt);
        const int m = (int)cnt * bs;
        gather_B(nodes, cnt, B, bs, k, M);
        double *R = &Rall[(size_t)x * k * k];
        if (m < k || !qr_thin(m, k, M, R) || !rank_ok(R, k)) return false;
        for (size_t aa = 0; aa < cnt; ++aa)
            for (int p = 0; p < bs; ++p)
                for (int c = 0; c < k; ++c)
                    T.Q[((size_t)nodes[aa] * bs + p) * k + c] = M[(size_t)c * m + aa * bs + p];
        return true;
    };
    std::vector<uint8_t> ok(na, 0);
    parallel_for(na, [&](int64_t lo, int64_t hi, int) {
        std::vector<double> Mt;
        for (int64_t x = lo; x < hi; ++x)
            if (off[x + 1] > off[x]) ok[x] = factor(x, Mt) ? 1 : 0;
    });
    // rank-deficient aggregates merge into the neighbour aggregate with the
    // largest summed strength (ties: smaller id); a grown aggregate is
    // factored again when visited
    std::vector<double> M;
    int64_t a = 0;
    while (a < na) {
        const int32_t *nodes;
        size_t cnt;
        members(a, nodes, cnt);
        if (cnt == 0) {
            ++a;
            continue;
        }
        if (changed[a] ? factor(a, M) : ok[a] != 0) {
            ++a;
            continue;
        }
        std::vector<std::pair<int32_t, double>> score;
        const Strength &S = strength();
        for (size_t u = 0; u < cnt; ++u) {
            const int32_t i = nodes[u];
            for (int64_t kk = A.ptr[i]; kk < A.ptr[i + 1]; ++kk) {
                const int32_t c = A.col[kk];
                if (c == i) continue;
                const int32_t t = agg[c];
                if (t < 0 || t == a) continue;
                bool found = false;
                for (auto &sc : score)
                    if (sc.first == t) {
                        sc.second += S.s[kk];
                        found = true;
                        break;
                    }
                if (!found) score.push_back({t, S.s[kk]});
            }
        }
        TE_REQUIRE(!score.empty(), TE_ERANK, "aggregate %lld is rank deficient and has no neighbour", (long long)a);
        int32_t best = score[0].first;
        double bsv = score[0].second;
        for (auto &sc : score)
            if (sc.second > bsv || (sc.second == bsv && sc.first < best)) {
                best = sc.first;
                bsv = sc.second;
            }
        std::vector<int32_t> merged;
        {
            const int32_t *bn;
            size_t bc;
            members(best, bn, bc);
            merged.assign(bn, bn + bc);
        }
        merged.insert(merged.end(), nodes, nodes + cnt);
        std::sort(merged.begin(), merged.end());
        for (size_t u = 0; u < cnt; ++u) agg[nodes[u]] = best;
        moved[best] = std::move(merged);
        changed[best] = 1;
        moved[a].clear();
        changed[a] = 1;
        a = (best < a) ? best : a + 1;
    }
    std::vector<int32_t> remap(na, -1);
    for (int64_t x = 0; x < na; ++x) {
        const int32_t *nodes;
        size_t cnt;
        members(x, nodes, cnt);
        if (cnt) remap[x] = (int32_t)T.nc++;
    }
    T.agg.assign(n, -1);
    for (int64_t i = 0; i < n; ++i)
        if (agg[i] >= 0) T.agg[i] = remap[agg[i]];
    T.Bc.assign((size_t)T.nc * k * k, 0.0);
    for (int64_t x = 0; x < na; ++x)
        if (remap[x] >= 0)
            std::copy(&Rall[(size_t)x * k * k], &Rall[(size_t)(x + 1) * k * k], &T.Bc[(size_t)remap[x] * k * k]);
    return T;
}

// ---------------------------------------------------------------------------
// SELL packing
// ---------------------------------------------------------------------------
// Rows sorted by descending length inside windows of `window` rows (ties in
// natural order), so the 64 rows of a slice have nearly equal lengths while
// x stays local to the window.
std::vector<int32_t> window_sorted_order(const std::vector<int64_t> &ptr, int64_t window) {
    const int64_t n = (int64_t)ptr.size() - 1;
    std::vector<int32_t> ord(n);
    for (int64_t i = 0; i < n; ++i) ord[i] = (int32_t)i;
    const int64_t nw = (n + window - 1) / window;
    // one window is a few thousand rows of work: every thread takes windows
    parallel_for(
        nw,
        [&](int64_t lo, int64_t hi, int) {
            for (int64_t wi = lo; wi < hi; ++wi) {
                const int64_t w0 = wi * window, w1 = std::min(n, w0 + window);
                std::sort(ord.begin() + w0, ord.begin() + w1, [&](int32_t a, int32_t b) {
                    const int64_t la = ptr[a + 1] - ptr[a], lb = ptr[b + 1] - ptr[b];
                    return la != lb ? la > lb : a < b;
                });
            }
        },
        1);
    return ord;
}

// ---------------------------------------------------------------------------
// Lanczos estimate of the largest eigenvalue of D^-1/2 A D^-1/2 (device)
// ---------------------------------------------------------------------------
static double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
    const int m = (int)a.size();
    if (m == 1) return a[0];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // number of eigenvalues < x (Sturm sequence of the LDL^T pivots)
    auto count_below = [&](double x) {
        int c = 0;
        double d = a[0] - x;
        if (d < 0) ++c;
        for (int i = 1; i < m; ++i) {
            double dd = d == 0.0 ? 1e-300 : d;
            d = (a[i] - x) - b[i - 1] * b[i - 1] / dd;
            if (d < 0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        double mid = 0.5 * (lo + hi);
        if (count_below(mid) < m) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static double dev_dot(const double *x, const double *y, int64_t n, DBuf<double> &part, DBuf<double> &res,
                      hipStream_t s) {
    dot_partials(x, y, n, 1, part.p, s);
    reduce_partials(part.p, dot_nblocks(n), 1, res.p, s);
    double h = 0.0;
    TE_CHECK_HIP(hipMemcpyAsync(&h, res.p, sizeof(double), hipMemcpyDeviceToHost, s));
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return h;
}

static double lanczos_estimate(const Level &L, int steps, uint64_t seed, hipStream_t s) {
    const int64_t n = L.n * L.bs;
    DBuf<double> v(n), vp(n), w(n), t(n), dh(n), part(dot_nblocks(n) + 1), res(1);
    dev_rsqrt(L.dstore.p, dh.p, n, s);
    lanczos_start(v.p, L.perm.p, L.n, L.bs, seed, s);
    double nv = std::sqrt(dev_dot(v.p, v.p, n, part, res, s));
    scal(v.p, 1.0 / nv, n, s);
    TE_CHECK_HIP(hipMemsetAsync(vp.p, 0, n * sizeof(double), s));
    std::vector<double> al, be;
    double beta_prev = 0.0;
    for (int j = 0; j < steps; ++j) {
        scale_mul(v.p, dh.p, t.p, n, s);
        sell_apply<double>(L.A, t.p, w.p, nullptr, 0, 1, s);
        lanczos_w(w.p, dh.p, vp.p, beta_prev, n, s);
        double a = dev_dot(w.p, v.p, n, part, res, s);
        axpy<double>(w.p, v.p, -a, n, s);
        double b = std::sqrt(dev_dot(w.p, w.p, n, part, res, s));
        al.push_back(a);
        if (j == steps - 1 || b <= 1e-12 * (std::fabs(a) + beta_prev)) break;
        be.push_back(b);
        std::swap(vp.p, v.p);  // v_prev <- v
        // v <- w / b
        TE_CHECK_HIP(hipMemcpyAsync(v.p, w.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        scal(v.p, 1.0 / b, n, s);
        beta_prev = b;
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    return tridiag_max_eig(al, be);
}

// ---------------------------------------------------------------------------
// the setup
// ---------------------------------------------------------------------------

// The level's columns on the host (level 0 keeps them on the device unless a
// host step needs them; the coarse levels always have them).
static void host_cols(Level &L, const DBsr &D, hipStream_t s) {
    const int64_t nnzb = L.Ah.ptr.empty() ? 0 : L.Ah.ptr.back();
    if ((int64_t)L.Ah.col.size() != nnzb) download(L.Ah.col, D.col, (size_t)nnzb, s);
}

static int64_t host_nnzb(const HBsr &H) { return H.ptr.empty() ? 0 : H.ptr.back(); }

// Columns of a level in natural numbering: the host copy, or for a mesh level
// without one, read back from the packed lane-per-row operator (storage row r
// holds natural row perm[r], its entries in their original order, columns
// stored in the storage numbering).
static std::vector<int32_t> level_cols(const Level &L) {
    if ((int64_t)L.Ah.col.size() == host_nnzb(L.Ah)) return L.Ah.col;
    const Sell &S = L.A;
    TE_REQUIRE(S.format == FMT_SELL, TE_EINVAL, "level %d has no host pattern", L.index);
    hipStream_t s = nullptr;
    std::vector<int32_t> sc, off, rl;
    download(sc, S.col.p, S.col.n, s);
    download(off, S.slice_off.p, (size_t)S.nslices + 1, s);
    download(rl, S.rowlen.p, S.rowlen.n, s);
    std::vector<int32_t> col((size_t)host_nnzb(L.Ah));
    for (int64_t r = 0; r < S.nrows; ++r) {
        const int64_t o = L.perm_h[r], d0 = L.Ah.ptr[o], sl = r / SELL_C, ln = r % SELL_C;
        TE_REQUIRE(rl[r] == L.Ah.ptr[o + 1] - d0, TE_EHIP, "packed row %lld has the wrong length", (long long)r);
        for (int64_t k = 0; k < rl[r]; ++k) col[d0 + k] = L.perm_h[sc[(size_t)(off[sl] + k) * SELL_C + ln]];
    }
    return col;
}

// Lane-per-row SELL for operators with 3-row blocks (many short rows); one
// wave per row for 6-row blocks (coarse operators, restrictions).
static int fmt_for(int br) { return br >= 6 ? FMT_ROWWAVE : FMT_SELL; }

// Storage order, packed operator and point diagonal of a level; dnat gets
// the diagonal in natural numbering (device) for the prolongator smoothing.
static void finish_level(Level &L, const DBsr &D, const amg_options &o, DBuf<double> &dnat, hipStream_t s) {
    L.perm_h = window_sorted_order(L.Ah.ptr, 4096);
    L.iperm_h.assign(L.n, 0);
    parallel_for(L.n, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) L.iperm_h[L.perm_h[i]] = (int32_t)i;
    });
    dev_pack(L.A, D, L.Ah.ptr, L.perm_h, L.iperm_h, nullptr, o.build_fp32 != 0, s, fmt_for(L.bs),
             o.coarse_sym && L.bs == 6);
    if (L.A.sym() && o.build_fp32) {
        // the float32 V-cycle keeps full storage: its halved value stream does
        // not pay for the gathered mirror blocks
        dev_pack(L.A32, D, L.Ah.ptr, L.perm_h, L.iperm_h, nullptr, true, s, fmt_for(L.bs));
        L.A32.val.release();
        L.A.val32.release();
    }
    upload(L.perm, L.perm_h, s);
    dev_diag(D, dnat, s);
    // diagonal, its reciprocals and the positivity check in storage order on the device
    const int64_t nd = std::max<int64_t>(L.n * L.bs, 1);
    L.dstore.alloc(nd);
    L.dinv.alloc(nd);
    if (o.build_fp32) L.dinv32.alloc(nd);
    const int64_t bad = dev_diag_store(dnat.p, L.perm.p, L.n, L.bs, L.dstore.p, L.dinv.p,
                                       o.build_fp32 ? L.dinv32.p : nullptr, s);
    TE_REQUIRE(bad < 0, TE_EINVAL, "non-positive diagonal entry at level %d row %lld", L.index, (long long)bad);
}

static void set_cheb(Level &L, const amg_options &o) {
    const double b = o.cheb_safety * L.lam, a = b / o.cheb_ratio;
    L.theta = 0.5 * (b + a);
    L.delta = 0.5 * (b - a);
    const double sigma = L.theta / L.delta;
    double rho = 1.0 / sigma;
    L.c1.clear();
    L.c2.clear();
    for (int k = 0; k + 1 < o.cheb_degree; ++k) {
        double rn = 1.0 / (2.0 * sigma - rho);
        L.c1.push_back(rn * rho);
        L.c2.push_back(2.0 * rn / L.delta);
        rho = rn;
    }
}

static void alloc_work(amg_handle *h, hipStream_t) {
    const int m = h->opt.max_nrhs;
    for (auto &L : h->L) {
        const size_t n = (size_t)L.n * L.bs * m;
        L.w64.g.alloc(n);
        L.w64.x.alloc(n);
        L.w64.r.alloc(n);
        L.w64.d.alloc(n);
        L.w64.d2.alloc(n);
        L.w64.s.alloc(n);
        if (h->opt.build_fp32) {
            L.w32.g.alloc(n);
            L.w32.x.alloc(n);
            L.w32.r.alloc(n);
            L.w32.d.alloc(n);
            L.w32.d2.alloc(n);
            L.w32.s.alloc(n);
        }
    }
    const size_t n0 = (size_t)h->L[0].n * 3 * m;
    h->u.alloc(n0);
    h->r.alloc(n0);
    h->r_old.alloc(n0);
    h->z.alloc(n0);
    h->p.alloc(n0);
    h->q.alloc(n0);
    h->t.alloc(n0);
    h->b.alloc(n0);
    // partial sums of the level-0 products: at most one per slice (any launch
    // configuration) or one per 4 rows (several right-hand sides)
    int np = std::max<int>(dot_nblocks(h->L[0].n * 3), (int)(h->L[0].A.nslices + 8));
    np = std::max<int>(np, (int)((h->L[0].n + 3) / 4 + 8));
    h->partials.alloc((size_t)np * m * 2 + 64);
    h->sums.alloc(4 * 64);
    h->scal.alloc(cg_scalars_bytes());
    h->colsel.alloc(64);
}

int setup_impl(const te_bsr *A, const double *coords, const uint8_t *dir_mask, const amg_options *opt_in,
               const int32_t *const *agg_given, int n_given, amg_handle **out, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    TE_REQUIRE(A && coords && out, TE_EINVAL, "NULL argument");
    TE_REQUIRE(A->n_brows > 0 && A->row_ptr && A->col_idx && A->val, TE_EINVAL, "empty or NULL matrix");
    amg_options o;
    if (opt_in) o = *opt_in;
    else amg_options_default(&o);
    TE_REQUIRE(o.max_nrhs >= 1 && o.max_nrhs <= 64, TE_EINVAL, "max_nrhs must be in 1..64");
    TE_REQUIRE(o.cheb_degree >= 1 && o.cheb_degree <= 8, TE_EINVAL, "cheb_degree must be in 1..8");
    TE_REQUIRE(o.max_levels >= 1 && o.max_levels <= 16, TE_EINVAL, "max_levels must be in 1..16");
    TE_REQUIRE(o.lanczos_steps >= 1, TE_EINVAL, "lanczos_steps must be >= 1");
    TE_REQUIRE(o.aggregation == TE_AGG_GREEDY || o.aggregation == TE_AGG_MIS2, TE_EINVAL,
               "aggregation must be TE_AGG_GREEDY or TE_AGG_MIS2");
    g_threads = o.host_threads;
    auto h = std::make_unique<amg_handle>();
    h->opt = o;
    const int64_t n = A->n_brows;
    const bool verbose = std::getenv("TE_VERBOSE") != nullptr;
    auto note = [&](const char *what, int l, int64_t nn, int64_t nz) {
        if (!verbose) return;
        double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[te setup %7.2fs] level %d: %s (n=%lld, nnzb=%lld)\n", t, l, what, (long long)nn,
                     (long long)nz);
        std::fflush(stderr);
    };
    // level 0: the pattern on the host (aggregation, storage order), the
    // values stay in the caller's device arrays
    Level L0;
    L0.index = 0;
    L0.bs = 3;
    L0.n = n;
    L0.Ah.br = L0.Ah.bc = 3;
    L0.Ah.nr = L0.Ah.nc = n;
    download(L0.Ah.ptr, A->row_ptr, (size_t)n + 1, s);
    TE_REQUIRE(L0.Ah.ptr[0] == 0 && L0.Ah.ptr[n] == A->nnzb, TE_EINVAL, "row_ptr inconsistent with nnzb");
    for (int64_t i = 0; i < n; ++i)
        TE_REQUIRE(L0.Ah.ptr[i + 1] >= L0.Ah.ptr[i], TE_EINVAL, "row_ptr decreases at row %lld", (long long)i);
    note("row pointers checked", 0, n, A->nnzb);
    // the columns stay on the device: the host needs them only for the greedy
    // rule or a rank-deficient merge (host_cols below)
    {
        const int64_t i = dev_check_pattern(A->row_ptr, A->col_idx, n, s);
        TE_REQUIRE(i < 0, TE_EINVAL, "row %lld has a column index out of range or out of ascending order, or no diagonal block", (long long)i);
    }
    note("columns checked", 0, n, A->nnzb);
    h->pattern_hash = dev_pattern_hash(A->row_ptr, A->col_idx, n, s);
    DBsr D0;  // view of the caller's matrix
    D0.br = D0.bc = 3;
    D0.nr = D0.nc = n;
    D0.nnzb = A->nnzb;
    D0.ptr = A->row_ptr;
    D0.col = A->col_idx;
    D0.val = A->val;
    // near-nullspace of the current level on the device (level 0: the rigid-body
    // modes about the node centroid); a host copy is made only when the
    // tentative prolongator has to take the host path
    DBuf<double> dB;
    {
        double c[3];
        dev_centroid(coords, n, c, s);
        dev_rigid_body_modes(coords, dir_mask, n, c, dB, s);
    }
    note("near-nullspace", 0, n, 0);
    std::vector<double> B;
    const int k = 6;
    h->L.push_back(std::move(L0));
    DBsr owned;               // operator of the current level below the mesh level
    const DBsr *cur = &D0;    // natural-numbering operator of the current level
    DBsr Pn, Rn;              // transfers of the previous level, waiting for this level's storage order
    std::vector<int64_t> Pn_ptr, Rn_ptr;
    bool pending = false;
    for (int l = 0;; ++l) {
        Level &L = h->L[l];
        note("pack operator", l, L.n, host_nnzb(L.Ah));
        DBuf<double> dnat;
        finish_level(L, *cur, o, dnat, s);
        note("operator packed", l, L.n, host_nnzb(L.Ah));
        if (pending) {
            Level &U = h->L[l - 1];
            const auto pord = window_sorted_order(Pn_ptr, 4096);
            dev_pack(U.P, Pn, Pn_ptr, pord, L.iperm_h, &U.iperm_h, o.build_fp32 != 0, s, fmt_for(Pn.br));
            // restriction rows in this level's own storage order: contiguous output
            dev_pack(U.R, Rn, Rn_ptr, L.perm_h, U.iperm_h, nullptr, o.build_fp32 != 0, s, fmt_for(Rn.br));
            Pn.release();
            Rn.release();
            pending = false;
            note("transfer operators packed", l - 1, 0, 0);
        }
        const int64_t ndof = L.n * L.bs;
        bool coarsest = ndof <= o.coarse_max || l == o.max_levels - 1;
        if (!coarsest) {
            L.lam = lanczos_estimate(L, o.lanczos_steps, 0x5EEDull + (uint64_t)l, s);
            L.dstore.release();
            set_cheb(L, o);
            note("eigenvalue estimate", l, L.n, 0);
            const double theta = o.theta0 * std::ldexp(1.0, -l);
            const bool par = o.aggregation == TE_AGG_MIS2 && !(agg_given && l < n_given);
            Strength S;
            DBuf<double> ds;
            dev_strength(*cur, ds, s);
            if (!par) download(S.s, ds.p, (size_t)cur->nnzb, s);
            auto strength = [&]() -> const Strength & {
                if (S.s.empty() && cur->nnzb) download(S.s, ds.p, (size_t)cur->nnzb, s);
                return S;
            };
            note("strength", l, L.n, cur->nnzb);
            std::vector<int32_t> agg;
            int64_t na;
            if (agg_given && l < n_given) {
                TE_REQUIRE(agg_given[l], TE_EINVAL, "aggregate map of level %d is NULL", l);
                agg.assign(agg_given[l], agg_given[l] + L.n);
                na = 0;
                for (int32_t a : agg) {
                    TE_REQUIRE(a >= -1 && a < L.n, TE_EINVAL, "aggregate id %d out of range at level %d", a, l);
                    na = std::max<int64_t>(na, (int64_t)a + 1);
                }
            } else if (par) {
                na = dev_aggregate_mis2(*cur, ds, theta, kMisSeed + (uint64_t)l, kTieRtol, agg, s);
            } else {
                host_cols(L, *cur, s);
                na = greedy_aggregate(L.Ah, S, theta, agg);
            }
            coarsest = na == 0;
            if (!coarsest) {
                note("aggregated", l, na, 0);
                // per-aggregate QR on the device; the host path (which can merge a
                // rank-deficient aggregate into a neighbour) when that fails
                Tentative T;
                DBuf<double> dQ, dBc;
                bool on_device;
                {
                    std::vector<int64_t> off(na + 1, 0);
                    for (int64_t i = 0; i < L.n; ++i)
                        if (agg[i] >= 0) ++off[agg[i] + 1];
                    for (int64_t x = 0; x < na; ++x) off[x + 1] += off[x];
                    std::vector<int32_t> mem(off[na]);
                    std::vector<int64_t> fill(off.begin(), off.end() - 1);
                    for (int64_t i = 0; i < L.n; ++i)
                        if (agg[i] >= 0) mem[fill[agg[i]]++] = (int32_t)i;
                    on_device = dev_tentative(off, mem, dB, L.n, L.bs, kRankRtol, dQ, dBc, s);
                }
                if (on_device) {
                    T.nc = na;
                    T.agg = std::move(agg);
                } else {
                    if (B.empty()) download(B, dB.p, (size_t)L.n * L.bs * k, s);
                    host_cols(L, *cur, s);
                    T = tentative(L.Ah, strength, agg, na, B, L.bs, k);
                    upload(dQ, T.Q, s);
                    upload(dBc, T.Bc, s);
                }
                DBsr Af;  // filtered operator of the prolongator smoothing (option)
                if (o.smooth_filtered) dev_filtered(*cur, ds, theta, Af, s);
                S = Strength();
                ds.release();
                note(on_device ? "tentative prolongator (device)" : "tentative prolongator (host)", l, T.nc, 0);
                DBuf<int32_t> dagg;
                upload(dagg, T.agg, s);
                DBsr P, AP, R, Ac;
                dev_smoothed_p(o.smooth_filtered ? Af : *cur, dagg, T.nc, dQ, dnat, 4.0 / (3.0 * L.lam), P, s);
                Af.release();
                note("smoothed P", l, P.nr, P.nnzb);
                dev_mult(*cur, P, AP, s);
                note("A P", l, AP.nr, AP.nnzb);
                dev_transpose(P, R, s);
                dev_mult(R, AP, Ac, s, true);
                note("Galerkin", l, Ac.nr, Ac.nnzb);
                AP.release();
                coarsest = (double)Ac.nr * k > o.max_coarse_ratio * (double)ndof;
                if (!coarsest) {
                    L.agg = T.agg;
                    L.p_nnzb = P.nnzb;
                    Level N;
                    N.index = l + 1;
                    N.bs = k;
                    N.n = Ac.nr;
                    dev_pattern_to_host(Ac, N.Ah, s);
                    dB = std::move(dBc);
                    B.clear();
                    download(Pn_ptr, P.ptr, (size_t)P.nr + 1, s);
                    download(Rn_ptr, R.ptr, (size_t)R.nr + 1, s);
                    Pn = std::move(P);
                    Rn = std::move(R);
                    pending = true;
                    owned = std::move(Ac);  // releases this level's operator (already packed)
                    cur = &owned;
                    h->L.push_back(std::move(N));
                    continue;
                }
            }
        }
        // this level is the coarsest: its values on the host for the dense factor
        TE_REQUIRE(ndof <= 12000, TE_EINVAL, "coarsest level has %lld DOF, too many for the dense factor",
                   (long long)ndof);
        dev_to_host(*cur, L.Ah, s);
        L.dstore.release();
        break;
    }
    owned.release();
    // coarsest level: dense inverse of (A + A^T)/2 in storage order
    {
        Level &C = h->L.back();
        C.lam = 0.0;
        const int64_t nc = C.n * C.bs;
        std::vector<double> M((size_t)nc * nc, 0.0);
        const int b = C.bs;
        for (int64_t i = 0; i < C.n; ++i)
            for (int64_t kk = C.Ah.ptr[i]; kk < C.Ah.ptr[i + 1]; ++kk) {
                const int64_t j = C.Ah.col[kk];
                const int64_t si = C.iperm_h[i], sj = C.iperm_h[j];
                for (int p = 0; p < b; ++p)
                    for (int q = 0; q < b; ++q) {
                        double v = 0.5 * C.Ah.val[(size_t)kk * b * b + p * b + q];
                        M[(size_t)(si * b + p) * nc + sj * b + q] += v;
                        M[(size_t)(sj * b + q) * nc + si * b + p] += v;
                    }
            }
        dev_dense_inverse_spd(M, (int)nc, h->Ainv, s);
        h->nc = (int)nc;
    }
    note("coarse factor", (int)h->L.size() - 1, h->nc, 0);
    alloc_work(h.get(), s);
    TE_CHECK_HIP(hipStreamSynchronize(s));
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return TE_OK;
}

// Values of A_l in natural numbering from the packed operator: storage row r
// holds natural row perm[r] with its blocks in the natural order.
static void unpack_values(const Level &L, std::vector<double> &val) {
    const Sell &S = L.A;
    const int bb = S.br * S.bc;
    hipStream_t s = nullptr;
    std::vector<double> sv;
    download(sv, S.val.p, S.val.n, s);
    val.assign((size_t)host_nnzb(L.Ah) * bb, 0.0);
    if (S.format == FMT_ROWWAVE && S.sym()) {
        // blocks on/above the diagonal in the row's natural order, the others
        // as the transposes of their mirrors, in the same order
        std::vector<int64_t> rptr, lptr;
        std::vector<int32_t> lidx;
        download(rptr, S.rptr.p, (size_t)S.nrows + 1, s);
        download(lptr, S.lptr.p, (size_t)S.nrows + 1, s);
        download(lidx, S.lidx.p, (size_t)lptr[S.nrows], s);
        const int b = S.br;
        for (int64_t r = 0; r < S.nrows; ++r) {
            const int64_t o = L.perm_h[r];
            int64_t u = rptr[r], l = lptr[r];
            for (int64_t k = L.Ah.ptr[o]; k < L.Ah.ptr[o + 1]; ++k) {
                double *dst = &val[(size_t)k * bb];
                if (L.iperm_h[L.Ah.col[k]] >= r) {
                    std::copy(&sv[(size_t)u * bb], &sv[(size_t)(u + 1) * bb], dst);
                    ++u;
                } else {
                    const double *m = &sv[(size_t)lidx[l] * bb];
                    for (int p = 0; p < b; ++p)
                        for (int q = 0; q < b; ++q) dst[p * b + q] = m[q * b + p];
                    ++l;
                }
            }
        }
    } else if (S.format == FMT_ROWWAVE) {
        std::vector<int64_t> rptr;
        download(rptr, S.rptr.p, (size_t)S.nrows + 1, s);
        for (int64_t r = 0; r < S.nrows; ++r) {
            const int64_t o = L.perm_h[r], d0 = L.Ah.ptr[o];
            for (int64_t k = 0; k < rptr[r + 1] - rptr[r]; ++k)
                for (int x = 0; x < bb; ++x) val[(size_t)(d0 + k) * bb + x] = sv[(size_t)(rptr[r] + k) * bb + x];
        }
    } else {
        std::vector<int32_t> off;
        download(off, S.slice_off.p, (size_t)S.nslices + 1, s);
        for (int64_t r = 0; r < S.nrows; ++r) {
            const int64_t o = L.perm_h[r], d0 = L.Ah.ptr[o], len = L.Ah.ptr[o + 1] - d0;
            const int64_t sl = r / SELL_C, ln = r % SELL_C;
            for (int64_t k = 0; k < len; ++k)
                for (int x = 0; x < bb; ++x)
                    val[(size_t)(d0 + k) * bb + x] =
                        sv[(size_t)(((int64_t)off[sl] + k) * bb * SELL_C + sell_val_off<sell_vw<double>()>(x, bb, (int)ln))];
        }
    }
}

}  // namespace te

using namespace te;

extern "C" const char *te_last_error(void) { return te::last_error(); }
extern "C" int te_version(void) { return 100; }

extern "C" void amg_options_default(amg_options *o) {
    if (!o) return;
    o->theta0 = 0.08;
    o->coarse_max = 3000;
    o->max_levels = 10;
    o->lanczos_steps = 20;
    o->cheb_degree = 2;
    o->cheb_ratio = 10.0;
    o->cheb_safety = 1.1;
    o->max_coarse_ratio = 0.8;
    o->build_fp32 = 1;
    o->host_threads = 0;
    o->max_nrhs = 1;
    o->coarse_sym = 1;
    o->aggregation = TE_AGG_MIS2;
    o->smooth_filtered = 0;
}

extern "C" int amg_setup(const te_bsr *A, const double *coords, const uint8_t *dir_mask, const amg_options *opt,
                         amg_handle **out, hipStream_t stream) {
    return guarded([&] { return setup_impl(A, coords, dir_mask, opt, nullptr, 0, out, stream); });
}

extern "C" int amg_setup_with_aggregates(const te_bsr *A, const double *coords, const uint8_t *dir_mask,
                                         const amg_options *opt, const int32_t *const *agg, int32_t n_levels_given,
                                         amg_handle **out, hipStream_t stream) {
    return guarded([&] {
        TE_REQUIRE(agg || n_levels_given == 0, TE_EINVAL, "agg is NULL");
        return setup_impl(A, coords, dir_mask, opt, agg, n_levels_given, out, stream);
    });
}

// The matrix of the CG products from now on: same pattern as the setup
// matrix, new values, packed in the level-0 storage order; the hierarchy
// (level-0 smoother included) stays the one built at setup.
static int set_operator_impl(amg_handle *h, const te_bsr *A, hipStream_t s) {
    TE_REQUIRE(h, TE_EINVAL, "handle is NULL");
    if (!A) {
        h->Aop = Sell();
        h->has_op = false;
        return TE_OK;
    }
    Level &L0 = h->L[0];
    TE_REQUIRE(A->row_ptr && A->col_idx && A->val, TE_EINVAL, "NULL matrix array");
    TE_REQUIRE(A->n_brows == L0.n && A->nnzb == host_nnzb(L0.Ah), TE_EINVAL,
               "operator has %lld block rows and %lld blocks, the setup matrix %lld and %lld", (long long)A->n_brows,
               (long long)A->nnzb, (long long)L0.n, (long long)host_nnzb(L0.Ah));
    TE_REQUIRE(dev_pattern_hash(A->row_ptr, A->col_idx, A->n_brows, s) == h->pattern_hash, TE_EINVAL,
               "operator pattern differs from the setup matrix's");
    DBsr D;
    D.br = D.bc = 3;
    D.nr = D.nc = A->n_brows;
    D.nnzb = A->nnzb;
    D.ptr = A->row_ptr;
    D.col = A->col_idx;
    D.val = A->val;
    Sell S;
    dev_pack(S, D, L0.Ah.ptr, L0.perm_h, L0.iperm_h, nullptr, false, s, FMT_SELL);
    h->Aop = std::move(S);
    h->has_op = true;
    TE_CHECK_HIP(hipStreamSynchronize(s));
    return TE_OK;
}

extern "C" int amg_set_operator(amg_handle *h, const te_bsr *A, hipStream_t stream) {
    return guarded([&] { return set_operator_impl(h, A, stream); });
}

extern "C" int amg_destroy(amg_handle *h) {
    delete h;
    return TE_OK;
}

extern "C" int amg_get_info(const amg_handle *h, amg_info *info) {
    return guarded([&] {
        TE_REQUIRE(h && info, TE_EINVAL, "NULL argument");
        std::memset(info, 0, sizeof *info);
        info->n_levels = (int32_t)h->L.size();
        int64_t bytes = h->Ainv.bytes();
        for (size_t l = 0; l < h->L.size() && l < 16; ++l) {
            const Level &L = h->L[l];
            info->n_dof[l] = L.n * L.bs;
            info->nnzb[l] = host_nnzb(L.Ah);
            info->bs[l] = L.bs;
            info->lambda_hat[l] = L.lam;
            info->p_nnzb[l] = L.p_nnzb;
            bytes += L.A.bytes() + L.A32.bytes() + L.P.bytes() + L.R.bytes() + L.dinv.bytes() + L.dinv32.bytes() +
                     L.perm.bytes();
        }
        info->setup_ms = h->setup_ms;
        info->bytes_device = bytes;
        return TE_OK;
    });
}

extern "C" int amg_get_aggregates(const amg_handle *h, int32_t level, int32_t *agg_host) {
    return guarded([&] {
        TE_REQUIRE(h && agg_host, TE_EINVAL, "NULL argument");
        TE_REQUIRE(level >= 0 && level + 1 < (int)h->L.size(), TE_EINVAL, "level %d has no aggregates", level);
        std::copy(h->L[level].agg.begin(), h->L[level].agg.end(), agg_host);
        return TE_OK;
    });
}

extern "C" int amg_get_level_matrix(const amg_handle *h, int32_t level, int64_t *n_rows_out, int64_t *nnzb_out,
                                    int64_t *row_ptr, int32_t *col, double *val) {
    return guarded([&] {
        TE_REQUIRE(h && n_rows_out && nnzb_out, TE_EINVAL, "NULL argument");
        TE_REQUIRE(level >= 0 && level < (int)h->L.size(), TE_EINVAL, "bad level %d", level);
        const Level &L = h->L[level];
        const HBsr &M = L.Ah;
        *n_rows_out = M.nr;
        *nnzb_out = host_nnzb(M);
        if (row_ptr) std::copy(M.ptr.begin(), M.ptr.end(), row_ptr);
        if (col) {
            const std::vector<int32_t> c = level_cols(L);
            std::copy(c.begin(), c.end(), col);
        }
        if (val) {
            std::vector<double> v;
            unpack_values(L, v);
            std::copy(v.begin(), v.end(), val);
        }
        return TE_OK;
    });
}
