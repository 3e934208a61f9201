// Hierarchy data structures shared by the setup and the solve.
#pragma once

#include <functional>
#include <memory>

#include "te_internal.h"

namespace te {

template <typename T>
struct Work {
    DBuf<T> g, x, r, d, d2, s;
};

struct Level {
    int index = 0;
    int bs = 3;                    // block size (3 on the mesh level, 6 below)
    int64_t n = 0;                 // block rows
    HBsr Ah;                       // pattern in natural numbering (host; values only on the coarsest level)
    int64_t p_nnzb = 0;            // stored blocks of the prolongator to the next level
    std::vector<int32_t> agg;      // aggregate of each node (natural), -1 isolated
    std::vector<int32_t> perm_h;   // storage position -> natural index
    std::vector<int32_t> iperm_h;  // natural index -> storage position
    DBuf<double> dstore;           // point diagonal in storage order (setup only)
    Sell A, P, R;                  // device operators, storage numbering
    Sell A32;                      // float32 operator in full storage when A keeps only its upper blocks
    DBuf<int32_t> perm;
    DBuf<double> dinv;
    DBuf<float> dinv32;
    double lam = 0.0;              // largest-eigenvalue estimate of D^-1 A
    double theta = 0.0, delta = 0.0;
    std::vector<double> c1, c2;    // Chebyshev step coefficients
    Work<double> w64;
    Work<float> w32;
};

// The level operator a precision runs on: float32 work uses the full-storage
// copy where the float64 operator is stored by its upper blocks.
template <typename T>
inline Sell &level_op(Level &L) {
    if constexpr (sizeof(T) == 4) return L.A32.nrows ? L.A32 : L.A;
    else return L.A;
}

// fn(lo, hi, thread) over [0, n) on the host threads, one thread per `grain`
// items at most
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t, int)> &fn, int64_t grain = 256);
int setup_impl(const te_bsr *A, const double *coords, const uint8_t *dir_mask, const amg_options *opt,
               const int32_t *const *agg_given, int n_given, amg_handle **out, hipStream_t s);

}  // namespace te

namespace te {
// Event pairs around kernel launches, one list per kernel class.
struct Prof {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev[TE_K_COUNT];
    int used[TE_K_COUNT] = {};
    void reset(bool enable, hipStream_t st) {
        on = enable;
        s = st;
        for (int c = 0; c < TE_K_COUNT; ++c) used[c] = 0;
    }
    void begin(int c) {
        if (!on) return;
        if ((int)ev[c].size() < 2 * (used[c] + 1)) {
            hipEvent_t a, b;
            TE_CHECK_HIP(hipEventCreate(&a));
            TE_CHECK_HIP(hipEventCreate(&b));
            ev[c].push_back(a);
            ev[c].push_back(b);
        }
        TE_CHECK_HIP(hipEventRecord(ev[c][2 * used[c]], s));
    }
    void end(int c) {
        if (!on) return;
        TE_CHECK_HIP(hipEventRecord(ev[c][2 * used[c] + 1], s));
        ++used[c];
    }
    ~Prof() {
        for (auto &v : ev)
            for (auto e : v) (void)hipEventDestroy(e);
    }
};
}  // namespace te

namespace te {
// Executable graphs of the preconditioner of a solve, one per (precision,
// number of right-hand sides); launch configurations are baked in, so the
// autotuner clears them.  Captured on a stream of their own (the caller's
// may be the null stream, which cannot be captured) and launched on the
// caller's.
struct GraphSet {
    std::vector<std::pair<int, hipGraphExec_t>> g;
    hipStream_t cap = nullptr;
    hipGraphExec_t find(int key) const {
        for (const auto &e : g)
            if (e.first == key) return e.second;
        return nullptr;
    }
    void clear() {
        for (auto &e : g) (void)hipGraphExecDestroy(e.second);
        g.clear();
    }
    ~GraphSet() {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
    }
};
}  // namespace te

struct amg_handle {
    amg_options opt;
    te::Prof prof;
    te::GraphSet vgraphs;
    std::vector<te::Level> L;
    te::DBuf<double> Ainv;         // coarsest level: dense inverse, storage order
    int nc = 0;
    double setup_ms = 0.0;
    // the matrix of the CG products when it is not the one the hierarchy was
    // built for (amg_set_operator): same pattern, level-0 storage order
    te::Sell Aop;
    bool has_op = false;
    uint64_t pattern_hash = 0;     // of the setup matrix's row pointers and columns
    // solve workspace (level-0 storage order, [n][3][nrhs])
    te::DBuf<double> u, r, r_old, z, p, q, t, b;
    te::DBuf<double> partials, sums;
    te::DBuf<char> scal;
    te::DBuf<int32_t> colsel;      // [64] column selector of copy_cols
    // launch shape of amg_pcg_solve_multi over a set of handles (te_autotune_multi):
    // persistent grid multiplier and work-item order (0: as given, 1: largest first)
    int multi_grid = 1, multi_order = 0;
    // block-CG workspace, allocated by the first block solve and kept:
    // Gram partials and results, the two small coefficient matrices, X/R partials
    te::DBuf<double> bgpart, bgout, bsmall, bxpart;
};

namespace te {
// The operator of the CG products (the setup matrix, or the one set by
// amg_set_operator), with the tuned launch configuration of the setup matrix.
inline Sell &cg_operator(amg_handle *h) {
    if (!h->has_op) return h->L[0].A;
    h->Aop.tune64 = h->L[0].A.tune64;
    h->Aop.tune32 = h->L[0].A.tune32;
    return h->Aop;
}
}  // namespace te
