// Autotuner: picks the launch configuration of every level operator of a
// hierarchy by timing the candidates on the operator itself (median of 5
// launches after one warm-up, HIP events on the solve stream), separately
// for the float64 and float32 copies: for one right-hand side the waves per
// workgroup, slices (rows) per wave, XCD block order and non-temporal value
// loads, and for the operators stored one wave per row whether a slot's
// lanes share the x entries by lane permutes; for the hierarchy's max_nrhs right-hand sides (when above one) the
// block rows per workgroup of the multi-RHS products.  Choices can be stored
// in and re-read from a small JSON file keyed by the operator's shape class
// (and the number of right-hand sides), so a second run on a similar problem
// applies them without timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <utility>

#include "te_amg.h"

namespace te {

namespace {

std::string key_of(const Sell &A, const char *dtype) {
    const double per_row = A.nrows ? (double)A.nnzb / (double)A.nrows : 0.0;
    const int rbucket = A.nrows > 0 ? (int)std::floor(std::log2((double)A.nrows)) : 0;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s-%dx%d-%s-rows2^%d-bpr%d",
                  A.format == FMT_SELL ? "sell" : (A.sym() ? "rsym" : "roww"), A.br, A.bc, dtype, rbucket,
                  (int)std::lround(per_row));
    return buf;
}

std::map<std::string, Tune> read_cache(const char *path) {
    std::map<std::string, Tune> c;
    if (!path) return c;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // lines of the form:  "key": [wpb, spw, remap, nt, mwpb, mtile, msplit, xb]  (the last four optional)
        auto a = line.find('"'), b = line.find('"', a + 1), l = line.find('['), r = line.find(']');
        if (a == std::string::npos || b == std::string::npos || l == std::string::npos || r == std::string::npos)
            continue;
        Tune t;
        std::string nums = line.substr(l + 1, r - l - 1);
        std::replace(nums.begin(), nums.end(), ',', ' ');
        std::istringstream is(nums);
        if (is >> t.wpb >> t.spw >> t.remap >> t.nt) {
            int m = 0, mt = 0, sp = 0;
            if (is >> m && (m == 4 || m == 8 || m == 16)) t.mwpb = m;   // checked against the format at launch
            if (is >> mt && (mt == 0 || mt == 16 || mt == 32 || mt == 64)) t.mtile = mt;
            if (is >> sp) t.msplit = sp ? 1 : 0;
            int xb = 0;
            if (is >> xb) t.xb = xb ? 1 : 0;   // used by the row-wave operators only
            c[line.substr(a + 1, b - a - 1)] = t;
        }
    }
    return c;
}

void write_cache(const char *path, const std::map<std::string, Tune> &c) {
    if (!path) return;
    std::ofstream f(path);
    TE_REQUIRE(f.good(), TE_EINVAL, "cannot write the tuning cache %s", path);
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : c) {
        f << "  \"" << kv.first << "\": [" << kv.second.wpb << ", " << kv.second.spw << ", " << kv.second.remap
          << ", " << kv.second.nt << ", " << kv.second.mwpb << ", " << kv.second.mtile << ", " << kv.second.msplit
          << ", " << kv.second.xb << "]"
          << (++i < c.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

template <typename T>
float time_op(Sell &A, Tune &slot, const Tune &cand, const T *x, T *y, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
              int nrhs = 1) {
    slot = cand;
    sell_apply<T>(A, x, y, nullptr, 0, nrhs, s);  // warm-up
    float t[5];
    for (int r = 0; r < 5; ++r) {
        TE_CHECK_HIP(hipEventRecord(e0, s));
        sell_apply<T>(A, x, y, nullptr, 0, nrhs, s);
        TE_CHECK_HIP(hipEventRecord(e1, s));
        TE_CHECK_HIP(hipEventSynchronize(e1));
        TE_CHECK_HIP(hipEventElapsedTime(&t[r], e0, e1));
    }
    std::sort(t, t + 5);
    return t[2];
}

// Waves per workgroup and, on the SELL layout with more than 16 columns,
// the column tile (16, 32 or 64 columns per pass over the matrix, or 0: one
// row per wave with a lane per column) of the nrhs-column products; the
// single-RHS choice in `slot` is kept.
template <typename T>
void tune_multi(Sell &A, Tune &slot, const std::string &key, const T *x, T *y, int nrhs,
                std::map<std::string, Tune> &cache, hipStream_t s, hipEvent_t e0, hipEvent_t e1, std::string &report) {
    const Tune keep = slot;
    Tune best = keep;
    float best_t = INFINITY, def_t = 0.f;
    const bool tiles = A.format == FMT_SELL && nrhs > 16;
    const std::pair<int, int> shapes[] = {{0, 0}, {64, 0}, {32, 0}, {16, 0}, {32, 1}, {16, 1}};
    for (const auto &sh : shapes) {
        const int mt = sh.first;
        if (!tiles && (mt != keep.mtile || sh.second)) continue;
        for (int m : {4, 8, 16}) {
            if (m == 16 && A.format == FMT_SELL) continue;   // the SELL kernel takes at most 8 waves
            Tune c = keep;
            c.mwpb = m;
            c.mtile = mt;
            c.msplit = sh.second;
            const float t = time_op<T>(A, slot, c, x, y, s, e0, e1, nrhs);
            if (m == 4 && mt == keep.mtile && !sh.second) def_t = t;
            if (t < best_t) {
                best_t = t;
                best = c;
            }
        }
    }
    slot = best;
    cache[key] = slot;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s best %d waves per workgroup, tile %d%s: %.4f ms (default %.4f ms)\n",
                  key.c_str(), best.mwpb, best.mtile, best.msplit ? " over the XCDs" : "", best_t, def_t);
    report += buf;
}

template <typename T>
void tune_one(Sell &A, Tune &slot, const char *dtype, const T *x, T *y, std::map<std::string, Tune> &cache,
              bool use_cache, hipStream_t s, hipEvent_t e0, hipEvent_t e1, std::string &report, int nrhs) {
    if (A.nrows == 0) return;
    const std::string key = key_of(A, dtype);
    const std::string mkey = key + "-nrhs" + std::to_string(nrhs);
    if (use_cache) {
        auto it = cache.find(key);
        auto mt = cache.find(mkey);
        if (it != cache.end() && (nrhs == 1 || mt != cache.end())) {
            slot = it->second;
            if (nrhs > 1) {
                slot.mwpb = A.format == FMT_SELL ? std::min(mt->second.mwpb, 8) : mt->second.mwpb;
                slot.mtile = mt->second.mtile;
                slot.msplit = mt->second.msplit;
            }
            report += key + " cached\n";
            return;
        }
    }
    Tune best;
    float best_t = INFINITY, def_t = 0.f;
    // the shared x entries exist for one wave per row (blocks no wider than tall)
    const int nxb = A.format == FMT_ROWWAVE && A.bc <= A.br ? 2 : 1;
    for (int xb = 0; xb < nxb; ++xb)
        for (int wpb : {1, 2, 4, 8})
            for (int spw : {1, 2, 4})
                for (int remap : {0, 1})
                    for (int nt : {0, 1}) {
                        Tune c{wpb, spw, remap, nt};
                        c.xb = xb;
                        const float t = time_op<T>(A, slot, c, x, y, s, e0, e1);
                        if (wpb == 4 && spw == 1 && remap == 1 && nt == 0 && xb == 0) def_t = t;
                        if (t < best_t) {
                            best_t = t;
                            best = c;
                        }
                    }
    slot = best;
    cache[key] = best;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s best [%d,%d,%d,%d%s] %.4f ms (default %.4f ms)\n", key.c_str(), best.wpb,
                  best.spw, best.remap, best.nt, best.xb ? ",shared-x" : "", best_t, def_t);
    report += buf;
    if (nrhs > 1) tune_multi<T>(A, slot, mkey, x, y, nrhs, cache, s, e0, e1, report);
}

int autotune_impl(amg_handle *h, const char *cache_path, int32_t use_cache, char *report_out, int64_t report_len,
                  hipStream_t s) {
    TE_REQUIRE(h, TE_EINVAL, "NULL handle");
    h->vgraphs.clear();  // their launches use the configurations about to change
    auto cache = read_cache(use_cache ? cache_path : nullptr);
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
    std::string rep;
    const int m = h->opt.max_nrhs;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &L = h->L[l];
        const bool next = l + 1 < h->L.size();
        tune_one<double>(L.A, L.A.tune64, "f64", L.w64.d.p, L.w64.s.p, cache, use_cache, s, e0, e1, rep, m);
        if (next) {
            Level &N = h->L[l + 1];
            tune_one<double>(L.P, L.P.tune64, "f64", N.w64.x.p, L.w64.s.p, cache, use_cache, s, e0, e1, rep, m);
            tune_one<double>(L.R, L.R.tune64, "f64", L.w64.s.p, N.w64.g.p, cache, use_cache, s, e0, e1, rep, m);
        }
        if (h->opt.build_fp32) {
            tune_one<float>(level_op<float>(L), level_op<float>(L).tune32, "f32", L.w32.d.p, L.w32.s.p, cache,
                            use_cache, s, e0, e1, rep, m);
            if (next) {
                Level &N = h->L[l + 1];
                tune_one<float>(L.P, L.P.tune32, "f32", N.w32.x.p, L.w32.s.p, cache, use_cache, s, e0, e1, rep, m);
                tune_one<float>(L.R, L.R.tune32, "f32", L.w32.s.p, N.w32.g.p, cache, use_cache, s, e0, e1, rep, m);
            }
        }
    }
    // the work vectors held timing garbage: nothing reads them before writing
    if (cache_path) write_cache(cache_path, cache);
    if (report_out && report_len > 0) {
        std::snprintf(report_out, (size_t)report_len, "%s", rep.c_str());
    }
    return TE_OK;
}

}  // namespace
}  // namespace te

extern "C" int te_autotune(amg_handle *h, const char *cache_path, int32_t use_cache, char *report,
                           int64_t report_len, hipStream_t stream) {
    return te::guarded([&] { return te::autotune_impl(h, cache_path, use_cache, report, report_len, stream); });
}
