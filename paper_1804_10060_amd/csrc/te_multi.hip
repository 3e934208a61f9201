// Multi-mesh solve: many independent systems (each with its own SA-AMG
// hierarchy from amg_setup) advanced together.  Every phase of the CG
// iteration is ONE persistent launch over a queue of (mesh, level, row-tile)
// work items, so meshes of uneven size share the GPU instead of running
// small launches one after another; one whole iteration is captured once as
// a HIP graph and replayed.  Each mesh keeps its own CG recurrence, its own
// stop test (the device stops a mesh whose recurrence residual passes; the
// host then checks the true residual), so mesh i gets the standalone solve
// of its right-hand side up to the summation order of the dot products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "te_amg.h"
#include "te_multi_kernels.h"

namespace te {

namespace {

struct Phase {
    int kind = 0;            // 0 sparse product, 1 vector op, 2 dense coarse
    int br = 0, bc = 0;
    int epi = 0;             // sparse: which epilogue
    int vop = 0;             // vector op
    DBuf<char> items;
    DBuf<int64_t> tile0;
    DBuf<int32_t> mesh_of;
    int nitems = 0;
    int64_t ntiles = 0;
    const double *coef = nullptr;  // per-mesh scalar for vector ops
    int gmult = 1;                 // persistent grid: gmult x the resident workgroups
};

enum Epis { E_DOT, E_RESID, E_RESIDN, E_SET, E_ADD, E_INIT, E_STEP_LZ, E_STEP_L, E_STEP_Z, E_STEP };

template <class Item>
void upload_items(Phase &P, const std::vector<Item> &items, const std::vector<int64_t> &tiles,
                  const std::vector<int32_t> &mesh, hipStream_t s) {
    P.nitems = (int)items.size();
    std::vector<int64_t> t0(items.size() + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) t0[i + 1] = t0[i] + tiles[i];
    P.ntiles = t0.back();
    std::vector<char> raw(items.size() * sizeof(Item));
    if (!items.empty()) std::memcpy(raw.data(), items.data(), raw.size());
    upload(P.items, raw, s);
    upload(P.tile0, t0, s);
    upload(P.mesh_of, mesh, s);
}

inline int64_t tiles_of(const Sell &A) {
    const int64_t units = A.format == FMT_SELL ? A.nslices : A.nrows;
    return (units + GW - 1) / GW;
}

template <class Epi>
GItem<double, Epi> gitem(const Sell &A, const double *x, const Epi &e, int mesh) {
    GItem<double, Epi> g{};
    g.fmt = A.format;
    if (A.format == FMT_SELL) g.sv = view<double>(A, A.val.p);
    else g.rv = rview<double>(A, A.val.p);
    g.x = x;
    g.epi = e;
    g.mesh = mesh;
    return g;
}

struct MultiState {
    int n = 0;
    std::vector<amg_handle *> H;
    bool flexible = false;
    int deg = 2;
    int Lmax = 1;
    int gmult = 1;            // grid multiplier of every grouped launch
    std::vector<int> order;   // mesh order of the work items
    // device scalars
    DBuf<double> rz, pq, alpha, beta, rr, bb, tol2, sums;
    DBuf<int32_t> active, cand, flag, iters, tailmask;
    DBuf<double> partials;
    MultiScal S{};
    // phases
    Phase ap, update, dotrz, pupdate, tres, dense;
    std::vector<Phase> jac, pre, resid, restrict_, prolong, postinit, post;  // per level (and step)
    std::vector<std::vector<Phase>> pre_steps, post_steps;
};

const double *level_g(amg_handle *h, int l) { return l == 0 ? h->r.p : h->L[l].w64.g.p; }
double *level_x(amg_handle *h, int l) { return l == 0 ? h->z.p : h->L[l].w64.x.p; }

template <int BR, int BC>
void launch_sparse(const Phase &P, const int32_t *active, double *partials, hipStream_t s) {
    switch (P.epi) {
        case E_DOT: group_launch<BR, BC, EpiDot>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                 partials, s, P.gmult); break;
        case E_RESID:
            group_launch<BR, BC, EpiResid<double, false>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                          partials, s, P.gmult);
            break;
        case E_RESIDN:
            group_launch<BR, BC, EpiResid<double, true>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                         partials, s, P.gmult);
            break;
        case E_SET:
            group_launch<BR, BC, EpiSet<double>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                 partials, s, P.gmult);
            break;
        case E_ADD:
            group_launch<BR, BC, EpiAdd<double>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                 partials, s, P.gmult);
            break;
        case E_INIT:
            group_launch<BR, BC, EpiChebInit<double>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                      partials, s, P.gmult);
            break;
        case E_STEP_LZ:
            group_launch<BR, BC, EpiChebStep<double, true, true>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                                  partials, s, P.gmult);
            break;
        case E_STEP_L:
            group_launch<BR, BC, EpiChebStep<double, true, false>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                                   partials, s, P.gmult);
            break;
        case E_STEP_Z:
            group_launch<BR, BC, EpiChebStep<double, false, true>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                                   partials, s, P.gmult);
            break;
        default:
            group_launch<BR, BC, EpiChebStep<double, false, false>>(P.items.p, P.tile0.p, P.nitems, P.ntiles, active,
                                                                    partials, s, P.gmult);
    }
}

void run(const Phase &P, const int32_t *active, double *partials, hipStream_t s) {
    if (P.nitems == 0) return;
    if (P.kind == 0) {
        const int key = P.br * 10 + P.bc;
        if (key == 33) launch_sparse<3, 3>(P, active, partials, s);
        else if (key == 66) launch_sparse<6, 6>(P, active, partials, s);
        else if (key == 36) launch_sparse<3, 6>(P, active, partials, s);
        else if (key == 63) launch_sparse<6, 3>(P, active, partials, s);
        else TE_REQUIRE(false, TE_EINVAL, "unsupported block shape in a grouped phase");
    } else if (P.kind == 1) {
        const VItem *it = (const VItem *)P.items.p;
        switch (P.vop) {
            case VOP_UPDATE: group_vec_launch<VOP_UPDATE>(it, P.tile0.p, P.nitems, P.ntiles, active,
                                                          P.coef, partials, s, P.gmult); break;
            case VOP_DOTRZ: group_vec_launch<VOP_DOTRZ>(it, P.tile0.p, P.nitems, P.ntiles, active,
                                                        P.coef, partials, s, P.gmult); break;
            case VOP_PUPDATE: group_vec_launch<VOP_PUPDATE>(it, P.tile0.p, P.nitems, P.ntiles, active,
                                                            P.coef, partials, s, P.gmult); break;
            case VOP_JACOBI: group_vec_launch<VOP_JACOBI>(it, P.tile0.p, P.nitems, P.ntiles, active,
                                                          P.coef, partials, s, P.gmult); break;
            default: group_vec_launch<VOP_DOTSELF>(it, P.tile0.p, P.nitems, P.ntiles, active,
                                                   P.coef, partials, s, P.gmult);
        }
    } else {
        const unsigned g = (unsigned)std::min<int64_t>(P.ntiles, (int64_t)GROUP_GRID * P.gmult);
        hipLaunchKernelGGL(k_group_dense, dim3(g), dim3(BLK), 0, s, (const DItem *)P.items.p, P.tile0.p, P.nitems,
                           active);
        TE_CHECK_HIP(hipGetLastError());
    }
}

void reduce(const Phase &P, int nv, double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_group_reduce, dim3(P.nitems, nv), dim3(WAVE), 0, s, partials, P.tile0.p, P.mesh_of.p, nv,
                       out);
    TE_CHECK_HIP(hipGetLastError());
}

// ---- building the phase tables ---------------------------------------------
void build_phases(MultiState &M, hipStream_t s) {
    const int n = M.n;
    // CG phases on level 0
    {
        std::vector<GItem<double, EpiDot>> it;
        std::vector<int64_t> t;
        std::vector<int32_t> mo;
        std::vector<GItem<double, EpiResid<double, true>>> it2;
        std::vector<VItem> up, rz, pu;
        std::vector<int64_t> tv;
        for (int m : M.order) {
            amg_handle *h = M.H[m];
            const Sell &A = h->L[0].A;
            it.push_back(gitem(A, h->p.p, EpiDot{h->p.p, h->q.p}, m));
            it2.push_back(gitem(A, h->u.p, EpiResid<double, true>{h->b.p, h->t.p}, m));
            t.push_back(tiles_of(A));
            mo.push_back(m);
            const int64_t nv = h->L[0].n * 3;
            up.push_back(VItem{h->u.p, h->r.p, M.flexible ? h->r_old.p : nullptr, h->p.p, h->q.p, 0.0, nv, m});
            rz.push_back(VItem{h->r.p, nullptr, M.flexible ? h->r_old.p : nullptr, h->z.p, nullptr, 0.0, nv, m});
            pu.push_back(VItem{h->p.p, nullptr, nullptr, h->z.p, nullptr, 0.0, nv, m});
            tv.push_back((nv + VTILE - 1) / VTILE);
        }
        M.ap.kind = 0; M.ap.br = 3; M.ap.bc = 3; M.ap.epi = E_DOT;
        upload_items(M.ap, it, t, mo, s);
        M.tres.kind = 0; M.tres.br = 3; M.tres.bc = 3; M.tres.epi = E_RESIDN;
        upload_items(M.tres, it2, t, mo, s);
        M.update.kind = 1; M.update.vop = VOP_UPDATE; M.update.coef = M.alpha.p;
        upload_items(M.update, up, tv, mo, s);
        M.dotrz.kind = 1; M.dotrz.vop = VOP_DOTRZ;
        upload_items(M.dotrz, rz, tv, mo, s);
        M.pupdate.kind = 1; M.pupdate.vop = VOP_PUPDATE; M.pupdate.coef = M.beta.p;
        upload_items(M.pupdate, pu, tv, mo, s);
    }
    const int steps = M.deg - 1;
    M.jac.resize(M.Lmax);
    M.resid.resize(M.Lmax);
    M.restrict_.resize(M.Lmax);
    M.prolong.resize(M.Lmax);
    M.postinit.resize(M.Lmax);
    M.pre_steps.resize(M.Lmax);
    M.post_steps.resize(M.Lmax);
    for (int l = 0; l + 1 < M.Lmax; ++l) {
        std::vector<VItem> jv;
        std::vector<int64_t> jt, tr, tp, tres_;
        std::vector<int32_t> mo;
        std::vector<GItem<double, EpiResid<double, false>>> ri;
        std::vector<GItem<double, EpiSet<double>>> rs;
        std::vector<GItem<double, EpiAdd<double>>> pa;
        std::vector<GItem<double, EpiChebInit<double>>> pinit;
        std::vector<std::vector<GItem<double, EpiChebStep<double, true, true>>>> s_lz(steps);
        std::vector<std::vector<GItem<double, EpiChebStep<double, true, false>>>> s_l(steps);
        std::vector<std::vector<GItem<double, EpiChebStep<double, false, true>>>> s_z(steps);
        std::vector<std::vector<GItem<double, EpiChebStep<double, false, false>>>> s_n(steps);
        int bs = 0, rbr = 0, rbc = 0, pbr = 0, pbc = 0;
        for (int m : M.order) {
            amg_handle *h = M.H[m];
            if (l + 1 >= (int)h->L.size()) continue;
            Level &L = h->L[l];
            Level &N = h->L[l + 1];
            bs = L.bs;
            rbr = L.R.br; rbc = L.R.bc; pbr = L.P.br; pbc = L.P.bc;
            const double *g = level_g(h, l);
            double *x = level_x(h, l);
            Work<double> &W = L.w64;
            const int64_t nv = L.n * L.bs;
            jv.push_back(VItem{W.d.p, nullptr, nullptr, g, L.dinv.p, 1.0 / L.theta, nv, m});
            jt.push_back((nv + VTILE - 1) / VTILE);
            mo.push_back(m);
            ri.push_back(gitem(L.A, x, EpiResid<double, false>{g, W.s.p}, m));
            tres_.push_back(tiles_of(L.A));
            rs.push_back(gitem(L.R, W.s.p, EpiSet<double>{N.w64.g.p}, m));
            tr.push_back(tiles_of(L.R));
            pa.push_back(gitem(L.P, level_x(h, l + 1), EpiAdd<double>{x}, m));
            tp.push_back(tiles_of(L.P));
            pinit.push_back(gitem(L.A, x, EpiChebInit<double>{g, L.dinv.p, W.r.p, W.d.p, 1.0 / L.theta}, m));
            // Chebyshev steps: the d buffers alternate d -> d2 -> d ...
            for (int k = 0; k < steps; ++k) {
                const bool last = k + 1 == steps;
                double *dc = (k % 2 == 0) ? W.d.p : W.d2.p;
                double *dn = (k % 2 == 0) ? W.d2.p : W.d.p;
                const double *rin_pre = (k == 0) ? g : W.r.p;
                if (last && k == 0) s_lz[k].push_back(gitem(L.A, dc, EpiChebStep<double, true, true>{rin_pre, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
                else if (last) s_l[k].push_back(gitem(L.A, dc, EpiChebStep<double, true, false>{rin_pre, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
                else if (k == 0) s_z[k].push_back(gitem(L.A, dc, EpiChebStep<double, false, true>{rin_pre, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
                else s_n[k].push_back(gitem(L.A, dc, EpiChebStep<double, false, false>{rin_pre, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
            }
        }
        if (mo.empty()) continue;
        M.jac[l].kind = 1; M.jac[l].vop = VOP_JACOBI;
        upload_items(M.jac[l], jv, jt, mo, s);
        M.resid[l].kind = 0; M.resid[l].br = bs; M.resid[l].bc = bs; M.resid[l].epi = E_RESID;
        upload_items(M.resid[l], ri, tres_, mo, s);
        M.restrict_[l].kind = 0; M.restrict_[l].br = rbr; M.restrict_[l].bc = rbc; M.restrict_[l].epi = E_SET;
        upload_items(M.restrict_[l], rs, tr, mo, s);
        M.prolong[l].kind = 0; M.prolong[l].br = pbr; M.prolong[l].bc = pbc; M.prolong[l].epi = E_ADD;
        upload_items(M.prolong[l], pa, tp, mo, s);
        M.postinit[l].kind = 0; M.postinit[l].br = bs; M.postinit[l].bc = bs; M.postinit[l].epi = E_INIT;
        upload_items(M.postinit[l], pinit, tres_, mo, s);
        // pre-smoothing steps start from x = 0; post-smoothing steps accumulate
        M.pre_steps[l].resize(steps);
        M.post_steps[l].resize(steps);
        for (int k = 0; k < steps; ++k) {
            const bool last = k + 1 == steps;
            Phase &Pp = M.pre_steps[l][k];
            Pp.kind = 0; Pp.br = bs; Pp.bc = bs;
            if (last && k == 0) { Pp.epi = E_STEP_LZ; upload_items(Pp, s_lz[k], tres_, mo, s); }
            else if (last) { Pp.epi = E_STEP_L; upload_items(Pp, s_l[k], tres_, mo, s); }
            else if (k == 0) { Pp.epi = E_STEP_Z; upload_items(Pp, s_z[k], tres_, mo, s); }
            else { Pp.epi = E_STEP; upload_items(Pp, s_n[k], tres_, mo, s); }
            // post-smoothing: same operators, rin = r after the init, never x = 0
            std::vector<GItem<double, EpiChebStep<double, true, false>>> q_l;
            std::vector<GItem<double, EpiChebStep<double, false, false>>> q_n;
            for (int m : M.order) {
                amg_handle *h = M.H[m];
                if (l + 1 >= (int)h->L.size()) continue;
                Level &L = h->L[l];
                Work<double> &W = L.w64;
                double *x = level_x(h, l);
                double *dc = (k % 2 == 0) ? W.d.p : W.d2.p;
                double *dn = (k % 2 == 0) ? W.d2.p : W.d.p;
                if (last) q_l.push_back(gitem(L.A, dc, EpiChebStep<double, true, false>{W.r.p, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
                else q_n.push_back(gitem(L.A, dc, EpiChebStep<double, false, false>{W.r.p, dc, L.dinv.p, W.r.p, dn, x, L.c1[k], L.c2[k]}, m));
            }
            Phase &Pq = M.post_steps[l][k];
            Pq.kind = 0; Pq.br = bs; Pq.bc = bs;
            if (last) { Pq.epi = E_STEP_L; upload_items(Pq, q_l, tres_, mo, s); }
            else { Pq.epi = E_STEP; upload_items(Pq, q_n, tres_, mo, s); }
        }
    }
    // dense coarse solves, each mesh on its own coarsest level
    {
        std::vector<DItem> di;
        std::vector<int64_t> dt;
        std::vector<int32_t> mo;
        for (int m : M.order) {
            amg_handle *h = M.H[m];
            const int c = (int)h->L.size() - 1;
            di.push_back(DItem{h->Ainv.p, level_g(h, c), level_x(h, c), (int64_t)h->nc, m});
            dt.push_back(((int64_t)h->nc + WPB - 1) / WPB);
            mo.push_back(m);
        }
        M.dense.kind = 2;
        upload_items(M.dense, di, dt, mo, s);
    }
    for (Phase *P : {&M.ap, &M.update, &M.dotrz, &M.pupdate, &M.tres, &M.dense}) P->gmult = M.gmult;
    for (auto *V : {&M.jac, &M.resid, &M.restrict_, &M.prolong, &M.postinit})
        for (Phase &P : *V) P.gmult = M.gmult;
    for (auto *V : {&M.pre_steps, &M.post_steps})
        for (auto &row : *V)
            for (Phase &P : row) P.gmult = M.gmult;
}

// The work-item order of the grouped phases: the meshes as given (0), or
// largest first (1: ties by index), so the largest tiles start first.
std::vector<int> mesh_order(amg_handle *const *hs, int n, int how) {
    std::vector<int> o(n);
    for (int m = 0; m < n; ++m) o[m] = m;
    if (how == 1)
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return hs[a]->L[0].n > hs[b]->L[0].n; });
    return o;
}

// z = M^-1 r for every mesh whose flag in `mask` is set
void vcycle_all(MultiState &M, const int32_t *mask, hipStream_t s) {
    for (int l = 0; l + 1 < M.Lmax; ++l) {
        if (M.jac[l].nitems == 0) continue;
        run(M.jac[l], mask, nullptr, s);
        for (auto &P : M.pre_steps[l]) run(P, mask, nullptr, s);
        run(M.resid[l], mask, nullptr, s);
        run(M.restrict_[l], mask, nullptr, s);
    }
    run(M.dense, mask, nullptr, s);
    for (int l = M.Lmax - 2; l >= 0; --l) {
        if (M.prolong[l].nitems == 0) continue;
        run(M.prolong[l], mask, nullptr, s);
        run(M.postinit[l], mask, nullptr, s);
        for (auto &P : M.post_steps[l]) run(P, mask, nullptr, s);
    }
}

// the tail of an iteration: z = M r, beta, p = z + beta p
void tail(MultiState &M, const int32_t *mask, hipStream_t s) {
    vcycle_all(M, mask, s);
    run(M.dotrz, mask, M.partials.p, s);
    reduce(M.dotrz, 2, M.partials.p, M.sums.p, s);
    hipLaunchKernelGGL(k_multi_beta, dim3((M.n + 63) / 64), dim3(64), 0, s, M.S, mask, M.sums.p, M.n,
                       M.flexible ? 1 : 0);
    TE_CHECK_HIP(hipGetLastError());
    run(M.pupdate, mask, nullptr, s);
}

void iteration(MultiState &M, hipStream_t s) {
    run(M.ap, M.active.p, M.partials.p, s);
    reduce(M.ap, 1, M.partials.p, M.sums.p, s);
    hipLaunchKernelGGL(k_multi_alpha, dim3((M.n + 63) / 64), dim3(64), 0, s, M.S, M.sums.p, M.n);
    run(M.update, M.active.p, M.partials.p, s);
    reduce(M.update, 1, M.partials.p, M.sums.p, s);
    hipLaunchKernelGGL(k_multi_rr, dim3((M.n + 63) / 64), dim3(64), 0, s, M.S, M.sums.p, M.n);
    TE_CHECK_HIP(hipGetLastError());
    tail(M, M.active.p, s);
}

__global__ void k_set_rz(MultiScal S, const double *__restrict__ rzf, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n || !S.active[m]) return;
    const double v = rzf[2 * m];
    if (!(v > 0.0)) {
        S.flag[m] = (v != v) ? 3 : 2;
        S.active[m] = 0;
    }
    S.rz[m] = v;
}

template <class T>
void fetch_vec(std::vector<T> &h, const T *d, int n, hipStream_t s) {
    h.resize(n);
    TE_CHECK_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
}

int multi_impl(amg_handle **hs, int n, const double *const *b, double *const *u, const pcg_options *opt_in,
               pcg_report *rep, hipStream_t user) {
    TE_REQUIRE(hs && n >= 1 && b && u, TE_EINVAL, "bad argument");
    pcg_options o;
    if (opt_in) o = *opt_in;
    else pcg_options_default(&o);
    TE_REQUIRE(o.precision == TE_PREC_FP64, TE_EINVAL, "the multi-mesh solve runs in float64");
    MultiState M;
    M.n = n;
    M.H.assign(hs, hs + n);
    M.deg = hs[0]->opt.cheb_degree;
    // launch shape chosen by te_autotune_multi for this set (kept in the handles)
    M.gmult = std::max(1, hs[0]->multi_grid);
    M.order = mesh_order(hs, n, hs[0]->multi_order);
    for (int m = 0; m < n; ++m) {
        TE_REQUIRE(hs[m] && b[m] && u[m], TE_EINVAL, "NULL handle or vector %d", m);
        TE_REQUIRE(!hs[m]->has_op, TE_EINVAL, "handle %d has an operator set by amg_set_operator, which the "
                   "multi-mesh solve does not take", m);
        TE_REQUIRE(hs[m]->opt.cheb_degree == M.deg && M.deg >= 2, TE_EINVAL,
                   "all meshes need the same Chebyshev degree >= 2");
        M.Lmax = std::max<int>(M.Lmax, (int)hs[m]->L.size());
    }
    for (int m = 0; m < n; ++m)
        for (size_t l = 1; l < hs[m]->L.size(); ++l)
            TE_REQUIRE(hs[m]->L[l].bs == 6, TE_EINVAL, "unexpected coarse block size");
    // private stream and events; on every exit, errors included, the
    // caller's stream is made to wait for the private stream's work before
    // both are released
    struct StreamGuard {
        hipStream_t user, s = nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr, evj = nullptr;
        ~StreamGuard() {
            if (s && evj && hipEventRecord(evj, s) == hipSuccess) (void)hipStreamWaitEvent(user, evj, 0);
            for (hipEvent_t e : {ev0, ev1, evj})
                if (e) (void)hipEventDestroy(e);
            if (s) (void)hipStreamDestroy(s);
        }
    } sg{user};
    TE_CHECK_HIP(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
    TE_CHECK_HIP(hipEventCreate(&sg.ev0));
    TE_CHECK_HIP(hipEventCreate(&sg.ev1));
    TE_CHECK_HIP(hipEventCreateWithFlags(&sg.evj, hipEventDisableTiming));
    hipStream_t s = sg.s;
    hipEvent_t ev0 = sg.ev0, ev1 = sg.ev1, evj = sg.evj;
    TE_CHECK_HIP(hipEventRecord(evj, user));
    TE_CHECK_HIP(hipStreamWaitEvent(s, evj, 0));
    TE_CHECK_HIP(hipEventRecord(ev0, s));

    for (auto *p : {&M.rz, &M.pq, &M.alpha, &M.beta, &M.rr, &M.bb, &M.tol2}) p->alloc(n);
    M.sums.alloc(2 * n);
    for (auto *p : {&M.active, &M.cand, &M.flag, &M.iters, &M.tailmask}) {
        p->alloc(n);
        TE_CHECK_HIP(hipMemsetAsync(p->p, 0, n * sizeof(int32_t), s));
    }
    TE_CHECK_HIP(hipMemsetAsync(M.alpha.p, 0, n * sizeof(double), s));
    TE_CHECK_HIP(hipMemsetAsync(M.beta.p, 0, n * sizeof(double), s));
    M.S = MultiScal{M.rz.p, M.pq.p, M.alpha.p, M.beta.p, M.rr.p, M.bb.p, M.tol2.p,
                    M.active.p, M.cand.p, M.flag.p, M.iters.p};
    build_phases(M, s);
    int64_t maxt = 0;
    for (const Phase *P : {&M.ap, &M.update, &M.dotrz}) maxt = std::max(maxt, P->ntiles);
    M.partials.alloc(2 * maxt + 2);

    // inputs into each mesh's storage order
    for (int m = 0; m < n; ++m) {
        amg_handle *h = hs[m];
        permute_gather(b[m], h->b.p, h->L[0].perm.p, h->L[0].n, 3, 1, s);
        permute_gather(u[m], h->u.p, h->L[0].perm.p, h->L[0].n, 3, 1, s);
    }
    // |b|^2 and the initial residual
    {
        Phase bb;
        std::vector<VItem> it;
        std::vector<int64_t> t;
        std::vector<int32_t> mo;
        for (int m = 0; m < n; ++m) {
            const int64_t nv = hs[m]->L[0].n * 3;
            it.push_back(VItem{nullptr, nullptr, nullptr, hs[m]->b.p, nullptr, 0.0, nv, m});
            t.push_back((nv + VTILE - 1) / VTILE);
            mo.push_back(m);
        }
        bb.kind = 1;
        bb.vop = VOP_DOTSELF;
        upload_items(bb, it, t, mo, s);
        DBuf<double> part(2 * bb.ntiles + 2);
        run(bb, nullptr, part.p, s);
        reduce(bb, 1, part.p, M.bb.p, s);
    }
    run(M.tres, nullptr, M.partials.p, s);
    reduce(M.tres, 1, M.partials.p, M.sums.p, s);
    std::vector<double> bbh, rrh;
    fetch_vec(bbh, M.bb.p, n, s);
    fetch_vec(rrh, M.sums.p, n, s);
    TE_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> act(n, 0), conv(n, 0), replaced(n, 0);
    std::vector<double> tol2(n, o.rtol * o.rtol);
    for (int m = 0; m < n; ++m) {
        TE_REQUIRE(std::isfinite(bbh[m]) && std::isfinite(rrh[m]), TE_ENAN, "NaN/Inf in mesh %d", m);
        if (bbh[m] == 0.0) {
            conv[m] = 1;
            TE_CHECK_HIP(hipMemsetAsync(hs[m]->u.p, 0, hs[m]->L[0].n * 3 * sizeof(double), s));
        } else if (rrh[m] <= tol2[m] * bbh[m]) {
            conv[m] = 1;
        } else {
            act[m] = 1;
        }
    }
    // the residual of the initial guess is r; z = M r; p = z
    for (int m = 0; m < n; ++m)
        TE_CHECK_HIP(hipMemcpyAsync(hs[m]->r.p, hs[m]->t.p, hs[m]->L[0].n * 3 * sizeof(double),
                                    hipMemcpyDeviceToDevice, s));
    TE_CHECK_HIP(hipMemcpyAsync(M.tol2.p, tol2.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    TE_CHECK_HIP(hipMemcpyAsync(M.active.p, act.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    vcycle_all(M, M.active.p, s);
    run(M.dotrz, M.active.p, M.partials.p, s);
    reduce(M.dotrz, 2, M.partials.p, M.sums.p, s);
    hipLaunchKernelGGL(k_set_rz, dim3((n + 63) / 64), dim3(64), 0, s, M.S, M.sums.p, n);
    TE_CHECK_HIP(hipGetLastError());
    for (int m = 0; m < n; ++m)
        if (act[m])
            TE_CHECK_HIP(hipMemcpyAsync(hs[m]->p.p, hs[m]->z.p, hs[m]->L[0].n * 3 * sizeof(double),
                                        hipMemcpyDeviceToDevice, s));

    // capture one iteration and the tail (for residual replacement) as graphs
    hipGraph_t g_it = nullptr, g_tail = nullptr;
    hipGraphExec_t x_it = nullptr, x_tail = nullptr;
    TE_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    iteration(M, s);
    TE_CHECK_HIP(hipStreamEndCapture(s, &g_it));
    TE_CHECK_HIP(hipGraphInstantiate(&x_it, g_it, nullptr, nullptr, 0));
    TE_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    tail(M, M.tailmask.p, s);
    TE_CHECK_HIP(hipStreamEndCapture(s, &g_tail));
    TE_CHECK_HIP(hipGraphInstantiate(&x_tail, g_tail, nullptr, nullptr, 0));
    struct GraphGuard {
        hipGraph_t a, b;
        hipGraphExec_t c, d;
        ~GraphGuard() {
            if (c) (void)hipGraphExecDestroy(c);
            if (d) (void)hipGraphExecDestroy(d);
            if (a) (void)hipGraphDestroy(a);
            if (b) (void)hipGraphDestroy(b);
        }
    } gg{g_it, g_tail, x_it, x_tail};

    std::vector<int32_t> flags, cand, itv;
    std::vector<double> trh;
    int n_active = 0;
    for (int m = 0; m < n; ++m) n_active += act[m];
    for (int it = 0; n_active > 0 && it < o.maxit; ++it) {
        TE_CHECK_HIP(hipGraphLaunch(x_it, s));
        fetch_vec(act, M.active.p, n, s);
        fetch_vec(cand, M.cand.p, n, s);
        fetch_vec(flags, M.flag.p, n, s);
        TE_CHECK_HIP(hipStreamSynchronize(s));
        for (int m = 0; m < n; ++m) {
            TE_REQUIRE(flags[m] != 3, TE_ENAN, "NaN in the CG recurrence of mesh %d", m);
            TE_REQUIRE(flags[m] == 0, TE_EINDEF, "CG breakdown in mesh %d (%s)", m,
                       flags[m] == 1 ? "(p,Ap) <= 0" : "(r,z) <= 0");
        }
        bool any = false;
        for (int m = 0; m < n; ++m) any = any || cand[m];
        if (any) {
            // true residual of the meshes whose recurrence passed
            run(M.tres, M.cand.p, M.partials.p, s);
            reduce(M.tres, 1, M.partials.p, M.sums.p, s);
            fetch_vec(trh, M.sums.p, n, s);
            TE_CHECK_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> tm(n, 0);
            bool any_tail = false;
            for (int m = 0; m < n; ++m) {
                if (!cand[m]) continue;
                cand[m] = 0;
                if (trh[m] <= tol2[m] * bbh[m]) {
                    conv[m] = 1;
                } else if (replaced[m] < o.max_replace) {
                    ++replaced[m];
                    TE_CHECK_HIP(hipMemcpyAsync(hs[m]->r.p, hs[m]->t.p, hs[m]->L[0].n * 3 * sizeof(double),
                                                hipMemcpyDeviceToDevice, s));
                    tm[m] = 1;
                    act[m] = 1;
                    any_tail = true;
                }
            }
            TE_CHECK_HIP(hipMemcpyAsync(M.cand.p, cand.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
            if (any_tail) {
                TE_CHECK_HIP(hipMemcpyAsync(M.tailmask.p, tm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
                TE_CHECK_HIP(hipGraphLaunch(x_tail, s));
                TE_CHECK_HIP(hipMemcpyAsync(M.active.p, act.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
                TE_CHECK_HIP(hipStreamSynchronize(s));
            }
        }
        n_active = 0;
        for (int m = 0; m < n; ++m) n_active += act[m];
    }
    // final true residuals and outputs
    run(M.tres, nullptr, M.partials.p, s);
    reduce(M.tres, 1, M.partials.p, M.sums.p, s);
    for (int m = 0; m < n; ++m) permute_scatter(hs[m]->u.p, u[m], hs[m]->L[0].perm.p, hs[m]->L[0].n, 3, 1, s);
    TE_CHECK_HIP(hipEventRecord(ev1, s));
    fetch_vec(trh, M.sums.p, n, s);
    fetch_vec(itv, M.iters.p, n, s);
    TE_CHECK_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    TE_CHECK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    bool all = true;
    for (int m = 0; m < n; ++m) {
        const double rel = bbh[m] > 0 ? std::sqrt(trh[m] / bbh[m]) : 0.0;
        const int c = bbh[m] == 0.0 ? 1 : (rel <= o.rtol ? 1 : 0);
        all = all && c;
        if (rep) {
            rep[m].max_iters = itv[m];
            rep[m].time_ms = ms;
            if (rep[m].iters) rep[m].iters[0] = itv[m];
            if (rep[m].converged) rep[m].converged[0] = c;
            if (rep[m].relres_true) rep[m].relres_true[0] = rel;
        }
    }
    return all ? TE_OK : TE_ENOTCONV;
}

}  // namespace
}  // namespace te

namespace te {
namespace {
// Launch shape of the grouped phases for one set of hierarchies: the
// persistent grid (1, 2 or 4 times the resident workgroups) and the work-item
// order (meshes as given, or largest first), timed on one V-cycle of every
// mesh plus the level-0 product (median of 5 after a warm-up, HIP events),
// the best kept in every handle.  Overwrites the handles' solve workspace.
int autotune_multi_impl(amg_handle **hs, int n, char *report, int64_t len, hipStream_t s) {
    TE_REQUIRE(hs && n >= 1, TE_EINVAL, "bad argument");
    MultiState M;
    M.n = n;
    M.H.assign(hs, hs + n);
    M.deg = hs[0]->opt.cheb_degree;
    for (int m = 0; m < n; ++m) {
        TE_REQUIRE(hs[m], TE_EINVAL, "NULL handle %d", m);
        TE_REQUIRE(hs[m]->opt.cheb_degree == M.deg && M.deg >= 2, TE_EINVAL,
                   "all meshes need the same Chebyshev degree >= 2");
        M.Lmax = std::max<int>(M.Lmax, (int)hs[m]->L.size());
        for (size_t l = 1; l < hs[m]->L.size(); ++l)
            TE_REQUIRE(hs[m]->L[l].bs == 6, TE_EINVAL, "unexpected coarse block size");
    }
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    TE_CHECK_HIP(hipEventCreate(&ev.a));
    TE_CHECK_HIP(hipEventCreate(&ev.b));
    DBuf<int32_t> ones;
    upload(ones, std::vector<int32_t>(n, 1), s);
    std::string rep;
    float best_t = INFINITY, def_t = 0.f;
    int best_g = 1, best_o = 0;
    for (int how : {0, 1}) {
        for (int gm : {1, 2, 4}) {
            M.order = mesh_order(hs, n, how);
            M.gmult = gm;
            build_phases(M, s);
            DBuf<double> part(2 * M.ap.ntiles + 2);
            auto once = [&] {
                vcycle_all(M, ones.p, s);
                run(M.ap, ones.p, part.p, s);
            };
            once();
            float t[5];
            for (int r = 0; r < 5; ++r) {
                TE_CHECK_HIP(hipEventRecord(ev.a, s));
                once();
                TE_CHECK_HIP(hipEventRecord(ev.b, s));
                TE_CHECK_HIP(hipEventSynchronize(ev.b));
                TE_CHECK_HIP(hipEventElapsedTime(&t[r], ev.a, ev.b));
            }
            std::sort(t, t + 5);
            if (how == 0 && gm == 1) def_t = t[2];
            if (t[2] < best_t) {
                best_t = t[2];
                best_g = gm;
                best_o = how;
            }
        }
    }
    for (int m = 0; m < n; ++m) {
        hs[m]->multi_grid = best_g;
        hs[m]->multi_order = best_o;
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "multi-mesh %d systems: grid %dx resident, %s order: %.4f ms per V-cycle + "
                  "product (default %.4f ms)\n", n, best_g, best_o ? "largest-first" : "given", best_t, def_t);
    rep += buf;
    if (report && len > 0) std::snprintf(report, (size_t)len, "%s", rep.c_str());
    return TE_OK;
}
}  // namespace
}  // namespace te

extern "C" int te_autotune_multi(amg_handle **h, int32_t n, char *report, int64_t report_len, hipStream_t stream) {
    return te::guarded([&] { return te::autotune_multi_impl(h, n, report, report_len, stream); });
}

extern "C" int amg_pcg_solve_multi(amg_handle **h, int32_t n, const double *const *b, double *const *u,
                                   const pcg_options *opt, pcg_report *rep, hipStream_t stream) {
    return te::guarded([&] { return te::multi_impl(h, n, b, u, opt, rep, stream); });
}
