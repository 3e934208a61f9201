"""Oracle: smoothed-aggregation AMG preconditioner for 3D elasticity
(test infrastructure only; see the package docstring).

What the paper fixes (Sec. 2.1.3 and Sec. 5.1): smoothed aggregation
(Vanek, Mandel & Brezina 1996) with the six rigid-body modes as the
near-nullspace, a Chebyshev smoother whose largest eigenvalue must be
estimated well (with more Krylov steps than a library default), control of
the coarsening rate, and a comparatively large coarse grid.  Where the paper
is silent the following readings are taken (each is a parameter):

* strength:   s_IJ = |A_IJ|_F / sqrt(|A_II|_F |A_JJ|_F), strong if I != J and
              s_IJ >= theta_l, theta_l = theta_0 2^-l, theta_0 = 0.08; the
              Frobenius sums run over block entries in row-major order.
* aggregation: two phases.  The greedy rule (option "greedy") is
              sequential in node order.  Phase 1 makes a new
              aggregate of I and its strong neighbours when all of them are
              free; phase 2 attaches each remaining node to the aggregate (of
              a phase-1 snapshot) of its strongest neighbour, strengths within
              a relative 1e-9 counting as equal and then the smaller aggregate
              id winning.  Nodes with no strong neighbour (e.g. clamped) are
              isolated and left out of every aggregate.
* parallel aggregation (option "mis2", the default): the phase-1 roots
              are the maximal distance-2 independent set of the strong graph
              (made symmetric) chosen by fixed priorities in parallel rounds
              (Luby's rounds
              with fixed keys; Bell, Dalton & Olson 2012 use them for
              aggregation).  With fixed keys the rounds select exactly the
              set the sequential phase 1 selects when it visits the nodes in
              descending key order (Blelloch, Fineman & Shun 2012).  Key of
              node I on level l: (splitmix64((0xA66 + l) ^ I) >> 33, I).
              Aggregates are numbered by ascending root; phase 2 as above.
* tentative P: per aggregate (nodes ascending) the thin QR B_J = Q_J R_J with
              diag(R_J) > 0; rank deficiency (min |R_kk| < 1e-10 max |R_kk|)
              merges the aggregate into its neighbour aggregate of largest
              summed strength.
* eigenvalue: largest Ritz value of 20 Lanczos steps on D^-1/2 A D^-1/2, start
              vector from splitmix64 with seed 0x5EED + level.
* smoothing:  P = (I - omega D^-1 A) P_tent, omega = 4 / (3 lambda_hat).
              Option smooth_filtered: A replaced by A^F, the strong blocks
              (the symmetric strong graph of the MIS-2 rule) and the diagonal
              of each block row, every dropped block added to the row's
              diagonal block (so A^F acts on the translations as A does);
              D and lambda_hat stay those of A.
* Galerkin:   A_c = P^T A P, coarse block size = near-nullspace size (6).
* stop:       coarse DOF <= coarse_max (3000) or 10 levels or a coarsening
              ratio above 0.8; the coarsest level is solved by a dense
              Cholesky factor of (A + A^T)/2.
* smoother:   Chebyshev of degree 2 on D^-1 A over [b/10, b], b = 1.1 lambda_hat
              (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
              Alg. 12.1), point-Jacobi D.
* cycle:      V-cycle, pre-smooth from zero, residual, coarse correction,
              post-smooth with the same polynomial (symmetric M^-1).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .rng import splitmix64_vec, uniform01_vec

TIE_RTOL = 1e-9
RANK_RTOL = 1e-10


@dataclasses.dataclass
class AMGOptions:
    theta0: float = 0.08
    coarse_max: int = 3000
    max_levels: int = 10
    lanczos_steps: int = 20
    cheb_degree: int = 2
    cheb_ratio: float = 10.0     # a = b / cheb_ratio
    cheb_safety: float = 1.1     # b = cheb_safety * lambda_hat
    max_coarse_ratio: float = 0.8
    aggregation: str = "mis2"  # or "greedy"
    smooth_filtered: bool = False


class RankError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# Strength of connection and aggregation
# ---------------------------------------------------------------------------

def _block_fro(data):
    """Frobenius norm of each block, summing squares in row-major order."""
    flat = data.reshape(data.shape[0], -1)
    acc = np.zeros(flat.shape[0])
    for e in range(flat.shape[1]):
        acc = acc + flat[:, e] * flat[:, e]
    return np.sqrt(acc)


def strength(A: sp.bsr_matrix):
    """Per stored block: s_IJ (0 on the diagonal).  Returns (rows, cols, s)."""
    n = A.shape[0] // A.blocksize[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    fro = _block_fro(A.data)
    dnorm = np.zeros(n)
    isdiag = rows == cols
    dnorm[rows[isdiag]] = fro[isdiag]
    s = fro / np.sqrt(dnorm[rows] * dnorm[cols])
    s[isdiag] = 0.0
    return rows, cols, s


def aggregate(A: sp.bsr_matrix, theta: float):
    """Greedy aggregation.  Returns (agg[N] with -1 for isolated nodes,
    n_agg, strong-neighbour lists with strengths)."""
    n = A.shape[0] // A.blocksize[0]
    rows, cols, s = strength(A)
    strong = (s >= theta) & (rows != cols)
    ptr = A.indptr
    nbrs = []
    for i in range(n):
        sl = slice(ptr[i], ptr[i + 1])
        sel = strong[sl]
        nbrs.append((cols[sl][sel], s[sl][sel]))
    agg = np.full(n, -1, np.int64)
    n_agg = 0
    # phase 1: new aggregate of I and all its strong neighbours when all free
    for i in range(n):
        nb, _ = nbrs[i]
        if nb.size == 0 or agg[i] >= 0:
            continue
        if np.all(agg[nb] < 0):
            agg[i] = n_agg
            agg[nb] = n_agg
            n_agg += 1
    return _attach_rest(agg, nbrs), n_agg, (rows, cols, s)


def _attach_rest(agg, nbrs):
    """Phase 2: every node with strong neighbours that is not in a phase-1
    aggregate joins the phase-1 aggregate of its strongest aggregated
    neighbour (relative ties within TIE_RTOL: the smaller aggregate id)."""
    n = agg.shape[0]
    agg = agg.copy()
    snap = agg.copy()
    for i in range(n):
        nb, sv = nbrs[i]
        if nb.size == 0 or snap[i] >= 0:
            continue
        best_s, best_a = -1.0, -1
        for j, sj in zip(nb.tolist(), sv.tolist()):
            a = snap[j]
            if a < 0:
                continue
            if best_a < 0 or sj > best_s * (1.0 + TIE_RTOL):
                best_s, best_a = sj, a
            elif sj >= best_s * (1.0 - TIE_RTOL) and a < best_a:
                best_s, best_a = sj, a
        assert best_a >= 0, "non-isolated node with no aggregated strong neighbour"
        agg[i] = best_a
    return agg


MIS_SEED = 0xA66
IN, UNDECIDED, OUT = 2, 1, 0


def mis_keys(n, seed):
    """Fixed priority key of each node: (splitmix64(seed ^ I) >> 33, I) packed
    as prio * 2^30 + I (I < 2^30)."""
    assert n < (1 << 30)
    prio = (splitmix64_vec(seed, n) >> np.uint64(33)).astype(np.int64)
    return prio * (1 << 30) + np.arange(n, dtype=np.int64)


def symmetric_strong(A: sp.bsr_matrix, theta: float):
    """Per stored block: strong if s_IJ >= theta or s_JI >= theta (I != J).
    The two agree for a symmetric A up to rounding; taking both makes the
    strong graph symmetric by construction.  Returns (flag, (rows, cols, s))."""
    rows, cols, s = strength(A)
    own = (s >= theta) & (rows != cols)
    n = A.shape[0] // A.blocksize[0]
    key = rows * n + cols
    order = np.argsort(key)
    tkey = cols * n + rows
    tpos = order[np.searchsorted(key[order], tkey)]   # entry k = (I, J) -> position of (J, I)
    assert np.array_equal(key[tpos], tkey), "pattern not symmetric"
    return own | own[tpos], (rows, cols, s)


def mis2_rounds(n, rows, cols, flag, keys):
    """Distance-2 maximal independent set of the graph given by the flagged
    entries, by rounds: key*(I) = (state, key) with IN > UNDECIDED > OUT;
    m1(I) = max of key* over I and its neighbours, m2(I) = max of m1 over I
    and its neighbours (= over all nodes within distance 2).  An undecided
    node whose m2 is its own key* joins the set; an undecided node whose m2
    belongs to a member is excluded.  Returns (in_set bool[n], rounds)."""
    r, c = rows[flag], cols[flag]
    has = np.zeros(n, bool)
    has[r] = True
    state = np.where(has, UNDECIDED, OUT).astype(np.int64)
    rounds = 0
    while np.any(state == UNDECIDED):
        k = state * (1 << 61) + keys
        m1 = k.copy()
        np.maximum.at(m1, r, k[c])
        m2 = m1.copy()
        np.maximum.at(m2, r, m1[c])
        und = state == UNDECIDED
        join = und & (m2 == k)
        drop = und & ((m2 >> 61) == IN)
        state[join] = IN
        state[drop] = OUT
        rounds += 1
    return state == IN, rounds


def aggregate_mis2(A: sp.bsr_matrix, theta: float, seed: int):
    """Parallel aggregation: phase-1 roots by mis2_rounds on the symmetric
    strong graph, aggregates numbered by ascending root, phase-1 aggregate =
    root and its strong neighbours, then phase 2 (_attach_rest).
    Returns (agg, n_agg, (rows, cols, s))."""
    n = A.shape[0] // A.blocksize[0]
    flag, sinfo = symmetric_strong(A, theta)
    rows, cols, s = sinfo
    roots, _ = mis2_rounds(n, rows, cols, flag, mis_keys(n, seed))
    agg = np.full(n, -1, np.int64)
    ids = np.cumsum(roots) - 1
    agg[roots] = ids[roots]
    sel = flag & roots[rows]
    hits = np.bincount(cols[sel], minlength=n)
    assert hits.max(initial=0) <= 1 and not np.any(roots[cols[sel]]), "phase-1 aggregates overlap"
    agg[cols[sel]] = ids[rows[sel]]
    ptr = A.indptr
    nbrs = [(cols[ptr[i]:ptr[i + 1]][flag[ptr[i]:ptr[i + 1]]], s[ptr[i]:ptr[i + 1]][flag[ptr[i]:ptr[i + 1]]])
            for i in range(n)]
    return _attach_rest(agg, nbrs), int(roots.sum()), sinfo


# ---------------------------------------------------------------------------
# Tentative prolongator
# ---------------------------------------------------------------------------

def _qr_pos(Bj):
    Q, R = np.linalg.qr(Bj, mode="reduced")
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None]


def _rank_ok(R):
    d = np.abs(np.diag(R))
    return d.min() >= RANK_RTOL * d.max() and d.max() > 0


def _groups(agg, n_agg):
    """members[a] = ascending node list of aggregate a."""
    order = np.argsort(agg, kind="stable")
    sa = agg[order]
    members = [[] for _ in range(n_agg)]
    start = np.searchsorted(sa, np.arange(n_agg), side="left")
    stop = np.searchsorted(sa, np.arange(n_agg), side="right")
    for a in range(n_agg):
        members[a] = order[start[a]:stop[a]].tolist()
    return members


def tentative_prolongator(agg, n_agg, B, bs, strength_info):
    """P_tent (scalar CSR, (bs N) x (6 n_agg')) and coarse near-nullspace
    B_c (6 n_agg' x 6), after the rank-deficiency merge.  Returns
    (P_tent, Bc, agg) with agg renumbered compactly (creation order kept)."""
    n = agg.size
    k = B.shape[1]
    Bn = B.reshape(n, bs, k)
    agg = agg.copy()
    members = _groups(agg, n_agg)
    rows, cols, s = strength_info
    a_id = 0
    while a_id < len(members):
        nodes = sorted(members[a_id])
        if not nodes:
            a_id += 1
            continue
        Bj = Bn[nodes].reshape(-1, k)
        if Bj.shape[0] >= k and _rank_ok(np.linalg.qr(Bj, mode="r")):
            a_id += 1
            continue
        # merge into the neighbouring aggregate with the largest summed strength
        score = {}
        sel = np.isin(rows, nodes) & (rows != cols)
        for c, sv in zip(cols[sel].tolist(), s[sel].tolist()):
            t = int(agg[c])
            if t >= 0 and t != a_id:
                score[t] = score.get(t, 0.0) + sv
        if not score:
            raise RankError(f"aggregate {a_id} is rank deficient and has no neighbour")
        best = max(score.items(), key=lambda kv: (kv[1], -kv[0]))[0]
        members[best] = sorted(members[best] + nodes)
        members[a_id] = []
        agg[nodes] = best
        a_id = best if best < a_id else a_id + 1
    live = [a for a in range(len(members)) if members[a]]
    nc = len(live)
    new_agg = np.full(n, -1, np.int64)
    Qrows = np.zeros((n, bs, k))
    Bc = np.zeros((nc * k, k))
    for J, a in enumerate(live):
        nodes = np.array(sorted(members[a]), np.int64)
        new_agg[nodes] = J
        Q, R = _qr_pos(Bn[nodes].reshape(-1, k))
        Qrows[nodes] = Q.reshape(len(nodes), bs, k)
        Bc[J * k:(J + 1) * k] = R
    # CSR: every DOF of an aggregated node has k entries in its aggregate's columns
    live_dof = np.repeat(new_agg >= 0, bs)
    counts = np.where(live_dof, k, 0)
    indptr = np.zeros(n * bs + 1, np.int64)
    np.cumsum(counts, out=indptr[1:])
    dof_agg = np.repeat(new_agg, bs)[live_dof]
    indices = (dof_agg[:, None] * k + np.arange(k)[None, :]).ravel()
    data = Qrows.reshape(n * bs, k)[live_dof].ravel()
    P = sp.csr_matrix((data, indices, indptr), shape=(n * bs, nc * k))
    return P, Bc, new_agg


# ---------------------------------------------------------------------------
# Eigenvalue estimate, prolongator smoothing, Galerkin product
# ---------------------------------------------------------------------------

def point_diagonal(A):
    return A.diagonal().astype(np.float64)


def lanczos_max(A, D, steps, seed):
    """Largest Ritz value of `steps` Lanczos steps (no reorthogonalisation) on
    S = D^-1/2 A D^-1/2 from the splitmix64 start vector."""
    n = A.shape[0]
    dh = 1.0 / np.sqrt(D)
    v = uniform01_vec(seed, n) - 0.5
    v = v / np.linalg.norm(v)
    v_prev = np.zeros(n)
    beta_prev = 0.0
    alphas, betas = [], []
    for j in range(steps):
        w = dh * (A @ (dh * v)) - beta_prev * v_prev
        a = float(w @ v)
        w = w - a * v
        b = float(np.linalg.norm(w))
        alphas.append(a)
        if j == steps - 1 or b <= 1e-12 * (abs(a) + beta_prev):
            break
        betas.append(b)
        v_prev, v, beta_prev = v, w / b, b
    if len(alphas) == 1:
        return alphas[0]
    ev = sla.eigvalsh_tridiagonal(np.array(alphas), np.array(betas[:len(alphas) - 1]))
    return float(ev.max())


def filtered_operator(A: sp.bsr_matrix, theta: float):
    """A^F: per block row the diagonal block plus the dropped blocks (summed
    in stored order), and the strong off-diagonal blocks unchanged."""
    flag, (rows, cols, _) = symmetric_strong(A, theta)
    diag = rows == cols
    keep = flag | diag
    data = A.data.copy()
    n = A.shape[0] // A.blocksize[0]
    dpos = np.full(n, -1, np.int64)
    dpos[rows[diag]] = np.flatnonzero(diag)
    assert np.all(dpos >= 0), "a block row without its diagonal block"
    dropped = np.flatnonzero(~keep)
    for k in dropped.tolist():            # stored order within each row
        data[dpos[rows[k]]] += A.data[k]
    counts = np.bincount(rows[keep], minlength=n)
    indptr = np.concatenate([[0], np.cumsum(counts)])
    return sp.bsr_matrix((data[keep], cols[keep], indptr), shape=A.shape)


def smooth_prolongator(A, D, P_tent, lam_hat):
    omega = 4.0 / (3.0 * lam_hat)
    return (P_tent - omega * sp.diags(1.0 / D) @ (A.tocsr() @ P_tent)).tocsr()


def galerkin(A, P, bs_c=6):
    Ac = (P.T.tocsr() @ (A.tocsr() @ P)).tocsr()
    return Ac.tobsr(blocksize=(bs_c, bs_c))


# ---------------------------------------------------------------------------
# Hierarchy
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Level:
    A: sp.bsr_matrix
    bs: int
    D: np.ndarray
    lam: float = 0.0
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    agg: np.ndarray | None = None
    chol: tuple | None = None


def setup(A: sp.bsr_matrix, B: np.ndarray, opt: AMGOptions = AMGOptions(), aggregates=None):
    """Build the hierarchy.  `aggregates` optionally fixes the aggregate map of
    each level (list of int arrays); otherwise opt.aggregation's rule is used."""
    levels = []
    bs = A.blocksize[0]
    Al, Bl = A, B
    for l in range(opt.max_levels):
        D = point_diagonal(Al)
        lev = Level(A=Al, bs=bs, D=D)
        levels.append(lev)
        ndof = Al.shape[0]
        if ndof <= opt.coarse_max or l == opt.max_levels - 1:
            break
        lev.lam = lanczos_max(Al, D, opt.lanczos_steps, 0x5EED + l)
        theta = opt.theta0 * 2.0 ** (-l)
        if aggregates is not None and l < len(aggregates):
            _, _, sinfo = aggregate(Al, theta)
            agg = np.asarray(aggregates[l], np.int64)
            n_agg = int(agg.max()) + 1 if agg.size and agg.max() >= 0 else 0
        elif opt.aggregation == "mis2":
            agg, n_agg, sinfo = aggregate_mis2(Al, theta, MIS_SEED + l)
        else:
            agg, n_agg, sinfo = aggregate(Al, theta)
        if n_agg == 0:
            break
        P_tent, Bc, agg = tentative_prolongator(agg, n_agg, Bl, bs, sinfo)
        P = smooth_prolongator(filtered_operator(Al, theta) if opt.smooth_filtered else Al, D, P_tent, lev.lam)
        Ac = galerkin(Al, P, Bc.shape[1])
        if Ac.shape[0] > opt.max_coarse_ratio * ndof:
            break
        lev.P, lev.R, lev.agg = P, P.T.tocsr(), agg
        Al, Bl, bs = Ac, Bc, Bc.shape[1]
    last = levels[-1]
    last.P = last.R = None
    dense = last.A.toarray()
    last.chol = sla.cho_factor(0.5 * (dense + dense.T), lower=True)
    # every non-coarsest level needs its eigenvalue estimate for smoothing
    for l, lev in enumerate(levels[:-1]):
        if lev.lam == 0.0:
            lev.lam = lanczos_max(lev.A, lev.D, opt.lanczos_steps, 0x5EED + l)
    return levels


# ---------------------------------------------------------------------------
# Smoother and cycle
# ---------------------------------------------------------------------------

def chebyshev(A, D, g, x0, lam_hat, degree=2, ratio=10.0, safety=1.1):
    """Chebyshev iteration on D^-1 A over [b/ratio, b], b = safety * lam_hat
    (Saad Alg. 12.1 with the residual preconditioned by D^-1)."""
    b = safety * lam_hat
    a = b / ratio
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = x0.copy()
    r = g - A @ x
    d = (r / D) / theta
    for k in range(degree):
        x = x + d
        if k < degree - 1:
            r = r - A @ d
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (r / D)
            rho = rho_new
    return x


def vcycle(levels, g, l=0, opt: AMGOptions = AMGOptions()):
    lev = levels[l]
    if lev.chol is not None:
        return sla.cho_solve(lev.chol, g)
    x = chebyshev(lev.A, lev.D, g, np.zeros_like(g), lev.lam, opt.cheb_degree, opt.cheb_ratio, opt.cheb_safety)
    s = g - lev.A @ x
    x = x + lev.P @ vcycle(levels, lev.R @ s, l + 1, opt)
    return chebyshev(lev.A, lev.D, g, x, lev.lam, opt.cheb_degree, opt.cheb_ratio, opt.cheb_safety)


def operator_complexity(levels):
    return sum(lv.A.nnz for lv in levels) / levels[0].A.nnz
