"""Oracle: classical algebraic multigrid for the scalar thermal problem
(test infrastructure only; see the package docstring).

What the paper fixes (Sec. 5.1): the thermal correction is solved by CG
preconditioned with a classical AMG (the paper uses BoomerAMG; classical AMG
suits scalar equations) with a hybrid Gauss-Seidel smoother from the work it
cites (Baker, Falgout, Kolev & Yang 2011).  The rest are readings, each a
parameter:

* strength (Ruge & Stueben): row i strongly depends on j != i when
  -a_ij >= theta max_{k != i} (-a_ik) and that maximum is positive;
  theta = 0.25.
* coarsening: PMIS (De Sterck, Yang & Heys 2006) with fixed keys: a point
  that strongly influences no point is F from the start; then, in rounds,
  every undecided point whose key is larger than the keys of all its
  undecided strong neighbours (either direction) becomes C, and every
  undecided point that strongly depends on a new C point becomes F.  Key of
  point i on level l: (|S_i^T|, splitmix64((0xC1A5 + l) ^ i) >> 24, i)
  compared lexicographically, |S_i^T| the number of points that strongly
  depend on i.  C points are numbered in ascending order.
* interpolation: direct interpolation (Stueben 2001): for an F point i with
  strong C neighbours C_i, w_ij = -alpha_i a_ij / a_ii for negative and
  -beta_i a_ij / a_ii for positive a_ij (j in C_i), with alpha_i the ratio of
  the sums of negative off-diagonal entries over all neighbours and over C_i,
  beta_i the same for positive entries; without a positive entry in C_i the
  positive entries are added to the diagonal.  An F point without strong C
  neighbours has an empty row.  C points inject.
* coarse operator A_c = P^T A P; stop at <= coarse_max rows (500), 10
  levels, or a coarse level keeping more than 0.9 of the rows; the coarsest
  level is solved exactly (dense LU).
* smoother: the l1 hybrid Gauss-Seidel of the cited work: the rows are cut
  into blocks of `block` consecutive rows (128); inside a block Gauss-Seidel,
  across blocks Jacobi (values from before the sweep), with the diagonal
  a_ii + sum over columns outside the block of |a_ij| (convergent for any
  SPD matrix).  Pre-smoothing one forward sweep from zero, post-smoothing
  one backward sweep: the V-cycle is symmetric for a symmetric A.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .rng import splitmix64_vec

THETA = 0.25
KEY_SEED = 0xC1A5
F_PT, U_PT, C_PT = 0, 1, 2


@dataclasses.dataclass
class CAMGOptions:
    theta: float = THETA
    coarse_max: int = 500
    max_levels: int = 10
    max_coarse_ratio: float = 0.9
    block: int = 128


def strength(A: sp.csr_matrix, theta=THETA):
    """Per stored entry: True where row i strongly depends on column j."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    off = A.indices != rows
    neg = np.where(off, -A.data, -np.inf)
    m = np.full(n, -np.inf)
    np.maximum.at(m, rows, neg)
    return off & (m[rows] > 0) & (-A.data >= theta * m[rows])


def pmis(A: sp.csr_matrix, S, level, with_rounds=False):
    """C/F splitting by PMIS rounds with fixed keys.  Returns (state[n],
    rounds), state C_PT or F_PT; with_rounds adds the round in which each
    point was decided (0 for the points made F at the start)."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    infl = np.bincount(cols[S], minlength=n)                     # |S_i^T|
    rnd = (splitmix64_vec(KEY_SEED + level, n) >> np.uint64(24)).astype(np.int64)  # 40 bits
    state = np.where(infl > 0, U_PT, F_PT)
    # strong neighbours in either direction, as (i, j) pairs
    er, ec = rows[S], cols[S]
    gi = np.concatenate([er, ec])
    gj = np.concatenate([ec, er])
    rounds = 0
    when = np.zeros(n, np.int64)
    while np.any(state == U_PT):
        und = state == U_PT
        # i is a local maximum if no undecided strong neighbour j has a larger key
        bigger = (infl[gj] > infl[gi]) | ((infl[gj] == infl[gi]) & ((rnd[gj] > rnd[gi]) |
                                                                    ((rnd[gj] == rnd[gi]) & (gj > gi))))
        beaten = np.zeros(n, bool)
        beaten[gi[und[gj] & bigger]] = True
        newc = und & ~beaten
        dep = np.zeros(n, bool)
        dep[er[newc[ec]]] = True                                  # depends on a new C point
        state = np.where(newc, C_PT, np.where(und & dep, F_PT, state))
        rounds += 1
        when[und & (state != U_PT)] = rounds
    if with_rounds:
        return state, rounds, when
    return state, rounds


def direct_interpolation(A: sp.csr_matrix, S, state):
    """P (n x n_C, CSR) by direct interpolation; C points numbered ascending."""
    n = A.shape[0]
    cidx = np.cumsum(state == C_PT) - 1
    nc = int((state == C_PT).sum())
    Pr, Pc, Pv = [], [], []
    for i in range(n):
        if state[i] == C_PT:
            Pr.append(i)
            Pc.append(cidx[i])
            Pv.append(1.0)
            continue
        lo, hi = A.indptr[i], A.indptr[i + 1]
        cols = A.indices[lo:hi]
        vals = A.data[lo:hi]
        strong = S[lo:hi]
        diag = 0.0
        sn = sp_ = 0.0          # sums over all off-diagonal neighbours (negative, positive)
        cn = cp = 0.0           # sums over the strong C neighbours
        ci = []
        for j, a, s in zip(cols.tolist(), vals.tolist(), strong.tolist()):
            if j == i:
                diag += a
                continue
            if a < 0:
                sn += a
            else:
                sp_ += a
            if s and state[j] == C_PT:
                ci.append((j, a))
                if a < 0:
                    cn += a
                else:
                    cp += a
        if not ci:
            continue
        if cp == 0.0:
            diag += sp_
        alpha = sn / cn if cn != 0.0 else 0.0
        beta = sp_ / cp if cp != 0.0 else 0.0
        for j, a in ci:
            Pr.append(i)
            Pc.append(cidx[j])
            Pv.append(-(alpha if a < 0 else beta) * a / diag)
    return sp.csr_matrix((Pv, (Pr, Pc)), shape=(n, nc))


@dataclasses.dataclass
class CLevel:
    A: sp.csr_matrix
    dl1: np.ndarray | None = None        # a_ii + l1 row sums outside the block
    A_in: sp.csr_matrix | None = None    # entries inside the row's block
    A_out: sp.csr_matrix | None = None   # entries outside it
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    state: np.ndarray | None = None
    lu: tuple | None = None


def _split_blocks(A, block):
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    inside = (rows // block) == (A.indices // block)
    A_in = sp.csr_matrix((np.where(inside, A.data, 0.0), A.indices, A.indptr), shape=A.shape)
    A_out = sp.csr_matrix((np.where(inside, 0.0, A.data), A.indices, A.indptr), shape=A.shape)
    l1 = np.zeros(n)
    np.add.at(l1, rows, np.where(inside, 0.0, np.abs(A.data)))
    return A_in, A_out, A.diagonal() + l1


def setup(A: sp.csr_matrix, opt: CAMGOptions = CAMGOptions()):
    levels = []
    Al = A.tocsr()
    Al.sort_indices()
    for l in range(opt.max_levels):
        lev = CLevel(A=Al)
        levels.append(lev)
        n = Al.shape[0]
        if n <= opt.coarse_max or l == opt.max_levels - 1:
            break
        S = strength(Al, opt.theta)
        state, _ = pmis(Al, S, l)
        nc = int((state == C_PT).sum())
        if nc == 0 or nc > opt.max_coarse_ratio * n:
            break
        P = direct_interpolation(Al, S, state)
        R = P.T.tocsr()
        Ac = (R @ (Al @ P)).tocsr()
        Ac.sort_indices()
        lev.P, lev.R, lev.state = P, R, state
        Al = Ac
    last = levels[-1]
    last.lu = sla.lu_factor(last.A.toarray())
    for lev in levels[:-1]:
        lev.A_in, lev.A_out, lev.dl1 = _split_blocks(lev.A, opt.block)
    return levels


def hybrid_gs(lev: CLevel, g, x, block, forward=True):
    """One l1 hybrid Gauss-Seidel sweep (in place on a copy of x): blocks
    of `block` rows, Gauss-Seidel inside (ascending rows if forward, else
    descending), Jacobi across (values from before the sweep)."""
    n = g.size
    x_old = x.copy()
    out_part = lev.A_out @ x_old
    x = x.copy()
    order = range(block) if forward else range(block - 1, -1, -1)
    starts = np.arange(0, n, block)
    A_in = lev.A_in
    for k in order:
        idx = starts + k
        idx = idx[idx < n]
        if idx.size == 0:
            continue
        r = g[idx] - out_part[idx] - A_in[idx] @ x
        x[idx] = x[idx] + r / lev.dl1[idx]
    return x


def vcycle(levels, g, l=0, opt: CAMGOptions = CAMGOptions()):
    lev = levels[l]
    if lev.lu is not None:
        return sla.lu_solve(lev.lu, g)
    x = hybrid_gs(lev, g, np.zeros_like(g), opt.block, forward=True)
    s = g - lev.A @ x
    x = x + lev.P @ vcycle(levels, lev.R @ s, l + 1, opt)
    return hybrid_gs(lev, g, x, opt.block, forward=False)
