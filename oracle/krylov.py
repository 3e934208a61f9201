"""Oracle: preconditioned conjugate gradients (test infrastructure only).

CG for symmetric positive-definite systems with a preconditioner M^-1, as the
paper uses it (Sec. 2.1.2, left preconditioning; Sec. 5.1, CG + AMG), in the
form of Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.1:

    r = b - A u;  z = M^-1 r;  p = z
    repeat:  q = A p;  alpha = (r,z)/(p,q);  u += alpha p;  r -= alpha q
             stop test;  z' = M^-1 r';  beta;  p = z' + beta p

with beta = (r',z')/(r,z) (standard) or, for a preconditioner that is not a
fixed linear operator (single-precision V-cycle), the flexible choice
beta = (z', r' - r)/(z, r) (Notay, SIAM J. Sci. Comput. 22, 2000).

Stopping rule (a reading; the paper states a preconditioned relative
residual): the recurrence residual |r|_2 <= rtol |b|_2 triggers a check of the
true residual |b - A u|_2; if that also passes the solve ends, otherwise r is
replaced by the true residual and the iteration continues (at most 3 times).
Breakdown when (p,Ap) <= 0 or (r,z) <= 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np


class Breakdown(RuntimeError):
    pass


@dataclasses.dataclass
class Result:
    u: np.ndarray
    iters: int
    converged: bool
    relres_true: float
    history: list


def pcg(A, b, M=None, u0=None, rtol=1e-8, maxit=500, flexible=False, max_replace=3):
    """A: callable or matrix; M: callable (r -> z) or None for identity."""
    mat = A if callable(A) else (lambda x: A @ x)
    prec = M if M is not None else (lambda r: r.copy())
    bnorm = float(np.linalg.norm(b))
    u = np.zeros_like(b) if u0 is None else u0.astype(np.float64).copy()
    if bnorm == 0.0:
        return Result(np.zeros_like(b), 0, True, 0.0, [0.0])
    r = b - mat(u)
    hist = [float(np.linalg.norm(r)) / bnorm]
    replaced = 0
    it = 0
    # a good initial guess may already pass
    if hist[-1] <= rtol:
        return Result(u, 0, True, hist[-1], hist)
    z = prec(r)
    rz = float(r @ z)
    if rz <= 0:
        raise Breakdown("(r,z) <= 0")
    p = z.copy()
    while it < maxit:
        q = mat(p)
        pq = float(p @ q)
        if pq <= 0:
            raise Breakdown("(p,Ap) <= 0")
        alpha = rz / pq
        u = u + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        rn = float(np.linalg.norm(r)) / bnorm
        hist.append(rn)
        if rn <= rtol:
            rt = b - mat(u)
            rtn = float(np.linalg.norm(rt)) / bnorm
            if rtn <= rtol:
                return Result(u, it, True, rtn, hist)
            if replaced >= max_replace:
                return Result(u, it, False, rtn, hist)
            replaced += 1
            r = rt
        z_new = prec(r)
        rz_new = float(r @ z_new)
        if rz_new <= 0:
            raise Breakdown("(r,z) <= 0")
        if flexible:
            beta = float(z_new @ (r - r_old)) / rz
        else:
            beta = rz_new / rz
        p = z_new + beta * p
        rz = rz_new
    rt = b - mat(u)
    return Result(u, it, False, float(np.linalg.norm(rt)) / bnorm, hist)


def pcg_multi(A, Bm, M=None, U0=None, **kw):
    """Independent CG recurrences, one per column of Bm [n, k]; column j is by
    definition the single right-hand-side solve of Bm[:, j]."""
    res = []
    for j in range(Bm.shape[1]):
        res.append(pcg(A, Bm[:, j], M, None if U0 is None else U0[:, j], **kw))
    return res


@dataclasses.dataclass
class BlockResult:
    U: np.ndarray
    iters: int
    converged: list
    relres_true: list
    ranks: list


def _orth(W, drop_tol):
    """Orthonormal basis of the columns of W from the eigen-decomposition of
    W^T W; directions whose singular value is below drop_tol times the
    largest are dropped."""
    G = W.T @ W
    lam, V = np.linalg.eigh(0.5 * (G + G.T))
    if lam[-1] <= 0.0:
        return W[:, :0]
    keep = lam > (drop_tol ** 2) * lam[-1]
    return W @ (V[:, keep] / np.sqrt(lam[keep]))


def block_pcg(A, B, M=None, U0=None, rtol=1e-8, maxit=500, max_replace=3, drop_tol=1e-6):
    """Block preconditioned CG over the columns of B [n, m] (O'Leary, Linear
    Algebra Appl. 29, 1980): one Krylov space shared by all columns,

        R = B - A X;  Z = M^-1 R;  P = orth(Z)
        repeat:  Q = A P;  alpha = (P^T Q)^-1 (P^T R);  X += P alpha;  R -= Q alpha
                 stop test;  Z = M^-1 R;  beta = -(P^T Q)^-1 (Q^T Z);  P = orth(Z + P beta)

    with the search block orthonormalised every step and its numerically
    dependent directions dropped, which keeps P^T A P invertible when columns
    converge or become dependent (the breakdown-free form of Ji and Li, 2017;
    Dubrulle, ETNA 12, 2001).  The rank test is on the singular values of the
    block relative to the largest (drop_tol; computed from the Gram matrix,
    whose rounding puts numerically dependent directions near sqrt(eps), so
    the default is 1e-6).  M: callable on one column (applied per column).
    Stop test per column as in pcg(): the recurrence residual triggers a true
    residual check of every column once all columns pass."""
    mat = A if callable(A) else (lambda x: A @ x)
    prec = M if M is not None else (lambda r: r.copy())
    n, m = B.shape
    bnorm = np.linalg.norm(B, axis=0)
    X = np.zeros_like(B) if U0 is None else U0.astype(np.float64).copy()

    def matb(Y):
        return np.stack([mat(Y[:, j]) for j in range(Y.shape[1])], axis=1) if Y.shape[1] else Y.copy()

    def precb(Y):
        return np.stack([prec(Y[:, j]) for j in range(Y.shape[1])], axis=1)

    def rel(Rm):
        return np.where(bnorm > 0, np.linalg.norm(Rm, axis=0) / np.where(bnorm > 0, bnorm, 1.0), 0.0)

    R = B - matb(X)
    ranks = []
    it = 0
    replaced = 0
    if np.all(rel(R) <= rtol):
        return BlockResult(X, 0, [True] * m, rel(R).tolist(), ranks)
    Z = precb(R)
    P = _orth(Z, drop_tol)
    while it < maxit and P.shape[1] > 0:
        ranks.append(P.shape[1])
        Q = matb(P)
        PQ = P.T @ Q
        alpha = np.linalg.solve(PQ, P.T @ R)
        X = X + P @ alpha
        R = R - Q @ alpha
        it += 1
        if np.all(rel(R) <= rtol):
            Rt = B - matb(X)
            rt = rel(Rt)
            if np.all(rt <= rtol):
                return BlockResult(X, it, [True] * m, rt.tolist(), ranks)
            if replaced >= max_replace:
                return BlockResult(X, it, (rt <= rtol).tolist(), rt.tolist(), ranks)
            replaced += 1
            R = Rt
        Z = precb(R)
        beta = -np.linalg.solve(PQ, Q.T @ Z)
        P = _orth(Z + P @ beta, drop_tol)
    rt = rel(B - matb(X))
    return BlockResult(X, it, (rt <= rtol).tolist(), rt.tolist(), ranks)
