"""Oracle: the nonlinear heat equation of the thermal step and its Newton
solve (test infrastructure only; see the package docstring).

What the paper fixes (Sec. 3, eq. wf_thermal; Sec. 3.2; Sec. 5.2, 5.3): the
temperature T_{m+1} in the Lagrange space V_h satisfies, with the theta-method
at theta = 1 (backward Euler, Sec. 5.3) or without the time term (steady,
Sec. 5.2),

    F_T(T; s) = int rho c_v (T - T_m)/dt s + int kappa grad T . grad s
                + int_Gamma h (T - T_bc) s ds = 0      for all s in V_h,

with kappa and c_v depending on T (so F_T is nonlinear), solved by Newton's
method (Sec. 3.2) from an initial 400 K (steady, Sec. 5.2) to a relative
residual of 1e-9, each correction by CG preconditioned with classical AMG
(Sec. 5.1; ``oracle.camg``).  The full linearisation is not symmetric
(Sec. 3.2 keeps CG all the same).

Readings (the paper is silent or its sign is ambiguous):
* Robin term: the paper writes kappa grad T . n = beta (T - T_bc) and the
  boundary integral with a minus sign; for the exchange to take heat out of
  the body when T > T_bc the coefficient is -h with h >= 0, so the boundary
  term here is + int h (T - T_bc) s.  h and T_bc are constant per boundary
  triangle.
* Coefficients: each material gives kappa(T) and c_v(T) as piecewise-linear
  tables, constant beyond the ends (as the elastic tables), and rho per
  material; a cell takes its material's values at the exact mean of T_h over
  the cell (the rule of the elastic materials), so kappa and c_v are constant
  per cell and every integral is exact (degree-2 stiffness, mass and face
  mass integrands).  The table slope used in the Jacobian is that of the
  segment [T_k, T_{k+1}) holding the mean (0 beyond the ends).
* Newton: T <- T + d with J(T) d = -F(T); stop when |F(T)|_2 <= rtol |F(T_0)|_2
  (rtol 1e-9) or |F(T)|_2 <= atol (1e-8, in the units of F: watts), the
  absolute floor that ends a step starting near a steady state, where 1e-9
  of the initial residual lies below rounding; the correction solved by
  preconditioned CG to a relative residual of 1e-8 (lin_rtol).
"""
from __future__ import annotations

import dataclasses
import functools
from fractions import Fraction
from math import factorial

import numpy as np
import scipy.sparse as sp

from . import fem


def table_value_slope(T, table_T, table_v):
    """Piecewise-linear table (constant beyond the ends): value at T and the
    slope of the segment [T_k, T_{k+1}) holding T (0 outside)."""
    val = np.interp(T, table_T, table_v)
    k = np.searchsorted(table_T, T, side="right") - 1
    inside = (k >= 0) & (k < len(table_T) - 1)
    kk = np.clip(k, 0, len(table_T) - 2)
    slope = (table_v[kk + 1] - table_v[kk]) / (table_T[kk + 1] - table_T[kk])
    return val, np.where(inside, slope, 0.0)


def cell_weights(degree):
    """(1/|K|) int phi_c: the weights of the cell mean of T_h."""
    _, _, M = fem.reference_tables(degree)
    return M.sum(axis=0)


@functools.lru_cache(maxsize=None)
def face_mass(degree):
    """(1/|F|) int_F phi_a phi_b on a triangle (P1: l_a; P2: vertices
    l_a (2 l_a - 1), edges 4 l_a l_b in the order 01, 02, 12), exact from
    int_F l0^a l1^b l2^c ds = a! b! c! 2! |F| / (a+b+c+2)!."""
    def lam(k, c=1):
        e = [0, 0, 0]
        e[k] = 1
        return {tuple(e): Fraction(c)}

    def mul(p, q):
        out = {}
        for ep, cp in p.items():
            for eq, cq in q.items():
                e = tuple(a + b for a, b in zip(ep, eq))
                out[e] = out.get(e, Fraction(0)) + cp * cq
        return out

    if degree == 1:
        phis = [lam(a) for a in range(3)]
    else:
        phis = []
        for a in range(3):
            q = mul(lam(a, 2), lam(a))
            e = [0, 0, 0]
            e[a] = 1
            q[tuple(e)] = q.get(tuple(e), Fraction(0)) - 1
            phis.append(q)
        phis += [mul(lam(a, 4), lam(b)) for a, b in fem.FACE_EDGES]
    n = len(phis)
    out = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            tot = Fraction(0)
            for (a, b, c), coef in mul(phis[i], phis[j]).items():
                tot += coef * Fraction(factorial(a) * factorial(b) * factorial(c) * 2, factorial(a + b + c + 2))
            out[i, j] = float(tot)
    return out


@dataclasses.dataclass
class ThermalProblem:
    """Inputs of one thermal solve.  tables: T, kappa, cv [n_mat][n_pts],
    rho [n_mat]; faces [F][3|6] with h, T_bc per face (may be empty)."""
    coords: np.ndarray
    cells: np.ndarray
    degree: int
    T_tab: np.ndarray
    kappa_tab: np.ndarray
    cv_tab: np.ndarray
    rho: np.ndarray
    cell_material: np.ndarray
    faces: np.ndarray
    h: np.ndarray
    T_bc: np.ndarray


def problem_from_meshgen(mesh, mats, robin):
    return ThermalProblem(mesh.coords, mesh.cells.astype(np.int64), mesh.degree, mats.T, mats.kappa, mats.cv,
                          mats.rho, np.asarray(mats.cell_material), robin.faces.astype(np.int64), robin.h, robin.T_bc)


def assemble(P: ThermalProblem, T, T_old=None, dt=None):
    """Residual F[N] of eq. wf_thermal at T (with the backward-Euler time term
    when dt is given) and its Jacobian J = dF/dT (scipy CSR, the node
    pattern).  Every integral exact."""
    cells = P.cells
    n = P.coords.shape[0]
    vol, G = fem.cell_geometry(P.coords, cells)
    S, _, M = fem.reference_tables(P.degree)
    dots = np.einsum("ckm,clm->ckl", G, G)
    Kref = vol[:, None, None] * np.einsum("abkl,ckl->cab", S, dots)      # int grad phi_a . grad phi_b
    w = cell_weights(P.degree)
    Tc = T[cells]
    Tbar = Tc @ w
    kap = np.empty(cells.shape[0])
    dkap = np.empty_like(kap)
    cv = np.empty_like(kap)
    dcv = np.empty_like(kap)
    rho = np.empty_like(kap)
    for m in np.unique(P.cell_material).tolist():
        sel = P.cell_material == m
        kap[sel], dkap[sel] = table_value_slope(Tbar[sel], P.T_tab[m], P.kappa_tab[m])
        cv[sel], dcv[sel] = table_value_slope(Tbar[sel], P.T_tab[m], P.cv_tab[m])
        rho[sel] = P.rho[m]
    KT = np.einsum("cab,cb->ca", Kref, Tc)
    Fe = kap[:, None] * KT
    Je = kap[:, None, None] * Kref + dkap[:, None, None] * KT[:, :, None] * w[None, None, :]
    if dt is not None:
        Mref = vol[:, None, None] * M[None, :, :]
        MdT = np.einsum("cab,cb->ca", Mref, Tc - T_old[cells])
        c = rho / dt
        Fe = Fe + (c * cv)[:, None] * MdT
        Je = Je + (c * cv)[:, None, None] * Mref + (c * dcv)[:, None, None] * MdT[:, :, None] * w[None, None, :]
    F = np.zeros(n)
    np.add.at(F, cells.ravel(), Fe.ravel())
    npe = cells.shape[1]
    rows = np.repeat(cells, npe, axis=1).ravel()
    cols = np.tile(cells, (1, npe)).ravel()
    vals = Je.ravel()
    if len(P.faces):
        f = P.faces
        x = P.coords[f[:, :3]]
        area = 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)
        Mf = area[:, None, None] * face_mass(P.degree)[None]
        fint = area[:, None] * fem.face_basis_integrals(P.degree)[None, :]
        Ff = P.h[:, None] * (np.einsum("fab,fb->fa", Mf, T[f]) - P.T_bc[:, None] * fint)
        np.add.at(F, f.ravel(), Ff.ravel())
        nf = f.shape[1]
        rows = np.concatenate([rows, np.repeat(f, nf, axis=1).ravel()])
        cols = np.concatenate([cols, np.tile(f, (1, nf)).ravel()])
        vals = np.concatenate([vals, (P.h[:, None, None] * Mf).ravel()])
    J = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    J.sum_duplicates()
    J.sort_indices()
    return F, J


@dataclasses.dataclass
class NewtonResult:
    T: np.ndarray
    iters: int
    converged: bool
    res_history: list
    lin_iters: list


def newton(P: ThermalProblem, T0, linear_solve, T_old=None, dt=None, rtol=1e-9, maxit=25, atol=1e-8):
    """Newton's method on F_T = 0 (Sec. 3.2): linear_solve(J, rhs, k) returns
    (d, lin_iters) with J d = rhs for Newton iteration k."""
    T = np.array(T0, dtype=np.float64, copy=True)
    F, J = assemble(P, T, T_old, dt)
    f0 = float(np.linalg.norm(F))
    hist = [f0]
    lin = []
    stop = max(rtol * f0, atol)
    for k in range(maxit):
        if hist[-1] <= stop:
            return NewtonResult(T, k, True, hist, lin)
        d, li = linear_solve(J, -F, k)
        lin.append(li)
        T = T + d
        F, J = assemble(P, T, T_old, dt)
        hist.append(float(np.linalg.norm(F)))
    return NewtonResult(T, maxit, hist[-1] <= stop, hist, lin)


class ReusedPreconditioner:
    """The linear solves of Newton's method with a kept classical-AMG
    preconditioner (a reading of Sec. 5.3, where the thermal preconditioner is
    rebuilt only at steps of rapid change): built from the Jacobian of the
    first correction and kept across Newton steps and time steps; rebuilt
    before the next correction when a correction needed more than
    rebuild_factor times the CG iterations of the first correction after the
    last build.  Each correction: PCG from zero to lin_rtol."""

    def __init__(self, amg_options=None, lin_rtol=1e-8, lin_maxit=500, rebuild_factor=1.5):
        from . import camg
        self.camg = camg
        self.opt = amg_options or camg.CAMGOptions()
        self.lin_rtol, self.lin_maxit, self.factor = lin_rtol, lin_maxit, rebuild_factor
        self.levels = None
        self.base = -1
        self.stale = True
        self.builds = 0

    def __call__(self, J, rhs, k):
        from . import krylov
        if self.levels is None or self.stale:
            self.levels = self.camg.setup(J, self.opt)
            self.base, self.stale = -1, False
            self.builds += 1
        r = krylov.pcg(J, rhs, lambda v: self.camg.vcycle(self.levels, v, opt=self.opt), rtol=self.lin_rtol,
                       maxit=self.lin_maxit)
        if self.base < 0:
            self.base = r.iters
        elif r.iters > self.factor * self.base:
            self.stale = True
        return r.u, r.iters
