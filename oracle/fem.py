"""Oracle: Lagrange P1/P2 tetrahedral assembly of the linear thermoelastic
problem (test infrastructure only; see the package docstring).

Problem (Sec. 3, eqs. elasticity_bvp and u-dbc, weak form wf_elastic; the
boundary pressure term and temperature-dependent materials are in their own
section below): find u_h in [V_h]^3, u_h = u_bc on Gamma_D, with

    a(u, v) = int lam div u div v + 2 mu eps(u):eps(v) dx
            = int C:eps_T : grad v dx + int f.v dx,
    eps_T   = alpha (T - T_ref) I,  so  C:eps_T = (3 lam + 2 mu) alpha (T - T_ref) I.

Writing u = phi_b e_j and v = phi_a e_i gives the 3x3 coupling block of nodes
a, b (component i of the test function, j of the trial function)

    K[(a,i),(b,j)] = int lam d_i phi_a d_j phi_b + mu d_j phi_a d_i phi_b
                         + mu delta_ij grad phi_a . grad phi_b,
    b[(a,i)]       = (3 lam + 2 mu) alpha int (T_h - T_ref) d_i phi_a + int f_i phi_a.

The isotropic stiffness tensor is read from (E, nu) through the Lame constants
(the paper only names an elastic stiffness tensor).  T_h is the nodal
interpolant of T in the same Lagrange space as u.  Every integral is exact:
the integrands are polynomials in the barycentric coordinates, integrated with
  int_K l0^a l1^b l2^c l3^d dx = a! b! c! d! 3! |K| / (a+b+c+d+3)!.
"""
from __future__ import annotations

import dataclasses
import functools
from fractions import Fraction
from math import factorial

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# Barycentric polynomial algebra (exact, rational)
# ---------------------------------------------------------------------------

EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def _poly_mul(p, q):
    out = {}
    for ep, cp in p.items():
        for eq, cq in q.items():
            e = tuple(a + b for a, b in zip(ep, eq))
            out[e] = out.get(e, Fraction(0)) + cp * cq
    return out


def _poly_add(p, q, s=Fraction(1)):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, Fraction(0)) + s * c
    return out


def _lam(k, c=1):
    e = [0, 0, 0, 0]
    e[k] = 1
    return {tuple(e): Fraction(c)}


def _const(c):
    return {(0, 0, 0, 0): Fraction(c)}


def _integral_over_volume(p):
    """(1/|K|) int_K p dx for p in barycentric monomials."""
    tot = Fraction(0)
    for (a, b, c, d), coef in p.items():
        num = factorial(a) * factorial(b) * factorial(c) * factorial(d) * factorial(3)
        tot += coef * Fraction(num, factorial(a + b + c + d + 3))
    return tot


def basis(degree):
    """Lagrange basis on the tetrahedron in barycentric coordinates.
    P1: phi_a = l_a.  P2: vertices l_a (2 l_a - 1), edges 4 l_a l_b in the
    order (01, 02, 03, 12, 13, 23)."""
    if degree == 1:
        return [_lam(a) for a in range(4)]
    phis = [_poly_add(_poly_mul(_lam(a, 2), _lam(a)), _lam(a), Fraction(-1)) for a in range(4)]
    phis += [_poly_mul(_lam(a, 4), _lam(b)) for a, b in EDGES]
    return phis


def _d_dlam(p, k):
    out = {}
    for e, c in p.items():
        if e[k] > 0:
            e2 = list(e)
            e2[k] -= 1
            out[tuple(e2)] = out.get(tuple(e2), Fraction(0)) + c * e[k]
    return out


@functools.lru_cache(maxsize=None)
def reference_tables(degree):
    """Exact tables (as float64), all divided by |K|:
    S[a,b,k,l] = int (dphi_a/dl_k)(dphi_b/dl_l);  W[c,a,k] = int phi_c dphi_a/dl_k;
    M[a,c] = int phi_a phi_c."""
    phis = basis(degree)
    n = len(phis)
    dphi = [[_d_dlam(p, k) for k in range(4)] for p in phis]
    S = np.zeros((n, n, 4, 4))
    W = np.zeros((n, n, 4))
    M = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            M[a, b] = float(_integral_over_volume(_poly_mul(phis[a], phis[b])))
            for k in range(4):
                W[a, b, k] = float(_integral_over_volume(_poly_mul(phis[a], dphi[b][k])))
                for l in range(4):
                    S[a, b, k, l] = float(_integral_over_volume(_poly_mul(dphi[a][k], dphi[b][l])))
    return S, W, M


def lame(E, nu):
    """Lame constants of an isotropic material."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


# ---------------------------------------------------------------------------
# Element geometry and element tensors
# ---------------------------------------------------------------------------

def cell_geometry(coords, cells):
    """vol[C] = |det J|/6 and G[C,k,i] = d_i l_k for the affine map of each cell
    (vertices are the first four cell nodes)."""
    x = coords[cells[:, :4]]  # [C,4,3]
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # rows k = grad l_{k+1}
    G = np.empty((cells.shape[0], 4, 3))
    G[:, 1:, :] = Jinv
    G[:, 0, :] = -Jinv.sum(axis=1)
    return np.abs(det) / 6.0, G


def element_stiffness(vol, G, lam, mu, degree):
    """K_e[C, a, i, b, j] for the bilinear form above (exact integration);
    lam and mu are scalars or per-cell arrays."""
    S, _, _ = reference_tables(degree)
    GG = np.einsum("cki,clj->cklij", G, G)           # G[k,i] G[l,j]
    dots = np.einsum("ckm,clm->ckl", G, G)           # grad l_k . grad l_l
    eye = np.eye(3)
    lam = np.reshape(lam, (-1, 1, 1, 1, 1))
    mu = np.reshape(mu, (-1, 1, 1, 1, 1))
    kern = lam * GG + mu * GG.transpose(0, 1, 2, 4, 3) + mu * dots[:, :, :, None, None] * eye
    # kern[c,k,l,i,j] = lam G_ki G_lj + mu G_kj G_li + mu delta_ij G_k.G_l
    Ke = np.einsum("abkl,cklij->caibj", S, kern)
    return vol[:, None, None, None, None] * Ke


def element_load(vol, G, dT_cell, f_cell, lam, mu, alpha, degree):
    """b_e[C, a, i]: thermal load plus consistent body-force load; lam, mu and
    alpha are scalars or per-cell arrays."""
    _, W, M = reference_tables(degree)
    c_alpha = np.reshape((3.0 * np.asarray(lam) + 2.0 * np.asarray(mu)) * np.asarray(alpha), (-1, 1, 1))
    # sum_c dT_c int phi_c d_i phi_a = sum_c dT_c sum_k W[c,a,k] G[k,i]
    be = c_alpha * np.einsum("cn,nak,cki->cai", dT_cell, W, G) * vol[:, None, None]
    if f_cell is not None:
        be = be + vol[:, None, None] * np.einsum("an,cni->cai", M, f_cell)
    return be


# ---------------------------------------------------------------------------
# Global assembly into 3x3-block compressed rows
# ---------------------------------------------------------------------------

def sparsity(cells, n_nodes):
    """Block pattern: I ~ J when both belong to one cell (closed star).
    Returns (row_ptr[N+1], col_idx[nnzb]) with sorted columns."""
    c = cells.astype(np.int64)
    npe = c.shape[1]
    I = np.repeat(c, npe, axis=1).ravel()
    J = np.tile(c, (1, npe)).ravel()
    keys = np.unique(I * n_nodes + J)
    rows = keys // n_nodes
    cols = keys % n_nodes
    row_ptr = np.zeros(n_nodes + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n_nodes), out=row_ptr[1:])
    return row_ptr, cols


def assemble(coords, cells, degree, E, nu, alpha, T_ref, T, f=None, chunk=200_000):
    """Unconstrained global stiffness (scipy BSR, 3x3 blocks) and load b[N,3]
    of one material (E, nu, alpha scalars) or of per-cell coefficients
    (arrays over the cells)."""
    n = coords.shape[0]
    lam, mu = lame(np.asarray(E, dtype=np.float64), np.asarray(nu, dtype=np.float64))
    alpha = np.asarray(alpha, dtype=np.float64)
    per_cell = lam.ndim > 0

    def part(v, s0, s1):
        return v[s0:s1] if per_cell else v

    row_ptr, cols = sparsity(cells, n)
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr)) * n + cols
    val = np.zeros((cols.size, 3, 3))
    b = np.zeros((n, 3))
    npe = cells.shape[1]
    for s in range(0, cells.shape[0], chunk):
        cc = cells[s:s + chunk].astype(np.int64)
        vol, G = cell_geometry(coords, cc)
        s1 = s + cc.shape[0]
        Ke = element_stiffness(vol, G, part(lam, s, s1), part(mu, s, s1), degree)  # [c,a,i,b,j]
        dT = T[cc] - T_ref
        fc = None if f is None else f[cc]
        be = element_load(vol, G, dT, fc, part(lam, s, s1), part(mu, s, s1),
                          alpha[s:s1] if per_cell else alpha, degree)
        I = np.repeat(cc, npe, axis=1)   # [c, a*npe+b] -> node a
        J = np.tile(cc, (1, npe))
        pos = np.searchsorted(keys, (I * n + J).ravel())
        blocks = Ke.transpose(0, 1, 3, 2, 4).reshape(-1, 3, 3)  # [c*a*b, i, j]
        np.add.at(val, pos, blocks)
        np.add.at(b, cc.ravel(), be.reshape(-1, 3))
    A = sp.bsr_matrix((val, cols, row_ptr), shape=(3 * n, 3 * n))
    return A, b


def assemble_rows(coords, cells, degree, E, nu, alpha, T_ref, T, rows, f=None):
    """Block rows `rows` of the unconstrained system, computed from the cells
    that touch them only (exact for those rows).  Returns a dict
    row -> (cols[int], blocks[k,3,3], b_row[3])."""
    rows = np.asarray(rows, dtype=np.int64)
    touch = np.isin(cells, rows).any(axis=1)
    sub = cells[touch].astype(np.int64)
    lam, mu = lame(E, nu)
    vol, G = cell_geometry(coords, sub)
    Ke = element_stiffness(vol, G, lam, mu, degree)
    be = element_load(vol, G, T[sub] - T_ref, None if f is None else f[sub], lam, mu, alpha, degree)
    out = {}
    npe = sub.shape[1]
    for r in rows.tolist():
        acc = {}
        brow = np.zeros(3)
        cs, as_ = np.nonzero(sub == r)
        for c, a in zip(cs.tolist(), as_.tolist()):
            brow += be[c, a]
            for bb in range(npe):
                J = int(sub[c, bb])
                acc[J] = acc.get(J, 0.0) + Ke[c, a, :, bb, :]
        cols = np.array(sorted(acc))
        out[r] = (cols, np.array([acc[j] for j in cols]), brow)
    return out


# ---------------------------------------------------------------------------
# Temperature-dependent materials and boundary pressure
# ---------------------------------------------------------------------------
# Sec. 3 lets the stiffness tensor C and alpha_L depend on temperature and
# the weak form wf_elastic carries the boundary term - int p_bc n . v ds on
# Gamma_N (traction sigma n = p_bc n); Sec. 4.2 shows normalised
# temperature tables for several materials.  Readings: each material gives
# E, nu and alpha_L as piecewise-linear tables in T, constant beyond their
# ends; a cell takes the values of its material at the mean of T_h over the
# cell (so C and alpha_L are constant per cell); p_bc is constant on each
# boundary triangle.

@dataclasses.dataclass
class MaterialTables:
    """T[m, k] ascending sample temperatures of material m, and E, nu, alpha
    at those temperatures (all [n_materials, n_points])."""
    T: np.ndarray
    E: np.ndarray
    nu: np.ndarray
    alpha: np.ndarray


def cell_mean(T, cells, degree):
    """Mean of the Lagrange interpolant T_h over each cell:
    sum_c T_c (1/|K|) int phi_c, with int phi_c = sum_a int phi_a phi_c
    (the basis sums to one)."""
    _, _, M = reference_tables(degree)
    return T[cells] @ M.sum(axis=0)


def cell_coefficients(T, cells, degree, cell_material, tables: MaterialTables):
    """Per-cell (E, nu, alpha) of each cell's material at its mean temperature."""
    Tm = cell_mean(T, cells, degree)
    E = np.empty(cells.shape[0])
    nu = np.empty_like(E)
    alpha = np.empty_like(E)
    for m in np.unique(cell_material).tolist():
        sel = cell_material == m
        E[sel] = np.interp(Tm[sel], tables.T[m], tables.E[m])
        nu[sel] = np.interp(Tm[sel], tables.T[m], tables.nu[m])
        alpha[sel] = np.interp(Tm[sel], tables.T[m], tables.alpha[m])
    return E, nu, alpha


FACE_EDGES = [(0, 1), (0, 2), (1, 2)]


@functools.lru_cache(maxsize=None)
def face_basis_integrals(degree):
    """(1/|F|) int_F phi_a ds for the Lagrange basis on a triangle in
    barycentric coordinates (P1: l_a; P2: vertices l_a (2 l_a - 1), then
    4 l_a l_b on the edges 01, 02, 12), from
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
            q[(0, 0, 0)] = Fraction(0)
            e = [0, 0, 0]
            e[a] = 1
            q[tuple(e)] = q.get(tuple(e), Fraction(0)) - 1
            phis.append(q)
        phis += [mul(lam(a, 4), lam(b)) for a, b in FACE_EDGES]
    out = []
    for p in phis:
        tot = Fraction(0)
        for (a, b, c), coef in p.items():
            tot += coef * Fraction(factorial(a) * factorial(b) * factorial(c) * 2, factorial(a + b + c + 2))
        out.append(float(tot))
    return np.array(out)


def pressure_load(coords, faces, degree, p):
    """b[N, 3] of the boundary term int_F p n . v ds summed over the faces
    (traction p n; faces [F, 3] (P1) or [F, 6] (P2: vertices, then the edge
    nodes 01, 02, 12); n = (x1 - x0) x (x2 - x0) / |.|, outward for faces
    ordered counterclockwise seen from outside)."""
    faces = np.asarray(faces, dtype=np.int64)
    x = coords[faces[:, :3]]
    nv = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    two_area = np.linalg.norm(nv, axis=1)
    n = nv / two_area[:, None]
    w = face_basis_integrals(degree)
    contrib = (np.asarray(p, dtype=np.float64) * 0.5 * two_area)[:, None, None] * w[None, :, None] * n[:, None, :]
    b = np.zeros((coords.shape[0], 3))
    np.add.at(b, faces.ravel(), contrib.reshape(-1, 3))
    return b


def assemble_materials(coords, cells, degree, cell_material, tables, T_ref, T, f=None, faces=None, face_p=None):
    """Unconstrained system with per-cell temperature-dependent coefficients
    and the boundary pressure load: (A, b[N, 3])."""
    E, nu, alpha = cell_coefficients(T, np.asarray(cells, dtype=np.int64), degree, np.asarray(cell_material), tables)
    A, b = assemble(coords, cells, degree, E, nu, alpha, T_ref, T, f)
    if faces is not None and len(faces):
        b = b + pressure_load(coords, faces, degree, face_p)
    return A, b


def assemble_rows_materials(coords, cells, degree, cell_material, tables, T_ref, T, rows, f=None, faces=None,
                            face_p=None):
    """Block rows `rows` of the unconstrained multi-material system with the
    boundary pressure, from the cells and faces that touch them only.
    Returns a dict row -> (cols[int], blocks[k,3,3], b_row[3])."""
    rows = np.asarray(rows, dtype=np.int64)
    cells = np.asarray(cells, dtype=np.int64)
    touch = np.isin(cells, rows).any(axis=1)
    sub = cells[touch]
    E, nu, alpha = cell_coefficients(T, sub, degree, np.asarray(cell_material)[touch], tables)
    lam, mu = lame(E, nu)
    vol, G = cell_geometry(coords, sub)
    Ke = element_stiffness(vol, G, lam, mu, degree)
    be = element_load(vol, G, T[sub] - T_ref, None if f is None else f[sub], lam, mu, alpha, degree)
    bp = None
    if faces is not None and len(faces):
        faces = np.asarray(faces, dtype=np.int64)
        ft = np.isin(faces, rows).any(axis=1)
        bp = pressure_load(coords, faces[ft], degree, np.asarray(face_p)[ft])
    out = {}
    npe = sub.shape[1]
    for r in rows.tolist():
        acc = {}
        brow = np.zeros(3) if bp is None else bp[r].copy()
        cs, as_ = np.nonzero(sub == r)
        for c, a in zip(cs.tolist(), as_.tolist()):
            brow += be[c, a]
            for bb in range(npe):
                J = int(sub[c, bb])
                acc[J] = acc.get(J, 0.0) + Ke[c, a, :, bb, :]
        cols = np.array(sorted(acc))
        out[r] = (cols, np.array([acc[j] for j in cols]), brow)
    return out


# ---------------------------------------------------------------------------
# Dirichlet conditions and near-nullspace
# ---------------------------------------------------------------------------

def apply_dirichlet(A, b, mask, u_bc=None):
    """Symmetric elimination that keeps every DOF in the system: the lifting
    b -= A[:, D] u_D, then rows and columns of constrained DOFs are zeroed,
    their diagonal set to 1 and b_D = u_D.  Returns new (A, b[3N])."""
    m = mask.reshape(-1).astype(bool)
    bf = b.reshape(-1).astype(np.float64).copy()
    uD = np.zeros_like(bf) if u_bc is None else np.where(m, u_bc.reshape(-1), 0.0)
    bf = bf - A @ uD
    bf[m] = uD[m]
    A = A.copy()
    nb = A.shape[0] // 3
    rows = np.repeat(np.arange(nb), np.diff(A.indptr))
    keep_r = (~m).reshape(nb, 3)[rows][:, :, None]
    keep_c = (~m).reshape(nb, 3)[A.indices][:, None, :]
    A.data = A.data * keep_r * keep_c
    diag = np.nonzero(rows == A.indices)[0]
    md = m.reshape(nb, 3)[rows[diag]]
    for i in range(3):
        A.data[diag, i, i] = np.where(md[:, i], 1.0, A.data[diag, i, i])
    return A, bf


def rigid_body_modes(coords, mask=None):
    """B[3N, 6]: translations e_x, e_y, e_z and rotations about the node
    centroid, (-(y-yc), x-xc, 0), (0, -(z-zc), y-yc), (z-zc, 0, -(x-xc));
    rows of constrained DOFs set to zero."""
    n = coords.shape[0]
    c = coords - coords.mean(axis=0)
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = 1.0
    B[:, 1, 1] = 1.0
    B[:, 2, 2] = 1.0
    B[:, 0, 3] = -c[:, 1]
    B[:, 1, 3] = c[:, 0]
    B[:, 1, 4] = -c[:, 2]
    B[:, 2, 4] = c[:, 1]
    B[:, 0, 5] = c[:, 2]
    B[:, 2, 5] = -c[:, 0]
    B = B.reshape(3 * n, 6)
    if mask is not None:
        B[mask.reshape(-1).astype(bool)] = 0.0
    return B


def assemble_problem(prob, u_bc=None):
    """Convenience: assemble + Dirichlet for a meshgen.Problem.
    Returns (A_dirichlet, b_dirichlet[3N], A_free, b_free[N,3])."""
    m = prob.mesh
    A0, b0 = assemble(m.coords, m.cells, m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T, prob.f)
    A, b = apply_dirichlet(A0, b0, prob.mask, u_bc)
    return A, b, A0, b0


def cell_strain_stress(coords, cells, degree, u, E, nu, alpha, T_ref, T, points):
    """Strain and stress at barycentric `points` [P,4] of every cell, for the
    closed-form checks: eps = sym grad u_h, sigma = C:(eps - alpha dT_h I)."""
    lam, mu = lame(E, nu)
    vol, G = cell_geometry(coords, cells.astype(np.int64))
    phis = basis(degree)
    dphi = [[_d_dlam(p, k) for k in range(4)] for p in phis]

    def ev(p, l):
        return sum(float(c) * np.prod([l[i] ** e[i] for i in range(4)]) for e, c in p.items())

    ue = u.reshape(-1, 3)[cells]  # [C, n, 3]
    Te = T[cells] - T_ref
    out_eps, out_sig = [], []
    for l in points:
        dv = np.array([[ev(dphi[a][k], l) for k in range(4)] for a in range(len(phis))])  # [n,4]
        ph = np.array([ev(p, l) for p in phis])
        grad_phi = np.einsum("ak,cki->cai", dv, G)  # [C,n,3]
        gu = np.einsum("cai,caj->cij", ue, grad_phi)  # d_j u_i
        eps = 0.5 * (gu + gu.transpose(0, 2, 1))
        dT = Te @ ph
        tr = np.trace(eps, axis1=1, axis2=2) - 3 * alpha * dT
        sig = 2 * mu * (eps - alpha * dT[:, None, None] * np.eye(3)) + lam * tr[:, None, None] * np.eye(3)
        out_eps.append(eps)
        out_sig.append(sig)
    return np.array(out_eps), np.array(out_sig)
