"""Pins of the thermal oracle (eq. wf_thermal, Newton) and of the classical
AMG oracle against closed forms, finite differences, exact solutions,
conservation, library routines and hand-worked cases."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import camg, fem, krylov, thermal


def _tri_quadrature(f, n=7):
    """int over the reference triangle (area 1/2) by a Gauss-Legendre product
    rule on the collapsed square (exact for polynomials of degree <= 2n-2)."""
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    tot = 0.0
    for a, wa in zip(u, wu):
        for b, wb in zip(u, wu):
            # (a, b) on the square -> (s, t) = (a, b (1 - a)) on the triangle
            tot += wa * wb * (1.0 - a) * f(a, b * (1.0 - a))
    return tot


@pytest.mark.parametrize("deg", [1, 2])
def test_face_mass_matches_quadrature(deg):
    def phi(s, t):
        l0, l1, l2 = 1.0 - s - t, s, t
        if deg == 1:
            return np.array([l0, l1, l2])
        L = [l0, l1, l2]
        return np.array([L[a] * (2 * L[a] - 1) for a in range(3)] +
                        [4 * L[a] * L[b] for a, b in fem.FACE_EDGES])
    n = 3 if deg == 1 else 6
    ref = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            ref[i, j] = 2.0 * _tri_quadrature(lambda s, t: phi(s, t)[i] * phi(s, t)[j])   # per unit area
    assert np.abs(thermal.face_mass(deg) - ref).max() < 1e-14
    if deg == 1:
        assert np.allclose(thermal.face_mass(1), (np.ones((3, 3)) + np.eye(3)) / 12.0, atol=1e-16)


def test_table_value_and_slope():
    Tt = np.array([300.0, 400.0, 600.0])
    v = np.array([10.0, 20.0, 10.0])
    val, sl = thermal.table_value_slope(np.array([250.0, 300.0, 350.0, 400.0, 500.0, 600.0, 700.0]), Tt, v)
    assert np.allclose(val, [10, 10, 15, 20, 15, 10, 10])
    assert np.allclose(sl, [0, 0.1, 0.1, -0.05, -0.05, 0, 0])


def _small_problem(deg, robin=True, seed=0):
    m = mg.disc_mesh(3, 12, 2, deg)
    P = thermal.problem_from_meshgen(m, mg.disc_thermal_materials(m), mg.disc_robin_faces(m))
    if not robin:
        P.faces = P.faces[:0]
        P.h = P.h[:0]
        P.T_bc = P.T_bc[:0]
    rng = np.random.default_rng(seed)
    return m, P, rng


@pytest.mark.parametrize("deg", [1, 2])
@pytest.mark.parametrize("transient", [False, True])
def test_jacobian_equals_finite_differences(deg, transient):
    m, P, rng = _small_problem(deg)
    T = rng.uniform(300.0, 900.0, m.n_nodes)
    T_old = T - rng.uniform(0.0, 30.0, m.n_nodes) if transient else None
    dt = 7.0 if transient else None
    _, J = thermal.assemble(P, T, T_old, dt)
    Jd = J.toarray()
    h = 1e-3
    for j in rng.choice(m.n_nodes, 12, replace=False).tolist():
        e = np.zeros(m.n_nodes)
        e[j] = h
        Fp, _ = thermal.assemble(P, T + e, T_old, dt)
        Fm, _ = thermal.assemble(P, T - e, T_old, dt)
        col = (Fp - Fm) / (2 * h)
        # the table slope is piecewise constant: a cell mean crossing a table
        # sample inside [T-h, T+h] would make the difference one-sided; the
        # random temperatures keep the means away from the samples
        assert np.abs(col - Jd[:, j]).max() <= 1e-6 * np.abs(Jd).max(), j


def _cube_slab(deg, n=3):
    m = mg.cube_mesh(n, deg)
    faces = mg.boundary_faces(m)
    x = m.coords[faces[:, :3].astype(np.int64)]
    left = np.all(np.abs(x[..., 0]) < 1e-12, axis=1)
    right = np.all(np.abs(x[..., 0] - 1.0) < 1e-12, axis=1)
    keep = left | right
    return m, faces[keep], left[keep]


@pytest.mark.parametrize("deg", [1, 2])
def test_steady_slab_with_robin_ends_is_exact(deg):
    """kappa constant, Robin at x = 0 (h0, Tb0) and x = 1 (h1, Tb1), the other
    faces insulated: T = A + B x with -kappa B + h0 (A - Tb0) = 0 and
    kappa B + h1 (A + B - Tb1) = 0; linear, so the FE solution is exact."""
    m, faces, left = _cube_slab(deg)
    kappa, h0, h1, Tb0, Tb1 = 17.0, 40.0, 260.0, 300.0, 800.0
    Tt = np.array([[200.0, 1200.0]])
    P = thermal.ThermalProblem(m.coords, m.cells.astype(np.int64), deg, Tt, np.array([[kappa, kappa]]),
                               np.array([[500.0, 500.0]]), np.array([8000.0]),
                               np.zeros(m.n_cells, np.int64), faces.astype(np.int64),
                               np.where(left, h0, h1), np.where(left, Tb0, Tb1))
    M = np.array([[h0, -kappa], [h1, kappa + h1]])
    A, B = np.linalg.solve(M, [h0 * Tb0, h1 * Tb1])
    res = thermal.newton(P, np.full(m.n_nodes, 400.0), lambda J, r, k: (spla.spsolve(J.tocsc(), r), 1))
    T_ex = A + B * m.coords[:, 0]
    assert res.converged and res.iters <= 2
    assert np.abs(res.T - T_ex).max() <= 1e-9 * np.abs(T_ex).max()


def test_uniform_exterior_temperature_is_the_steady_state():
    m, P, _ = _small_problem(2)
    P.T_bc = np.full_like(P.T_bc, 512.5)
    F, _ = thermal.assemble(P, np.full(m.n_nodes, 512.5))
    assert np.abs(F).max() <= 1e-12 * np.abs(thermal.assemble(P, np.full(m.n_nodes, 400.0))[0]).max()


@pytest.mark.parametrize("deg", [1, 2])
def test_insulated_backward_euler_step_conserves_heat(deg):
    """No exchange with the exterior: the time term of F_T summed over all
    test functions (which sum to one) is sum_c rho c_v(Tbar_c) int_c (T -
    T_old) / dt, and the diffusion term sums to zero, so the Newton solution
    keeps that weighted heat content; with constant c_v it keeps int T."""
    m, P, rng = _small_problem(deg, robin=False)
    T_old = 300.0 + 400.0 * (m.coords[:, 0] > 0) + rng.uniform(0, 50, m.n_nodes)
    res = thermal.newton(P, T_old, lambda J, r, k: (spla.spsolve(J.tocsc(), r), 1), T_old=T_old, dt=50.0)
    assert res.converged
    vol, _ = fem.cell_geometry(m.coords, m.cells.astype(np.int64))
    w = thermal.cell_weights(deg)
    Tbar = res.T[m.cells] @ w
    cv = np.empty(m.n_cells)
    rho = P.rho[P.cell_material]
    for k in range(3):
        sel = P.cell_material == k
        cv[sel] = np.interp(Tbar[sel], P.T_tab[k], P.cv_tab[k])
    dmean = (res.T - T_old)[m.cells] @ w
    heat = rho * cv * vol * dmean
    assert abs(heat.sum()) <= 1e-10 * np.abs(heat).sum()
    assert np.abs(res.T - T_old).max() > 1.0      # it did diffuse


def test_newton_converges_quadratically_with_linear_conductivity():
    m, P, _ = _small_problem(2)
    Tt = P.T_tab[0]
    P.kappa_tab = np.stack([20.0 * (1.0 + 1.5e-3 * (Tt - 300.0))] * 3)   # linear in T: a smooth kappa
    res = thermal.newton(P, np.full(m.n_nodes, 400.0), lambda J, r, k: (spla.spsolve(J.tocsc(), r), 1),
                         rtol=1e-13)
    h = np.array(res.res_history) / res.res_history[0]
    assert res.converged and res.iters <= 6
    # quadratic: e_{k+1} <= C e_k^2 once in the basin
    for k in range(1, len(h) - 1):
        if h[k] < 1e-2 and h[k + 1] > 1e-14:
            assert h[k + 1] <= 50.0 * h[k] ** 2


def test_newton_with_cg_and_classical_amg_matches_direct_newton():
    m, P, _ = _small_problem(2)
    T0 = np.full(m.n_nodes, 400.0)
    direct = thermal.newton(P, T0, lambda J, r, k: (spla.spsolve(J.tocsc(), r), 1))
    cache = {}

    def lin(J, r, k):
        if k == 0:
            cache["lev"] = camg.setup(J, camg.CAMGOptions(coarse_max=100, block=64))
        res = krylov.pcg(J, r, lambda v: camg.vcycle(cache["lev"], v, opt=camg.CAMGOptions(block=64)), rtol=1e-10)
        return res.u, res.iters
    it = thermal.newton(P, T0, lin)
    assert it.converged and direct.converged and len(cache["lev"]) >= 2
    assert np.linalg.norm(it.T - direct.T) <= 1e-9 * np.linalg.norm(direct.T)


# ---------------------------------------------------------------------------
# classical AMG
# ---------------------------------------------------------------------------

def _lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_strength_hand_worked():
    A = sp.csr_matrix(np.array([[4.0, -1.0, -0.2, 0.5],
                                [-1.0, 4.0, -1.0, 0.0],
                                [-0.2, -1.0, 4.0, -1.0],
                                [0.5, 0.0, -1.0, 4.0]]))
    S = camg.strength(A, 0.25)
    # row 0: max -a = 1 -> strong for -a >= 0.25: column 1 only (0.2 < 0.25; 0.5 positive)
    want = {(0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2)}
    rows = np.repeat(np.arange(4), np.diff(A.indptr))
    got = {(int(r), int(c)) for r, c, s in zip(rows, A.indices, S) if s}
    assert got == want


def _pmis_properties(A, S, level):
    """C points picked in one round are not strong neighbours (either
    direction); if i strongly depends on j and both are C, i was picked in an
    earlier round (else j's round would have made i an F point); every point
    made F in a round strongly depends on a C point of that round."""
    state, _, when = camg.pmis(A, S, level, with_rounds=True)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    C = state == camg.C_PT
    both = S & C[rows] & C[cols]
    assert np.all(when[rows[both]] < when[cols[both]])
    fr = (~C) & (when > 0)
    depC = np.zeros(n, bool)
    sel = S & C[cols] & (when[cols] == when[rows])
    depC[rows[sel]] = True
    assert np.all(depC[fr])
    return state


def test_pmis_on_a_path_hand_worked():
    """Path 0-1-2-3-4 (1D Laplacian, every neighbour strong, |S_i^T| = 1 at
    the ends and 2 inside): the keys order the inner points by their random
    bits; PMIS picks local maxima among undecided neighbours."""
    A = _lap1d(5)
    S = camg.strength(A)
    state, rounds = camg.pmis(A, S, 0)
    from oracle.rng import splitmix64
    infl = [1, 2, 2, 2, 1]
    key = [(infl[i], splitmix64((camg.KEY_SEED ^ i) & ((1 << 64) - 1)) >> 24, i) for i in range(5)]
    # replay the rounds by hand from the definition
    st = ["U"] * 5
    while "U" in st:
        newc = [i for i in range(5) if st[i] == "U" and
                all(not (st[j] == "U" and key[j] > key[i]) for j in (i - 1, i + 1) if 0 <= j < 5)]
        for i in newc:
            st[i] = "C"
        for i in range(5):
            if st[i] == "U" and any(j in newc for j in (i - 1, i + 1)):
                st[i] = "F"
    assert [("C" if s == camg.C_PT else "F") for s in state] == st
    _pmis_properties(A, S, 0)


def test_pmis_properties_on_random_and_mesh_graphs():
    rng = np.random.default_rng(3)
    for trial in range(5):
        n = 60
        M = sp.random(n, n, density=0.08, random_state=rng, data_rvs=lambda k: -rng.uniform(0.1, 1.0, k))
        M = (M + M.T).tocsr()
        A = (M + sp.diags(np.asarray(-M.sum(axis=1)).ravel() + 1.0)).tocsr()
        A.sort_indices()
        S = camg.strength(A)
        _pmis_properties(A, S, trial)
    m, P, _ = _small_problem(2)
    _, J = thermal.assemble(P, np.full(m.n_nodes, 500.0))
    _pmis_properties(J, camg.strength(J), 0)


def test_direct_interpolation_preserves_constants_for_zero_row_sums():
    """Without exchange with the exterior the conduction matrix has zero row
    sums; direct interpolation then reproduces constants on every F point
    with strong C neighbours, and C points inject."""
    m, P, _ = _small_problem(1, robin=False)
    _, J = thermal.assemble(P, np.full(m.n_nodes, 500.0))
    assert np.abs(np.asarray(J.sum(axis=1)).ravel()).max() <= 1e-12 * np.abs(J.data).max()
    S = camg.strength(J)
    state, _ = camg.pmis(J, S, 0)
    Pm = camg.direct_interpolation(J, S, state)
    rs = np.asarray(Pm.sum(axis=1)).ravel()
    has = np.diff(Pm.indptr) > 0
    assert np.all(np.abs(rs[has] - 1.0) <= 1e-12)
    C = state == camg.C_PT
    assert np.all(np.diff(Pm.indptr)[C] == 1) and np.all(Pm[C].toarray().max(axis=1) == 1.0)


def test_hybrid_gs_limits():
    rng = np.random.default_rng(1)
    A = _lap1d(40) + sp.diags(rng.uniform(0.1, 0.5, 40))
    A = A.tocsr()
    g = rng.standard_normal(40)
    x0 = rng.standard_normal(40)
    # one block holding every row: plain forward Gauss-Seidel
    lev = camg.CLevel(A=A)
    lev.A_in, lev.A_out, lev.dl1 = camg._split_blocks(A, 64)
    x = camg.hybrid_gs(lev, g, x0, 64, forward=True)
    L = sp.tril(A).tocsr()
    U = sp.triu(A, 1).tocsr()
    ref = spla.spsolve_triangular(L, g - U @ x0, lower=True)
    assert np.abs(x - ref).max() <= 1e-13 * np.abs(ref).max()
    # blocks of one row: l1 Jacobi
    lev.A_in, lev.A_out, lev.dl1 = camg._split_blocks(A, 1)
    x = camg.hybrid_gs(lev, g, x0, 1, forward=False)
    d = A.diagonal() + (abs(A).sum(axis=1).A.ravel() - np.abs(A.diagonal()))
    assert np.abs(x - (x0 + (g - A @ x0) / d)).max() <= 1e-13


def test_vcycle_symmetric_and_single_level_exact():
    m, P, _ = _small_problem(2, robin=True)
    _, J = thermal.assemble(P, np.full(m.n_nodes, 500.0))   # uniform T: J symmetric (no slope term acts)
    Js = (0.5 * (J + J.T)).tocsr()
    opt = camg.CAMGOptions(coarse_max=80, block=32)
    lev = camg.setup(Js, opt)
    assert len(lev) >= 3
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(Js.shape[0]), rng.standard_normal(Js.shape[0])
    Mx, My = camg.vcycle(lev, x, opt=opt), camg.vcycle(lev, y, opt=opt)
    assert abs(y @ Mx - x @ My) <= 1e-11 * abs(y @ Mx)
    assert x @ Mx > 0
    one = camg.setup(Js, camg.CAMGOptions(coarse_max=10 ** 6))
    assert len(one) == 1
    z = camg.vcycle(one, x)
    assert np.abs(Js @ z - x).max() <= 1e-10 * np.abs(x).max()
