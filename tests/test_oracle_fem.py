"""Pins of the oracle's finite-element assembly against things other than
itself: closed forms, invariants, textbook formulas and exact solutions."""
import itertools

import numpy as np
import pytest

import meshgen as mg
from oracle import fem
from tests.conftest import read_golden


# ---------------------------------------------------------------------------
# Inputs and identities
# ---------------------------------------------------------------------------

def test_paper_dof_identities():
    rows = read_golden("paper_dof_identities.txt")
    for r in rows:
        if len(r) == 2:
            assert 3 * int(r[0]) == int(r[1])
        else:
            assert int(r[0]) * 8 ** int(r[1]) == int(r[2])


def test_p2_nodes_equal_p1_nodes_of_doubled_grid():
    # P2 on a mesh has the DOF count of P1 on the once-refined mesh (Sec. 5.2.1)
    for n in (2, 3):
        assert mg.cube_mesh(n, 2).n_nodes == mg.cube_mesh(2 * n, 1).n_nodes
    assert mg.disc_mesh(3, 10, 2, 2).n_nodes == mg.disc_mesh(6, 20, 4, 1).n_nodes


def test_workload_sizes():
    m = mg.cube_mesh(16, 1)
    assert (m.n_nodes, m.n_cells, m.n_dof) == (4913, 24576, 14739)
    row_ptr, cols = fem.sparsity(m.cells, m.n_nodes)
    assert cols.size == 66961
    assert int(mg.cube_clamp_x0(m)[:, 0].sum()) == 289
    nr, nth, nz, d = mg.DISC_P2_12M
    assert (2 * nr + 1) * (2 * nth) * (2 * nz + 1) == 4_014_400
    assert nr * nth * nz * 6 == 2_875_392


def test_cells_positively_oriented_and_volume():
    for m, vol in [(mg.cube_mesh(3, 2), 1.0), (mg.cube_mesh(4, 1), 1.0)]:
        v, _ = fem.cell_geometry(m.coords, m.cells.astype(np.int64))
        x = m.coords[m.cells[:, :4]]
        det = np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 2))
        assert det.min() > 0
        assert abs(v.sum() - vol) < 1e-13
    # disc volume converges to the annulus volume pi (ro^2 - ri^2) t from below
    m = mg.disc_mesh(4, 64, 2, 1)
    v, _ = fem.cell_geometry(m.coords, m.cells.astype(np.int64))
    exact = np.pi * (0.5 ** 2 - 0.1 ** 2) * 0.05
    assert 0 < exact - v.sum() < 2e-3 * exact


# ---------------------------------------------------------------------------
# Reference tables
# ---------------------------------------------------------------------------

def test_lame_constants_closed_form():
    lam, mu = fem.lame(1.0, 0.3)
    assert abs(lam - 0.3 / (1.3 * 0.4)) < 1e-15 and abs(mu - 1 / 2.6) < 1e-15
    assert abs(3 * lam + 2 * mu - 2.5) < 1e-14          # = E / (1 - 2 nu)
    lam, mu = fem.lame(200e9, 0.3)
    assert abs((3 * lam + 2 * mu) * 1.2e-5 - 6.0e6) < 1e-3


def test_p2_mass_matrix_matches_textbook():
    ref = np.array(read_golden("p2_tet_mass_420.txt"), dtype=float)
    _, _, M = fem.reference_tables(2)
    assert np.abs(M * 420 - ref).max() < 1e-12


def test_p1_mass_matrix_closed_form():
    _, _, M = fem.reference_tables(1)
    assert np.abs(M - (np.ones((4, 4)) + np.eye(4)) / 20).max() < 1e-15


def test_reference_gradient_tables_partition_of_unity():
    # sum_a phi_a = 1 => sum_a dphi_a/dl_k = 0 after projecting out the
    # constraint sum_k l_k = 1; in the integrated form sum_c W[c,a,k] over
    # nodes c of phi_c = 1 gives int dphi_a/dl_k.
    for deg in (1, 2):
        S, W, M = fem.reference_tables(deg)
        assert abs(M.sum() - 1) < 1e-14
        intd = W.sum(axis=0)  # [a,k] = int dphi_a/dl_k / |K|
        # P1: dphi_a/dl_k = delta_ak; P2 vertex: (4 l_a - 1) -> 0; edge: 4 l_b -> 1
        if deg == 1:
            assert np.abs(intd - np.eye(4)).max() < 1e-15
        else:
            assert np.abs(intd[:4]).max() < 1e-15
            for e, (a, b) in enumerate(fem.EDGES):
                row = np.zeros(4)
                row[a] = row[b] = 1.0
                assert np.abs(intd[4 + e] - row).max() < 1e-15


# ---------------------------------------------------------------------------
# Element matrices
# ---------------------------------------------------------------------------

def _rand_tet(seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(4, 3))
    if np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], 1)) < 0:
        x[[1, 2]] = x[[2, 1]]
    return x


def _p2_nodes(x):
    return np.vstack([x] + [0.5 * (x[a] + x[b]) for a, b in fem.EDGES])


@pytest.mark.parametrize("deg", [1, 2])
def test_element_stiffness_spectrum_and_rbm(deg):
    x = _rand_tet(3)
    coords = x if deg == 1 else _p2_nodes(x)
    cells = np.arange(coords.shape[0])[None, :]
    vol, G = fem.cell_geometry(coords, cells)
    K = fem.element_stiffness(vol, G, 0.7, 0.45, deg)[0].reshape(3 * coords.shape[0], -1)
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    w = np.linalg.eigvalsh(K)
    assert (np.abs(w) < 1e-12 * w.max()).sum() == 6
    assert w[6] > 1e-8 * w.max()
    B = fem.rigid_body_modes(coords)
    assert np.abs(K @ B).max() <= 1e-13 * np.abs(K).max() * np.abs(B).max()


def test_p1_element_stiffness_equals_voigt_btcb():
    # Constant-strain tetrahedron: K = vol B^T C B in Voigt notation
    x = _rand_tet(11)
    E, nu = 3.0, 0.27
    lam, mu = fem.lame(E, nu)
    vol, G = fem.cell_geometry(x, np.arange(4)[None, :])
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[:3, :3] += 2 * mu * np.eye(3)
    C[3:, 3:] = mu * np.eye(3)
    Bv = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = G[0, a]
        # strains (xx, yy, zz, 2yz, 2xz, 2xy)
        Bv[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz], [0, gz, gy], [gz, 0, gx], [gy, gx, 0]]
    Kv = vol[0] * Bv.T @ C @ Bv
    K = fem.element_stiffness(vol, G, lam, mu, 1)[0].reshape(12, 12)
    assert np.abs(K - Kv).max() <= 1e-13 * np.abs(Kv).max()


def test_p2_element_stiffness_equals_quadrature():
    # degree-2 integrand: the 4-point rule (a, b, b, b) is exact
    x = _rand_tet(5)
    coords = _p2_nodes(x)
    vol, G = fem.cell_geometry(coords, np.arange(10)[None, :])
    lam, mu = 1.3, 0.8
    K = fem.element_stiffness(vol, G, lam, mu, 2)[0].reshape(30, 30)
    a, b = 0.5854101966249685, 0.1381966011250105
    Kq = np.zeros((30, 30))
    for q in range(4):
        l = np.full(4, b)
        l[q] = a
        # gradients of the P2 basis at l
        dl = np.zeros((10, 4))
        for v in range(4):
            dl[v, v] = 4 * l[v] - 1
        for e, (i, j) in enumerate(fem.EDGES):
            dl[4 + e, i] = 4 * l[j]
            dl[4 + e, j] = 4 * l[i]
        gp = dl @ G[0]  # [10,3]
        for A_, B_ in itertools.product(range(10), range(10)):
            blk = lam * np.outer(gp[A_], gp[B_]) + mu * np.outer(gp[B_], gp[A_]) + mu * (gp[A_] @ gp[B_]) * np.eye(3)
            Kq[3 * A_:3 * A_ + 3, 3 * B_:3 * B_ + 3] += vol[0] / 4 * blk
    assert np.abs(K - Kq).max() <= 1e-13 * np.abs(K).max()


# ---------------------------------------------------------------------------
# Global system
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("deg,n", [(1, 3), (2, 2)])
def test_global_stiffness_rbm_nullspace_and_symmetry(deg, n):
    m = mg.cube_mesh(n, deg)
    T = 300 + np.random.default_rng(0).uniform(0, 50, m.n_nodes)
    A, b = fem.assemble(m.coords, m.cells, deg, 1.0, 0.3, 1e-3, 300.0, T)
    K = A.toarray()
    B = fem.rigid_body_modes(m.coords)
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K @ B).max() <= 1e-13 * np.abs(K).max() * np.abs(B).max()
    w = np.linalg.eigvalsh(K)
    assert (np.abs(w) < 1e-11 * w.max()).sum() == 6
    # thermal load is self-equilibrated: orthogonal to every rigid-body mode
    assert np.abs(b.reshape(-1) @ B).max() <= 1e-13 * np.abs(b).sum() * np.abs(B).max()


@pytest.mark.parametrize("deg", [1, 2])
def test_constant_body_force_total(deg):
    m = mg.cube_mesh(2, deg)
    f = np.tile([1.5, -2.0, 0.25], (m.n_nodes, 1))
    _, b = fem.assemble(m.coords, m.cells, deg, 1.0, 0.3, 0.0, 300.0, np.full(m.n_nodes, 300.0), f)
    assert np.abs(b.sum(axis=0) - np.array([1.5, -2.0, 0.25])).max() < 1e-13


def _solve_dense_dirichlet(A, b, mask, u_bc):
    """Independent path: partitioned solve K_ff u_f = b_f - K_fD u_D."""
    K = A.toarray()
    m = mask.reshape(-1).astype(bool)
    u = np.zeros(K.shape[0])
    u[m] = u_bc.reshape(-1)[m]
    rhs = b.reshape(-1)[~m] - K[np.ix_(~m, m)] @ u[m]
    u[~m] = np.linalg.solve(K[np.ix_(~m, ~m)], rhs)
    return u


def _three_two_one(m):
    """Six DOFs that remove rigid motion: all of the corner x0, two of x1, one of x2."""
    c = m.coords
    i0 = int(np.argmin(np.linalg.norm(c - c.min(axis=0), axis=1)))
    far = c[i0] + np.array([1.0, 0, 0])
    i1 = int(np.argmin(np.linalg.norm(c - far, axis=1)))
    i2 = int(np.argmin(np.linalg.norm(c - (c[i0] + np.array([0, 1.0, 0])), axis=1)))
    mask = np.zeros((m.n_nodes, 3), np.uint8)
    mask[i0] = 1
    mask[i1, 1:] = 1
    mask[i2, 2] = 1
    return mask, c[i0]


@pytest.mark.parametrize("deg", [1, 2])
def test_free_body_uniform_heating_closed_form(deg):
    """Uniform dT on an unconstrained body: u = alpha dT (x - x0) + rigid, zero
    stress.  Prescribing the exact values at 3-2-1 supports gives it at every node."""
    m = mg.cube_mesh(3, deg) if deg == 1 else mg.cube_mesh(2, deg)
    alpha, dT = 1e-3, 7.0
    A0, b0 = fem.assemble(m.coords, m.cells, deg, 1.0, 0.3, alpha, 300.0, np.full(m.n_nodes, 300.0 + dT))
    mask, x0 = _three_two_one(m)
    u_ex = alpha * dT * (m.coords - x0)
    A, b = fem.apply_dirichlet(A0, b0, mask, u_ex)
    u = np.linalg.solve(A.toarray(), b)
    assert np.abs(u - u_ex.reshape(-1)).max() <= 1e-10 * np.abs(u_ex).max()
    # independent partitioned solve agrees (checks the elimination)
    u2 = _solve_dense_dirichlet(A0, b0, mask, u_ex)
    assert np.abs(u - u2).max() <= 1e-10 * np.abs(u_ex).max()
    _, sig = fem.cell_strain_stress(m.coords, m.cells, deg, u, 1.0, 0.3, alpha, 300.0,
                                    np.full(m.n_nodes, 300.0 + dT), [np.full(4, 0.25)])
    assert np.abs(sig).max() <= 1e-9 * (2.5 * alpha * dT)


def test_free_body_linear_temperature_p2_closed_form():
    """T = T_ref + dT0 + g.x: u = alpha[(dT0 + g.x) x - |x|^2 g / 2] + rigid has
    eps(u) = alpha dT I, so zero stress; u is quadratic, so exact in P2."""
    m = mg.cube_mesh(2, 2)
    alpha, dT0, g = 2e-3, 3.0, np.array([1.0, -2.0, 0.5])
    x = m.coords
    dT = dT0 + x @ g
    u_ex = alpha * (dT[:, None] * x - 0.5 * (x * x).sum(1)[:, None] * g[None, :])
    A0, b0 = fem.assemble(x, m.cells, 2, 1.0, 0.3, alpha, 300.0, 300.0 + dT)
    mask, _ = _three_two_one(m)
    A, b = fem.apply_dirichlet(A0, b0, mask, u_ex)
    u = np.linalg.solve(A.toarray(), b)
    assert np.abs(u - u_ex.reshape(-1)).max() <= 1e-10 * np.abs(u_ex).max()
    pts = [np.array([0.1, 0.2, 0.3, 0.4]), np.full(4, 0.25)]
    eps, sig = fem.cell_strain_stress(x, m.cells, 2, u, 1.0, 0.3, alpha, 300.0, 300.0 + dT, pts)
    assert np.abs(sig).max() <= 1e-8 * 2.5 * alpha * np.abs(dT).max()


@pytest.mark.parametrize("deg,thermal", [(1, False), (2, False), (1, True), (2, True)])
def test_patch_test(deg, thermal):
    """Linear displacement imposed on the boundary: the interior is exact."""
    m = mg.cube_mesh(3, deg) if deg == 1 else mg.cube_mesh(2, deg)
    rng = np.random.default_rng(4)
    Gm = rng.normal(size=(3, 3)) * 1e-2
    c = rng.normal(size=3) * 1e-2
    alpha, dT = (1e-3, 5.0) if thermal else (0.0, 0.0)
    u_ex = m.coords @ (Gm + alpha * dT * np.eye(3)).T + c
    gi = m.grid_index
    top = gi.max()
    on_bnd = (gi == 0).any(1) | (gi == top).any(1)
    mask = mg.clamp_mask(m, on_bnd)
    A0, b0 = fem.assemble(m.coords, m.cells, deg, 2.0, 0.25, alpha, 300.0, np.full(m.n_nodes, 300.0 + dT))
    A, b = fem.apply_dirichlet(A0, b0, mask, u_ex)
    u = np.linalg.solve(A.toarray(), b)
    assert np.abs(u - u_ex.reshape(-1)).max() <= 1e-10 * np.abs(u_ex).max()


def test_dirichlet_elimination_structure():
    prob = mg.cube_problem(3, 1)
    A, b, A0, b0 = fem.assemble_problem(prob)
    K = A.toarray()
    m = prob.mask.reshape(-1).astype(bool)
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.all(K[m][:, m] == np.eye(m.sum()))
    assert np.all(K[m][:, ~m] == 0) and np.all(K[~m][:, m] == 0)
    assert np.all(b[m] == 0)
    assert np.linalg.eigvalsh(K).min() > 0


def test_assemble_rows_matches_full_assembly():
    prob = mg.disc_problem(3, 12, 2, 2, seed=1)
    m = prob.mesh
    A, b = fem.assemble(m.coords, m.cells, 2, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T)
    rows = [0, 7, 100, m.n_nodes - 1]
    got = fem.assemble_rows(m.coords, m.cells, 2, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T, rows)
    for r in rows:
        cols, blocks, brow = got[r]
        sl = slice(A.indptr[r], A.indptr[r + 1])
        assert np.array_equal(cols, A.indices[sl])
        assert np.abs(blocks - A.data[sl]).max() <= 1e-13 * np.abs(A.data).max()
        assert np.abs(brow - b[r]).max() <= 1e-13 * np.abs(b).max()


def test_rigid_body_modes_definition():
    c = np.array([[0.0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]])
    B = fem.rigid_body_modes(c).reshape(4, 3, 6)
    xc = c.mean(0)
    w = np.array([0.3, -0.2, 0.7])
    # a rotation about the centroid: omega x (x - xc); our columns 3..5 are the
    # rotations about z, x and y with omega = e_z, e_x, e_y respectively
    for col, axis in [(3, 2), (4, 0), (5, 1)]:
        om = np.zeros(3)
        om[axis] = 1.0
        assert np.abs(B[:, :, col] - np.cross(om, c - xc)).max() < 1e-15
    assert np.abs(B[:, :, :3] - np.eye(3)[None]).max() == 0
    mask = np.zeros((4, 3), np.uint8)
    mask[2, 1] = 1
    Bm = fem.rigid_body_modes(c, mask).reshape(4, 3, 6)
    assert np.all(Bm[2, 1] == 0) and np.any(Bm[2, 0] != 0)
    del w
