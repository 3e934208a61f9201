"""Pins of the oracle's temperature-dependent multi-material assembly and
boundary pressure (Sec. 3: C and alpha_L depend on T; wf_elastic's term
int p_bc n . v ds on Gamma_N).  Each pin holds by the mathematics, not by
retyping the oracle: closed forms of elastic states that the P1/P2 spaces
contain exactly, exact integrals of the face basis, the exact mean of a
quadratic over a tetrahedron, and special cases that reduce to the
single-material assembly."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import fem


def _solve(A, b, mask, u_bc=None):
    Ad, bd = fem.apply_dirichlet(A, b, mask, u_bc)
    return spla.spsolve(Ad.tocsc(), bd).reshape(-1, 3)


def _faces(mesh, pred):
    return mg.boundary_faces(mesh, pred)


def test_face_basis_integrals_closed_form():
    # P1: each hat function integrates to |F|/3; P2: the vertex functions
    # l(2l - 1) integrate to zero and the edge functions 4 l_a l_b to |F|/3
    assert np.allclose(fem.face_basis_integrals(1), [1 / 3] * 3, rtol=0, atol=1e-15)
    assert np.allclose(fem.face_basis_integrals(2), [0, 0, 0, 1 / 3, 1 / 3, 1 / 3], rtol=0, atol=1e-15)


@pytest.mark.parametrize("degree", [1, 2])
def test_pressure_resultant(degree):
    """A uniform pressure on a closed surface has zero resultant; on one face
    of the unit cube the resultant is p * area * n."""
    m = mg.cube_mesh(3, degree)
    allf = _faces(m, None)
    b = fem.pressure_load(m.coords, allf, degree, np.full(len(allf), 2.5))
    assert np.abs(b.sum(axis=0)).max() <= 1e-13
    top = _faces(m, lambda c: c[:, 2] > 1 - 1e-12)
    b = fem.pressure_load(m.coords, top, degree, np.full(len(top), -3.0))
    assert np.allclose(b.sum(axis=0), [0.0, 0.0, -3.0], rtol=0, atol=1e-13)
    # the moment about the face centre vanishes for a uniform pressure
    x = m.coords - np.array([0.5, 0.5, 1.0])
    assert np.abs(np.cross(x, b).sum(axis=0)).max() <= 1e-13


@pytest.mark.parametrize("degree", [1, 2])
def test_cell_mean_is_exact(degree):
    """Mean of the interpolant over a tetrahedron: T = x^2 is reproduced by P2,
    and its mean over a tetrahedron with vertices x_i is
    (sum_i x_i^2 + sum_{i<j} x_i x_j) / 10; a linear T (P1) has the vertex average."""
    rng = np.random.default_rng(4)
    m = mg.cube_mesh(2, degree)
    X = m.coords + 0.05 * rng.normal(size=m.coords.shape)   # interior distortion keeps cells valid
    cells = m.cells.astype(np.int64)
    xv = X[cells[:, :4], 0]
    if degree == 2:
        # midside nodes at the midpoints of the distorted straight edges
        Xm = X.copy()
        for k, (a, b) in enumerate(fem.EDGES):
            Xm[cells[:, 4 + k]] = 0.5 * (X[cells[:, a]] + X[cells[:, b]])
        T = Xm[:, 0] ** 2
        pair = sum(xv[:, i] * xv[:, j] for i in range(4) for j in range(i + 1, 4))
        exact = ((xv ** 2).sum(axis=1) + pair) / 10.0
    else:
        T = 3.0 * X[:, 0] - X[:, 1] + 7.0
        exact = T[cells].mean(axis=1)
    assert np.allclose(fem.cell_mean(T, cells, degree), exact, rtol=1e-13, atol=1e-13)


def test_constant_tables_reduce_to_one_material():
    m = mg.cube_mesh(3, 2)
    rng = np.random.default_rng(1)
    T = 300.0 + 50.0 * rng.random(m.n_nodes)
    Tp = np.array([[200.0, 900.0], [100.0, 1000.0]])
    tab = fem.MaterialTables(Tp, np.full((2, 2), 7.0), np.full((2, 2), 0.27), np.full((2, 2), 2e-3))
    cm = (np.arange(m.n_cells) % 2).astype(np.int32)
    A1, b1 = fem.assemble_materials(m.coords, m.cells, 2, cm, tab, 300.0, T)
    A0, b0 = fem.assemble(m.coords, m.cells, 2, 7.0, 0.27, 2e-3, 300.0, T)
    assert np.abs((A1 - A0).tocsr()).max() <= 1e-13 * np.abs(A0).max()
    assert np.abs(b1 - b0).max() <= 1e-13 * np.abs(b0).max()


@pytest.mark.parametrize("degree", [1, 2])
def test_layered_bar_under_end_traction(degree):
    """Layers x in [0,1/3), [1/3,2/3), [2/3,1] of three materials with nu = 0,
    E from their tables at the (uniform) temperature, traction p e_x on x = 1,
    symmetry planes x = 0, y = 0, z = 0: the exact solution
    u_x = p int_0^x ds / E(s), u_y = u_z = 0 is piecewise linear across the
    layer planes, so P1 and P2 reproduce it exactly."""
    m = mg.cube_mesh(6, degree)
    cen = m.coords[m.cells[:, :4].astype(np.int64)].mean(axis=1)
    cm = np.minimum(2, (3.0 * cen[:, 0]).astype(np.int64)).astype(np.int32)
    Tp = np.array([[300.0, 500.0, 800.0]] * 3)
    E = np.array([[3.0, 2.0, 1.0], [10.0, 8.0, 4.0], [1.0, 1.5, 3.0]])
    tab = fem.MaterialTables(Tp, E, np.zeros((3, 3)), np.full((3, 3), 1e-3))
    Tu = 650.0
    T = np.full(m.n_nodes, Tu)
    p = 0.7
    faces = _faces(m, lambda c: c[:, 0] > 1 - 1e-12)
    A, b = fem.assemble_materials(m.coords, m.cells, degree, cm, tab, Tu, T, faces=faces,
                                  face_p=np.full(len(faces), p))
    X = m.coords
    mask = np.zeros((m.n_nodes, 3), np.uint8)
    mask[:, 0] = X[:, 0] < 1e-12
    mask[:, 1] = X[:, 1] < 1e-12
    mask[:, 2] = X[:, 2] < 1e-12
    u = _solve(A, b, mask)
    Eu = np.array([np.interp(Tu, Tp[k], E[k]) for k in range(3)])
    edges = np.array([0.0, 1 / 3, 2 / 3, 1.0])
    ux = np.zeros(m.n_nodes)
    for k in range(3):
        ux += p / Eu[k] * np.clip(X[:, 0] - edges[k], 0.0, edges[k + 1] - edges[k])
    assert np.abs(u[:, 0] - ux).max() <= 1e-10 * np.abs(ux).max()
    assert np.abs(u[:, 1:]).max() <= 1e-10 * np.abs(ux).max()


@pytest.mark.parametrize("degree", [1, 2])
def test_hydrostatic_pressure_and_heating_of_a_free_cube(degree):
    """Uniform traction p n on the whole surface of the unit cube, heated
    uniformly from T_ref to T1, E, nu, alpha_L from temperature tables at
    T1: sigma = p I, so eps = (p / (3K) + alpha (T1 - T_ref)) I with
    K = E / (3 (1 - 2 nu)) and u = eps x about the corner held by the three
    symmetry planes."""
    m = mg.cube_mesh(4, degree)
    Tp = np.array([[250.0, 600.0, 1000.0]])
    E, nu, al = np.array([[5.0, 4.0, 2.0]]), np.array([[0.2, 0.3, 0.35]]), np.array([[1e-3, 2e-3, 4e-3]])
    tab = fem.MaterialTables(Tp, E, nu, al)
    T_ref, T1, p = 300.0, 700.0, -0.9
    T = np.full(m.n_nodes, T1)
    faces = _faces(m, None)
    cm = np.zeros(m.n_cells, np.int32)
    A, b = fem.assemble_materials(m.coords, m.cells, degree, cm, tab, T_ref, T, faces=faces,
                                  face_p=np.full(len(faces), p))
    X = m.coords
    mask = np.stack([X[:, k] < 1e-12 for k in range(3)], axis=1).astype(np.uint8)
    u = _solve(A, b, mask)
    E1, nu1, a1 = (np.interp(T1, Tp[0], v[0]) for v in (E, nu, al))
    eps = p / (E1 / (1 - 2 * nu1)) + a1 * (T1 - T_ref)
    assert np.abs(u - eps * X).max() <= 1e-10 * abs(eps)


def test_multi_material_operator_keeps_symmetry_and_rigid_modes():
    m = mg.disc_mesh(3, 12, 2, 2)
    mat = mg.disc_materials(m)
    rng = np.random.default_rng(2)
    T = 300.0 + 600.0 * rng.random(m.n_nodes)
    A, _ = fem.assemble_materials(m.coords, m.cells, 2, mat.cell_material,
                                  fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha), 300.0, T)
    A = A.tocsr()
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    B = fem.rigid_body_modes(m.coords)
    assert np.abs(A @ B).max() <= 1e-9 * abs(A).max()


def test_tables_clamp_beyond_their_ends():
    Tp = np.array([[400.0, 600.0]])
    tab = fem.MaterialTables(Tp, np.array([[2.0, 1.0]]), np.array([[0.25, 0.25]]), np.array([[1e-3, 3e-3]]))
    m = mg.cube_mesh(1, 1)
    for Tv, Ee, ae in ((100.0, 2.0, 1e-3), (500.0, 1.5, 2e-3), (5000.0, 1.0, 3e-3)):
        E, nu, a = fem.cell_coefficients(np.full(m.n_nodes, Tv), m.cells.astype(np.int64), 1,
                                         np.zeros(m.n_cells, np.int32), tab)
        assert np.allclose(E, Ee) and np.allclose(a, ae) and np.allclose(nu, 0.25)


def test_sampled_rows_equal_the_full_assembly():
    m = mg.disc_mesh(3, 12, 2, 2)
    mat = mg.disc_materials(m)
    tab = fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha)
    T = mg.disc_temperature_ramp(m, 1)
    faces, p = mg.disc_pressure_faces(m)
    A, b = fem.assemble_materials(m.coords, m.cells, 2, mat.cell_material, tab, 300.0, T, faces=faces, face_p=p)
    A = A.tocsr()
    rows = np.array([0, 5, m.n_nodes // 2, m.n_nodes - 1] + list(np.unique(faces[:4, 3:].ravel())))
    got = fem.assemble_rows_materials(m.coords, m.cells, 2, mat.cell_material, tab, 300.0, T, rows, faces=faces,
                                      face_p=p)
    for r in rows.tolist():
        cols, blocks, brow = got[r]
        for k, c in enumerate(cols.tolist()):
            ref = A[3 * r:3 * r + 3, 3 * c:3 * c + 3].toarray()
            assert np.allclose(blocks[k], ref, rtol=0, atol=1e-12 * abs(A).max())
        assert np.allclose(brow, b[r], rtol=0, atol=1e-12 * np.abs(b).max())
