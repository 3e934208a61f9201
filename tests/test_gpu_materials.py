"""GPU assembly with temperature-dependent materials and boundary pressure
(fe_assemble_thermoelastic_materials) against the oracle.

Tolerances as for the one-material assembly: each entry is a sum of at most 24
element contributions of a few float64 products, so two correct
implementations differ by a small multiple of eps * max|K| (bar 1e-13 max|A|,
1e-13 max|b|); the cell coefficients come from the same table interpolation
and Lame formulas, which adds a few ulps per cell.  At full size the rows of b
are bounded by their own summed magnitudes (cancellation between the thermal,
body-force and pressure terms)."""
import numpy as np
import pytest

import meshgen as mg
from oracle import fem
from tests.gpu_util import dev, matrix_to_host, problem_on_device, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _gpu(prob, mat, faces=None, p=None, u_bc=None):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    d = problem_on_device(prob)
    m = prob.mesh
    say("assemble_materials", prob.name, "N =", m.n_nodes, "faces", 0 if faces is None else len(faces))
    A, b = te.assemble_materials(d["coords"], d["cells"], m.degree, (mat.T, mat.E, mat.nu, mat.alpha),
                                 dev(mat.cell_material.astype(np.int32)), prob.T_ref, d["T"], f=d["f"],
                                 faces=None if faces is None else dev(faces.astype(np.int32)),
                                 face_p=None if p is None else dev(p, torch.float64), mask=d["mask"],
                                 u_bc=None if u_bc is None else dev(u_bc, torch.float64))
    return A, b


def _oracle(prob, mat, faces=None, p=None, u_bc=None):
    m = prob.mesh
    tab = fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha)
    A0, b0 = fem.assemble_materials(m.coords, m.cells, m.degree, mat.cell_material, tab, prob.T_ref, prob.T, prob.f,
                                    faces=faces, face_p=p)
    return fem.apply_dirichlet(A0, b0, prob.mask, u_bc)


def _compare(prob, mat, faces=None, p=None, u_bc=None):
    A, b = _gpu(prob, mat, faces, p, u_bc)
    rp, col, val = matrix_to_host(A)
    Ao, bo = _oracle(prob, mat, faces, p, u_bc)
    assert np.array_equal(rp, Ao.indptr) and np.array_equal(col, Ao.indices)
    assert np.abs(val - Ao.data).max() <= TOL * np.abs(Ao.data).max()
    assert np.abs(b.cpu().numpy() - bo).max() <= TOL * np.abs(bo).max()
    return A, b


@pytest.mark.parametrize("deg", [1, 2])
def test_disc_three_materials_with_pressure_match_oracle(deg):
    prob = mg.disc_problem(6, 26, 2, deg, seed=3)   # ragged node count, several kernel tiles
    faces, p = mg.disc_pressure_faces(prob.mesh)
    _compare(prob, mg.disc_materials(prob.mesh), faces, p)


def test_body_force_dirichlet_values_and_out_of_range_temperatures():
    """Temperatures below and above the tables (clamped), a body force,
    random constrained DOFs with prescribed values, pressure on every face."""
    prob = mg.cube_problem(4, 2)
    m = prob.mesh
    rng = np.random.default_rng(7)
    prob.T = 100.0 + 1200.0 * rng.random(m.n_nodes)
    prob.f = rng.normal(size=(m.n_nodes, 3)) * 1e3
    prob.mask = (rng.uniform(size=(m.n_nodes, 3)) < 0.15).astype(np.uint8)
    u_bc = rng.normal(size=(m.n_nodes, 3)) * 1e-3
    Tp, E, nu, al = mg.turbine_material_tables()
    cen = m.coords[m.cells[:, :4].astype(np.int64)].mean(axis=1)
    mat = mg.Materials(Tp, E / 1e11, nu, al, (cen[:, 2] > 0.5).astype(np.int32) + (cen[:, 0] > 0.5))
    faces = mg.boundary_faces(m)
    _compare(prob, mat, faces, rng.normal(size=len(faces)), u_bc)


def test_constant_tables_equal_the_one_material_assembly():
    """One material with constant tables gives the plain assembly bit for bit
    (same Lame constants, same kernels)."""
    import paper_1804_10060_amd as te
    prob = mg.disc_problem(5, 20, 2, 2, seed=1)
    m = prob.mesh
    mat = mg.Materials(np.array([[200.0, 1200.0]]), np.full((1, 2), prob.E), np.full((1, 2), prob.nu),
                       np.full((1, 2), prob.alpha), np.zeros(m.n_cells, np.int32))
    A1, b1 = _gpu(prob, mat)
    d = problem_on_device(prob)
    A0, b0 = te.assemble(d["coords"], d["cells"], 2, prob.E, prob.nu, prob.alpha, prob.T_ref, d["T"], mask=d["mask"])
    torch = torch_cuda()
    assert torch.equal(A1.val, A0.val) and torch.equal(b1, b0)


@pytest.mark.parametrize("deg", [1, 2])
def test_layered_bar_solve_reproduces_the_closed_form(deg):
    """Three layers with nu = 0 under end traction (oracle pin of the same
    closed form): GPU assembly + AMG solve to rtol 1e-8."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.cube_problem(6, deg)
    m = prob.mesh
    prob.T = np.full(m.n_nodes, 650.0)
    prob.T_ref = 650.0
    X = m.coords
    prob.mask = np.stack([X[:, k] < 1e-12 for k in range(3)], axis=1).astype(np.uint8)
    cen = X[m.cells[:, :4].astype(np.int64)].mean(axis=1)
    Tp = np.array([[300.0, 500.0, 800.0]] * 3)
    E = np.array([[3.0, 2.0, 1.0], [10.0, 8.0, 4.0], [1.0, 1.5, 3.0]])
    mat = mg.Materials(Tp, E, np.zeros((3, 3)), np.full((3, 3), 1e-3),
                       np.minimum(2, (3.0 * cen[:, 0]).astype(np.int64)).astype(np.int32))
    faces = mg.boundary_faces(m, lambda c: c[:, 0] > 1 - 1e-12)
    pval = 0.7
    A, b = _gpu(prob, mat, faces, np.full(len(faces), pval))
    d = problem_on_device(prob)
    h = te.AMG(A, d["coords"], d["mask"])
    u, rep = h.solve(b)
    assert rep.converged == [1]
    u = u.cpu().numpy().reshape(-1, 3)
    Eu = np.array([np.interp(650.0, Tp[k], E[k]) for k in range(3)])
    edges = np.array([0.0, 1 / 3, 2 / 3, 1.0])
    ux = sum(pval / Eu[k] * np.clip(X[:, 0] - edges[k], 0.0, edges[k + 1] - edges[k]) for k in range(3))
    err = max(np.abs(u[:, 0] - ux).max(), np.abs(u[:, 1:]).max())
    say(f"layered bar P{deg}: {rep.iters[0]} iterations, max error {err / np.abs(ux).max():.2e} of max u")
    assert err <= 1e-7 * np.abs(ux).max()


def test_invalid_material_inputs_rejected():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.cube_problem(2, 1)
    m = prob.mesh
    d = problem_on_device(prob)
    Tp, E, nu, al = mg.turbine_material_tables()
    good = np.zeros(m.n_cells, np.int32)

    def run(tables, cm, faces=None):
        return te.assemble_materials(d["coords"], d["cells"], 1, tables, dev(cm), 300.0, d["T"],
                                     faces=None if faces is None else dev(faces),
                                     face_p=None if faces is None else dev(np.ones(len(faces)), torch.float64))

    bad = good.copy()
    bad[5] = 3
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        run((Tp, E, nu, al), bad)
    Tbad = Tp.copy()
    Tbad[1, 2] = Tbad[1, 1]
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        run((Tbad, E, nu, al), good)
    nubad = nu.copy()
    nubad[0, 0] = 0.5
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        run((Tp, E, nubad, al), good)
    faces = mg.boundary_faces(m)
    faces[2, 1] = m.n_nodes + 3
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        run((Tp, E, nu, al), good, faces)


@pytest.mark.timeout(900)
def test_full_size_disc_p2_three_materials_with_pressure():
    """The 12,043,200-DOF P2 disc with hub, web and rim materials and the rim
    and top pressures: sampled rows assembled by the oracle (cells and faces
    touching them) against the GPU's, then a solve to rtol 1e-8 checked on the
    host with scipy."""
    import time
    import scipy.sparse as sp
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(*mg.DISC_P2_12M, seed=0)
    m = prob.mesh
    mat = mg.disc_materials(m)
    faces, p = mg.disc_pressure_faces(m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A, b = _gpu(prob, mat, faces, p)
    torch.cuda.synchronize()
    say(f"assembly with materials and pressure: {(time.perf_counter() - t0) * 1e3:.0f} ms ({len(faces)} faces)")
    rp, col, val = matrix_to_host(A)
    bh = b.cpu().numpy().reshape(-1, 3)
    tab = fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 12), faces[rng.integers(0, len(faces), 8), 3],
                                     [0, m.n_nodes - 1]]))
    ref = fem.assemble_rows_materials(m.coords, m.cells, 2, mat.cell_material, tab, prob.T_ref, prob.T, rows,
                                      faces=faces, face_p=p)
    mask = prob.mask.astype(bool)
    for r in rows.tolist():
        cols_o, blocks_o, b_o = ref[r]
        assert np.array_equal(col[rp[r]:rp[r + 1]], cols_o), f"row {r} pattern"
        blocks_o = blocks_o.copy()
        for k, cc in enumerate(cols_o.tolist()):
            for a in range(3):
                for q in range(3):
                    if mask[r, a] or mask[cc, q]:
                        blocks_o[k, a, q] = 1.0 if (cc == r and a == q) else 0.0
        g = val[rp[r]:rp[r + 1]]
        assert np.abs(g - blocks_o).max() <= TOL * np.abs(blocks_o).max(), f"row {r} blocks"
        b_o = np.where(mask[r], 0.0, b_o)
        # magnitude of the summed terms of this row's load (thermal, pressure)
        assert np.all(np.abs(bh[r] - b_o) <= 1e-12 * (np.abs(b_o) + np.abs(bh[r]).max() + 1e-300)), f"row {r} b"
    d = problem_on_device(prob)
    h = te.AMG(A, d["coords"], d["mask"])
    u, rep = h.solve(b)
    say(f"solve: {rep.iters[0]} iterations, {rep.time_ms:.1f} ms")
    assert rep.converged == [1]
    M = sp.bsr_matrix((val, col, rp), shape=(3 * A.n, 3 * A.n))
    bb = b.cpu().numpy()
    assert np.linalg.norm(bb - M @ u.cpu().numpy()) <= 1.0000001e-8 * np.linalg.norm(bb)
