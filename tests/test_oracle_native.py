"""Pins of the C++ oracle (oracle/native): element by element against the
NumPy oracle at small sizes (same aggregates at every level, operators,
eigenvalue estimates, V-cycle and CG iterates), and the closed forms that pin
the NumPy oracle, run against the C++ one directly."""
import numpy as np
import pytest

import meshgen as mg
from oracle import amg, fem, krylov, native
from tests.test_oracle_fem import _three_two_one


def _rel(a, b):
    a = a.toarray() if hasattr(a, "toarray") else a
    b = b.toarray() if hasattr(b, "toarray") else b
    return float(np.abs(a - b).max() / max(np.abs(a).max(), 1e-300))


CASES = [("cube4_p1", lambda: mg.cube_problem(4, 1), 50), ("cube3_p2", lambda: mg.cube_problem(3, 2), 100),
         ("disc8x34x2_p2", lambda: mg.disc_problem(8, 34, 2, 2, seed=3), 3000)]


@pytest.mark.parametrize("name,make,cmax", CASES)
@pytest.mark.parametrize("rule", ["mis2", "greedy"])
def test_native_equals_numpy_oracle(name, make, cmax, rule):
    prob = make()
    A, b, _, _ = fem.assemble_problem(prob)
    S = native.System.from_problem(prob)
    assert _rel(A, S.matrix()) <= 1e-13 and _rel(b, S.b()) <= 1e-13
    lev = amg.setup(A, fem.rigid_body_modes(prob.mesh.coords, prob.mask),
                    amg.AMGOptions(coarse_max=cmax, aggregation=rule))
    H = native.Hierarchy(S, coarse_max=cmax, aggregation=rule)
    assert len(H.levels) == len(lev) >= 2
    for l in range(len(lev) - 1):
        assert np.array_equal(H.aggregates(l), lev[l].agg), f"aggregates differ at level {l}"
        assert _rel(lev[l].P, H.P(l)) <= 1e-12
        assert _rel(lev[l].R, H.R(l)) <= 1e-12
        assert abs(H.levels[l].lam - lev[l].lam) <= 1e-12 * lev[l].lam
    for l in range(len(lev)):
        assert _rel(lev[l].A, H.A(l)) <= 1e-12
    r = np.random.default_rng(5).standard_normal(b.size)
    z0 = amg.vcycle(lev, r)
    assert np.abs(H.vcycle(r) - z0).max() <= 1e-11 * np.abs(z0).max()
    ro = krylov.pcg(A, b, lambda v: amg.vcycle(lev, v), rtol=1e-8)
    rn = H.pcg(S.b(), rtol=1e-8)
    assert rn.converged and rn.iters == ro.iters
    assert np.linalg.norm(rn.u - ro.u) <= 1e-10 * np.linalg.norm(ro.u)
    # flexible CG with a fixed preconditioner is CG (the FCG pin of the NumPy oracle)
    rf = H.pcg(S.b(), rtol=1e-8, flexible=True)
    assert rf.iters == rn.iters and np.linalg.norm(rf.u - rn.u) <= 1e-10 * np.linalg.norm(rn.u)


def test_native_thread_count_does_not_change_the_result():
    prob = mg.disc_problem(8, 34, 2, 2, seed=1)
    out = []
    for t in (1, 3):
        S = native.System.from_problem(prob, threads=t)
        H = native.Hierarchy(S, threads=t)
        out.append((S.b(), H.pcg(S.b()).u, [H.aggregates(l) for l in range(len(H.levels) - 1)]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert all(np.array_equal(a, b) for a, b in zip(out[0][2], out[1][2]))


@pytest.mark.parametrize("deg", [1, 2])
def test_native_rbm_nullspace_symmetry_and_equilibrium(deg):
    m = mg.cube_mesh(3 if deg == 1 else 2, deg)
    T = 300 + np.random.default_rng(0).uniform(0, 50, m.n_nodes)
    S = native.System(m.coords, m.cells, deg, 1.0, 0.3, 1e-3, 300.0, T)
    K = S.matrix().toarray()
    B = fem.rigid_body_modes(m.coords)
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K @ B).max() <= 1e-13 * np.abs(K).max() * np.abs(B).max()
    b = S.b()
    assert np.abs(b @ B).max() <= 1e-13 * np.abs(b).sum() * np.abs(B).max()
    # constant body force: the consistent load sums to f times the volume (1)
    f = np.tile([1.5, -2.0, 0.25], (m.n_nodes, 1))
    Sf = native.System(m.coords, m.cells, deg, 1.0, 0.3, 0.0, 300.0, np.full(m.n_nodes, 300.0), f)
    assert np.abs(Sf.b().reshape(-1, 3).sum(0) - [1.5, -2.0, 0.25]).max() < 1e-13


@pytest.mark.parametrize("deg", [1, 2])
def test_native_free_body_uniform_heating_closed_form(deg):
    """u = alpha dT (x - x0) at every node when the 3-2-1 supports carry it."""
    m = mg.cube_mesh(3, deg) if deg == 1 else mg.cube_mesh(2, deg)
    alpha, dT = 1e-3, 7.0
    mask, x0 = _three_two_one(m)
    u_ex = alpha * dT * (m.coords - x0)
    S = native.System(m.coords, m.cells, deg, 1.0, 0.3, alpha, 300.0, np.full(m.n_nodes, 300.0 + dT), mask=mask,
                      u_bc=u_ex)
    u = np.linalg.solve(S.matrix().toarray(), S.b())
    assert np.abs(u - u_ex.reshape(-1)).max() <= 1e-10 * np.abs(u_ex).max()


@pytest.mark.parametrize("deg", [1, 2])
def test_native_thermal_patch_test(deg):
    """u = (G + alpha dT I) x + c imposed on the boundary is exact inside."""
    m = mg.cube_mesh(3, deg) if deg == 1 else mg.cube_mesh(2, deg)
    rng = np.random.default_rng(4)
    Gm = rng.normal(size=(3, 3)) * 1e-2
    c = rng.normal(size=3) * 1e-2
    alpha, dT = 1e-3, 5.0
    u_ex = m.coords @ (Gm + alpha * dT * np.eye(3)).T + c
    gi = m.grid_index
    on_bnd = (gi == 0).any(1) | (gi == gi.max()).any(1)
    mask = mg.clamp_mask(m, on_bnd)
    S = native.System(m.coords, m.cells, deg, 2.0, 0.25, alpha, 300.0, np.full(m.n_nodes, 300.0 + dT), mask=mask,
                      u_bc=u_ex)
    u = np.linalg.solve(S.matrix().toarray(), S.b())
    assert np.abs(u - u_ex.reshape(-1)).max() <= 1e-10 * np.abs(u_ex).max()


def test_native_pcg_reaches_the_dense_solution():
    prob = mg.cube_problem(4, 2)
    S = native.System.from_problem(prob)
    H = native.Hierarchy(S, coarse_max=100)
    assert len(H.levels) >= 2
    r = H.pcg(S.b(), rtol=1e-12)
    u = np.linalg.solve(S.matrix().toarray(), S.b())
    assert r.converged and np.linalg.norm(r.u - u) <= 1e-10 * np.linalg.norm(u)
