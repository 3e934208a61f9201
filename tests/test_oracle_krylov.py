"""Pins of the oracle's (flexible) preconditioned CG and of the end-to-end
oracle solve: library special cases, dense direct solves, monotonicity and the
behaviour the paper describes."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import amg, fem, krylov


def _system(prob):
    A, b, _, _ = fem.assemble_problem(prob)
    B = fem.rigid_body_modes(prob.mesh.coords, prob.mask)
    return A, b, B


def test_cg_without_preconditioner_equals_scipy_iterates():
    A, b, _ = _system(mg.cube_problem(3, 1))
    for k in (1, 3, 8):
        ours = krylov.pcg(A, b, None, rtol=1e-30, maxit=k)
        ref, _ = spla.cg(A, b, x0=np.zeros_like(b), rtol=1e-30, atol=0.0, maxiter=k)
        assert np.linalg.norm(ours.u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_pcg_energy_error_monotone_and_dense_solution():
    A, b, B = _system(mg.cube_problem(4, 2))
    lv = amg.setup(A, B, amg.AMGOptions(coarse_max=500))
    u_ex = np.linalg.solve(A.toarray(), b)
    errs = []
    for k in range(1, 12):
        r = krylov.pcg(A, b, lambda v: amg.vcycle(lv, v), rtol=1e-30, maxit=k)
        e = r.u - u_ex
        errs.append(float(e @ (A @ e)))
    assert all(e2 <= e1 * (1 + 1e-9) for e1, e2 in zip(errs, errs[1:]))
    res = krylov.pcg(A, b, lambda v: amg.vcycle(lv, v), rtol=1e-12)
    assert res.converged
    assert np.linalg.norm(res.u - u_ex) <= 1e-10 * np.linalg.norm(u_ex)


@pytest.mark.parametrize("deg,n", [(1, 3), (2, 2), (1, 4)])
def test_tiny_meshes_dense_direct_solve(deg, n):
    A, b, B = _system(mg.cube_problem(n, deg))
    u_ex = np.linalg.solve(A.toarray(), b)
    lv = amg.setup(A, B, amg.AMGOptions(coarse_max=60))
    res = krylov.pcg(A, b, lambda v: amg.vcycle(lv, v), rtol=1e-13)
    assert np.linalg.norm(res.u - u_ex) <= 1e-11 * np.linalg.norm(u_ex)


def test_flexible_cg_equals_pcg_with_fixed_preconditioner():
    A, b, B = _system(mg.cube_problem(6, 1))
    lv = amg.setup(A, B, amg.AMGOptions(coarse_max=300))
    M = lambda v: amg.vcycle(lv, v)  # noqa: E731
    r1 = krylov.pcg(A, b, M, rtol=1e-10)
    r2 = krylov.pcg(A, b, M, rtol=1e-10, flexible=True)
    assert r1.iters == r2.iters
    assert np.linalg.norm(r1.u - r2.u) <= 1e-9 * np.linalg.norm(r1.u)


def test_true_residual_stop_rule_and_zero_rhs():
    A, b, B = _system(mg.cube_problem(3, 1))
    res = krylov.pcg(A, b, None, rtol=1e-8)
    assert res.converged and res.relres_true <= 1e-8
    assert np.linalg.norm(b - A @ res.u) <= 1e-8 * np.linalg.norm(b)
    z = krylov.pcg(A, np.zeros_like(b), None)
    assert z.iters == 0 and np.all(z.u == 0)
    # an exact initial guess needs no iteration
    g = krylov.pcg(A, b, None, u0=np.linalg.solve(A.toarray(), b), rtol=1e-8)
    assert g.iters == 0


def test_indefinite_preconditioner_detected():
    A, b, B = _system(mg.cube_problem(3, 1))
    with pytest.raises(krylov.Breakdown):
        krylov.pcg(A, b, lambda r: -r, rtol=1e-8)


# ---------------------------------------------------------------------------
# Behaviour the paper describes (Sec. 2.1.2, 2.1.3, 5.1)
# ---------------------------------------------------------------------------

def test_unpreconditioned_cg_grows_with_refinement():
    its = []
    for n in (4, 8):
        A, b, _ = _system(mg.cube_problem(n, 1))
        its.append(krylov.pcg(A, b, None, rtol=1e-8, maxit=5000).iters)
    assert its[1] > 1.5 * its[0]


def test_amg_iterations_bounded_under_refinement():
    its = []
    for n in (4, 8, 12):
        A, b, B = _system(mg.cube_problem(n, 1))
        lv = amg.setup(A, B, amg.AMGOptions(coarse_max=200))
        its.append(krylov.pcg(A, b, lambda v, lv=lv: amg.vcycle(lv, v), rtol=1e-8).iters)
    assert max(its) <= 25
    assert its[-1] <= its[0] + 6


def test_translation_only_nullspace_is_worse():
    # Sec. 2.1.3: without the rotational modes SA-AMG degrades
    prob = mg.disc_problem(8, 34, 2, 1)
    A, b, B = _system(prob)
    full = amg.setup(A, B, amg.AMGOptions(coarse_max=300))
    # translations only: a 3-column near-nullspace hierarchy
    part = amg.setup(A, B[:, :3], amg.AMGOptions(coarse_max=300))
    it_full = krylov.pcg(A, b, lambda v: amg.vcycle(full, v), rtol=1e-8).iters
    it_part = krylov.pcg(A, b, lambda v: amg.vcycle(part, v), rtol=1e-8, maxit=2000).iters
    assert it_part > it_full


def test_underestimated_eigenvalue_breaks_cg():
    # Sec. 5.1: an underestimated lambda_max loses positive definiteness
    A, b, B = _system(mg.cube_problem(8, 2))
    lv = amg.setup(A, B, amg.AMGOptions(coarse_max=300))
    good = krylov.pcg(A, b, lambda v: amg.vcycle(lv, v), rtol=1e-8)
    for l in lv[:-1]:
        l.lam *= 0.3
    failed = False
    try:
        bad = krylov.pcg(A, b, lambda v: amg.vcycle(lv, v), rtol=1e-8, maxit=10 * good.iters)
        failed = (not bad.converged) or bad.iters > 2 * good.iters
    except krylov.Breakdown:
        failed = True
    assert failed


# ---------------------------------------------------------------------------
# block CG (O'Leary 1980) with orthonormalised search blocks
# ---------------------------------------------------------------------------

def _laplace1d(n):
    import scipy.sparse as sp
    return sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_block_cg_with_one_column_is_cg():
    """m = 1: the search block is the normalised CG direction, so the
    iterates are those of CG."""
    A = _laplace1d(60)
    rng = np.random.default_rng(3)
    b = rng.normal(size=60)
    M = lambda r: r / 2.0
    res = krylov.pcg(A, b, M, rtol=1e-10)
    blk = krylov.block_pcg(A, b[:, None], M, rtol=1e-10)
    assert blk.iters == res.iters
    assert np.abs(blk.U[:, 0] - res.u).max() <= 1e-10 * np.abs(res.u).max()


def test_block_cg_terminates_in_n_over_m_steps():
    """Finite termination: with m right-hand sides the shared Krylov space of
    an n x n SPD matrix is exhausted after ceil(n / m) steps."""
    n, m = 48, 8
    A = _laplace1d(n)
    rng = np.random.default_rng(5)
    B = rng.normal(size=(n, m))
    blk = krylov.block_pcg(A, B, rtol=1e-11, maxit=n // m)
    assert blk.iters <= n // m and all(blk.converged)
    X = np.linalg.solve(A.toarray(), B)
    assert np.abs(blk.U - X).max() <= 1e-9 * np.abs(X).max()


def test_block_cg_drops_dependent_directions():
    """Dependent right-hand sides (a multiple, a sum, a zero column) make the
    first block rank deficient: the dependent directions are dropped and every
    column is still solved."""
    A = _laplace1d(40)
    rng = np.random.default_rng(7)
    b0, b1 = rng.normal(size=40), rng.normal(size=40)
    B = np.stack([b0, 2.0 * b0, b0 + b1, b1, np.zeros(40)], axis=1)
    blk = krylov.block_pcg(A, B, lambda r: r / 2.0, rtol=1e-10)
    assert blk.ranks[0] == 2 and all(blk.converged)
    X = np.linalg.solve(A.toarray(), B)
    assert np.abs(blk.U - X).max() <= 1e-8 * np.abs(X).max()


def test_block_cg_with_amg_solves_the_disc_load_cases():
    """Twelve bump load cases on a small P1 disc with the oracle's AMG: every
    column meets the true residual, agrees with its direct solve to the
    accuracy the residual allows, and the shared Krylov space needs fewer
    steps than the slowest single solve."""
    prob = mg.disc_problem(8, 34, 2, 1, seed=0)
    m = prob.mesh
    A0, _ = fem.assemble(m.coords, m.cells, 1, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T)
    cols = []
    for s in range(1000, 1012):
        _, b = fem.assemble(m.coords, m.cells, 1, prob.E, prob.nu, prob.alpha, prob.T_ref,
                            mg.disc_temperature_bumps(m, s))
        cols.append(fem.apply_dirichlet(A0, b, prob.mask)[1])
    A, _ = fem.apply_dirichlet(A0, cols[0], prob.mask)
    B = np.stack(cols, axis=1)
    opt = amg.AMGOptions(coarse_max=300)
    levels = amg.setup(A, fem.rigid_body_modes(m.coords, prob.mask), opt)
    M = lambda r: amg.vcycle(levels, r, opt=opt)
    blk = krylov.block_pcg(A, B, M)
    assert all(blk.converged) and max(blk.relres_true) <= 1e-8
    X = spla.spsolve(A.tocsc(), B)
    assert np.abs(blk.U - X).max() <= 1e-6 * np.abs(X).max()
    single = max(krylov.pcg(A, B[:, j], M).iters for j in range(B.shape[1]))
    assert blk.iters < single
