"""GPU block CG over the columns of a multi-RHS solve (pcg_options.block)
against the oracle's block_pcg.

Both run O'Leary's block recurrence with the search block orthonormalised each
step; the oracle orthonormalises by an eigendecomposition of the Gram matrix
and the library by a pivoted Cholesky factor, which span the same space while
the block has full rank, so the iterates agree up to rounding.  Bar: the
iteration counts within one, every column's true residual <= 1e-8 recomputed
here from the oracle's matrix, and each column within 1e-8 (relative) of the
oracle's block solution, the bar of the single-solve parity test."""
import numpy as np
import pytest

import meshgen as mg
from oracle import amg, fem, krylov
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_system(prob, seeds):
    """Dirichlet-eliminated A and the bump load cases of `seeds` as columns."""
    m = prob.mesh
    A0, _ = fem.assemble(m.coords, m.cells, m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T)
    cols = []
    for s in seeds:
        _, b = fem.assemble(m.coords, m.cells, m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref,
                            mg.disc_temperature_bumps(m, s))
        cols.append(fem.apply_dirichlet(A0, b, prob.mask)[1])
    A, _ = fem.apply_dirichlet(A0, cols[0], prob.mask)
    return A, np.stack(cols, axis=1)


def _gpu_block(prob, B, coarse_max, **kw):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    A, _, d = gpu_assemble(prob)
    m = B.shape[1]
    say("amg_setup", prob.name, "nrhs", m)
    h = te.AMG(A, d["coords"], d["mask"], coarse_max=coarse_max, max_nrhs=max(m, 1))
    Bd = dev(np.ascontiguousarray(B.reshape(-1, 3, m)), torch.float64)
    say("block pcg", prob.name, "nrhs", m)
    U, rep = h.solve(Bd, block=True, **kw)
    return h, U.cpu().numpy().reshape(-1, m), rep


def _oracle_block(prob, A, B, coarse_max):
    opt = amg.AMGOptions(coarse_max=coarse_max)
    levels = amg.setup(A, fem.rigid_body_modes(prob.mesh.coords, prob.mask), opt)
    return krylov.block_pcg(A, B, lambda r: amg.vcycle(levels, r, opt=opt))


def _check(A, B, U, rep, blk):
    bn = np.linalg.norm(B, axis=0)
    rt = np.linalg.norm(B - A @ U, axis=0)
    assert np.all(rt <= 1.0000001e-8 * bn + 1e-300), rt / np.maximum(bn, 1e-300)
    assert all(rep.converged) and all(blk.converged)
    assert abs(rep.iters[0] - blk.iters) <= 1 and len(set(rep.iters)) == 1
    for j in range(B.shape[1]):
        un = np.linalg.norm(blk.U[:, j])
        assert np.linalg.norm(U[:, j] - blk.U[:, j]) <= 1e-8 * un + 1e-300, f"column {j}"


@pytest.mark.parametrize("deg", [1, 2])
def test_block_cg_matches_oracle_on_disc_load_cases(deg):
    prob = mg.disc_problem(8, 34, 2, deg, seed=0)
    A, B = _oracle_system(prob, range(1000, 1012))
    h, U, rep = _gpu_block(prob, B, 300)
    blk = _oracle_block(prob, A, B, 300)
    say(f"P{deg}: block CG iterations gpu {rep.iters[0]} oracle {blk.iters} (ranks {blk.ranks[:3]}...)")
    _check(A, B, U, rep, blk)
    # fewer steps than the slowest of the independent recurrences
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    _, rep1 = h.solve(dev(np.ascontiguousarray(B.reshape(-1, 3, B.shape[1])), torch.float64))
    assert rep.iters[0] < max(rep1.iters)


def test_dependent_zero_and_duplicate_columns():
    """Six independent load cases, then a zero column, a duplicate, and
    combinations of the first ones: the block loses rank at the start and the
    dependent directions are dropped; every column still meets the residual."""
    prob = mg.disc_problem(8, 34, 2, 1, seed=0)
    A, B6 = _oracle_system(prob, range(2000, 2006))
    rng = np.random.default_rng(3)
    extra = [np.zeros(B6.shape[0]), B6[:, 2].copy(), B6 @ rng.normal(size=6), B6[:, :2] @ np.array([1.0, -2.0])]
    B = np.concatenate([B6, np.stack(extra, axis=1)], axis=1)
    h, U, rep = _gpu_block(prob, B, 300)
    blk = _oracle_block(prob, A, B, 300)
    say(f"dependent columns: gpu {rep.iters[0]} oracle {blk.iters}, oracle ranks {blk.ranks[:3]}")
    assert blk.ranks[0] == 6
    assert np.all(U[:, 6] == 0.0)
    _check(A, B, U, rep, blk)


def test_ragged_column_count_and_the_two_pass_reductions():
    """Five columns (not a power of two) on a 19,680-node disc: more row
    workgroups than the one-pass reduction takes, Gram passes with a ragged
    tail of rows per workgroup; checked on the host against scipy."""
    import scipy.sparse as sp
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(40, 120, 3, 1, seed=1)
    m = prob.mesh
    A, _, d = gpu_assemble(prob)
    Ts = np.stack([mg.disc_temperature_bumps(m, s) for s in range(40, 45)])
    B = te.assemble_load(d["coords"], d["cells"], 1, prob.E, prob.nu, prob.alpha, prob.T_ref,
                         dev(Ts, torch.float64), mask=d["mask"])
    h = te.AMG(A, d["coords"], d["mask"], max_nrhs=8)
    U, rep = h.solve(B, block=True)
    U1, rep1 = h.solve(B)
    say(f"5 columns, {m.n_nodes} nodes: block CG {rep.iters[0]}, independent {rep1.iters}")
    assert all(rep.converged) and rep.iters[0] <= max(rep1.iters)
    M = sp.bsr_matrix((A.val.cpu().numpy(), A.col_idx.cpu().numpy(), A.row_ptr.cpu().numpy()),
                      shape=(3 * A.n, 3 * A.n)).tocsr()
    Bh, Uh = B.cpu().numpy().reshape(-1, 5), U.cpu().numpy().reshape(-1, 5)
    bn = np.linalg.norm(Bh, axis=0)
    assert np.all(np.linalg.norm(Bh - M @ Uh, axis=0) <= 1.0000001e-8 * bn)
    # both solutions solve the system to 1e-8, so they agree to what the
    # condition number lets the residual bound (loosely: 1e-5 relative)
    U1h = U1.cpu().numpy().reshape(-1, 5)
    assert np.all(np.linalg.norm(Uh - U1h, axis=0) <= 1e-5 * np.linalg.norm(U1h, axis=0))


def test_block_cg_edge_cases():
    """One column (the plain recurrence), a zero block, an exact initial
    guess, and block with mixed precision (rejected)."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 1, seed=2)
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"], max_nrhs=4)
    u1, r1 = h.solve(b, block=True)
    u0, r0 = h.solve(b)
    assert r1.iters == r0.iters and torch.equal(u1, u0)
    Z = torch.zeros((A.n, 3, 3), dtype=torch.float64, device=b.device)
    uz, rz = h.solve(Z, block=True)
    assert rz.iters == [0, 0, 0] and all(rz.converged) and torch.count_nonzero(uz) == 0
    B = torch.stack([b.reshape(-1, 3), 2 * b.reshape(-1, 3), -b.reshape(-1, 3)], dim=2).contiguous()
    U, rep = h.solve(B, block=True)
    assert all(rep.converged)
    U2, rep2 = h.solve(B, u0=U, block=True)
    assert rep2.iters == [0, 0, 0] and torch.equal(U2, U)
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        h.solve(B, block=True, precision="mixed")
