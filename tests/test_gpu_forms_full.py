"""The batching forms at the sizes the form benchmarks time.

* 64 seeded bump load cases on the 1,993,320-DOF P1 disc as one block solve
  (64 CG recurrences sharing the products, then block CG);
* 32 P1 discs of 14,400 to 534,276 DOF in one multi-mesh solve.

Bar: every column / mesh meets the true relative residual 1e-8, recomputed on
the host with scipy from the assembled system (not by the library); each
sampled column or mesh equals its standalone float64 solve to the rounding of
the reduction order (1e-10, or 1e-6 when the stop lands one iteration apart);
and for the block solve, sampled rows assembled by the oracle itself confirm a
column's solution, as in the full-size single solve."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _host_matrix(A):
    rp, col, val = A.row_ptr.cpu().numpy(), A.col_idx.cpu().numpy(), A.val.cpu().numpy()
    return sp.bsr_matrix((val, col, rp), shape=(3 * A.n, 3 * A.n)).tocsr()


def _close(u, v, same_iters):
    return np.linalg.norm(u - v) <= (1e-10 if same_iters else 1e-6) * np.linalg.norm(v)


@pytest.mark.timeout(900)
def test_block_rhs_64_cases_on_the_2m_dof_disc():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    nr, nth, nz, deg = mg.DISC_P1_2M
    prob = mg.disc_problem(nr, nth, nz, deg, seed=0)
    m = prob.mesh
    A, _, d = gpu_assemble(prob)
    seeds = list(range(1000, 1064))
    Ts = np.stack([mg.disc_temperature_bumps(m, s) for s in seeds])
    B = te.assemble_load(d["coords"], d["cells"], deg, prob.E, prob.nu, prob.alpha, prob.T_ref,
                         dev(Ts, torch.float64), mask=d["mask"])
    say("setup 2M-DOF P1 disc, 64 right-hand sides")
    h = te.AMG(A, d["coords"], d["mask"], max_nrhs=64)
    U, rep = h.solve(B)
    say(f"block solve: iterations {min(rep.iters)}..{max(rep.iters)}, {rep.time_ms:.1f} ms")
    assert all(rep.converged)
    M = _host_matrix(A)
    Bh = B.cpu().numpy()
    Uh = U.cpu().numpy()
    for j in range(64):
        bj, uj = Bh[:, :, j].reshape(-1), Uh[:, :, j].reshape(-1)
        assert np.linalg.norm(bj - M @ uj) <= 1.0000001e-8 * np.linalg.norm(bj), f"column {j}"
    for j in (0, 37, 63):
        bj = B[:, :, j].reshape(-1).contiguous()
        u1, r1 = h.solve(bj)
        assert abs(r1.iters[0] - rep.iters[j]) <= 1
        assert _close(Uh[:, :, j].reshape(-1), u1.cpu().numpy(), r1.iters[0] == rep.iters[j]), f"column {j}"
    # column 37 against rows assembled by the oracle from its own temperature field
    from oracle import fem
    j = 37
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 16), [0, m.n_nodes - 1]]))
    ref = fem.assemble_rows(m.coords, m.cells, deg, prob.E, prob.nu, prob.alpha, prob.T_ref, Ts[j], rows)
    mask = prob.mask.astype(bool)
    u3 = Uh[:, :, j]
    bnorm = np.linalg.norm(Bh[:, :, j])
    for r in rows.tolist():
        cols_o, blocks_o, b_o = ref[r]
        blocks_o = blocks_o.copy()
        for k, cc in enumerate(cols_o.tolist()):
            for p in range(3):
                for q in range(3):
                    if mask[r, p] or mask[cc, q]:
                        blocks_o[k, p, q] = 1.0 if (cc == r and p == q) else 0.0
        b_o = np.where(mask[r], 0.0, b_o)
        Au = np.einsum("kpq,kq->p", blocks_o, u3[cols_o])
        scale = np.einsum("kpq,kq->p", np.abs(blocks_o), np.abs(u3[cols_o])) + np.abs(b_o)
        assert np.all(np.abs(b_o - Au) <= 1e-8 * bnorm + 1e-13 * scale), f"row {r}"
    # the same 64 columns by block CG: one shared Krylov space
    Ub, repb = h.solve(B, block=True)
    say(f"block CG: {repb.iters[0]} iterations, {repb.time_ms:.1f} ms")
    assert all(repb.converged) and repb.iters[0] < max(rep.iters)
    Ubh = Ub.cpu().numpy()
    for j in range(64):
        bj, uj = Bh[:, :, j].reshape(-1), Ubh[:, :, j].reshape(-1)
        assert np.linalg.norm(bj - M @ uj) <= 1.0000001e-8 * np.linalg.norm(bj), f"block CG column {j}"


@pytest.mark.timeout(900)
def test_multi_mesh_32_discs():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    hs, bs, mats = [], [], []
    for (nr, nth, nz, seed) in mg.multi_mesh_sizes(32, lo=1e4, hi=5e5):
        prob = mg.disc_problem(nr, nth, nz, 1, seed=0)
        prob.T = mg.disc_temperature_bumps(prob.mesh, seed)
        A, b, d = gpu_assemble(prob)
        hs.append(te.AMG(A, d["coords"], d["mask"]))
        bs.append(b)
        mats.append(_host_matrix(A))
    say("multi-mesh solve of", len(hs), "discs")
    us, rep = te.solve_multi(hs, bs)
    assert all(rep["converged"])
    for i, (h, b, u, M) in enumerate(zip(hs, bs, us, mats)):
        bh, uh = b.cpu().numpy(), u.cpu().numpy()
        assert np.linalg.norm(bh - M @ uh) <= 1.0000001e-8 * np.linalg.norm(bh), f"mesh {i}"
        u1, r1 = h.solve(b)
        assert abs(r1.iters[0] - rep["iters"][i]) <= 1
        assert _close(uh, u1.cpu().numpy(), r1.iters[0] == rep["iters"][i]), f"mesh {i}"
    say("iterations", rep["iters"])
