"""Multi-mesh solve (one persistent launch per phase, iteration replayed as a
HIP graph): every mesh gets its standalone solve.

Bar: the per-mesh recurrences are the standalone ones; only the reduction
order of dot products differs, so iterates agree to rounding (1e-10 relative
when the iteration counts agree; a stop one iteration apart differs by one CG
update, below the 1e-8 residual level, so 1e-6 then), and every mesh reaches
the true relative residual 1e-8."""
import numpy as np
import pytest

import meshgen as mg
from oracle import amg, fem, krylov
from tests.gpu_util import gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(prob, **opts):
    import paper_1804_10060_amd as te
    A, b, d = gpu_assemble(prob)
    return te.AMG(A, d["coords"], d["mask"], **opts), b


def test_multi_mesh_equals_standalone_solves():
    import paper_1804_10060_amd as te
    torch_cuda()
    grids = [(3, 12, 2), (10, 40, 2), (6, 26, 3), (14, 60, 2), (4, 16, 2), (8, 34, 4)]
    hs, bs = [], []
    for i, (nr, nth, nz) in enumerate(grids):
        prob = mg.disc_problem(nr, nth, nz, 1, seed=i)
        prob.T = mg.disc_temperature_bumps(prob.mesh, 2000 + i)
        opts = {"coarse_max": 10 ** 6} if i == 0 else {"coarse_max": 400}  # mesh 0: one level only
        h, b = _setup(prob, **opts)
        hs.append(h)
        bs.append(b)
    assert hs[0].info()["n_levels"] == 1 and max(h.info()["n_levels"] for h in hs) >= 3
    say("solve_multi", len(hs), "meshes")
    us, rep = te.solve_multi(hs, bs)
    assert all(rep["converged"])
    for i, (h, b) in enumerate(zip(hs, bs)):
        u1, r1 = h.solve(b)
        d_it = abs(r1.iters[0] - rep["iters"][i])
        assert d_it <= 1, (i, r1.iters[0], rep["iters"][i])
        tol = 1e-10 if d_it == 0 else 1e-6
        err = float(((us[i] - u1).norm() / u1.norm()).cpu())
        say(f"mesh {i}: iters multi {rep['iters'][i]} single {r1.iters[0]} diff {err:.1e}")
        assert err <= tol
        assert rep["relres_true"][i] <= 1e-8
    # the multi-mesh autotuner (persistent grid, work-item order): the per-tile
    # partial sums and the per-mesh reductions over them keep their order, so
    # the tuned launches give the same iterates bit for bit
    report = te.autotune_multi(hs)
    say(report.strip())
    assert "grid" in report
    ut, rept = te.solve_multi(hs, bs)
    assert rept["iters"] == rep["iters"]
    for i in range(len(hs)):
        assert torch_cuda().equal(ut[i], us[i]), i


def test_multi_mesh_matches_oracle_and_zero_rhs():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    probs = [mg.cube_problem(6, 1), mg.disc_problem(5, 20, 2, 2, seed=3)]
    hs, bs = [], []
    for p in probs:
        h, b = _setup(p, coarse_max=300)
        hs.append(h)
        bs.append(b)
    # a third system: zero right-hand side with a non-zero guess -> u = 0, no iteration
    h3, _ = _setup(probs[0], coarse_max=300)
    hs.append(h3)
    bs.append(torch.zeros_like(bs[0]))
    u0s = [torch.zeros_like(bs[0]), torch.zeros_like(bs[1]), torch.ones_like(bs[0])]
    us, rep = te.solve_multi(hs, bs, u0s=u0s)
    assert rep["iters"][2] == 0 and float(us[2].abs().max()) == 0.0
    for i, p in enumerate(probs):
        A, b, _, _ = fem.assemble_problem(p)
        lv = amg.setup(A, fem.rigid_body_modes(p.mesh.coords, p.mask), amg.AMGOptions(coarse_max=300))
        res = krylov.pcg(A, b, lambda r: amg.vcycle(lv, r, opt=amg.AMGOptions(coarse_max=300)), rtol=1e-8)
        err = np.linalg.norm(us[i].cpu().numpy() - res.u) / np.linalg.norm(res.u)
        say(f"oracle mesh {i}: iters multi {rep['iters'][i]} oracle {res.iters} diff {err:.1e}")
        assert err <= 1e-8


def test_symmetric_coarse_storage_in_block_and_multi_mesh_solves():
    """coarse_sym = 1 takes the lower-block paths of the several-RHS product
    and of the grouped multi-mesh kernels: both give the solves of the full
    storage to rounding (same iteration counts +-1, 1e-10 / 1e-6 relative)."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    probs = [mg.disc_problem(6, 26, 2, 1, seed=4), mg.disc_problem(10, 40, 2, 1, seed=5)]
    hs_s, hs_f, bs = [], [], []
    for i, p in enumerate(probs):
        p.T = mg.disc_temperature_bumps(p.mesh, 3000 + i)
        A, b, d = gpu_assemble(p)
        hs_s.append(te.AMG(A, d["coords"], d["mask"], coarse_max=400, coarse_sym=1, max_nrhs=4))
        hs_f.append(te.AMG(A, d["coords"], d["mask"], coarse_max=400, coarse_sym=0, max_nrhs=4))
        bs.append(b)
    assert min(h.info()["n_levels"] for h in hs_s) >= 2

    def close(a, b, it_a, it_b):
        assert abs(it_a - it_b) <= 1
        tol = 1e-10 if it_a == it_b else 1e-6
        assert float(((a - b).norm() / b.norm()).cpu()) <= tol

    # several right-hand sides: b, 2b, -b on mesh 0
    B = torch.stack([bs[0], 2 * bs[0], -bs[0]], dim=-1).reshape(-1, 3, 3).contiguous()
    Us, rs = hs_s[0].solve(B)
    Uf, rf = hs_f[0].solve(B)
    for j in range(3):
        close(Us[:, :, j], Uf[:, :, j], rs.iters[j], rf.iters[j])
    # both meshes in one multi-mesh solve
    us, reps = te.solve_multi(hs_s, bs)
    uf, repf = te.solve_multi(hs_f, bs)
    assert all(reps["converged"]) and all(repf["converged"])
    for i in range(2):
        close(us[i], uf[i], reps["iters"][i], repf["iters"][i])
