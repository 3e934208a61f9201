"""GPU solutions against the oracle on the launch paths the benchmark times:
an autotuned hierarchy of a 214k-DOF P2 disc (float64 and mixed precision),
every right-hand side of a multi-RHS solve against the oracle's independent
recurrences (krylov.pcg_multi), and every launch configuration the autotuner
can choose against the oracle's level operators.  The C++ oracle
(oracle/native) runs on the host beside the GPU for the larger disc."""
import json
import os
import tempfile

import numpy as np
import pytest

import meshgen as mg
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_disc_214k_autotuned_matches_oracle():
    import paper_1804_10060_amd as te
    from oracle import krylov, native
    torch = torch_cuda()
    prob = mg.disc_problem(24, 104, 3, 2, seed=0)
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"], max_nrhs=4)
    say("autotune 214k disc")
    h.autotune()
    u64, r64 = h.solve(b)
    u32, r32 = h.solve(b, precision="mixed")
    say("oracle (C++) on the host")
    S = native.System.from_problem(prob)
    H = native.Hierarchy(S)
    ro = H.pcg(S.b(), rtol=1e-8)
    n_lev = h.info()["n_levels"]
    assert n_lev == len(H.levels) >= 3
    for l in range(n_lev - 1):
        assert np.array_equal(h.aggregates(l), H.aggregates(l)), f"aggregates differ at level {l}"
    e64 = _rel(u64.cpu().numpy(), ro.u)
    e32 = _rel(u32.cpu().numpy(), ro.u)
    say(f"fp64 iters {r64.iters[0]} mixed {r32.iters[0]} oracle {ro.iters}; err fp64 {e64:.2e} mixed {e32:.2e}")
    assert abs(r64.iters[0] - ro.iters) <= 1 and abs(r32.iters[0] - ro.iters) <= 1
    assert e64 <= 1e-8 and e32 <= 1e-8
    # four load cases as one multi-RHS solve: each column against the oracle's
    # independent recurrence of that column (oracle PCG with the oracle V-cycle)
    m = prob.mesh
    Ts = np.stack([mg.disc_temperature_bumps(m, s) for s in range(1000, 1004)])
    B = te.assemble_load(d["coords"], d["cells"], 2, prob.E, prob.nu, prob.alpha, prob.T_ref,
                         dev(Ts, torch.float64), mask=d["mask"])
    U, rep = h.solve(B)
    U = U.cpu().numpy()
    Ah = S.matrix()
    Bo = np.stack([native.System(m.coords, m.cells, 2, prob.E, prob.nu, prob.alpha, prob.T_ref, T,
                                 mask=prob.mask).b() for T in Ts], axis=1)
    res = krylov.pcg_multi(Ah, Bo, H.vcycle, rtol=1e-8)
    for j, rj in enumerate(res):
        ej = _rel(U[:, :, j].reshape(-1), rj.u)
        say(f"column {j}: iters {rep.iters[j]} oracle {rj.iters} err {ej:.2e}")
        assert abs(rep.iters[j] - rj.iters) <= 1 and ej <= 1e-8


def test_multi_rhs_columns_match_oracle_pcg_multi():
    """Every column of a five-column solve (float64 and mixed) against
    krylov.pcg_multi with the NumPy oracle's hierarchy, on a P2 and a P1 disc."""
    import paper_1804_10060_amd as te
    from oracle import amg, fem, krylov
    torch = torch_cuda()
    for dims in ((8, 34, 2, 2), (12, 40, 3, 1)):
        prob = mg.disc_problem(*dims, seed=2)
        m = prob.mesh
        A, _, d = gpu_assemble(prob)
        Ts = np.stack([mg.disc_temperature_bumps(m, s) for s in range(1010, 1015)])
        B = te.assemble_load(d["coords"], d["cells"], m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref,
                             dev(Ts, torch.float64), mask=d["mask"])
        h = te.AMG(A, d["coords"], d["mask"], max_nrhs=8, coarse_max=300)
        Ao, _, _, _ = fem.assemble_problem(prob)
        lev = amg.setup(Ao, fem.rigid_body_modes(m.coords, prob.mask), amg.AMGOptions(coarse_max=300))
        for l in range(len(lev) - 1):
            assert np.array_equal(h.aggregates(l), lev[l].agg)
        Bo = []
        for T in Ts:
            A0, b0 = fem.assemble(m.coords, m.cells, m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref, T)
            Bo.append(fem.apply_dirichlet(A0, b0, prob.mask)[1])
        Bo = np.stack(Bo, axis=1)
        assert np.abs(B.cpu().numpy().reshape(-1, 5) - Bo).max() <= 1e-12 * np.abs(Bo).max()
        M = lambda r: amg.vcycle(lev, r, opt=amg.AMGOptions(coarse_max=300))  # noqa: E731
        for prec, flexible in (("fp64", False), ("mixed", True)):
            U, rep = h.solve(B, precision=prec)
            U = U.cpu().numpy()
            res = krylov.pcg_multi(Ao, Bo, M, rtol=1e-8, flexible=flexible)
            for j, rj in enumerate(res):
                ej = _rel(U[:, :, j].reshape(-1), rj.u)
                assert abs(rep.iters[j] - rj.iters) <= 1, (dims, prec, j, rep.iters[j], rj.iters)
                assert ej <= 1e-8, (dims, prec, j, ej)
            say(f"{dims} {prec}: iters {rep.iters} oracle {[r.iters for r in res]}")


def test_every_tuner_candidate_matches_oracle_operators():
    """The autotuner picks among 48 launch configurations per operator
    (waves per workgroup 1/2/4/8, slices or rows per wave 1/2/4, XCD order,
    non-temporal loads), for the row-wave operators (6-row blocks) each also
    with the x entries shared by lane permutes.  Each one, imposed on every operator through the
    tuning cache, computes A_l x, P_l x and R_l x equal to the oracle's
    operators (float64 within the summation-order bound, float32 within its
    rounding)."""
    import paper_1804_10060_amd as te
    from oracle import amg, fem
    torch = torch_cuda()
    prob = mg.disc_problem(10, 40, 2, 2, seed=4)
    A, _, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"], coarse_max=300)
    Ao, _, _, _ = fem.assemble_problem(prob)
    lev = amg.setup(Ao, fem.rigid_body_modes(prob.mesh.coords, prob.mask), amg.AMGOptions(coarse_max=300))
    nl = len(lev)
    assert h.info()["n_levels"] == nl >= 2
    rng = np.random.default_rng(9)
    ops = []
    for l in range(nl - 1):
        n_l, n_c = lev[l].A.shape[0], lev[l + 1].A.shape[0]
        for op, M, nin in ((te.TE_OP_A, lev[l].A, n_l), (te.TE_OP_P, lev[l].P, n_c), (te.TE_OP_R, lev[l].R, n_l)):
            x = rng.standard_normal(nin)
            ops.append((l, op, x, M @ x, abs(M) @ np.abs(x)))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        h.autotune(path, use_cache=False)
        with open(path) as fh:
            keys = list(json.load(fh))
        assert keys
        n_cand = 0
        # xb: the row-wave operators' shared x entries (ignored by the SELL ones)
        for xb in (0, 1):
            for wpb in (1, 2, 4, 8):
                for spw in (1, 2, 4):
                    for remap in (0, 1):
                        for nt in (0, 1):
                            with open(path, "w") as fh:
                                json.dump({k: [wpb, spw, remap, nt, 4, 0, 0, xb] for k in keys}, fh)
                            h.autotune(path, use_cache=True)
                            for l, op, x, y_ref, scale in ops:
                                for prec, tol in ((te.TE_PREC_FP64, 1e-13), (te.TE_PREC_MIXED, 1e-5)):
                                    y = h.apply(l, op, dev(x, torch.float64), precision=prec).cpu().numpy()
                                    bad = np.abs(y - y_ref) > tol * scale + 1e-300
                                    assert not bad.any(), (xb, wpb, spw, remap, nt, l, op, prec)
                            n_cand += 1
    say(f"{n_cand} candidate configurations x {len(ops)} operators checked")
    assert n_cand == 96


def test_every_multi_rhs_candidate_matches_oracle_pcg_multi():
    """The multi-RHS launch shapes the autotuner times (row per wave with a
    lane per column; row groups with column tiles of 64, 32 or 16 per pass;
    tiles of 32 or 16 spread over the XCDs; 4 or 8 waves per workgroup), each
    imposed through the tuning cache on a 40-column solve (ragged tiles):
    every column equals the oracle's krylov.pcg_multi to 1e-8 with the
    iteration count within one."""
    import paper_1804_10060_amd as te
    from oracle import amg, fem, krylov
    torch = torch_cuda()
    prob = mg.disc_problem(8, 34, 2, 2, seed=6)
    A, _, d = gpu_assemble(prob)
    m = 40
    h = te.AMG(A, d["coords"], d["mask"], max_nrhs=m)
    Ao, _, _, _ = fem.assemble_problem(prob)
    lev = amg.setup(Ao, fem.rigid_body_modes(prob.mesh.coords, prob.mask))
    rng = np.random.default_rng(21)
    keep = (1.0 - prob.mask.reshape(-1))[:, None]
    Uo = rng.standard_normal((Ao.shape[0], m)) * keep
    Bo = Ao @ Uo
    ref = krylov.pcg_multi(Ao, Bo, lambda v: amg.vcycle(lev, v), rtol=1e-8)
    n = prob.mesh.n_nodes
    B = dev(np.ascontiguousarray(Bo.reshape(n, 3, m)), torch.float64)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        h.autotune(path, use_cache=False)
        with open(path) as fh:
            tuned = json.load(fh)
        multi = [k for k in tuned if k.endswith(f"-nrhs{m}")]
        assert multi
        n_cand = 0
        for mwpb in (4, 8):
            for mtile, msplit in ((0, 0), (64, 0), (32, 0), (16, 0), (32, 1), (16, 1)):
                cache = dict(tuned)
                for k in multi:
                    cache[k] = tuned[k][:4] + [mwpb, mtile, msplit]
                with open(path, "w") as fh:
                    json.dump(cache, fh)
                h.autotune(path, use_cache=True)
                U, rep = h.solve(B)
                U = U.cpu().numpy().reshape(-1, m)
                for j in range(m):
                    r = ref[j]
                    assert rep.converged[j] and abs(rep.iters[j] - r.iters) <= 1, (mwpb, mtile, msplit, j)
                    e = np.linalg.norm(U[:, j] - r.u) / np.linalg.norm(r.u)
                    assert e <= 1e-8, (mwpb, mtile, msplit, j, e)
                n_cand += 1
    say(f"{n_cand} multi-RHS launch shapes x {m} columns checked against the oracle")
