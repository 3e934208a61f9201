"""Transient runs: preconditioner reuse (amg_set_operator), the time-step
control of eq. dt_spec (te_timestep) and the driver that orders them,
against the oracle.

Bars: the reused-hierarchy solve follows the single-solve bar (iterations
within one, relative difference <= 1e-8 from the same initial guess); the
time-step decisions are exact (the largest change is a maximum of exactly
computed differences and the rule is the same float64 expression), so the
driver's step sequence equals the oracle's bit for bit; every step's
displacement meets the true relative residual 1e-8 on the system the oracle
assembles itself."""
import math

import numpy as np
import pytest

import meshgen as mg
from oracle import amg, fem, krylov, transient
from tests.gpu_util import dev, gpu_assemble, say, torch_cuda

pytestmark = pytest.mark.gpu


def _materials_setup(prob):
    m = prob.mesh
    mat = mg.disc_materials(m)
    faces, p = mg.disc_pressure_faces(m)
    return mat, faces, p


def _gpu_system(prob, mat, faces, p, T):
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    m = prob.mesh
    return te.assemble_materials(dev(m.coords, torch.float64), dev(m.cells.astype(np.int32)), m.degree,
                                 (mat.T, mat.E, mat.nu, mat.alpha), dev(mat.cell_material.astype(np.int32)),
                                 prob.T_ref, dev(T, torch.float64), faces=dev(faces.astype(np.int32)),
                                 face_p=dev(p, torch.float64), mask=dev(prob.mask))


def _oracle_system(prob, mat, faces, p, T):
    m = prob.mesh
    tab = fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha)
    A0, b0 = fem.assemble_materials(m.coords, m.cells, m.degree, mat.cell_material, tab, prob.T_ref, T, None,
                                    faces=faces, face_p=p)
    return fem.apply_dirichlet(A0, b0, prob.mask)


def test_reused_hierarchy_matches_oracle_and_reverts():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 2, seed=2)
    m = prob.mesh
    mat, faces, p = _materials_setup(prob)
    Ta, Tb = (293.0 + (prob.T - 293.0) * s for s in (0.5, 0.6))
    Aa, ba = _gpu_system(prob, mat, faces, p, Ta)
    Ab, bb = _gpu_system(prob, mat, faces, p, Tb)
    Aao, bao = _oracle_system(prob, mat, faces, p, Ta)
    Abo, bbo = _oracle_system(prob, mat, faces, p, Tb)
    h = te.AMG(Aa, dev(m.coords, torch.float64), dev(prob.mask), coarse_max=400)
    opt = amg.AMGOptions(coarse_max=400)
    lv = amg.setup(Aao, fem.rigid_body_modes(m.coords, prob.mask), opt)
    M = lambda r: amg.vcycle(lv, r, opt=opt)
    ua_o = krylov.pcg(Aao, bao, M).u
    ua, repa = h.solve(ba)
    h.set_operator(Ab)
    u, rep = h.solve(bb, u0=dev(ua_o, torch.float64))
    res = krylov.pcg(Abo, bbo, M, u0=ua_o)
    say(f"reused hierarchy: gpu {rep.iters[0]} iterations, oracle {res.iters}")
    assert rep.converged == [1] and abs(rep.iters[0] - res.iters) <= 1
    uh = u.cpu().numpy()
    assert np.linalg.norm(uh - res.u) <= 1e-8 * np.linalg.norm(res.u)
    assert np.linalg.norm(bbo - Abo @ uh) <= 1.0000001e-8 * np.linalg.norm(bbo)
    # the same guess on the setup matrix would not solve the new system
    assert np.linalg.norm(bbo - Aao @ uh) > 1e-6 * np.linalg.norm(bbo)
    # back to the setup matrix: the solve of the first system again, bit for bit
    h.set_operator(None)
    ua2, _ = h.solve(ba)
    assert torch.equal(ua, ua2)


def test_set_operator_rejects_other_patterns_and_the_multi_solve():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 1, seed=1)
    A, b, d = gpu_assemble(prob)
    h = te.AMG(A, d["coords"], d["mask"])
    other, _, _ = gpu_assemble(mg.cube_problem(4, 1))
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        h.set_operator(other)
    # same sizes, one column index moved: a different pattern
    col = A.col_idx.clone()
    rp = A.row_ptr.cpu().numpy()
    r = 7
    row_cols = set(col[rp[r]:rp[r + 1]].cpu().numpy().tolist())
    new_c = next(c for c in range(A.n) if c not in row_cols)
    col[rp[r + 1] - 1] = new_c
    moved = te.Matrix(A.row_ptr, col, A.val)
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        h.set_operator(moved)
    h.set_operator(A)
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        te.solve_multi([h], [b])
    h.set_operator(None)
    us, rep = te.solve_multi([h], [b])
    assert all(rep["converged"])


def test_timestep_matches_oracle_exactly():
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    rng = np.random.default_rng(4)
    n = 100003
    T_old = 300.0 + 600.0 * rng.random(n)
    for scale, dt, dT_max, eps in [(3.0, 1.0, 10.0, 0.9), (12.0, 2.5, 10.0, 0.9), (0.0, 4.0, 10.0, 0.5),
                                   (9.99, 0.1, 10.0, 1.0), (1e-3, 7.0, 10.0, 0.9)]:
        T_new = T_old + scale * (2.0 * rng.random(n) - 1.0)
        got = te.timestep(dev(T_new, torch.float64), dev(T_old, torch.float64), dt, dT_max, eps)
        want = transient.next_step(T_new, T_old, dt, dT_max, eps)
        assert got[0] == want[0] and got[1] == want[1] and got[2] == want[2], (got, want)
    bad = T_old.copy()
    bad[n // 2] = np.nan
    with pytest.raises(te.TeError, match="TE_ENAN"):
        te.timestep(dev(bad, torch.float64), dev(T_old, torch.float64), 1.0)
    with pytest.raises(te.TeError, match="TE_EINVAL"):
        te.timestep(dev(T_old, torch.float64), dev(T_old, torch.float64), -1.0)


def test_driver_follows_the_oracle_step_sequence():
    """Five steps of a heating history on a P2 disc with three materials and
    pressure, the first attempt 40 s long (halved until its change is within
    10 K): the same accepted times and lengths as the oracle, and every
    displacement solves its step's system as the oracle assembles it."""
    from paper_1804_10060_amd import transient as gt
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 2, seed=2)
    m = prob.mesh
    mat, faces, p = _materials_setup(prob)
    tau = 600.0

    def T_np(t):
        return 293.0 + (prob.T - 293.0) * (1.0 - math.exp(-t / tau))

    run = gt.ElasticTransient(dev(m.coords, torch.float64), dev(m.cells.astype(np.int32)), m.degree,
                              (mat.T, mat.E, mat.nu, mat.alpha), dev(mat.cell_material.astype(np.int32)), prob.T_ref,
                              dev(prob.mask), faces=dev(faces.astype(np.int32)), face_p=dev(p, torch.float64),
                              coarse_max=400)
    us = []
    orig = run.solve_at

    def keep(T):
        out = orig(T)
        us.append(out[0].cpu().numpy())
        return out

    run.solve_at = keep
    recs = run.run(lambda t: dev(T_np(t), torch.float64), 0.0, 1e9, 40.0, dT_max=10.0, eps=0.9, max_steps=5)
    run.close()
    ref = transient.step_sequence(T_np, 0.0, 1e9, 40.0, dT_max=10.0, eps=0.9, max_steps=5)
    say("steps", [(r.t, r.dt, r.rejected, r.iters) for r in recs])
    assert len(recs) == 6 and recs[1].rejected >= 1
    for r, o in zip(recs[1:], ref):
        assert (r.t, r.dt, r.max_change, r.rejected) == (o.t, o.dt, o.dT, o.rejected)
    assert recs[0].setup and not any(r.setup for r in recs[1:])
    for r, u in zip(recs, us):
        A, b = _oracle_system(prob, mat, faces, p, T_np(r.t))
        assert np.linalg.norm(b - A @ u) <= 1.0000001e-8 * np.linalg.norm(b), f"step at t = {r.t}"


def test_reused_hierarchy_with_mixed_precision_and_block_cg():
    """After amg_set_operator the float32 V-cycle (the setup matrix's copies)
    inside float64 flexible CG, and block CG over three columns, both solve
    the new system to the true residual on the oracle's own assembly."""
    import paper_1804_10060_amd as te
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 2, seed=2)
    m = prob.mesh
    mat, faces, p = _materials_setup(prob)
    Ta, Tb = (293.0 + (prob.T - 293.0) * s for s in (0.5, 0.6))
    Aa, ba = _gpu_system(prob, mat, faces, p, Ta)
    Ab, bb = _gpu_system(prob, mat, faces, p, Tb)
    Abo, bbo = _oracle_system(prob, mat, faces, p, Tb)
    h = te.AMG(Aa, dev(m.coords, torch.float64), dev(prob.mask), coarse_max=400, max_nrhs=4)
    h.set_operator(Ab)
    u, rep = h.solve(bb, precision="mixed")
    assert rep.converged == [1]
    uh = u.cpu().numpy()
    assert np.linalg.norm(bbo - Abo @ uh) <= 1.0000001e-8 * np.linalg.norm(bbo)
    B3 = torch.stack([bb.reshape(-1, 3), 0.5 * bb.reshape(-1, 3), ba.reshape(-1, 3)], dim=2).contiguous()
    U, repb = h.solve(B3, block=True)
    assert all(repb.converged)
    Uh = U.cpu().numpy().reshape(-1, 3)
    Bh = B3.cpu().numpy().reshape(-1, 3)
    for j in range(3):
        assert np.linalg.norm(Bh[:, j] - Abo @ Uh[:, j]) <= 1.0000001e-8 * np.linalg.norm(Bh[:, j]) + \
            1e-12 * np.linalg.norm(Bh[:, j]), f"column {j}"


def test_coupled_heat_and_elastic_steps_match_oracle():
    """Backward-Euler heat steps from 293 K (Sec. 5.3) with exterior
    temperatures and pressures ramping in time, each followed by the elastic
    solve at the new temperature on the reused hierarchy: the step times,
    lengths and rejections of eq. dt_spec, the temperatures and the
    displacements against the oracle running the same sequence (the
    thermal preconditioner kept and rebuilt by the same rule)."""
    from oracle import camg, thermal
    from paper_1804_10060_amd import heat
    from paper_1804_10060_amd import transient as gt
    torch = torch_cuda()
    prob = mg.disc_problem(6, 26, 2, 2, seed=2)
    prob.T_ref = 293.0
    m = prob.mesh
    mat, faces, p = _materials_setup(prob)
    tm = mg.disc_thermal_materials(m)
    rb = mg.disc_robin_faces(m)
    P = thermal.problem_from_meshgen(m, tm, rb)
    ramp = lambda t: min(1.0, t / 600.0)  # noqa: E731
    Tbc_np = lambda t: 293.0 + (rb.T_bc - 293.0) * ramp(t)  # noqa: E731
    p_np = lambda t: p * ramp(t)  # noqa: E731
    d_coords, d_cells = dev(m.coords, torch.float64), dev(m.cells.astype(np.int32))
    ts = heat.ThermalSolver(d_coords, d_cells, 2, heat.Tables.of(tm), dev(tm.cell_material.astype(np.int32)),
                            dev(rb.faces.astype(np.int32)), dev(rb.h, torch.float64), dev(rb.T_bc, torch.float64))
    el = gt.ElasticTransient(d_coords, d_cells, 2, (mat.T, mat.E, mat.nu, mat.alpha),
                             dev(mat.cell_material.astype(np.int32)), prob.T_ref, dev(prob.mask),
                             faces=dev(faces.astype(np.int32)), face_p=dev(p_np(0.0), torch.float64), coarse_max=400)
    us = []
    orig = el.solve_at

    def keep(T):
        out = orig(T)
        us.append(out[0].cpu().numpy())
        return out

    el.solve_at = keep
    run = gt.ThermoelasticTransient(ts, el, lambda t: dev(Tbc_np(t), torch.float64),
                                    lambda t: dev(p_np(t), torch.float64), coarse_max=200, block=64)
    recs, _ = run.run(dev(np.full(m.n_nodes, 293.0), torch.float64), 0.0, 1e9, 200.0, max_steps=4)
    el.close()
    pre = thermal.ReusedPreconditioner(camg.CAMGOptions(coarse_max=200, block=64))
    ref = transient.coupled_step_sequence(P, np.full(m.n_nodes, 293.0), Tbc_np, pre, 0.0, 1e9, 200.0, max_steps=4)
    say("coupled", [(round(r.t, 3), round(r.dt, 3), r.rejected, r.newton_iters, r.iters) for r in recs[1:]])
    say("oracle ", [(round(o.t, 3), round(o.dt, 3), o.rejected, o.newton_iters) for o in ref])
    assert len(recs) == 5 and recs[1].rejected >= 1
    # the same decisions; the times agree to the rounding of the largest change
    for r, o in zip(recs[1:], ref):
        assert r.rejected == o.rejected and r.newton_iters == o.newton_iters
        assert abs(r.t - o.t) <= 1e-9 * o.t and abs(r.max_change - o.dT) <= 1e-9 * o.dT
    # displacements: the oracle's elastic solve on its own assembly at its
    # own temperature, on the hierarchy of the first step, from the previous
    # displacement
    opt = amg.AMGOptions(coarse_max=400)
    A0, b0 = _oracle_system(prob, mat, faces, p_np(0.0), np.full(m.n_nodes, 293.0))
    lv = amg.setup(A0, fem.rigid_body_modes(m.coords, prob.mask), opt)
    M = lambda r: amg.vcycle(lv, r, opt=opt)  # noqa: E731
    u_prev = np.zeros(3 * m.n_nodes)
    assert np.abs(us[0]).max() == 0.0       # stress-free start: T = T_ref, no pressure
    for k, o in enumerate(ref):
        A, b = _oracle_system(prob, mat, faces, p_np(o.t), o.T)
        res = krylov.pcg(A, b, M, u0=u_prev)
        assert abs(recs[k + 1].iters - res.iters) <= 1
        assert np.linalg.norm(us[k + 1] - res.u) <= 1e-7 * np.linalg.norm(res.u), f"step {k}"
        u_prev = res.u
