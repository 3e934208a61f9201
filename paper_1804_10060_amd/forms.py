"""Measurements of the batched and learned forms against plain float64 PCG-AMG
on the same GPU, at the same true relative residual 1e-8.

    python -m paper_1804_10060_amd.forms [block|multi|learned|materials|aggregation|thermal|transient|all] [--quick]

Prints one JSON object.  Workloads (seeded, synthetic):
  block   : 64 thermal load cases (4-16 Gaussian bumps, U[0,500] K) on the
            P1 disc 104x452x13 (1,993,320 DOF): one 64-column solve (64 CG
            recurrences, and block CG) vs 64 single-column solves;
  multi   : 32 P1 discs with DOF log-uniform in [1e4, 5e5]: one multi-mesh
            solve (persistent launches, graph replay) vs 32 separate solves;
  learned : P1 disc 80x344x11 (1,003,104 DOF); 2000 training and 200
            held-out load fields solved by the library, the network trained
            by the library's kernels, then held-out solves from the learned
            guess vs from zero;
  materials: P2 disc 96x416x12 (12,043,200 DOF) with hub, web and rim
            materials (temperature tables) and rim/top pressure: assembly
            against the one-material assembly, and the solve;
  aggregation: P2 disc 96x416x12: AMG setup and solve with the device MIS-2
            aggregation against the host greedy aggregation, and with the
            prolongator smoothed by the filtered operator;
  thermal : P2 disc 96x416x12 (4,014,400 temperature DOF) with the hub, web
            and rim thermal tables and heat exchange on every boundary face:
            the steady Newton solve from 400 K (CG + classical AMG);
  transient: the same disc with the three materials and pressure, starting
            stress-free at 293 K while the exterior temperatures and the
            pressures ramp to their operating values over 600 s: 16 accepted
            steps of eq. dt_spec (dT_max 10 K, eps 0.9), each attempt one
            backward-Euler heat step by Newton, each accepted step an elastic
            solve on the first step's hierarchy from the previous
            displacement; against a new hierarchy and a zero guess at
            sampled steps.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

import meshgen as mg


# The P1 discs (block, multi-mesh and learned forms) use the greedy
# aggregation: with their index-ordered structured nodes it gives regular
# aggregates that precondition better than the default MIS-2 rule (17 against
# 23 iterations on the 2M-DOF disc); on the P2 discs the MIS-2 rule is better.
P1_AGGREGATION = "greedy"


def log(*a):
    print("[forms]", *a, file=sys.stderr, flush=True)


def _torch():
    import torch
    return torch


def block_form(quick=False):
    import paper_1804_10060_amd as te
    from paper_1804_10060_amd import learned
    torch = _torch()
    grid = (26, 113, 3) if quick else mg.DISC_P1_2M[:3]
    k = 16 if quick else 64
    pr = learned.Problem(*grid, max_nrhs=64, aggregation=P1_AGGREGATION)
    seeds = list(range(1000, 1000 + k))
    T = torch.from_numpy(np.stack([mg.disc_temperature_bumps(pr.mesh, s) for s in seeds])).to(pr.dev)
    fv = torch.zeros((k, 3), dtype=torch.float64, device=pr.dev)
    B = pr.loads(T, fv)
    log(f"block: {pr.mesh.n_dof} DOF, {k} load cases")
    pr.amg.solve(B[:, :, :2].contiguous())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr.amg.solve(B)
    torch.cuda.synchronize()
    t_untuned = time.perf_counter() - t0
    tune_report = pr.amg.autotune()   # launch configurations, including those of the k-column products
    log(tune_report)
    pr.amg.solve(B[:, :, :2].contiguous())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, rep = pr.amg.solve(B)
    torch.cuda.synchronize()
    t_block = time.perf_counter() - t0
    # block CG: one Krylov space over the k columns
    pr.amg.solve(B[:, :, :2].contiguous(), block=True)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ub, repb = pr.amg.solve(B, block=True)
    torch.cuda.synchronize()
    t_bcg = time.perf_counter() - t0
    singles, diffs, its = 0.0, [], []
    for j in range(k):
        bj = B[:, :, j].reshape(-1).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uj, rj = pr.amg.solve(bj)
        torch.cuda.synchronize()
        singles += time.perf_counter() - t0
        its.append(rj.iters[0])
        diffs.append(float((U[:, :, j].reshape(-1) - uj).norm() / uj.norm()))
    out = {"workload": f"P1 disc {grid[0]}x{grid[1]}x{grid[2]}, {pr.mesh.n_dof} DOF, {k} bump load cases",
           "n_dof": pr.mesh.n_dof, "nrhs": k, "block_s": t_block, "block_s_untuned": t_untuned, "singles_s": singles,
           "autotune": [ln for ln in tune_report.splitlines() if "nrhs" in ln],
           "speedup": singles / t_block, "block_iters_max": max(rep.iters), "single_iters_mean": float(np.mean(its)),
           "all_converged": bool(all(rep.converged)), "max_relres_true": max(rep.relres_true),
           "max_rel_diff_vs_single": max(diffs),
           "block_cg_s": t_bcg, "block_cg_iters": repb.iters[0], "block_cg_speedup": singles / t_bcg,
           "block_cg_all_converged": bool(all(repb.converged)), "block_cg_max_relres_true": max(repb.relres_true),
           "block_cg_max_rel_diff_vs_single": float(max((Ub[:, :, j] - U[:, :, j]).norm() / U[:, :, j].norm()
                                                        for j in range(k))),
           "dof_rhs_per_s_block": pr.mesh.n_dof * k / t_block, "dof_rhs_per_s_single": pr.mesh.n_dof * k / singles}
    log(json.dumps(out))
    return out


def multi_form(quick=False):
    import paper_1804_10060_amd as te
    torch = _torch()
    sizes = mg.multi_mesh_sizes(8 if quick else 32, lo=1e4, hi=(5e4 if quick else 5e5))
    hs, bs = [], []
    ndof = 0
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    for (nr, nth, nz, seed) in sizes:
        prob = mg.disc_problem(nr, nth, nz, 1, seed=0)
        prob.T = mg.disc_temperature_bumps(prob.mesh, seed)
        m = prob.mesh
        c = torch.from_numpy(m.coords).to(dev)
        A, b = te.assemble(c, torch.from_numpy(m.cells).to(dev), 1, prob.E, prob.nu, prob.alpha, prob.T_ref,
                           torch.from_numpy(prob.T).to(dev), mask=torch.from_numpy(prob.mask).to(dev))
        hs.append(te.AMG(A, c, torch.from_numpy(prob.mask).to(dev), aggregation=P1_AGGREGATION))
        bs.append(b)
        ndof += m.n_dof
    log(f"multi: {len(hs)} meshes, {ndof} DOF total, setup {time.perf_counter() - t0:.1f}s")
    te.solve_multi(hs[:2], bs[:2])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    te.solve_multi(hs, bs)
    torch.cuda.synchronize()
    t_untuned = time.perf_counter() - t0
    tune_multi = te.autotune_multi(hs)   # persistent grid and work order of the grouped launches
    log(tune_multi.strip())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, rep = te.solve_multi(hs, bs)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    seq, diffs, its = 0.0, [], []
    for h, b, u in zip(hs, bs, us):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u1, r1 = h.solve(b)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        its.append(r1.iters[0])
        diffs.append(float((u - u1).norm() / u1.norm()))
    out = {"workload": f"{len(hs)} P1 discs, DOF log-uniform, {ndof} DOF total",
           "multi_s_untuned": t_untuned, "autotune": tune_multi.strip(),
           "meshes": len(hs), "total_dof": ndof, "dof_per_mesh": [3 * int(h.info()['n_dof'][0] // 3) for h in hs],
           "multi_s": t_multi, "sequential_s": seq, "speedup": seq / t_multi,
           "iters_multi": rep["iters"], "iters_single": its, "all_converged": bool(all(rep["converged"])),
           "max_relres_true": max(rep["relres_true"]), "max_rel_diff_vs_single": max(diffs)}
    log(json.dumps({k: v for k, v in out.items() if k not in ("dof_per_mesh",)}))
    return out


def learned_form(quick=False):
    from paper_1804_10060_amd import learned
    grid = (16, 68, 3) if quick else mg.DISC_P1_1M[:3]
    n_train, n_test = (192, 16) if quick else (2000, 200)
    epochs = 24 if quick else 12
    pr = learned.Problem(*grid, max_nrhs=64, aggregation=P1_AGGREGATION)
    t0 = time.perf_counter()
    train = pr.generate(list(range(10000, 10000 + n_train)), log=log)
    test = pr.generate(list(range(20000, 20000 + n_test)), log=log)
    t_gen = time.perf_counter() - t0
    params, hist, t_train = pr.train(train, epochs=epochs, lr=2e-3, log=log)
    res = pr.evaluate(params, test)
    iz = [r["iters_zero"] for r in res]
    ig = [r["iters_guess"] for r in res]
    out = {"workload": f"P1 disc {grid[0]}x{grid[1]}x{grid[2]}, {pr.mesh.n_dof} DOF; {n_train} train / {n_test} "
                       f"held-out load fields", "n_dof": pr.mesh.n_dof, "train": n_train, "test": n_test,
           "epochs": epochs, "data_generation_s": t_gen, "training_s": t_train, "loss_first": hist[0],
           "loss_last": hist[-1], "iters_zero_mean": float(np.mean(iz)), "iters_guess_mean": float(np.mean(ig)),
           "ms_zero_mean": float(np.mean([r["ms_zero"] for r in res])),
           "ms_guess_mean": float(np.mean([r["ms_guess"] for r in res])),
           "ms_inference_mean": float(np.mean([r["ms_inference"] for r in res])),
           "ms_guess_plus_inference_mean": float(np.mean([r["ms_guess"] + r["ms_inference"] for r in res])),
           "guess_used_fraction": float(np.mean([r["guess_used"] for r in res])),
           "rel_err_scaled_guess_mean": float(np.mean([r["rel_err0"] for r in res])),
           "max_relres_true_guess": max(r["relres_true_guess"] for r in res),
           "max_rel_diff_vs_zero_start": max(r["rel_diff"] for r in res)}
    log(json.dumps(out))
    return out


def materials_form(quick=False):
    """The disc with hub, web and rim materials (temperature tables) and the
    rim and top pressures against the one-material disc: assembly and solve."""
    import paper_1804_10060_amd as te
    torch = _torch()
    grid = (24, 104, 3, 2) if quick else mg.DISC_P2_12M
    prob = mg.disc_problem(*grid, seed=0)
    m = prob.mesh
    dev = torch.device("cuda:0")
    c = torch.from_numpy(m.coords).to(dev)
    cl = torch.from_numpy(m.cells.astype(np.int32)).to(dev)
    T = torch.from_numpy(prob.T).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    mat = mg.disc_materials(m)
    faces, p = mg.disc_pressure_faces(m)
    cm = torch.from_numpy(mat.cell_material).to(dev)
    fd = torch.from_numpy(faces).to(dev)
    pd = torch.from_numpy(p).to(dev)

    def timed(fn, reps=3):
        out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / reps

    (A1, b1), t_plain = timed(lambda: te.assemble(c, cl, grid[3], prob.E, prob.nu, prob.alpha, prob.T_ref, T,
                                                  mask=mask))
    (A, b), t_mat = timed(lambda: te.assemble_materials(c, cl, grid[3], (mat.T, mat.E, mat.nu, mat.alpha), cm,
                                                        prob.T_ref, T, faces=fd, face_p=pd, mask=mask))
    del A1, b1
    h = te.AMG(A, c, mask)
    h.solve(b)
    u, rep = h.solve(b)
    out = {"workload": f"P2 disc {grid[0]}x{grid[1]}x{grid[2]}, {m.n_dof} DOF, 3 materials (hub, web, rim; "
                       f"E, nu, alpha_L tables 250-1000 K), pressure on {len(faces)} rim/top faces",
           "n_dof": m.n_dof, "assembly_one_material_ms": t_plain * 1e3, "assembly_materials_ms": t_mat * 1e3,
           "solve_ms": rep.time_ms, "iters": rep.iters[0], "relres_true": rep.relres_true[0],
           "dof_per_s": m.n_dof / (rep.time_ms * 1e-3)}
    log(json.dumps(out))
    return out


def aggregation_form(quick=False):
    """AMG setup and float64 solve with the host greedy aggregation and with
    the device MIS-2 aggregation, on the same assembled system."""
    import paper_1804_10060_amd as te
    torch = _torch()
    grid = (24, 104, 3, 2) if quick else mg.DISC_P2_12M
    prob = mg.disc_problem(*grid, seed=0)
    m = prob.mesh
    dev = torch.device("cuda:0")
    c = torch.from_numpy(m.coords).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    A, b = te.assemble(c, torch.from_numpy(m.cells.astype(np.int32)).to(dev), grid[3], prob.E, prob.nu, prob.alpha,
                       prob.T_ref, torch.from_numpy(prob.T).to(dev), mask=mask)
    out = {"workload": f"P2 disc {grid[0]}x{grid[1]}x{grid[2]}, {m.n_dof} DOF", "n_dof": m.n_dof}
    te.AMG(A, c, mask, aggregation="mis2").close()  # warm-up of the setup kernels
    for name, mode, filt in (("greedy", "greedy", 0), ("mis2", "mis2", 0), ("mis2_filtered", "mis2", 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = te.AMG(A, c, mask, aggregation=mode, smooth_filtered=filt)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        info = h.info()
        h.solve(b)
        u, rep = h.solve(b)
        out[name] = {"setup_s": t_setup, "levels_dof": info["n_dof"], "nnzb": info["nnzb"], "solve_ms": rep.time_ms,
                     "iters": rep.iters[0], "relres_true": rep.relres_true[0],
                     "setup_plus_solve_s": t_setup + rep.time_ms * 1e-3}
        h.close()
    log(json.dumps(out))
    return out


def _thermal_solver(torch, dev, m, degree):
    from paper_1804_10060_amd import heat
    tm = mg.disc_thermal_materials(m)
    rb = mg.disc_robin_faces(m)
    ts = heat.ThermalSolver(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.cells.astype(np.int32)).to(dev),
                            degree, heat.Tables.of(tm), torch.from_numpy(tm.cell_material.astype(np.int32)).to(dev),
                            torch.from_numpy(rb.faces.astype(np.int32)).to(dev), torch.from_numpy(rb.h).to(dev),
                            torch.from_numpy(rb.T_bc).to(dev))
    return ts, rb


def thermal_form(quick=False):
    """The steady heat equation of the disc by Newton from 400 K (Sec. 5.2):
    a warm-up solve, then the timed solve with a fresh preconditioner."""
    torch = _torch()
    grid = (24, 104, 3, 2) if quick else mg.DISC_P2_12M
    m = mg.disc_mesh(*grid)
    dev = torch.device("cuda:0")
    ts, rb = _thermal_solver(torch, dev, m, grid[3])
    T0 = torch.full((m.n_nodes,), 400.0, dtype=torch.float64, device=dev)
    ts.newton(T0)
    ts.reset_preconditioner()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T, rep = ts.newton(T0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"workload": f"steady heat equation, P2 disc {grid[0]}x{grid[1]}x{grid[2]}, {m.n_nodes} DOF, "
                       f"{rb.faces.shape[0]} exchange faces", "ms": wall * 1e3, "newton_iters": rep.iters,
           "lin_iters": rep.lin_iters, "assembly_ms": rep.assembly_ms, "setup_ms": rep.setup_ms,
           "cg_ms": rep.solve_ms, "res_history": rep.res_history, "T_min": float(T.min()), "T_max": float(T.max())}
    log(json.dumps(out))
    return out


def transient_form(quick=False):
    """Backward-Euler heat steps driving the elastic solves (the loop of a
    transient run, Sec. 3.3 and 5.3), the elastic hierarchy of the first step
    reused with the previous displacement as guess, against a new hierarchy
    per step from a zero guess at sampled steps."""
    from paper_1804_10060_amd import transient
    torch = _torch()
    grid = (24, 104, 3, 2) if quick else mg.DISC_P2_12M
    nsteps = 6 if quick else 16
    prob = mg.disc_problem(*grid, seed=0)
    prob.T_ref = 293.0
    m = prob.mesh
    dev = torch.device("cuda:0")
    mat = mg.disc_materials(m)
    faces, p = mg.disc_pressure_faces(m)
    c = torch.from_numpy(m.coords).to(dev)
    cl = torch.from_numpy(m.cells.astype(np.int32)).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    cm = torch.from_numpy(mat.cell_material).to(dev)
    tables = (mat.T, mat.E, mat.nu, mat.alpha)
    ts, rb = _thermal_solver(torch, dev, m, grid[3])
    T_bc = torch.from_numpy(rb.T_bc).to(dev)
    p_d = torch.from_numpy(p).to(dev)
    ramp_s, T0 = 600.0, 293.0

    def ramp(t):
        return min(1.0, t / ramp_s)

    def T_bc_of_t(t):
        return (T0 + (T_bc - T0) * ramp(t)).contiguous()

    def p_of_t(t):
        return (p_d * ramp(t)).contiguous()

    def elastic():
        return transient.ElasticTransient(c, cl, grid[3], tables, cm, prob.T_ref, mask,
                                          faces=torch.from_numpy(faces).to(dev), face_p=p_of_t(0.0))

    el = elastic()
    # the temperatures of sampled steps, kept for the comparison below
    keep_at = sorted({1, nsteps // 2, nsteps})
    temps, count, orig = {}, [0], el.solve_at

    def capture(T):
        if count[0] in keep_at:
            temps[count[0]] = T.clone()
        count[0] += 1
        return orig(T)

    el.solve_at = capture
    run = transient.ThermoelasticTransient(ts, el, T_bc_of_t, p_of_t)
    Tstart = torch.full((m.n_nodes,), T0, dtype=torch.float64, device=dev)
    recs, _ = run.run(Tstart, 0.0, 1e9, 10.0, dT_max=10.0, eps=0.9, max_steps=nsteps)
    el.close()
    fresh = {}
    for k, T in temps.items():
        r = elastic()
        r.kw["face_p"] = p_of_t(recs[k].t)
        u, rep, built, ta, to, tsol = r.solve_at(T)
        fresh[k] = {"iters": rep.iters[0], "assemble_ms": ta, "setup_ms": to, "solve_ms": tsol}
        r.close()
    steps = [dataclasses.asdict(s) for s in recs]
    later = recs[1:]
    elastic_ms = [s.assemble_ms + s.operator_ms + s.solve_ms for s in later]
    thermal_ms = [s.thermal_ms for s in later]
    fresh_ms = [v["assemble_ms"] + v["setup_ms"] + v["solve_ms"] for v in fresh.values()]
    out = {"workload": f"P2 disc {grid[0]}x{grid[1]}x{grid[2]}, {m.n_dof} elastic + {m.n_nodes} thermal DOF, 3 "
                       f"materials, exterior temperatures and pressures ramped over {ramp_s:.0f} s from a "
                       f"stress-free 293 K, dT_max 10 K, eps 0.9",
           "steps": steps, "t_end": recs[-1].t,
           "thermal_step_ms_mean": float(np.mean(thermal_ms)), "elastic_step_ms_mean": float(np.mean(elastic_ms)),
           "thermal_share": float(np.sum(thermal_ms) / (np.sum(thermal_ms) + np.sum(elastic_ms))),
           "elastic_iters_mean": float(np.mean([s.iters for s in later])),
           "thermal_rebuilds": int(sum(s.thermal_rebuilds for s in later)),
           "rejected_total": int(sum(s.rejected for s in later)),
           "fresh_sampled": fresh, "fresh_elastic_step_ms_mean": float(np.mean(fresh_ms)),
           "all_converged": bool(all(s.relres_true <= 1e-8 for s in recs))}
    log(json.dumps({k: v for k, v in out.items() if k != "steps"}))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["block", "multi", "learned", "materials", "aggregation",
                                                               "thermal", "transient", "all"])
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args()
    out = {}
    if a.which in ("block", "all"):
        out["block_rhs"] = block_form(a.quick)
    if a.which in ("multi", "all"):
        out["multi_mesh"] = multi_form(a.quick)
    if a.which in ("learned", "all"):
        out["learned_guess"] = learned_form(a.quick)
    if a.which in ("materials", "all"):
        out["materials"] = materials_form(a.quick)
    if a.which in ("aggregation", "all"):
        out["aggregation"] = aggregation_form(a.quick)
    if a.which in ("thermal", "all"):
        out["thermal"] = thermal_form(a.quick)
    if a.which in ("transient", "all"):
        out["transient"] = transient_form(a.quick)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
