#!/usr/bin/env python3
"""Benchmark: time to a true relative residual of 1e-8 for PCG + smoothed-
aggregation AMG on one MI355X, on the 12,043,200-DOF P2 turbine-disc proxy.

One step = one full solve from u0 = 0 (A, b and the hierarchy resident in
HBM, the preconditioner reused as in the paper's transient runs); assembly and
setup are timed once and reported beside it.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import statistics
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG-AMG time-to-rtol1e-8 and DOF/s; SpMV HBM GB/s; mixed/learned vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def ensure_built():
    lib = os.path.join(ROOT, "paper_1804_10060_amd", "libte_amd.so")
    if not os.path.exists(lib):
        log("library missing: building")
        from paper_1804_10060_amd import build as b
        b.build()


def algorithmic_bytes(info, n_rows, nnzb0, vt=8):
    """Bytes each level-0 kernel class must move per launch (values + column
    index per stored block, one int per row for the row length, and the
    vectors each epilogue reads or writes, vt bytes per entry, 3 per node)."""
    mat = nnzb0 * (9 * vt + 4) + n_rows * 4
    v = 3 * vt * n_rows  # one nodal vector
    out = {
        "Ap": mat + 2 * v,            # gather p, write q
        "pre_smooth": mat + 4 * v,    # gather d, read g, D^-1; write x
        "residual": mat + 3 * v,      # gather x, read g; write s
        "post_init": mat + 5 * v,     # gather x, read g, D^-1; write r, d
        "post_smooth": mat + 5 * v,   # gather d, read r, D^-1, x; write x
    }
    if info["n_levels"] > 1:
        nc = info["n_dof"][1] // 6
        pn = info["p_nnzb"][0]
        vc = 6 * vt * nc
        out["restrict"] = pn * (18 * vt + 4) + nc * 8 + v + vc
        out["prolong"] = pn * (18 * vt + 4) + n_rows * 8 + vc + 2 * v
    return out


def algorithmic_bytes_multi(n_rows, nnzb0, m, vt=8):
    """The mesh-level classes of an m-column solve: the matrix once, every
    per-column vector m times, D^-1 (one per row) once."""
    mat = nnzb0 * (9 * vt + 4) + n_rows * 4
    v = 3 * vt * n_rows
    return {"Ap": mat + 2 * v * m, "pre_smooth": mat + 3 * v * m + v, "residual": mat + 3 * v * m,
            "post_init": mat + 4 * v * m + v, "post_smooth": mat + 4 * v * m + v}


def cpu_baseline(sample_grid=(48, 208, 6, 2)):
    """The oracle in its C++17/OpenMP form (float64, the same algorithm and
    rtol) on all host cores the process may use, on a bounded sample of the
    workload: the P2 disc of the same recipe with half the cells per
    direction (1,573,728 DOF, an eighth of the headline disc)."""
    import meshgen as mg
    from oracle import native
    nr, nth, nz, deg = sample_grid
    prob = mg.disc_problem(nr, nth, nz, deg, seed=0)
    threads = native.max_threads()
    S = native.System.from_problem(prob)
    H = native.Hierarchy(S)
    r = H.pcg(S.b(), rtol=1e-8)
    n = prob.mesh.n_dof
    log(f"cpu oracle ({threads} threads): {n} DOF, assembly {S.time_assemble:.1f}s setup {H.time_setup:.1f}s "
        f"solve {r.time_solve:.1f}s, {r.iters} it")
    return {"value": n / r.time_solve, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": f"C++17/OpenMP oracle solve phase (PCG + SA-AMG, float64, rtol 1e-8, {r.iters} iterations) "
                      f"on the disc P2 {nr}x{nth}x{nz} ({n} DOF, 1/8 of the headline disc), same material and "
                      f"field recipe, {threads} OpenMP threads; its assembly {S.time_assemble:.2f}s and setup "
                      f"{H.time_setup:.2f}s are reported beside the value",
            "solve_s": r.time_solve, "setup_s": H.time_setup, "assembly_s": S.time_assemble, "iters": r.iters,
            "dof_per_s_setup_plus_solve": n / (H.time_setup + r.time_solve), "host_cpus": os.cpu_count()}


def cpu_baseline_full(grid=(96, 416, 12, 2), repeats=3, one_thread_grid=(48, 208, 6, 2)):
    """The protocol of a full CPU comparison: the C++ oracle on the headline
    disc with all host cores (assembly, setup and solve, median of `repeats`),
    and with one thread on the 1/8 disc (one run each; a one-thread run of the
    headline disc takes tens of minutes)."""
    import statistics

    import meshgen as mg
    from oracle import native
    out = {"threads": native.max_threads(), "host_cpus": os.cpu_count()}
    for key, g, th, rep in (("all_cores", grid, 0, repeats), ("one_thread", one_thread_grid, 1, 1)):
        prob = mg.disc_problem(*g, seed=0)
        runs = []
        for k in range(rep):
            S = native.System.from_problem(prob, threads=th)
            H = native.Hierarchy(S, threads=th)
            r = H.pcg(S.b(), rtol=1e-8)
            runs.append((S.time_assemble, H.time_setup, r.time_solve, r.iters))
            log(f"cpu oracle {key} run {k}: {prob.mesh.n_dof} DOF, assembly {runs[-1][0]:.1f}s setup "
                f"{runs[-1][1]:.1f}s solve {runs[-1][2]:.1f}s, {r.iters} it")
            H.free()
            S.free()
        med = [statistics.median(x[i] for x in runs) for i in range(3)]
        n = prob.mesh.n_dof
        out[key] = {"grid": list(g), "n_dof": n, "runs": len(runs), "assembly_s": med[0], "setup_s": med[1],
                    "solve_s": med[2], "iters": runs[0][3], "dof_per_s_solve": n / med[2],
                    "dof_per_s_setup_plus_solve": n / (med[1] + med[2]),
                    "threads": native.max_threads() if th == 0 else th}
    return out


def block_rhs_form(te, torch, dev):
    """64 thermal load cases on the 1,993,320-DOF P1 disc as one multi-RHS
    solve (and as block CG), against 64 single float64 solves on the same GPU;
    columns 0 and 63 against the stored oracle solutions of their cases."""
    import numpy as np

    import meshgen as mg
    from paper_1804_10060_amd._lib import KERNEL_CLASSES
    from tests import golden_c2
    prob = mg.disc_problem(*mg.DISC_P1_2M, seed=0)
    m = prob.mesh
    coords, cells = torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.cells).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    A, _ = te.assemble(coords, cells, 1, prob.E, prob.nu, prob.alpha, prob.T_ref, torch.from_numpy(prob.T).to(dev),
                       mask=mask)
    h = te.AMG(A, coords, mask, max_nrhs=64, aggregation="greedy")
    h.autotune()
    seeds = list(range(1000, 1064))
    Ts = torch.from_numpy(np.stack([mg.disc_temperature_bumps(m, s) for s in seeds])).to(dev)
    B = te.assemble_load(coords, cells, 1, prob.E, prob.nu, prob.alpha, prob.T_ref, Ts, mask=mask)
    h.solve(B[:, :, :2].contiguous())
    h.solve(B[:, :, :2].contiguous(), block=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, rep = h.solve(B)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    # per-class times of the 64-column mesh-level products (HIP events)
    _, prep = h.solve(B, profile=True)
    algo = algorithmic_bytes_multi(m.n_nodes, A.nnzb, B.shape[2])
    spmm = {}
    for i, name in enumerate(KERNEL_CLASSES):
        if name in algo and prep.kernel_launches[i]:
            avg = prep.kernel_ms[i] / prep.kernel_launches[i]
            spmm[name] = {"avg_ms": round(avg, 4), "algo_bytes": int(algo[name]),
                          "GBps": round(algo[name] / (avg * 1e-3) / 1e9, 1)}
    dom = max(spmm, key=lambda k: spmm[k]["avg_ms"] * prep.kernel_launches[KERNEL_CLASSES.index(k)])
    spmm_roofline = {"bound": "hbm", "kernel": dom, "achieved": spmm[dom]["GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(spmm[dom]["GBps"] / HBM_PEAK_GBS, 4),
                     "algo_bytes_per_launch": spmm[dom]["algo_bytes"]}
    t0 = time.perf_counter()
    Ub, repb = h.solve(B, block=True)
    torch.cuda.synchronize()
    t_bcg = time.perf_counter() - t0
    t_single, its = 0.0, []
    for j in range(len(seeds)):
        bj = B[:, :, j].reshape(-1).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rj = h.solve(bj)
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t0
        its.append(rj.iters[0])
    err = {}
    for j, seed in ((0, 1000), (63, 1063)):
        g = golden_c2.load(golden_c2.load_case_path(seed))
        es, ep = golden_c2.errors(U[:, :, j].reshape(-1).cpu().numpy(), g)
        eb, _ = golden_c2.errors(Ub[:, :, j].reshape(-1).cpu().numpy(), g)
        err[f"case{seed}"] = {"sampled": es, "projected": ep, "block_cg_sampled": eb, "iters": rep.iters[j],
                              "oracle_iters": g["iters"]}
    n = m.n_dof
    out = {"workload": f"P1 disc 104x452x13, {n} DOF, 64 bump load cases (seeds 1000-1063), greedy aggregation",
           "ms": round(t_multi * 1e3, 2), "singles_ms": round(t_single * 1e3, 2),
           "speedup_vs_fp64_singles": round(t_single / t_multi, 3), "iters_max": max(rep.iters),
           "single_iters_mean": float(np.mean(its)), "all_converged": bool(all(rep.converged)),
           "max_relres_true": max(rep.relres_true), "block_cg_ms": round(t_bcg * 1e3, 2),
           "block_cg_iters": repb.iters[0], "block_cg_speedup_vs_fp64_singles": round(t_single / t_bcg, 3),
           "dof_rhs_per_s": n * len(seeds) / t_multi, "err_vs_oracle": err,
           "spmm_kernels": spmm, "spmm_roofline": spmm_roofline}
    log(f"block rhs: 64 columns {t_multi * 1e3:.1f} ms, block CG {t_bcg * 1e3:.1f} ms, singles "
        f"{t_single * 1e3:.1f} ms; errors {err}")
    return out


def thermal_form(torch, dev, elastic_ms):
    """The steady thermal solve of the same disc (P2, 4,014,400 nodes; hub,
    web and rim thermal tables; heat exchange on every boundary face): Newton
    from 400 K to relative residual 1e-9 with CG and classical AMG (Sec. 5.1,
    5.2), timed beside the elastic solve, against the stored oracle
    temperature."""
    import numpy as np

    import meshgen as mg
    from paper_1804_10060_amd import heat
    from tests import golden_c2
    m = mg.disc_mesh(*mg.DISC_P2_12M)
    tm = mg.disc_thermal_materials(m)
    rb = mg.disc_robin_faces(m)
    ts = heat.ThermalSolver(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.cells).to(dev), 2,
                            heat.Tables.of(tm), torch.from_numpy(tm.cell_material.astype(np.int32)).to(dev),
                            torch.from_numpy(rb.faces).to(dev), torch.from_numpy(rb.h).to(dev),
                            torch.from_numpy(rb.T_bc).to(dev))
    T0 = torch.full((m.n_nodes,), 400.0, dtype=torch.float64, device=dev)
    ts.newton(T0)                      # warm-up (builds its preconditioner)
    ts.reset_preconditioner()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T, rep = ts.newton(T0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"workload": f"steady heat equation on the P2 disc 96x416x12, {m.n_nodes} thermal DOF, 3 materials, "
                       f"{rb.faces.shape[0]} heat-exchange faces; Newton from 400 K to relres 1e-9, CG + classical "
                       f"AMG", "ms": round(wall * 1e3, 2), "newton_iters": rep.iters, "lin_iters": rep.lin_iters,
           "assembly_ms": round(rep.assembly_ms, 2), "amg_setup_ms": round(rep.setup_ms, 2),
           "cg_ms": round(rep.solve_ms, 2), "dof_per_s": m.n_nodes / wall,
           "share_of_thermal_plus_elastic": round(wall * 1e3 / (wall * 1e3 + elastic_ms), 3)}
    if os.path.exists(golden_c2.THERMAL_PATH):
        g = golden_c2.load(golden_c2.THERMAL_PATH)
        es, ep = golden_c2.errors(T.cpu().numpy(), g)
        out["err_vs_oracle"] = {"sampled": es, "projected": ep, "newton_iters": rep.iters,
                                "oracle_newton_iters": g["iters"], "oracle_lin_iters": g["lin_iters"]}
    log(f"thermal: {wall * 1e3:.1f} ms, Newton {rep.iters}, CG {rep.lin_iters}; {out.get('err_vs_oracle')}")
    return out


def learned_form_small(torch):
    """The learned initial guess at a size the bench can afford: a P1 disc of
    13,872 DOF, the network trained by the library's kernels on 192 solves the
    library generates, then 16 held-out load fields solved from the scaled
    guess and from zero (the 1M-DOF protocol is forms.py learned)."""
    import numpy as np

    from paper_1804_10060_amd import learned
    pr = learned.Problem(16, 68, 3, max_nrhs=64, aggregation="greedy")
    train = pr.generate(list(range(10000, 10192)), log=lambda *a: None)
    test = pr.generate(list(range(20000, 20016)), log=lambda *a: None)
    params, hist, t_train = pr.train(train, epochs=24, lr=2e-3, log=lambda *a: None)
    res = pr.evaluate(params, test)
    out = {"workload": f"P1 disc 16x68x3, {pr.mesh.n_dof} DOF; 192 train / 16 held-out load fields",
           "training_s": round(t_train, 2), "loss_first": hist[0], "loss_last": hist[-1],
           "iters_zero_mean": float(np.mean([r["iters_zero"] for r in res])),
           "iters_guess_mean": float(np.mean([r["iters_guess"] for r in res])),
           "ms_zero_mean": float(np.mean([r["ms_zero"] for r in res])),
           "ms_guess_mean": float(np.mean([r["ms_guess"] for r in res])),
           "ms_inference_mean": float(np.mean([r["ms_inference"] for r in res])),
           "max_relres_true_guess": max(r["relres_true_guess"] for r in res),
           "max_rel_diff_vs_zero_start": max(r["rel_diff"] for r in res)}
    log(f"learned (small): {out['iters_guess_mean']:.2f} vs {out['iters_zero_mean']:.2f} iterations")
    return out


def multi_mesh_form(te, torch, dev):
    """32 P1 discs (DOF log-uniform in [1e4, 5e5], bump fields of seeds
    2000-2031) in one persistent graph-replayed launch sequence against 32
    single float64 solves; the smallest and the largest mesh against the
    stored oracle solutions of those meshes."""
    import numpy as np

    import meshgen as mg
    from tests import golden_c2
    sizes = mg.multi_mesh_sizes(32, lo=1e4, hi=5e5)
    hs, bs, probs = [], [], []
    for (nr, nth, nz, seed) in sizes:
        prob = mg.disc_problem(nr, nth, nz, 1, seed=0)
        prob.T = mg.disc_temperature_bumps(prob.mesh, seed)
        m = prob.mesh
        c = torch.from_numpy(m.coords).to(dev)
        mk = torch.from_numpy(prob.mask).to(dev)
        A, b = te.assemble(c, torch.from_numpy(m.cells).to(dev), 1, prob.E, prob.nu, prob.alpha, prob.T_ref,
                           torch.from_numpy(prob.T).to(dev), mask=mk)
        hs.append(te.AMG(A, c, mk, aggregation="greedy"))
        bs.append(b)
        probs.append(prob)
    te.solve_multi(hs[:2], bs[:2])
    tune_multi = te.autotune_multi(hs)
    log(tune_multi.strip())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, reps = te.solve_multi(hs, bs)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    t_seq = 0.0
    for h, b in zip(hs, bs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.solve(b)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
    dofs = [p.mesh.n_dof for p in probs]
    err = {}
    for i in golden_c2.MULTI_MESH_INDICES:
        g = golden_c2.load(golden_c2.multi_mesh_path(i))
        es, ep = golden_c2.errors(us[i].cpu().numpy(), g)
        err[f"mesh{i}_{dofs[i]}dof"] = {"sampled": es, "projected": ep, "iters": reps["iters"][i],
                                         "oracle_iters": g["iters"]}
    out = {"workload": f"32 P1 discs, {sum(dofs)} DOF in total ({min(dofs)}-{max(dofs)} each), bump fields, "
                       f"greedy aggregation", "ms": round(t_multi * 1e3, 2), "singles_ms": round(t_seq * 1e3, 2),
           "autotune": tune_multi.strip(),
           "speedup_vs_fp64_singles": round(t_seq / t_multi, 3),
           "all_converged": bool(all(reps["converged"])), "err_vs_oracle": err}
    log(f"multi-mesh: {t_multi * 1e3:.1f} ms vs {t_seq * 1e3:.1f} ms sequential; errors {err}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", default="96,416,12,2", help="disc nr,ntheta,nz,degree")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only the full CPU protocol: the oracle on the headline disc with all cores (median of 3) "
                         "and with one thread on the 1/8 disc; prints one JSON line")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision, thermal, 64-load-case and 32-mesh forms")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configurations")
    ap.add_argument("--coarse-sym", type=int, default=1, choices=(0, 1),
                    help="store the coarse operators by their upper triangle (amg_options.coarse_sym)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the build targets a single MI355X); --gpus {args.gpus} is not "
              f"supported", file=sys.stderr)
        sys.exit(2)
    if args.cpu_full:
        print(json.dumps({"cpu_baseline_full": cpu_baseline_full()}), flush=True)
        return
    os.environ.setdefault("TE_VERBOSE", "1")
    ensure_built()
    import numpy as np
    import torch

    import meshgen as mg
    import paper_1804_10060_amd as te
    from paper_1804_10060_amd._lib import KERNEL_CLASSES

    nr, nth, nz, deg = (int(x) for x in args.grid.split(","))
    log(f"generating disc P{deg} {nr}x{nth}x{nz}")
    prob = mg.disc_problem(nr, nth, nz, deg, seed=0)
    m = prob.mesh
    dev = torch.device("cuda:0")
    coords = torch.from_numpy(m.coords).to(dev)
    cells = torch.from_numpy(m.cells).to(dev)
    T = torch.from_numpy(prob.T).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    torch.cuda.synchronize()

    # HBM copy probe (context, and the reference kernel for counter scaling)
    probe = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    probe2 = torch.empty_like(probe)
    probe2.copy_(probe)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        probe2.copy_(probe)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * probe.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    # a read-only 1 GiB reduction: the second calibration point of the read counter
    probe.zero_()
    float(probe.sum())
    del probe, probe2
    log(f"copy probe: {copy_gbs:.0f} GB/s")

    log("assembly")
    torch.cuda.synchronize()
    ta = time.perf_counter()
    A, b = te.assemble(coords, cells, deg, prob.E, prob.nu, prob.alpha, prob.T_ref, T, mask=mask)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - ta
    log(f"assembly {t_asm * 1e3:.1f} ms, nnzb {A.nnzb}")
    log("AMG setup")
    ts = time.perf_counter()
    h = te.AMG(A, coords, mask, coarse_sym=args.coarse_sym)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - ts
    info = h.info()
    log(f"setup {t_setup:.1f}s levels {info['n_dof']}")

    tune_report, t_tune = "", 0.0
    if not args.no_tune:
        t0 = time.perf_counter()
        tune_report = h.autotune()
        t_tune = time.perf_counter() - t0
        log(f"autotune {t_tune:.2f}s\n" + tune_report)

    for w in range(args.warmup):
        u, rep = h.solve(b)
        log(f"warmup {w}: {rep.iters[0]} it, {rep.time_ms:.1f} ms, relres {rep.relres_true[0]:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for k in range(args.steps):
        u, rep = h.solve(b, profile=True)
        reps.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k, rep in enumerate(reps):
        log(f"step {k}: {rep.iters[0]} it, {rep.time_ms:.1f} ms, relres {rep.relres_true[0]:.2e}")
    assert all(r.converged[0] for r in reps), "solve did not converge"
    ms_per_step = (t1 - t0) / args.steps * 1e3
    value = m.n_dof * args.steps / (t1 - t0)

    # per-class kernel times over the timed region
    kms = np.zeros(len(KERNEL_CLASSES))
    kn = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
    for r in reps:
        kms += np.array(r.kernel_ms)
        kn += np.array(r.kernel_launches)
    algo = algorithmic_bytes(info, m.n_nodes, A.nnzb)
    kernels = {}
    for i, name in enumerate(KERNEL_CLASSES):
        if kn[i] == 0:
            continue
        avg = kms[i] / kn[i]
        ent = {"total_ms": round(kms[i] / args.steps, 3), "launches_per_step": int(kn[i] // args.steps),
               "avg_ms": round(avg, 4)}
        if name in algo:
            ent["algo_bytes"] = int(algo[name])
            ent["GBps"] = round(algo[name] / (avg * 1e-3) / 1e9, 1)
        kernels[name] = ent
    # CG vector work per iteration (float64): u += a p, r -= a q with the (r, r) partials (read u, r, p, q;
    # write u, r), (r, z) (read r, z), p = z + b p (read z, p; write p): 11 nodal vectors
    if "vector" in kernels and "Ap" in kernels:
        iters = kn[KERNEL_CLASSES.index("Ap")] / args.steps
        vb = 11 * 3 * 8 * m.n_nodes * iters
        kernels["vector"]["algo_bytes_per_step"] = int(vb)
        kernels["vector"]["GBps"] = round(vb / (kernels["vector"]["total_ms"] * 1e-3) / 1e9, 1)
    single = [k for k in ("Ap", "pre_smooth", "residual", "post_init", "post_smooth") if k in kernels]
    dom = max(single, key=lambda k: kernels[k]["total_ms"])
    achieved = kernels[dom]["GBps"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "kernel_symbol": {"post_smooth": "k_sell1<3,3,double,double,double,EpiChebStep<double,true,false>>",
                                  "pre_smooth": "k_sell1<3,3,double,double,double,EpiChebStep<double,true,true>>",
                                  "Ap": "k_sell1<3,3,double,double,double,EpiDot>",
                                  "residual": "k_sell1<3,3,double,double,double,EpiResid<double,false>>",
                                  "post_init": "k_sell1<3,3,double,double,double,EpiChebInit<double>>"}[dom],
                "algo_bytes_per_launch": kernels[dom]["algo_bytes"]}

    # HBM traffic of the dominant kernel from the committed counter runs,
    # valid only while the kernel source is the one that was measured
    tj = os.path.join(ROOT, "profiles", "disc_p2_12M_fp64_traffic.json")
    if os.path.exists(tj) and (nr, nth, nz, deg) == (96, 416, 12, 2):
        import hashlib
        t = json.load(open(tj))
        csrc = os.path.join(ROOT, "paper_1804_10060_amd", "csrc")
        digest = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                         for f in ("te_dev.h", "te_kernels.hip", "te_internal.h"))).hexdigest()
        if digest == t.get("kernel_source_sha256") and dom in t.get("per_launch", {}):
            roofline["traffic"] = t["per_launch"][dom]["traffic_bytes"]
            roofline["traffic_source"] = "profiles/disc_p2_12M_fp64_hbm_counters.md"

    # error against the stored float64 oracle solution of this disc
    err_vs_oracle = None
    golden = None
    if (nr, nth, nz, deg) == (96, 416, 12, 2):
        from tests import golden_c2
        golden = golden_c2.load()
        es, ep = golden_c2.errors(u.cpu().numpy(), golden)
        err_vs_oracle = {"sampled": es, "projected": ep, "oracle_iters": golden["iters"],
                         "aggregates_equal": all(golden_c2.agg_digest(h.aggregates(l)) == dg
                                                 for l, (_, dg) in golden["agg"].items()),
                         "source": "tests/golden/disc_p2_12m_oracle.txt (C++ oracle, 4096 sampled DOFs and 8 "
                                   "Gaussian projections)"}
        log(f"vs oracle: sampled {es:.2e}, projected {ep:.2e}")

    forms = {}
    if not args.no_forms:
        u64 = u.clone()
        um, repm = h.solve(b, precision="mixed")
        diff = float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64))
        forms["mixed_fp32_vcycle"] = {"ms": round(repm.time_ms, 2), "iters": repm.iters[0],
                                      "relres_true": repm.relres_true[0], "rel_diff_vs_fp64": diff,
                                      "speedup_vs_fp64": round(reps[-1].time_ms / repm.time_ms, 3)}
        # the float32 V-cycle kernels (values and vectors 4 bytes; the outer product stays float64)
        _, repp = h.solve(b, precision="mixed", profile=True)
        algo32 = algorithmic_bytes(info, m.n_nodes, A.nnzb, vt=4)
        k32 = {}
        for i, name in enumerate(KERNEL_CLASSES):
            if name in algo32 and name != "Ap" and repp.kernel_launches[i]:
                avg = repp.kernel_ms[i] / repp.kernel_launches[i]
                k32[name] = {"avg_ms": round(avg, 4), "algo_bytes": int(algo32[name]),
                             "GBps": round(algo32[name] / (avg * 1e-3) / 1e9, 1),
                             "frac": round(algo32[name] / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        forms["mixed_fp32_vcycle"]["fp32_kernels"] = k32
        if golden is not None:
            es, ep = golden_c2.errors(um.cpu().numpy(), golden)
            forms["mixed_fp32_vcycle"]["err_vs_oracle"] = {"sampled": es, "projected": ep}
        log(f"mixed: {repm.iters[0]} it, {repm.time_ms:.1f} ms, diff vs fp64 {diff:.2e}")
        forms["thermal_steady"] = thermal_form(torch, dev, ms_per_step)
        forms["block_rhs_64"] = block_rhs_form(te, torch, dev)
        forms["multi_mesh_32"] = multi_mesh_form(te, torch, dev)
        forms["learned_guess_small"] = learned_form_small(torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()

    out = {
        "metric": METRIC, "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"turbine-disc proxy r_in=0.1 r_out=0.5 t=0.05, structured Kuhn tets "
                               f"{nr}x{nth}x{nz}, P{deg}, {m.n_dof} DOF, E=200e9 nu=0.3 alpha=1.2e-5, "
                               f"T = 300->900 K ramp + 8 seeded hot spots (seed 0), bore clamped; "
                               f"PCG + SA-AMG (6 rigid-body modes, Chebyshev 2) to true relres 1e-8 from u0=0",
                   "n_dof": m.n_dof, "nnzb": A.nnzb, "levels_dof": info["n_dof"],
                   "iterations": reps[-1].iters[0], "parallelism": "single GPU"},
        "time_solve_ms": round(ms_per_step, 2),
        "time_solve_ms_median": round(statistics.median(r.time_ms for r in reps), 2),
        "time_solve_ms_min": round(min(r.time_ms for r in reps), 2),
        "time_assembly_ms": round(t_asm * 1e3, 2),
        "time_setup_ms": round(t_setup * 1e3, 1),
        "time_autotune_ms": round(t_tune * 1e3, 1),
        "dof_per_s_with_setup": m.n_dof / (t_asm + t_setup + ms_per_step * 1e-3),
        "err_vs_oracle": err_vs_oracle,
        "roofline": roofline,
        "kernels": kernels,
        "autotune": [ln for ln in tune_report.splitlines() if ln.strip()],
        "copy_probe_GBps": round(copy_gbs, 1),
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
