"""Writes tests/golden/disc_p1_2m_case{1000,1063}_oracle.txt: the float64
oracle's solutions of two of the 64 load cases of the block-RHS workload (P1
disc 104 x 452 x 13, 1,993,320 DOF; T = T_ref + 4-16 Gaussian bumps of the
case's seed; bore clamped; greedy aggregation, the rule the P1 forms use) at
rtol 1e-8, in the format of the 12M-DOF file (iterations, |u|_2, aggregate
digests, Gaussian projections, sampled DOFs).

Calls only the oracle (oracle/native) and the input generator:
    python tests/golden/make_disc_p1_2m_cases.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402
from oracle import native  # noqa: E402
from tests.golden_c2 import (LOAD_CASE_SEEDS, PROJ_SEEDS, agg_digest, load_case_path,  # noqa: E402
                             projection_vector, sample_indices)


def main():
    t0 = time.time()
    prob = mg.disc_problem(*mg.DISC_P1_2M, seed=0)
    m = prob.mesh
    H = None
    for seed in LOAD_CASE_SEEDS:
        T = mg.disc_temperature_bumps(m, seed)
        S = native.System(m.coords, m.cells, 1, prob.E, prob.nu, prob.alpha, prob.T_ref, T, mask=prob.mask)
        if H is None:  # the matrix does not depend on the load case
            H = native.Hierarchy(S, aggregation="greedy")
            Hs = S
        res = H.pcg(S.b(), rtol=1e-8)
        u = res.u
        n = u.size
        lines = [f"# Float64 oracle solution of load case {seed} (T = T_ref + bumps of seed {seed}) on the P1 disc",
                 "# 104x452x13 (1,993,320 DOF; bore clamped) at true relative residual 1e-8: greedy aggregation,",
                 "# theta0 0.08, coarse_max 3000, Chebyshev degree 2, 20 Lanczos steps, the solver of Sec. 5.1.",
                 "# Written by tests/golden/make_disc_p1_2m_cases.py with the C++ oracle (oracle/native).",
                 f"iters {res.iters}", f"relres {res.relres_true!r}", f"norm2 {float(np.linalg.norm(u))!r}",
                 "level_dof " + " ".join(str(l.n_rows * l.bs) for l in H.levels)]
        for l in range(len(H.levels) - 1):
            a = H.aggregates(l)
            lines.append(f"agg {l} {int(a.max()) + 1} {agg_digest(a)}")
        for s in PROJ_SEEDS:
            lines.append(f"proj {s} {float(projection_vector(s, n) @ u)!r}")
        for i in sample_indices(n).tolist():
            lines.append(f"sample {i} {float(u[i])!r}")
        with open(load_case_path(seed), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print(f"case {seed}: {res.iters} iterations, relres {res.relres_true:.2e}", flush=True)
    del Hs
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
