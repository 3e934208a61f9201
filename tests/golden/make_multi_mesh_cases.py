"""Writes tests/golden/multi_mesh{27,25}_oracle.txt: the float64 oracle's
solutions of the smallest (14,400 DOF) and the largest (534,276 DOF) of the 32
P1 discs of the multi-mesh workload (meshgen.multi_mesh_sizes(32), bump field
of each mesh's seed, bore clamped, greedy aggregation) at rtol 1e-8, in the
format of the 12M-DOF file.

Calls only the oracle (oracle/native) and the input generator:
    python tests/golden/make_multi_mesh_cases.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402
from oracle import native  # noqa: E402
from tests.golden_c2 import (MULTI_MESH_INDICES, PROJ_SEEDS, agg_digest, multi_mesh_path,  # noqa: E402
                             projection_vector, sample_indices)


def main():
    sizes = mg.multi_mesh_sizes(32, lo=1e4, hi=5e5)
    for i in MULTI_MESH_INDICES:
        nr, nth, nz, seed = sizes[i]
        prob = mg.disc_problem(nr, nth, nz, 1, seed=0)
        prob.T = mg.disc_temperature_bumps(prob.mesh, seed)
        S = native.System.from_problem(prob)
        H = native.Hierarchy(S, aggregation="greedy")
        res = H.pcg(S.b(), rtol=1e-8)
        u = res.u
        n = u.size
        lines = [f"# Float64 oracle solution of mesh {i} of the 32-mesh workload: P1 disc {nr}x{nth}x{nz} ({n} DOF),",
                 f"# bump field of seed {seed}, bore clamped, at true relative residual 1e-8: greedy aggregation,",
                 "# theta0 0.08, coarse_max 3000, Chebyshev degree 2, 20 Lanczos steps, the solver of Sec. 5.1.",
                 "# Written by tests/golden/make_multi_mesh_cases.py with the C++ oracle (oracle/native).",
                 f"iters {res.iters}", f"relres {res.relres_true!r}", f"norm2 {float(np.linalg.norm(u))!r}",
                 "level_dof " + " ".join(str(l.n_rows * l.bs) for l in H.levels)]
        for l in range(len(H.levels) - 1):
            a = H.aggregates(l)
            lines.append(f"agg {l} {int(a.max()) + 1} {agg_digest(a)}")
        for s in PROJ_SEEDS:
            lines.append(f"proj {s} {float(projection_vector(s, n) @ u)!r}")
        for j in sample_indices(n).tolist():
            lines.append(f"sample {j} {float(u[j])!r}")
        with open(multi_mesh_path(i), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print(f"mesh {i}: {n} DOF, {res.iters} iterations, relres {res.relres_true:.2e}", flush=True)


if __name__ == "__main__":
    main()
