"""Writes tests/golden/thermal_disc_p2_4m_oracle.txt: the float64 oracle's
steady temperature of the P2 disc 96 x 416 x 12 (4,014,400 nodes; hub, web
and rim with the thermal tables of meshgen.turbine_thermal_tables; heat
exchange on every boundary face, meshgen.disc_robin_faces), solved by Newton
from 400 K to relative residual 1e-9 (Sec. 5.2) with CG and classical AMG
(the kept preconditioner), in the format of the 12M-DOF file: Newton and CG
iterations, |T|_2, Gaussian projections and sampled nodes.

Calls only the oracle (oracle/thermal, oracle/camg, oracle/krylov) and the
input generator; about 15 minutes and 30 GB:
    python tests/golden/make_thermal_disc_p2.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402
from oracle import camg, thermal  # noqa: E402
from tests.golden_c2 import PROJ_SEEDS, THERMAL_PATH, projection_vector, sample_indices  # noqa: E402


def main():
    t0 = time.time()
    m = mg.disc_mesh(*mg.DISC_P2_12M)
    P = thermal.problem_from_meshgen(m, mg.disc_thermal_materials(m), mg.disc_robin_faces(m))
    pre = thermal.ReusedPreconditioner(camg.CAMGOptions())
    res = thermal.newton(P, np.full(m.n_nodes, 400.0), pre)
    T = res.T
    n = T.size
    lines = ["# Float64 oracle steady temperature of the P2 disc 96x416x12 (4,014,400 nodes), hub/web/rim thermal",
             "# tables, heat exchange on every boundary face; Newton from 400 K to relative residual 1e-9 with CG",
             "# and classical AMG (theta 0.25, PMIS, direct interpolation, l1 hybrid Gauss-Seidel blocks of 128,",
             "# coarse_max 500), the correction CG to 1e-8.  Written by tests/golden/make_thermal_disc_p2.py.",
             f"iters {res.iters}", "lin_iters " + " ".join(str(i) for i in res.lin_iters),
             "res_history " + " ".join(repr(float(h)) for h in res.res_history),
             f"norm2 {float(np.linalg.norm(T))!r}"]
    for s in PROJ_SEEDS:
        lines.append(f"proj {s} {float(projection_vector(s, n) @ T)!r}")
    for i in sample_indices(n).tolist():
        lines.append(f"sample {i} {float(T[i])!r}")
    with open(THERMAL_PATH, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {THERMAL_PATH}: {res.iters} Newton steps, CG {res.lin_iters}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
