"""Writes tests/golden/disc_p2_12m_oracle.txt: the float64 oracle's solution of
the 12,043,200-DOF P2 disc (96 x 416 x 12, temperature seed 0, bore clamped;
the headline workload) at rtol 1e-8, summarised for tests that cannot afford
the oracle run: iterations, true residual, the level sizes and a SHA-256 of
each level's aggregate map, |u|_2, projections of u on seeded Gaussian vectors
and u at seeded sample DOFs.

Calls only the oracle (the C++17/OpenMP form in oracle/native) and the input
generator.  Takes about 3 minutes and 45 GB of host memory on 8 cores:
    python tests/golden/make_disc_p2_12m.py
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

from tests.golden_c2 import PATH as OUT, agg_digest, projection_vector, sample_indices, PROJ_SEEDS  # noqa: E402


def main():
    t0 = time.time()
    prob = mg.disc_problem(*mg.DISC_P2_12M, seed=0)
    S = native.System.from_problem(prob)
    H = native.Hierarchy(S)
    res = H.pcg(S.b(), rtol=1e-8)
    u = res.u
    n = u.size
    lines = ["# Float64 oracle solution of the P2 disc 96x416x12 (12,043,200 DOF; temperature seed 0;",
             "# bore clamped) at true relative residual 1e-8: MIS-2 aggregation, theta0 0.08, coarse_max 3000,",
             "# Chebyshev degree 2, 20 Lanczos steps, the solver of Sec. 5.1.",
             "# Written by tests/golden/make_disc_p2_12m.py with the C++ oracle (oracle/native).",
             f"iters {res.iters}", f"relres {res.relres_true!r}", f"norm2 {float(np.linalg.norm(u))!r}",
             "level_dof " + " ".join(str(l.n_rows * l.bs) for l in H.levels)]
    for l in range(len(H.levels) - 1):
        a = H.aggregates(l)
        lines.append(f"agg {l} {int(a.max()) + 1} {agg_digest(a)}")
    for s in PROJ_SEEDS:
        lines.append(f"proj {s} {float(projection_vector(s, n) @ u)!r}")
    for i in sample_indices(n).tolist():
        lines.append(f"sample {i} {float(u[i])!r}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {OUT}: {res.iters} iterations, relres {res.relres_true:.2e}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
