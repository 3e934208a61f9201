"""The stored float64 oracle solution of the 12,043,200-DOF P2 disc
(tests/golden/disc_p2_12m_oracle.txt, written by
tests/golden/make_disc_p2_12m.py from the C++ oracle) and the error of a
solution against it.  Holds no arithmetic of the method: sampling rules and
the file format only."""
from __future__ import annotations

import hashlib
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "disc_p2_12m_oracle.txt")
N_SAMPLES = 4096
SAMPLE_SEED = 12_043_200
PROJ_SEEDS = list(range(1000, 1008))


def sample_indices(n_dof):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_dof, N_SAMPLES, replace=False))


def projection_vector(seed, n_dof):
    return np.random.default_rng(seed).standard_normal(n_dof)


def agg_digest(agg):
    return hashlib.sha256(np.ascontiguousarray(agg, dtype="<i4").tobytes()).hexdigest()


def load(path=PATH):
    g = {"agg": {}, "proj": {}, "sample_idx": [], "sample_val": []}
    with open(path) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "iters":
                g["iters"] = int(t[1])
            elif t[0] in ("relres", "norm2"):
                g[t[0]] = float(t[1])
            elif t[0] == "level_dof":
                g["level_dof"] = [int(x) for x in t[1:]]
            elif t[0] == "agg":
                g["agg"][int(t[1])] = (int(t[2]), t[3])
            elif t[0] == "proj":
                g["proj"][int(t[1])] = float(t[2])
            elif t[0] == "sample":
                g["sample_idx"].append(int(t[1]))
                g["sample_val"].append(float(t[2]))
    g["sample_idx"] = np.array(g["sample_idx"], np.int64)
    g["sample_val"] = np.array(g["sample_val"])
    return g


def errors(u, g):
    """(sampled, projected) estimates of |u - u_orc|_2 / |u_orc|_2: over the
    4096 stored DOFs, and from the 8 stored Gaussian projections (each
    (w, u - u_orc) has variance |u - u_orc|^2)."""
    u = np.asarray(u, np.float64).reshape(-1)
    d = u[g["sample_idx"]] - g["sample_val"]
    e_sample = float(np.linalg.norm(d) / np.linalg.norm(g["sample_val"]))
    sq = [(projection_vector(s, u.size) @ u - p) ** 2 for s, p in g["proj"].items()]
    e_proj = float(np.sqrt(np.mean(sq)) / g["norm2"])
    return e_sample, e_proj
