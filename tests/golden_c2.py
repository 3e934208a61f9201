"""Stored float64 oracle solutions of the benchmark workloads and the error
of a solution against them: the 12,043,200-DOF P2 disc
(tests/golden/disc_p2_12m_oracle.txt) and two load cases of the 64-case
1,993,320-DOF P1 disc (tests/golden/disc_p1_2m_case*_oracle.txt), written by
tests/golden/make_disc_p2_12m.py and make_disc_p1_2m_cases.py from the C++
oracle, and two meshes of the 32-mesh form (tests/golden/multi_mesh*_oracle.txt,
make_multi_mesh_cases.py).  Holds no arithmetic of the method: sampling rules and
the file format only."""
from __future__ import annotations

import hashlib
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PATH = os.path.join(GOLDEN, "disc_p2_12m_oracle.txt")
# the 64-load-case form: P1 disc 104 x 452 x 13, bump fields of seeds 1000..1063
LOAD_CASE_SEEDS = (1000, 1063)


def load_case_path(seed):
    return os.path.join(GOLDEN, f"disc_p1_2m_case{seed}_oracle.txt")


# the steady thermal solve of the P2 disc 96 x 416 x 12 (4,014,400 nodes)
THERMAL_PATH = os.path.join(GOLDEN, "thermal_disc_p2_4m_oracle.txt")

# the 32-mesh form: the smallest and the largest of meshgen.multi_mesh_sizes(32)
MULTI_MESH_INDICES = (27, 25)


def multi_mesh_path(index):
    return os.path.join(GOLDEN, f"multi_mesh{index}_oracle.txt")
N_SAMPLES = 4096
SAMPLE_SEED = 12_043_200
PROJ_SEEDS = list(range(1000, 1008))


def sample_indices(n_dof):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_dof, min(N_SAMPLES, n_dof), replace=False))


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
            elif t[0] == "lin_iters":
                g["lin_iters"] = [int(x) for x in t[1:]]
            elif t[0] == "res_history":
                g["res_history"] = [float(x) for x in t[1:]]
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
