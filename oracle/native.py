"""Oracle, large-size form: ctypes binding of the plain C++17/OpenMP
restatement in ``native/te_oracle.cpp`` of the float64 oracle (assembly of
eq. wf_elastic with Dirichlet elimination, smoothed-aggregation AMG of
Sec. 2.1.3 and 5.1, preconditioned CG of Sec. 2.1.2), for sizes the NumPy
oracle cannot reach (the 12M-DOF disc).

TEST INFRASTRUCTURE ONLY (see the package docstring).  It is pinned to the
NumPy oracle element by element at small sizes and by the same closed forms
(``tests/test_oracle_native.py``).  Built with g++ (no HIP); shares nothing
with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "te_oracle.cpp")
LIB = os.path.join(HERE, "native", "libte_oracle.so")

_lib = None


def build(verbose=False):
    """Compile the oracle library with g++ (always recompiles)."""
    cmd = ["g++", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed for the oracle:\n{r.stderr[-4000:]}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Opts(C.Structure):
    _fields_ = [("theta0", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("lanczos_steps", C.c_int32), ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
                ("cheb_safety", C.c_double), ("max_coarse_ratio", C.c_double), ("aggregation", C.c_int32),
                ("threads", C.c_int32)]


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ora_max_threads": ([], C.c_int),
        "ora_assemble": ([i64, i64, i32, vp, vp, d, d, d, d, vp, vp, vp, vp, i32], vp),
        "ora_sys_nnzb": ([vp], i64),
        "ora_sys_time": ([vp], d),
        "ora_sys_get": ([vp, vp, vp, vp, vp], None),
        "ora_sys_free": ([vp], None),
        "ora_setup": ([vp, C.POINTER(Opts), vp, i32, C.POINTER(vp)], C.c_int),
        "ora_hier_free": ([vp], None),
        "ora_levels": ([vp], i32),
        "ora_setup_time": ([vp], d),
        "ora_level_info": ([vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(d), C.POINTER(i64)],
                           None),
        "ora_level_matrix": ([vp, i32, i32, vp, vp, vp, C.POINTER(i64), C.POINTER(i64)], None),
        "ora_level_agg": ([vp, i32, vp], None),
        "ora_vcycle": ([vp, vp, vp], None),
        "ora_pcg": ([vp, vp, vp, d, i32, i32, i32, C.POINTER(i32), C.POINTER(d), vp, C.POINTER(d)], C.c_int),
    }
    for name, (a, r) in sig.items():
        f = getattr(lib, name)
        f.argtypes = a
        f.restype = r
    _lib = lib
    return lib


def _p(x):
    return None if x is None else x.ctypes.data


class System:
    """Assembled, Dirichlet-eliminated system held by the oracle library."""

    def __init__(self, coords, cells, degree, E, nu, alpha, T_ref, T, f=None, mask=None, u_bc=None, threads=0):
        lib = load()
        self._keep = [np.ascontiguousarray(coords, np.float64), np.ascontiguousarray(cells, np.int32),
                      np.ascontiguousarray(T, np.float64),
                      None if f is None else np.ascontiguousarray(f, np.float64),
                      None if mask is None else np.ascontiguousarray(mask, np.uint8),
                      None if u_bc is None else np.ascontiguousarray(u_bc, np.float64)]
        X, cl, Tt, ff, mm, ub = self._keep
        self.n = X.shape[0]
        self._h = lib.ora_assemble(self.n, cl.shape[0], int(degree), _p(X), _p(cl), float(E), float(nu), float(alpha),
                                   float(T_ref), _p(Tt), _p(ff), _p(mm), _p(ub), int(threads))
        self.nnzb = lib.ora_sys_nnzb(self._h)
        self.time_assemble = lib.ora_sys_time(self._h)

    @classmethod
    def from_problem(cls, prob, u_bc=None, threads=0):
        m = prob.mesh
        return cls(m.coords, m.cells, m.degree, prob.E, prob.nu, prob.alpha, prob.T_ref, prob.T, prob.f, prob.mask,
                   u_bc, threads)

    def b(self):
        out = np.empty(3 * self.n)
        load().ora_sys_get(self._h, None, None, None, _p(out))
        return out

    def matrix(self):
        ptr = np.empty(self.n + 1, np.int64)
        col = np.empty(self.nnzb, np.int32)
        val = np.empty((self.nnzb, 3, 3))
        load().ora_sys_get(self._h, _p(ptr), _p(col), _p(val), None)
        return sp.bsr_matrix((val, col, ptr), shape=(3 * self.n, 3 * self.n))

    def free(self):
        if self._h:
            load().ora_sys_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclasses.dataclass
class LevelInfo:
    n_rows: int
    nnzb: int
    bs: int
    lam: float
    p_nnzb: int


class RankError(RuntimeError):
    pass


class Hierarchy:
    def __init__(self, system: System, theta0=0.08, coarse_max=3000, max_levels=10, lanczos_steps=20, cheb_degree=2,
                 cheb_ratio=10.0, cheb_safety=1.1, max_coarse_ratio=0.8, aggregation="mis2", threads=0,
                 aggregates=None):
        lib = load()
        self.opts = Opts(theta0, coarse_max, max_levels, lanczos_steps, cheb_degree, cheb_ratio, cheb_safety,
                         max_coarse_ratio, 1 if aggregation == "mis2" else 0, threads)
        self.system = system
        h = C.c_void_p()
        arr = None
        n_given = 0
        if aggregates is not None:
            keep = [np.ascontiguousarray(a, np.int32) for a in aggregates]
            self._agg_keep = keep
            arr = (C.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
            n_given = len(keep)
        code = lib.ora_setup(system._h, C.byref(self.opts), arr, n_given, C.byref(h))
        self._h = h.value
        if code == -6:
            raise RankError("rank-deficient aggregate without a neighbour")
        if code != 0:
            raise RuntimeError(f"oracle setup failed ({code})")
        self.time_setup = lib.ora_setup_time(self._h)
        self.levels = []
        for l in range(lib.ora_levels(self._h)):
            nr, nz, bs, lam, pz = C.c_int64(), C.c_int64(), C.c_int32(), C.c_double(), C.c_int64()
            lib.ora_level_info(self._h, l, C.byref(nr), C.byref(nz), C.byref(bs), C.byref(lam), C.byref(pz))
            self.levels.append(LevelInfo(nr.value, nz.value, bs.value, lam.value, pz.value))

    def _mat(self, l, which):
        lib = load()
        nz, nr = C.c_int64(), C.c_int64()
        lib.ora_level_matrix(self._h, l, which, None, None, None, C.byref(nz), C.byref(nr))
        lv = self.levels[l]
        br, bc = {0: (lv.bs, lv.bs), 1: (lv.bs, 6), 2: (6, lv.bs)}[which]
        ptr = np.empty(nr.value + 1, np.int64)
        col = np.empty(nz.value, np.int32)
        val = np.empty((nz.value, br, bc))
        lib.ora_level_matrix(self._h, l, which, _p(ptr), _p(col), _p(val), None, None)
        ncols = {0: nr.value * bc, 1: self.levels[l + 1].n_rows * 6 if which else 0, 2: lv.n_rows * lv.bs}[which]
        return sp.bsr_matrix((val, col, ptr), shape=(nr.value * br, ncols))

    def A(self, l):
        return self._mat(l, 0)

    def P(self, l):
        return self._mat(l, 1)

    def R(self, l):
        return self._mat(l, 2)

    def aggregates(self, l):
        out = np.empty(self.levels[l].n_rows, np.int32)
        load().ora_level_agg(self._h, l, _p(out))
        return out

    def vcycle(self, r):
        r = np.ascontiguousarray(r, np.float64)
        z = np.empty_like(r)
        load().ora_vcycle(self._h, _p(r), _p(z))
        return z

    def pcg(self, b, u0=None, rtol=1e-8, maxit=500, max_replace=3, flexible=False):
        b = np.ascontiguousarray(b, np.float64)
        u = np.zeros_like(b) if u0 is None else np.array(u0, np.float64, copy=True)
        it, rel, t = C.c_int32(), C.c_double(), C.c_double()
        hist = np.full(maxit + 1, np.nan)
        code = load().ora_pcg(self._h, _p(b), _p(u), float(rtol), int(maxit), int(max_replace), int(flexible),
                              C.byref(it), C.byref(rel), _p(hist), C.byref(t))
        if code == -4:
            raise RuntimeError("oracle CG breakdown")
        return PcgResult(u, it.value, code == 0, rel.value, hist[:it.value + 1], t.value)

    def free(self):
        if self._h:
            load().ora_hier_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclasses.dataclass
class PcgResult:
    u: np.ndarray
    iters: int
    converged: bool
    relres_true: float
    history: np.ndarray
    time_solve: float


def max_threads():
    return load().ora_max_threads()
