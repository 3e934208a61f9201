"""Python binding of the thermal solve (include/te.h: fe_assemble_thermal,
camg_*, thermal_*): argument marshalling only, every step runs in the HIP
library.  The heat equation of eq. wf_thermal (Sec. 3) solved by Newton's
method (Sec. 3.2) with CG and classical AMG (Sec. 5.1)."""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import _lib
from ._lib import check, load


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, n, name):
    torch = _torch()
    if t is None:
        return
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA tensor of {dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    del torch


@dataclasses.dataclass
class CsrMatrix:
    """Scalar compressed rows on the device (te_csr)."""
    row_ptr: object   # int64 [n+1]
    col_idx: object   # int32 [nnz]
    val: object       # float64 [nnz]

    @property
    def n(self):
        return self.row_ptr.numel() - 1

    @property
    def nnz(self):
        return self.col_idx.numel()

    def c(self):
        return _lib.TeCsr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val.cpu().numpy(), self.col_idx.cpu().numpy(), self.row_ptr.cpu().numpy()),
                             shape=(self.n, self.n))


class Tables:
    """Host copies of the material tables, kept alive for the C call."""

    def __init__(self, T, kappa, cv, rho):
        self.T = np.ascontiguousarray(T, np.float64)
        self.kappa = np.ascontiguousarray(kappa, np.float64)
        self.cv = np.ascontiguousarray(cv, np.float64)
        self.rho = np.ascontiguousarray(rho, np.float64)
        nm, npt = self.T.shape
        if self.kappa.shape != (nm, npt) or self.cv.shape != (nm, npt) or self.rho.shape != (nm,):
            raise ValueError("table shapes disagree")
        self.c = _lib.TeThermalTables(nm, npt, self.T.ctypes.data, self.kappa.ctypes.data, self.cv.ctypes.data,
                                      self.rho.ctypes.data)

    @classmethod
    def of(cls, mats):
        return cls(mats.T, mats.kappa, mats.cv, mats.rho)


def _mesh(coords, cells, degree):
    torch = _torch()
    npe = 4 if degree == 1 else 10
    _need(coords, torch.float64, coords.shape[0] * 3, "coords")
    _need(cells, torch.int32, cells.shape[0] * npe, "cells")
    return _lib.TeMesh(coords.shape[0], cells.shape[0], degree, coords.data_ptr(), cells.data_ptr())


def _robin(faces, h, T_bc, degree):
    torch = _torch()
    if faces is None or faces.numel() == 0:
        return _lib.TeRobin(0, None, None, None)
    npf = 3 if degree == 1 else 6
    nf = faces.shape[0]
    _need(faces, torch.int32, nf * npf, "faces")
    _need(h, torch.float64, nf, "h")
    _need(T_bc, torch.float64, nf, "T_bc")
    return _lib.TeRobin(nf, faces.data_ptr(), h.data_ptr(), T_bc.data_ptr())


def assemble(coords, cells, degree, tables: Tables, cell_material, T, faces=None, h=None, T_bc=None, T_old=None,
             dt=0.0):
    """fe_assemble_thermal: (J, F) of eq. wf_thermal at T (steady when T_old is
    None, else one backward-Euler step of length dt)."""
    torch = _torch()
    lib = load()
    m = _mesh(coords, cells, degree)
    n = coords.shape[0]
    _need(T, torch.float64, n, "T")
    _need(T_old, torch.float64, n, "T_old")
    _need(cell_material, torch.int32, cells.shape[0], "cell_material")
    rp = torch.empty(n + 1, dtype=torch.int64, device=coords.device)
    nnz = C.c_int64(0)
    check(lib.fe_assemble_pattern(C.byref(m), _ptr(rp), C.byref(nnz), _stream()))
    col = torch.empty(nnz.value, dtype=torch.int32, device=coords.device)
    val = torch.empty(nnz.value, dtype=torch.float64, device=coords.device)
    F = torch.empty(n, dtype=torch.float64, device=coords.device)
    J = CsrMatrix(rp, col, val)
    jc = J.c()
    rb = _robin(faces, h, T_bc, degree)
    check(lib.fe_assemble_thermal(C.byref(m), C.byref(tables.c), _ptr(cell_material), C.byref(rb), _ptr(T),
                                  _ptr(T_old), float(dt), C.byref(jc), _ptr(F), _stream()))
    return J, F


def _camg_options(**kw):
    o = _lib.CamgOptions()
    load().camg_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown classical AMG option {k}")
        setattr(o, k, v)
    return o


class CAMG:
    """camg_setup / camg_apply / camg_pcg_solve / camg_destroy."""

    def __init__(self, A: CsrMatrix, **opts):
        self.opts = _camg_options(**opts)
        self._cd = load()
        self._h = C.c_void_p(0)
        ac = A.c()
        check(self._cd.camg_setup(C.byref(ac), C.byref(self.opts), C.byref(self._h), _stream()))
        self.n = A.n

    def __del__(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_cd", None)
        if h is not None and h.value and lib is not None:
            lib.camg_destroy(h)
            h.value = None

    def info(self):
        i = _lib.CamgInfo()
        check(load().camg_get_info(self._h, C.byref(i)))
        L = i.n_levels
        return {"n_levels": L, "n_rows": list(i.n_rows[:L]), "nnz": list(i.nnz[:L]), "p_nnz": list(i.p_nnz[:L]),
                "setup_ms": i.setup_ms}

    def splitting(self, level):
        n = self.info()["n_rows"][level]
        out = np.empty(n, np.int8)
        check(load().camg_get_splitting(self._h, level, C.c_void_p(out.ctypes.data)))
        return out

    def level_matrix(self, level, which=0):
        """A_l (0), P_l (1) or R_l (2) as a host scipy CSR matrix."""
        import scipy.sparse as sp
        lib = load()
        nr, nz = C.c_int64(0), C.c_int64(0)
        check(lib.camg_get_level_matrix(self._h, level, which, C.byref(nr), C.byref(nz), None, None, None))
        rp = np.empty(nr.value + 1, np.int64)
        col = np.empty(nz.value, np.int32)
        val = np.empty(nz.value, np.float64)
        check(lib.camg_get_level_matrix(self._h, level, which, C.byref(nr), C.byref(nz), C.c_void_p(rp.ctypes.data),
                                        C.c_void_p(col.ctypes.data), C.c_void_p(val.ctypes.data)))
        info = self.info()
        ncol = {0: nr.value, 1: info["n_rows"][level + 1] if which else 0, 2: info["n_rows"][level]}[which]
        return sp.csr_matrix((val, col, rp), shape=(nr.value, ncol))

    def apply(self, level, op, x, y=None):
        torch = _torch()
        _need(x, torch.float64, None, "x")
        if y is None:
            info = self.info()
            lv = level + 1 if op == _lib.TE_CAMG_R else level
            y = torch.zeros(info["n_rows"][lv], dtype=torch.float64, device=x.device)
        check(load().camg_apply(self._h, level, op, _ptr(x), _ptr(y), _stream()))
        return y

    def pcg(self, A: CsrMatrix, b, x0=None, rtol=1e-8, maxit=500, allow_notconv=False):
        torch = _torch()
        _need(b, torch.float64, self.n, "b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        it, rel = C.c_int32(0), C.c_double(0.0)
        ac = A.c()
        code = load().camg_pcg_solve(self._h, C.byref(ac), _ptr(b), _ptr(x), float(rtol), int(maxit), C.byref(it),
                                     C.byref(rel), _stream())
        check(code, allow=(_lib.TE_OK, _lib.TE_ENOTCONV) if allow_notconv else (_lib.TE_OK,))
        return x, it.value, rel.value


@dataclasses.dataclass
class NewtonReport:
    iters: int
    converged: bool
    rebuilds: int
    lin_iters: list
    res_history: list
    time_ms: float
    assembly_ms: float
    setup_ms: float
    solve_ms: float
    code: int


class ThermalSolver:
    """thermal_create / thermal_newton / thermal_destroy for one mesh."""

    def __init__(self, coords, cells, degree, tables: Tables, cell_material, faces=None, h=None, T_bc=None):
        torch = _torch()
        self._cd = load()
        m = _mesh(coords, cells, degree)
        _need(cell_material, torch.int32, cells.shape[0], "cell_material")
        rb = _robin(faces, h, T_bc, degree)
        self._h = C.c_void_p(0)
        check(self._cd.thermal_create(C.byref(m), C.byref(tables.c), _ptr(cell_material), C.byref(rb),
                                      C.byref(self._h), _stream()))
        self.n = coords.shape[0]
        self.n_faces = 0 if faces is None else faces.shape[0]

    def __del__(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_cd", None)
        if h is not None and h.value and lib is not None:
            lib.thermal_destroy(h)
            h.value = None

    def set_exterior(self, T_bc):
        _need(T_bc, _torch().float64, self.n_faces, "T_bc")
        check(load().thermal_set_exterior(self._h, _ptr(T_bc), _stream()))

    def reset_preconditioner(self):
        check(load().thermal_reset_preconditioner(self._h))

    def newton(self, T0, T_old=None, dt=0.0, rtol=1e-9, atol=1e-8, lin_rtol=1e-8, maxit=25, lin_maxit=500,
               rebuild_factor=1.5, allow_notconv=False, **amg_opts):
        """Newton solve of one (steady or backward-Euler) step from T0.
        Returns (T, NewtonReport)."""
        torch = _torch()
        _need(T0, torch.float64, self.n, "T0")
        _need(T_old, torch.float64, self.n, "T_old")
        T = T0.clone()
        o = _lib.NewtonOptions()
        load().newton_options_default(C.byref(o))
        o.rtol, o.atol, o.lin_rtol, o.maxit, o.lin_maxit = rtol, atol, lin_rtol, maxit, lin_maxit
        o.rebuild_factor = rebuild_factor
        for k, v in amg_opts.items():
            if not hasattr(o.amg, k):
                raise TypeError(f"unknown classical AMG option {k}")
            setattr(o.amg, k, v)
        r = _lib.NewtonReport()
        code = load().thermal_newton(self._h, _ptr(T), _ptr(T_old), float(dt), C.byref(o), C.byref(r), _stream())
        check(code, allow=(_lib.TE_OK, _lib.TE_ENOTCONV) if allow_notconv else (_lib.TE_OK,))
        return T, NewtonReport(r.iters, bool(r.converged), r.rebuilds, list(r.lin_iters[:r.iters]),
                               list(r.res_hist[:r.iters + 1]), r.time_ms, r.assembly_ms, r.setup_ms, r.solve_ms,
                               code)
