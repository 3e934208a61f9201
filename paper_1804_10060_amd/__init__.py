"""MI355X thermoelastic PCG + smoothed-aggregation AMG (Python binding).

Thin marshalling layer over the C ABI of include/te.h: every computation runs
in the HIP library libte_amd.so.  PyTorch supplies device memory and the
stream.  Importing this package does not touch the GPU; the library is loaded
on first use and a missing library raises (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import dataclasses

from . import _lib
from ._lib import (TE_OP_A, TE_OP_P, TE_OP_R, TE_OP_SMOOTH, TE_OP_VCYCLE, TE_PREC_FP64, TE_PREC_MIXED, TeError,
                   check, load)

__all__ = ["assemble", "assemble_load", "assemble_materials", "AMG", "MPNN", "solve_multi", "Matrix", "TeError", "load", "TE_PREC_FP64",
           "TE_PREC_MIXED", "TE_OP_A", "TE_OP_P", "TE_OP_R", "TE_OP_SMOOTH", "TE_OP_VCYCLE"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape=None, name="array"):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


@dataclasses.dataclass
class Matrix:
    """3x3-block compressed rows on the device (te_bsr)."""

    row_ptr: object   # int64 [N+1]
    col_idx: object   # int32 [nnzb]
    val: object       # float64 [nnzb, 3, 3]

    @property
    def n(self):
        return self.row_ptr.numel() - 1

    @property
    def nnzb(self):
        return self.col_idx.numel()

    def c(self):
        return _lib.TeBsr(self.n, self.nnzb, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())


def _mesh(coords, cells, degree):
    torch = _torch()
    npe = 4 if degree == 1 else 10
    _dev(coords, torch.float64, (coords.shape[0], 3), "coords")
    _dev(cells, torch.int32, (cells.shape[0], npe), "cells")
    return _lib.TeMesh(coords.shape[0], cells.shape[0], degree, coords.data_ptr(), cells.data_ptr())


def assemble(coords, cells, degree, E, nu, alpha, T_ref, T, f=None, mask=None, u_bc=None):
    """fe_assemble_pattern + fe_assemble_thermoelastic.  Returns (Matrix, b[3N])."""
    torch = _torch()
    lib = load()
    m = _mesh(coords, cells, degree)
    n = coords.shape[0]
    _dev(T, torch.float64, (n,), "T")
    _dev(f, torch.float64, (n, 3), "f")
    _dev(mask, torch.uint8, (n, 3), "mask")
    _dev(u_bc, torch.float64, (n, 3), "u_bc")
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=coords.device)
    nnzb = C.c_int64(0)
    check(lib.fe_assemble_pattern(C.byref(m), _ptr(row_ptr), C.byref(nnzb), _stream()))
    col = torch.empty(nnzb.value, dtype=torch.int32, device=coords.device)
    val = torch.empty((nnzb.value, 3, 3), dtype=torch.float64, device=coords.device)
    b = torch.empty(3 * n, dtype=torch.float64, device=coords.device)
    A = Matrix(row_ptr, col, val)
    mat = _lib.TeMaterial(E, nu, alpha, T_ref)
    bsr = A.c()
    check(lib.fe_assemble_thermoelastic(C.byref(m), C.byref(mat), _ptr(T), _ptr(f), _ptr(mask), _ptr(u_bc),
                                        C.byref(bsr), _ptr(b), _stream()))
    return A, b


def assemble_materials(coords, cells, degree, tables, cell_material, T_ref, T, f=None, faces=None, face_p=None,
                       mask=None, u_bc=None):
    """fe_assemble_pattern + fe_assemble_thermoelastic_materials.
    tables: (T, E, nu, alpha) host arrays [n_materials][n_points];
    cell_material: int32 [C]; faces/face_p: boundary pressure (int32 [F][3|6],
    float64 [F]) or None.  Returns (Matrix, b[3N])."""
    import numpy as np
    torch = _torch()
    lib = load()
    m = _mesh(coords, cells, degree)
    n = coords.shape[0]
    _dev(T, torch.float64, (n,), "T")
    _dev(cell_material, torch.int32, (cells.shape[0],), "cell_material")
    _dev(f, torch.float64, (n, 3), "f")
    _dev(mask, torch.uint8, (n, 3), "mask")
    _dev(u_bc, torch.float64, (n, 3), "u_bc")
    tab = [np.ascontiguousarray(a, dtype=np.float64) for a in tables]
    if tab[0].ndim != 2 or any(a.shape != tab[0].shape for a in tab):
        raise ValueError("tables must be four [n_materials][n_points] arrays")
    mt = _lib.TeMaterialTables(tab[0].shape[0], tab[0].shape[1], *[a.ctypes.data for a in tab], T_ref)
    pr = None
    if faces is not None and faces.shape[0] > 0:
        _dev(faces, torch.int32, (faces.shape[0], 3 if degree == 1 else 6), "faces")
        _dev(face_p, torch.float64, (faces.shape[0],), "face_p")
        pr = _lib.TePressure(faces.shape[0], faces.data_ptr(), face_p.data_ptr())
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=coords.device)
    nnzb = C.c_int64(0)
    check(lib.fe_assemble_pattern(C.byref(m), _ptr(row_ptr), C.byref(nnzb), _stream()))
    col = torch.empty(nnzb.value, dtype=torch.int32, device=coords.device)
    val = torch.empty((nnzb.value, 3, 3), dtype=torch.float64, device=coords.device)
    b = torch.empty(3 * n, dtype=torch.float64, device=coords.device)
    A = Matrix(row_ptr, col, val)
    bsr = A.c()
    check(lib.fe_assemble_thermoelastic_materials(C.byref(m), C.byref(mt), _ptr(cell_material), _ptr(T), _ptr(f),
                                                  C.byref(pr) if pr is not None else None, _ptr(mask), _ptr(u_bc),
                                                  C.byref(bsr), _ptr(b), _stream()))
    return A, b


def assemble_load(coords, cells, degree, E, nu, alpha, T_ref, T, f=None, mask=None):
    """fe_assemble_load for nrhs load cases: T [nrhs, N] -> b [N, 3, nrhs]."""
    torch = _torch()
    lib = load()
    m = _mesh(coords, cells, degree)
    n = coords.shape[0]
    nrhs = T.shape[0]
    _dev(T, torch.float64, (nrhs, n), "T")
    _dev(f, torch.float64, (nrhs, n, 3), "f")
    _dev(mask, torch.uint8, (n, 3), "mask")
    b = torch.empty((n, 3, nrhs), dtype=torch.float64, device=coords.device)
    mat = _lib.TeMaterial(E, nu, alpha, T_ref)
    check(lib.fe_assemble_load(C.byref(m), C.byref(mat), _ptr(T), _ptr(f), _ptr(mask), nrhs, _ptr(b), _stream()))
    return b


@dataclasses.dataclass
class SolveReport:
    iters: list
    converged: list
    relres_true: list
    history: object
    max_iters: int
    time_ms: float
    code: int
    kernel_ms: list
    kernel_launches: list


class AMG:
    """amg_setup / amg_pcg_solve / amg_destroy."""

    def __init__(self, A: Matrix, coords, mask=None, aggregates=None, **opts):
        torch = _torch()
        lib = load()
        n = A.n
        _dev(A.row_ptr, torch.int64, (n + 1,), "row_ptr")
        _dev(A.col_idx, torch.int32, None, "col_idx")
        _dev(A.val, torch.float64, (A.nnzb, 3, 3), "val")
        _dev(coords, torch.float64, (n, 3), "coords")
        _dev(mask, torch.uint8, (n, 3), "mask")
        o = _lib.AmgOptions()
        lib.amg_options_default(C.byref(o))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown AMG option {k}")
            if k == "aggregation" and isinstance(v, str):
                v = {"greedy": _lib.TE_AGG_GREEDY, "mis2": _lib.TE_AGG_MIS2}[v]
            setattr(o, k, v)
        self.opts = o
        self._cd = load()  # kept for __del__, which can run after module teardown
        self._h = C.c_void_p(0)
        bsr = A.c()
        if aggregates is None:
            check(lib.amg_setup(C.byref(bsr), _ptr(coords), _ptr(mask), C.byref(o), C.byref(self._h), _stream()))
        else:
            import numpy as np
            arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in aggregates]
            ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
            check(lib.amg_setup_with_aggregates(C.byref(bsr), _ptr(coords), _ptr(mask), C.byref(o), ptrs,
                                                len(arrs), C.byref(self._h), _stream()))
        self.n = n

    def __del__(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_cd", None)
        if h is not None and h.value and lib is not None:
            lib.amg_destroy(h)
            h.value = None  # in place: module globals may be gone at interpreter exit

    def close(self):
        self.__del__()

    # ---- introspection --------------------------------------------------
    def info(self):
        i = _lib.AmgInfo()
        check(load().amg_get_info(self._h, C.byref(i)))
        L = i.n_levels
        return {"n_levels": L, "n_dof": list(i.n_dof[:L]), "nnzb": list(i.nnzb[:L]), "bs": list(i.bs[:L]),
                "lambda_hat": list(i.lambda_hat[:L]), "p_nnzb": list(i.p_nnzb[:L]), "setup_ms": i.setup_ms,
                "bytes_device": i.bytes_device}

    def aggregates(self, level):
        import numpy as np
        n = self.info()["n_dof"][level] // self.info()["bs"][level]
        out = np.empty(n, np.int32)
        check(load().amg_get_aggregates(self._h, level, C.c_void_p(out.ctypes.data)))
        return out

    def level_matrix(self, level):
        """(row_ptr, col, val[nnzb, bs, bs]) of A_level in natural numbering (host numpy)."""
        import numpy as np
        nr, nz = C.c_int64(0), C.c_int64(0)
        lib = load()
        check(lib.amg_get_level_matrix(self._h, level, C.byref(nr), C.byref(nz), None, None, None))
        bs = self.info()["bs"][level]
        rp = np.empty(nr.value + 1, np.int64)
        col = np.empty(nz.value, np.int32)
        val = np.empty((nz.value, bs, bs), np.float64)
        check(lib.amg_get_level_matrix(self._h, level, C.byref(nr), C.byref(nz), C.c_void_p(rp.ctypes.data),
                                       C.c_void_p(col.ctypes.data), C.c_void_p(val.ctypes.data)))
        return rp, col, val

    def apply(self, level, op, x, y=None, precision=TE_PREC_FP64):
        torch = _torch()
        _dev(x, torch.float64, None, "x")
        if y is None:
            info = self.info()
            lv = level + 1 if op == TE_OP_R else level
            y = torch.zeros(info["n_dof"][lv], dtype=torch.float64, device=x.device)
        check(load().amg_apply(self._h, level, op, precision, _ptr(x), _ptr(y), _stream()))
        return y

    def autotune(self, cache_path=None, use_cache=True):
        """te_autotune: choose each operator's launch configuration; returns the text report."""
        buf = C.create_string_buffer(1 << 16)
        p = cache_path.encode() if cache_path else None
        check(load().te_autotune(self._h, p, int(use_cache), buf, len(buf), _stream()))
        return buf.value.decode()

    def energy_scale(self, b, u0):
        """u0 <- gamma u0, gamma = (b,u0)/(u0,A u0) (0 if the guess cannot beat zero); returns gamma."""
        torch = _torch()
        _dev(b, torch.float64, None, "b")
        _dev(u0, torch.float64, tuple(b.shape), "u0")
        g = C.c_double(0.0)
        check(load().amg_energy_scale(self._h, _ptr(b), _ptr(u0), C.byref(g), _stream()))
        return g.value

    def set_operator(self, A=None):
        """amg_set_operator: CG products with A (same pattern as the setup
        matrix) while the hierarchy stays; None goes back to the setup matrix."""
        if A is None:
            check(load().amg_set_operator(self._h, None, _stream()))
            return
        bsr = A.c()
        check(load().amg_set_operator(self._h, C.byref(bsr), _stream()))

    # ---- solve ----------------------------------------------------------
    def solve(self, b, u0=None, rtol=1e-8, maxit=500, precision="fp64", max_replace=3, history=False,
              allow_notconv=False, profile=False, block=False):
        """Returns (u, SolveReport).  b: [3N] or [N, 3, nrhs] float64 device tensor.
        block: one block CG over the nrhs columns instead of nrhs CG recurrences."""
        torch = _torch()
        import numpy as np
        nrhs = 1 if b.dim() == 1 else b.shape[-1]
        _dev(b, torch.float64, None, "b")
        if b.numel() != 3 * self.n * nrhs:
            raise ValueError("b has the wrong size")
        u = torch.zeros_like(b) if u0 is None else _dev(u0, torch.float64, tuple(b.shape), "u0").clone()
        o = _lib.PcgOptions()
        load().pcg_options_default(C.byref(o))
        o.rtol, o.maxit, o.max_replace, o.profile, o.block = rtol, maxit, max_replace, int(profile), int(block)
        o.precision = {"fp64": TE_PREC_FP64, "mixed": TE_PREC_MIXED}[precision] if isinstance(precision, str) \
            else precision
        iters = np.zeros(nrhs, np.int32)
        conv = np.zeros(nrhs, np.int32)
        rel = np.zeros(nrhs, np.float64)
        hist = np.zeros((maxit + 1) * nrhs, np.float64) if history else None
        rep = _lib.PcgReport()
        rep.iters, rep.converged, rep.relres_true = iters.ctypes.data, conv.ctypes.data, rel.ctypes.data
        rep.history = hist.ctypes.data if hist is not None else None
        code = load().amg_pcg_solve(self._h, _ptr(b), _ptr(u), nrhs, C.byref(o), C.byref(rep), _stream())
        check(code, allow=(_lib.TE_OK, _lib.TE_ENOTCONV) if allow_notconv else (_lib.TE_OK,))
        h = hist.reshape(maxit + 1, nrhs) if hist is not None else None
        return u, SolveReport(iters.tolist(), conv.tolist(), rel.tolist(), h, rep.max_iters, rep.time_ms, code,
                              list(rep.kernel_ms), list(rep.kernel_launches))


def timestep(T_new, T_old, dt, dT_max=10.0, eps=0.9, noalloc=False):
    """te_timestep (eq. dt_spec): returns (accept, dt_next, max_change) for a
    step of length dt from T_old to T_new (float64 device tensors, same size).
    noalloc=True calls te_timestep_noalloc (library scratch, no allocation)."""
    torch = _torch()
    _dev(T_new, torch.float64, None, "T_new")
    _dev(T_old, torch.float64, tuple(T_new.shape), "T_old")
    dn, acc, mc = C.c_double(0.0), C.c_int32(0), C.c_double(0.0)
    fn = load().te_timestep_noalloc if noalloc else load().te_timestep
    check(fn(_ptr(T_new), _ptr(T_old), T_new.numel(), float(dt), float(dT_max), float(eps), C.byref(dn),
             C.byref(acc), C.byref(mc), _stream()))
    return bool(acc.value), dn.value, mc.value


def autotune_multi(amgs):
    """te_autotune_multi: the grouped launch shape of solve_multi for this set
    of AMG handles (kept in them); returns the text report."""
    n = len(amgs)
    H = (C.c_void_p * n)(*[a._h.value for a in amgs])
    buf = C.create_string_buffer(1 << 12)
    check(load().te_autotune_multi(H, n, buf, len(buf), _stream()))
    return buf.value.decode()


def solve_multi(amgs, bs, u0s=None, rtol=1e-8, maxit=500, max_replace=3):
    """amg_pcg_solve_multi over several AMG handles.  Returns (us, reports)."""
    import numpy as np
    torch = _torch()
    n = len(amgs)
    us = [torch.zeros_like(b) if u0s is None else u0.clone() for b, u0 in zip(bs, u0s or [None] * n)]
    o = _lib.PcgOptions()
    load().pcg_options_default(C.byref(o))
    o.rtol, o.maxit, o.max_replace = rtol, maxit, max_replace
    H = (C.c_void_p * n)(*[a._h.value for a in amgs])
    B = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    U = (C.c_void_p * n)(*[u.data_ptr() for u in us])
    iters = np.zeros(n, np.int32)
    conv = np.zeros(n, np.int32)
    rel = np.zeros(n, np.float64)
    reps = (_lib.PcgReport * n)()
    for i in range(n):
        reps[i].iters = iters.ctypes.data + 4 * i
        reps[i].converged = conv.ctypes.data + 4 * i
        reps[i].relres_true = rel.ctypes.data + 8 * i
    code = load().amg_pcg_solve_multi(H, n, B, U, C.byref(o), reps, _stream())
    check(code, allow=(_lib.TE_OK, _lib.TE_ENOTCONV))
    return us, {"iters": iters.tolist(), "converged": conv.tolist(), "relres_true": rel.tolist(),
                "time_ms": reps[0].time_ms, "code": code}


class MPNN:
    """mpnn_create / features / forward / backward / Adam / guess (float32)."""

    def __init__(self, A: Matrix, coords):
        torch = _torch()
        lib = load()
        _dev(coords, torch.float64, (A.n, 3), "coords")
        self.n = A.n
        self.n_params = int(lib.mpnn_param_count())
        self._cd = lib  # kept for __del__, which can run after module teardown
        self._h = C.c_void_p(0)
        check(lib.mpnn_create(A.n, _ptr(A.row_ptr), _ptr(A.col_idx), _ptr(coords), C.byref(self._h), _stream()))
        self.device = coords.device

    def __del__(self):
        h, lib = getattr(self, "_h", None), getattr(self, "_cd", None)
        if h is not None and h.value and lib is not None:
            lib.mpnn_destroy(h)
            h.value = None  # in place: module globals may be gone at interpreter exit

    def features(self, T, T_ref, mask, f=None):
        torch = _torch()
        _dev(T, torch.float64, (self.n,), "T")
        _dev(mask, torch.uint8, (self.n, 3), "mask")
        _dev(f, torch.float64, (self.n, 3), "f")
        X = torch.empty((self.n, 10), dtype=torch.float32, device=self.device)
        check(load().mpnn_features(self._h, _ptr(T), T_ref, _ptr(f), _ptr(mask), _ptr(X), _stream()))
        return X

    def forward(self, params, X, mask):
        torch = _torch()
        _dev(params, torch.float32, (self.n_params,), "params")
        _dev(X, torch.float32, (self.n, 10), "X")
        _dev(mask, torch.uint8, (self.n, 3), "mask")
        y = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        check(load().mpnn_forward(self._h, _ptr(params), _ptr(X), _ptr(mask), _ptr(y), _stream()))
        return y

    def backward(self, params, target):
        """Gradient of the mean squared error of the last forward; returns (grad, loss)."""
        torch = _torch()
        _dev(target, torch.float32, (self.n, 3), "target")
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = C.c_double(0.0)
        check(load().mpnn_backward(self._h, _ptr(params), _ptr(target), _ptr(grad), C.byref(loss), _stream()))
        return grad, loss.value

    def backward_from(self, params, gy):
        """Gradient of a loss with dL/dy = gy (float [N, 3]) of the last forward."""
        torch = _torch()
        _dev(gy, torch.float32, (self.n, 3), "gy")
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        check(load().mpnn_backward_from(self._h, _ptr(params), _ptr(gy), _ptr(grad), _stream()))
        return grad

    def energy_grad(self, amg, target):
        """(gy, loss): relative energy error of the last forward's guess and its dL/dy."""
        torch = _torch()
        _dev(target, torch.float32, (self.n, 3), "target")
        gy = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        loss = C.c_double(0.0)
        check(load().mpnn_energy_grad(self._h, amg._h, _ptr(target), _ptr(gy), C.byref(loss), _stream()))
        return gy, loss.value

    def adam_step(self, params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        check(load().mpnn_adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, b1, b2,
                                    eps, _stream()))

    def guess(self):
        """u0 [3N] float64 from the last forward."""
        torch = _torch()
        u0 = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        check(load().mpnn_guess(self._h, _ptr(u0), _stream()))
        return u0
