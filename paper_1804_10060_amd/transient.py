"""The loop of a transient run (Sec. 3.2, 3.3 and Sec. 5.3): backward-Euler
heat steps (ThermoelasticTransient) driving elastic solves along the
temperature history (ElasticTransient).

Each accepted time step assembles the system at the new temperature (with
temperature-dependent materials the matrix changes), solves it starting from
the previous step's displacement, and either reuses the hierarchy built at
the first step (amg_set_operator: the CG runs on the new matrix, the V-cycle
stays) or builds a new one.  Steps follow eq. dt_spec through te_timestep:
the next step targets a largest temperature change of eps * dT_max, and a
step whose change exceeds dT_max is repeated with half the length.

ElasticTransient takes the temperature at each time from the caller
(`T_of_t`); ThermoelasticTransient computes it: every attempted step is one
backward-Euler step of the heat equation (eq. wf_thermal, theta = 1) solved
by Newton from the previous temperature with the exterior temperatures of
the step's end time, the thermal preconditioner kept across steps and
rebuilt by the library when a step's corrections need clearly more CG
iterations (the steps of rapid change, Sec. 5.3).  Every step of the
computation runs in the library; this module only orders the calls.
"""
from __future__ import annotations

import dataclasses
import time

from . import AMG, assemble_materials, timestep


@dataclasses.dataclass
class StepRecord:
    t: float            # time at the end of the step
    dt: float           # step length
    max_change: float   # largest temperature change over the step
    rejected: int       # attempts rejected (halved) before it
    iters: int          # CG iterations of its elastic solve
    relres_true: float
    setup: bool         # a hierarchy was built at this step
    assemble_ms: float  # wall times of the step's library calls
    operator_ms: float  # amg_setup or amg_set_operator
    solve_ms: float


class ElasticTransient:
    """Materials and loads of one mesh (device tensors as for
    assemble_materials); `reuse` keeps the first hierarchy for every step."""

    def __init__(self, coords, cells, degree, tables, cell_material, T_ref, mask, f=None, faces=None, face_p=None,
                 reuse=True, rtol=1e-8, **amg_opts):
        self.args = (coords, cells, degree, tables, cell_material, T_ref)
        self.kw = {"f": f, "faces": faces, "face_p": face_p, "mask": mask}
        self.coords, self.mask = coords, mask
        self.reuse, self.rtol, self.amg_opts = reuse, rtol, amg_opts
        self.h = None
        self.u = None

    def _sync(self):
        import torch
        torch.cuda.synchronize()

    def solve_at(self, T):
        """Assemble at temperature T and solve from the previous displacement.
        Returns (u, report, setup_built, assemble_ms, operator_ms, solve_ms)."""
        self._sync()
        t0 = time.perf_counter()
        A, b = assemble_materials(*self.args, T, **self.kw)
        self._sync()
        t1 = time.perf_counter()
        built = self.h is None or not self.reuse
        if built:
            if self.h is not None:
                self.h.close()
            self.h = AMG(A, self.coords, self.mask, **self.amg_opts)
        else:
            self.h.set_operator(A)
        self._sync()
        t2 = time.perf_counter()
        u, rep = self.h.solve(b, u0=self.u, rtol=self.rtol)
        self._sync()
        t3 = time.perf_counter()
        self.u = u
        return u, rep, built, (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3

    def run(self, T_of_t, t0, t_end, dt0, dT_max=10.0, eps=0.9, max_steps=None):
        """Solve at t0, then step to t_end (the last step cut to end there) or
        for max_steps accepted steps.  T_of_t(t) -> float64 device tensor [N].
        Returns the StepRecords, the first one for the state at t0."""
        t, dt = float(t0), float(dt0)
        T_old = T_of_t(t)
        u, rep, built, ta, to, ts = self.solve_at(T_old)
        recs = [StepRecord(t, 0.0, 0.0, 0, rep.iters[0], rep.relres_true[0], built, ta, to, ts)]
        while t < t_end and (max_steps is None or len(recs) <= max_steps):
            h = min(dt, t_end - t)
            rejected = 0
            while True:
                T_new = T_of_t(t + h)
                ok, dt_next, dT = timestep(T_new, T_old, h, dT_max, eps)
                if ok:
                    break
                rejected += 1
                h = dt_next
            u, rep, built, ta, to, ts = self.solve_at(T_new)
            t += h
            recs.append(StepRecord(t, h, dT, rejected, rep.iters[0], rep.relres_true[0], built, ta, to, ts))
            T_old = T_new
            dt = dt_next
        return recs

    def close(self):
        if self.h is not None:
            self.h.close()
            self.h = None


@dataclasses.dataclass
class CoupledRecord:
    t: float
    dt: float
    max_change: float
    rejected: int
    newton_iters: int       # Newton corrections of the accepted attempt
    lin_iters: list         # its CG iterations per correction
    thermal_rebuilds: int   # thermal preconditioner builds in this step (all attempts)
    thermal_ms: float       # wall time of the step's thermal solves (all attempts)
    iters: int              # elastic CG iterations
    relres_true: float
    setup: bool
    assemble_ms: float
    operator_ms: float
    solve_ms: float


class ThermoelasticTransient:
    """Heat steps driving the elastic solves of one mesh (Sec. 3.2: the
    thermal problem first, then the mechanical one at the new temperature).
    thermal: heat.ThermalSolver; elastic: ElasticTransient on the same mesh
    and node numbering; T_bc_of_t(t) -> device [n_faces] exterior
    temperatures; face_p_of_t(t) -> device [n_pressure_faces] or None (fixed
    pressure)."""

    def __init__(self, thermal, elastic: ElasticTransient, T_bc_of_t, face_p_of_t=None, **newton_kw):
        self.thermal, self.elastic = thermal, elastic
        self.T_bc_of_t, self.face_p_of_t = T_bc_of_t, face_p_of_t
        self.newton_kw = newton_kw

    def _elastic(self, t, T):
        if self.face_p_of_t is not None:
            self.elastic.kw["face_p"] = self.face_p_of_t(t)
        return self.elastic.solve_at(T)

    def run(self, T0, t0, t_end, dt0, dT_max=10.0, eps=0.9, max_steps=None):
        """The elastic state at t0 (temperature T0), then accepted steps to
        t_end (the last one cut to end there) or max_steps of them.  Returns
        (records, T) with the first record for t0."""
        t, dt = float(t0), float(dt0)
        T_old = T0.clone()
        u, rep, built, ta, to, ts = self._elastic(t, T_old)
        recs = [CoupledRecord(t, 0.0, 0.0, 0, 0, [], 0, 0.0, rep.iters[0], rep.relres_true[0], built, ta, to, ts)]
        while t < t_end and (max_steps is None or len(recs) <= max_steps):
            h = min(dt, t_end - t)
            rejected, rebuilds, th_ms = 0, 0, 0.0
            while True:
                self.thermal.set_exterior(self.T_bc_of_t(t + h))
                T_new, nrep = self.thermal.newton(T_old, T_old=T_old, dt=h, **self.newton_kw)
                rebuilds += nrep.rebuilds
                th_ms += nrep.time_ms
                ok, dt_next, dT = timestep(T_new, T_old, h, dT_max, eps)
                if ok:
                    break
                rejected += 1
                h = dt_next
            t += h
            u, rep, built, ta, to, ts = self._elastic(t, T_new)
            recs.append(CoupledRecord(t, h, dT, rejected, nrep.iters, nrep.lin_iters, rebuilds, th_ms, rep.iters[0],
                                      rep.relres_true[0], built, ta, to, ts))
            T_old = T_new
            dt = dt_next
        return recs, T_old
