"""Oracle: the time-step control around the elastic solve of a transient run
(test infrastructure only; see the package docstring).

What the paper fixes (Sec. 3.3, eq. dt_spec, and Sec. 5.3):

* the next step is the current one scaled so that the largest temperature
  change over it would be the target eps * dT_max:
      dt_next = eps * dT_max / max_x |T_new(x) - T_old(x)| * dt;
* a step whose largest change exceeds dT_max is repeated with half the step;
* the transient runs use dT_max = 10 K and backward Euler.

Where the paper is silent: a step with no change at all (the formula divides
by zero) doubles the step; eps is a parameter (0.9 in the measurements).

Preconditioner reuse (Sec. 5.3: the elastic preconditioner built at the first
step is reused for the later steps, and the previous solution is the initial
guess) needs nothing beyond krylov.pcg: the new step's matrix with the old
hierarchy's V-cycle as M and the previous displacement as u0.

The temperature of each step comes from one backward-Euler step (theta = 1,
Sec. 5.3) of the heat equation solved by Newton (oracle.thermal), the
exterior temperatures taken at the step's end time (coupled_step_sequence).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def next_step(T_new, T_old, dt, dT_max, eps):
    """Returns (accept, dt_next, dT) for a step of length dt that took the
    temperature from T_old to T_new: dT = max |T_new - T_old|; accepted iff
    dT <= dT_max; then dt_next = eps * dT_max / dT * dt (2 dt if dT = 0);
    rejected: dt_next = dt / 2 (the step is to be repeated)."""
    dT = float(np.max(np.abs(np.asarray(T_new, np.float64) - np.asarray(T_old, np.float64)))) if np.size(T_new) else 0.0
    if dT > dT_max:
        return False, 0.5 * dt, dT
    if dT == 0.0:
        return True, 2.0 * dt, dT
    return True, eps * dT_max / dT * dt, dT


@dataclasses.dataclass
class Step:
    t: float          # time at the end of the accepted step
    dt: float         # its length
    dT: float         # its largest temperature change
    rejected: int     # attempts rejected before it


def step_sequence(T_of_t, t0, t_end, dt0, dT_max=10.0, eps=0.9, max_steps=10000):
    """Accepted steps from t0 until t_end (the last step is cut to end at
    t_end) for a prescribed temperature history T_of_t(t) -> array."""
    steps = []
    t, dt = float(t0), float(dt0)
    T_old = np.asarray(T_of_t(t), np.float64)
    while t < t_end and len(steps) < max_steps:
        h = min(dt, t_end - t)
        rejected = 0
        while True:
            T_new = np.asarray(T_of_t(t + h), np.float64)
            ok, dt_next, dT = next_step(T_new, T_old, h, dT_max, eps)
            if ok:
                break
            rejected += 1
            h = dt_next
        t += h
        steps.append(Step(t, h, dT, rejected))
        T_old = T_new
        dt = dt_next
    return steps


@dataclasses.dataclass
class CoupledStep:
    t: float              # time at the end of the accepted step
    dt: float             # its length
    dT: float             # its largest temperature change
    rejected: int         # attempts rejected before it
    T: np.ndarray         # temperature at t
    newton_iters: int     # Newton corrections of the accepted attempt
    lin_iters: list       # CG iterations of each correction


def coupled_step_sequence(P, T0, T_bc_of_t, linear_solve, t0, t_end, dt0, dT_max=10.0, eps=0.9, max_steps=10000,
                          newton_kw=None):
    """The thermal half of a transient run (Sec. 3.2, 3.3, 5.3): each attempt
    solves one backward-Euler step of eq. wf_thermal by Newton from the
    previous temperature, with the exterior temperatures of the step's end
    time (P.T_bc is set to T_bc_of_t(t + h)); eq. dt_spec then accepts it or
    halves it (next_step).  linear_solve is the Newton correction solver
    (e.g. thermal.ReusedPreconditioner, kept across attempts and steps)."""
    from . import thermal
    steps = []
    t, dt = float(t0), float(dt0)
    T_old = np.asarray(T0, np.float64).copy()
    while t < t_end and len(steps) < max_steps:
        h = min(dt, t_end - t)
        rejected = 0
        while True:
            P.T_bc = np.asarray(T_bc_of_t(t + h), np.float64)
            res = thermal.newton(P, T_old, linear_solve, T_old=T_old, dt=h, **(newton_kw or {}))
            assert res.converged, "thermal Newton did not converge"
            ok, dt_next, dT = next_step(res.T, T_old, h, dT_max, eps)
            if ok:
                break
            rejected += 1
            h = dt_next
        t += h
        steps.append(CoupledStep(t, h, dT, rejected, res.T, res.iters, res.lin_iters))
        T_old = res.T
        dt = dt_next
    return steps
