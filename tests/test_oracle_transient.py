"""Pins of the oracle's time-step control (eq. dt_spec) and of preconditioner
reuse across steps.

* A temperature rising linearly in time: after the first accepted step every
  step is exactly eps * dT_max / max|rate| long and changes T by eps * dT_max
  (closed form), and the count of steps to t_end follows.
* A first step that is too long is halved until its change is within dT_max:
  ceil(log2(max|rate| dt0 / dT_max)) rejections.
* An exponential approach to an operating field: every accepted change is at
  most dT_max, the steps lengthen as the rate decays, and the step lengths
  satisfy eq. dt_spec one step to the next.
* No change doubles the step.
* The hierarchy built for one matrix preconditions CG on a changed matrix
  (temperature-dependent materials at a hotter field) to the direct solution
  of the changed system, and the previous solution as initial guess starts
  closer than zero."""
import math

import numpy as np
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import amg, fem, krylov, transient


def test_linear_rise_gives_uniform_steps():
    rng = np.random.default_rng(0)
    T0 = 300.0 + 50.0 * rng.random(500)
    rate = rng.uniform(-2.0, 5.0, 500)            # K/s, max |rate| = 5 at most
    rmax = np.abs(rate).max()
    T = lambda t: T0 + rate * t
    steps = transient.step_sequence(T, 0.0, 100.0, 0.5, dT_max=10.0, eps=0.9)
    h = 0.9 * 10.0 / rmax
    assert steps[0].rejected == 0 and math.isclose(steps[0].dt, 0.5)
    for s in steps[1:-1]:
        assert math.isclose(s.dt, h, rel_tol=1e-12) and math.isclose(s.dT, 9.0, rel_tol=1e-9)
    assert math.isclose(steps[-1].t, 100.0, rel_tol=1e-12)
    assert len(steps) == 1 + math.ceil((100.0 - 0.5) / h - 1e-9)


def test_too_long_first_step_is_halved():
    T0 = np.zeros(10)
    rate = np.linspace(0.0, 4.0, 10)
    for dt0, expect in [(2.5, 0), (2.6, 1), (10.0, 2), (40.0, 4), (41.0, 5)]:
        ok_first = transient.step_sequence(lambda t: T0 + rate * t, 0.0, 1e3, dt0, dT_max=10.0, eps=0.9)[0]
        assert ok_first.rejected == expect == max(0, math.ceil(math.log2(4.0 * dt0 / 10.0)))
        assert ok_first.dT <= 10.0 and math.isclose(ok_first.dt, dt0 / 2 ** expect)


def test_exponential_approach_respects_the_limit_and_the_rule():
    prob = mg.disc_problem(6, 26, 2, 1, seed=1)
    Top = prob.T
    tau = 600.0
    T = lambda t: 293.0 + (Top - 293.0) * (1.0 - math.exp(-t / tau))
    steps = transient.step_sequence(T, 0.0, 3000.0, 1.0, dT_max=10.0, eps=0.9)
    assert all(s.dT <= 10.0 for s in steps)
    # eq. dt_spec: dt_{m+1} = eps dT_max / dT_m * dt_m whenever the step was not cut or rejected
    for a, b in zip(steps[:-2], steps[1:-1]):
        if b.rejected == 0 and a.dT > 0:
            assert math.isclose(b.dt, 0.9 * 10.0 / a.dT * a.dt, rel_tol=1e-12)
    dts = [s.dt for s in steps[1:-1]]
    assert all(y >= x * (1 - 1e-9) for x, y in zip(dts, dts[1:]))   # the rate only decays


def test_no_change_doubles():
    ok, dt, dT = transient.next_step(np.ones(4), np.ones(4), 3.0, 10.0, 0.9)
    assert ok and dt == 6.0 and dT == 0.0
    ok, dt, dT = transient.next_step(np.array([0.0, 20.0]), np.zeros(2), 3.0, 10.0, 0.9)
    assert not ok and dt == 1.5 and dT == 20.0


def test_reused_hierarchy_solves_the_changed_system():
    prob = mg.disc_problem(6, 26, 2, 2, seed=2)
    m = prob.mesh
    mat = mg.disc_materials(m)
    tab = fem.MaterialTables(mat.T, mat.E, mat.nu, mat.alpha)
    systems = []
    for s in (0.5, 0.6):
        Ts = 293.0 + (prob.T - 293.0) * s
        A0, b0 = fem.assemble_materials(m.coords, m.cells, m.degree, mat.cell_material, tab, prob.T_ref, Ts, None)
        systems.append(fem.apply_dirichlet(A0, b0, prob.mask))
    (Aa, ba), (Ab, bb) = systems
    assert abs(Ab - Aa).max() > 1e-3 * abs(Aa).max()      # the materials make the matrix change
    opt = amg.AMGOptions(coarse_max=400)
    lv = amg.setup(Aa, fem.rigid_body_modes(m.coords, prob.mask), opt)
    M = lambda r: amg.vcycle(lv, r, opt=opt)
    ua = krylov.pcg(Aa, ba, M).u
    res = krylov.pcg(Ab, bb, M, u0=ua)
    direct = spla.spsolve(Ab.tocsc(), bb)
    assert res.converged and np.linalg.norm(bb - Ab @ res.u) <= 1e-8 * np.linalg.norm(bb)
    assert np.linalg.norm(res.u - direct) <= 1e-6 * np.linalg.norm(direct)
    assert np.linalg.norm(bb - Ab @ ua) < np.linalg.norm(bb)


def test_coupled_heat_steps_respect_the_limit_and_reach_the_steady_state():
    """Backward-Euler heat steps from 293 K with fixed exterior temperatures:
    every accepted step changes T by at most dT_max, the decisions follow
    next_step, a too-long first attempt is halved, and the temperature
    tends to the steady Newton solution of the same problem (the fixed point
    of the backward-Euler map is the steady solution)."""
    import scipy.sparse.linalg as spla

    from oracle import thermal
    m = mg.disc_mesh(3, 12, 2, 1)
    P = thermal.problem_from_meshgen(m, mg.disc_thermal_materials(m), mg.disc_robin_faces(m))
    Tbc = P.T_bc.copy()
    direct = lambda J, r, k: (spla.spsolve(J.tocsc(), r), 1)  # noqa: E731
    steps = transient.coupled_step_sequence(P, np.full(m.n_nodes, 293.0), lambda t: Tbc, direct, 0.0, 1e7, 50.0,
                                            dT_max=10.0, eps=0.9, max_steps=400)
    assert steps[0].rejected >= 1
    T_prev = np.full(m.n_nodes, 293.0)
    for s in steps:
        assert s.dT <= 10.0 and s.dT == float(np.abs(s.T - T_prev).max())
        T_prev = s.T
    # each step's length: the previous step's next length (eq. dt_spec), cut to
    # t_end, halved once per rejected attempt
    dt_next, t = 50.0, 0.0
    for s_ in steps:
        assert s_.dt == min(dt_next, 1e7 - t) / 2 ** s_.rejected
        dt_next = 2.0 * s_.dt if s_.dT == 0.0 else 0.9 * 10.0 / s_.dT * s_.dt
        t = s_.t
    P.T_bc = Tbc
    steady = thermal.newton(P, np.full(m.n_nodes, 400.0), direct)
    assert np.abs(steps[-1].T - steady.T).max() <= 1e-6 * np.abs(steady.T).max()
