"""CPU oracle for the thermoelastic PCG + smoothed-aggregation AMG path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this
package; the product path (the HIP library and its Python binding) never
does, and shares no code with it.

Everything here is plain, slow and written to be checked by eye against the
paper and the textbook methods it names, in float64:

* ``fem``     -- Lagrange P1/P2 tetrahedral assembly of the thermoelastic
                 weak form (Sec. 3, eq. wf_elastic), one material or
                 temperature-dependent tables per material with the boundary
                 pressure term, Dirichlet elimination, rigid-body
                 near-nullspace.
* ``amg``     -- smoothed-aggregation AMG (Sec. 2.1.3, Sec. 5.1): strength,
                 MIS-2 or greedy aggregation, tentative prolongator by QR, Lanczos
                 eigenvalue estimate, prolongator smoothing, Galerkin
                 product, Chebyshev smoother, V-cycle, coarse Cholesky.
* ``krylov``  -- preconditioned and flexible conjugate gradients
                 (Sec. 2.1.2), single and multiple right-hand sides.
* ``mpnn``    -- message-passing network forward/backward for the learned
                 initial guess.
* ``transient`` -- the time-step control of eq. dt_spec around the elastic
                 solve of a transient run (Sec. 3.3, Sec. 5.3).
* ``thermal`` -- the nonlinear heat equation of eq. wf_thermal (steady, or
                 one backward-Euler step) with its Newton Jacobian and
                 Newton's method (Sec. 3, 3.2, 5.2, 5.3).
* ``camg``    -- classical AMG for the scalar thermal corrections: strength,
                 PMIS coarsening, direct interpolation, Galerkin product, l1
                 hybrid Gauss-Seidel smoother, V-cycle (Sec. 5.1).
* ``native``  -- the assembly, smoothed-aggregation setup, V-cycle and PCG
                 restated in plain C++17/OpenMP (``native/te_oracle.cpp``),
                 for the sizes the NumPy oracle cannot reach.
* ``rng``     -- splitmix64 counter generator (Steele, Lea & Flood 2014).
"""
