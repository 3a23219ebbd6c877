"""Plain CPU FP64 oracle for time-stepper Arnoldi stability analysis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package.  It
is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline``
leg of ``bench.py``.  It shares no code, table or constant generator with the
HIP path; both sides only receive the same seeded inputs from ``workloads``.

Modules (each function cites the passage of Loiseau, Bucci, Cherubini & Robinet,
"Time-stepping and Krylov methods for large-scale instability problems",
arXiv:1804.03859, that it follows):

* ``cgle``        -- linear complex Ginzburg-Landau operator (Sec. 2.3.2, eq.
                     "ginzburg-landau equation"), 2nd-order finite differences,
                     Crank-Nicolson propagator.
* ``kolmogorov``  -- linearized 2D Navier-Stokes about a base flow (Sec. 3,
                     eq. "linearized Navier-Stokes equations") in vorticity form,
                     pseudo-spectral with 2/3 dealiasing, integrating-factor RK4.
* ``arnoldi``     -- m-step Arnoldi factorisation (Sec. 3.2.1, Algorithm 1) with
                     classical Gram-Schmidt applied twice, Ritz pairs, the Ritz
                     residual estimate (Sec. 3.2.2, eq. "Krylov convergence"),
                     wanted set and stop rule, lambda = log(mu)/T (Sec. 3.2).
* ``krylov_schur`` -- Krylov-Schur restart (Sec. 3.2.2, after Stewart 2001):
                     ordered real Schur form of the Krylov matrix, truncation to
                     the wanted part, re-expansion by Arnoldi steps.
* ``optimal``     -- adjoint propagators (discrete transposes of the Kolmogorov
                     and Ginzburg-Landau steppers) and the optimal perturbation:
                     Lanczos on M^dagger M (Sec. 2.3.1 SVD formulation, Sec. 3.3.2).
* ``fixedpoint``  -- nonlinear forced Navier-Stokes stepper and the fixed-point
                     solvers on it: selective frequency damping, recursive
                     projection method, BoostConv (Sec. 3.1).
* ``resolvent``   -- resolvent by forced time integration of the Ginzburg-Landau
                     equation (Sec. 2.3.2, Sec. 3.3.2) and its closed form for
                     Crank-Nicolson (the warped-frequency resolvent).
* ``rng``         -- splitmix64 + Box-Muller start-vector generator (published
                     definitions, Steele/Lea/Flood 2014 and Box & Muller 1958).
* ``mlp``         -- start-vector network (not in the paper): FP64 forward,
                     backward and Adam with the GPU's bfloat16 rounding points.
* ``learned``     -- packed spectral coordinates, the low-mode block target
                     made from Ritz vectors, and the start vector assembled
                     from a prediction (Algorithm 1 takes any start vector).

Parity status of every function is stated in its module header.
"""
