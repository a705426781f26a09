"""Plain FP64 CPU oracle for the rigidly constrained immersed-boundary Stokes solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constant tables); the only common
module is ``synthetic``, which draws seeded inputs and holds none of the
method's arithmetic.

What it computes, and from which passage of Kallemov, Bhalla, Griffith & Donev,
"An immersed boundary method for rigid bodies" (2016):

* ``kernel``      Peskin's four-point regularised delta (Sec. 3.1 uses a
                  tensor-product kernel; the four-point function itself is the
                  one of Peskin's 2002 review that Sec. 4.1 cites).
* ``grid``        MAC-grid operators A, G, D, L of Sec. 3.2 (eq. A_def).
* ``ib``          interpolation J and spreading S of Sec. 3.1 (eq. S_unweighted),
                  the periodic-steady spreading S' of Sec. 3.4
                  (eq. constrained_periodic), rigid marker velocities and the
                  body force / torque sums of Sec. 2.
* ``stokes``      exact periodic Stokes solution operator by FFT (Sec. 3.3,
                  eqs. Stokes_saddle and L_inv_periodic).
* ``constrained`` exact solution of eq. constrained_Stokes /
                  eq. constrained_periodic through the mobility M = J L^-1 S
                  (Sec. 3.3, eqs. lambda_sol and mob_def).
* ``dense``       the same system assembled densely and solved by LAPACK, the
                  independent check of ``constrained``.
* ``mobility``    analytic approximate mobilities of Sec. 4 (RPY tensor,
                  Brinkmanlet, self-mobility limits, 2D periodic forms).
* ``multigrid``   one geometric-multigrid V-cycle and the projection
                  preconditioner P_S^-1 of Sec. 5.2 (eq. P1_practical); the
                  paper does not give the V-cycle's internals, so the cycle
                  is the documented reading (RB Gauss-Seidel, cell averaging,
                  trilinear prolongation).
* ``precond``     the Schur-complement preconditioner of Sec. 5.1 with the
                  inner GMRES(N_s) of Sec. 5.2.
* ``navier``      explicit advection right-hand side for the unsteady runs
                  (a reading of the time integrator summarised in Sec. 3 and
                  Sec. 7.6).
* ``hasimoto``    periodic drag formulas used as pins (eqs. drag_periodic and
                  drag_periodic_2D).
* ``walls``       the slit channel: no-slip walls at both ends of the last
                  axis with the mirror extension of the appendix on physical
                  boundary conditions (operators, folded interpolation and
                  spreading, exact per-mode Stokes solve, V-cycle); Sec. 7
                  studies a sphere in such a channel.
* ``free``        free kinematics (Sec. 2 poses it, Sec. 8 names the enlarged
                  system and its body mobility N = (K* M^-1 K)^-1): bodies
                  moving under applied forces and torques, solved exactly.
"""
from . import kernel, grid, ib, stokes, constrained, dense, mobility, multigrid, precond, navier, hasimoto, free, walls  # noqa: F401
