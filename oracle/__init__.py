"""CPU oracle for the Schur-complement + PCG solve (test infrastructure).

This package is test infrastructure only: ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import it; the library and its Python binding never
do, and it imports nothing from them.  It shares no code with the GPU path; the only
module both sides use is the seeded input generator, which holds none of the method's
arithmetic.

Modules
  ref    -- ctypes front end of ``schur_pcg.c``: plain FP64 formation of S, gamma and the
            preconditioner, PCG (Algorithm 1), primal step and adjoint (O2).
  kkt    -- numpy FP64 dense references: the KKT system solved by LU (O1), the dense
            Schur product C G^-1 C^T, the LQR Riccati recursion, a banded Cholesky solve
            of S, and the dense adjoint (O4).
  exact  -- exact rational PCG with ``fractions.Fraction`` for tiny problems (O3).
  nmpc   -- numpy FP64 control step around the solve: linearisation of a pendulum-chain
            model into the LQ problem, the L1 merit and the parallel line search.
"""
