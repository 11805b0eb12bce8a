"""CPU oracle for the dual-porosity oil-water simulator's hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls into it, and it shares no code with the GPU library: the only common
module is ``synth`` (seeded input data, none of the method's arithmetic).

Everything is plain FP64 NumPy/SciPy, written to be read against the paper:

  physics.py  rock/fluid properties, transmissibilities, Peaceman well index,
              the fully implicit residual of the dual-porosity system and its
              analytic Jacobian (Sec. 2, Eqs. (1)-(10); Sec. 3 first paragraph)
  newton.py   Newton's method with a sparse direct solve, the timestep loop and
              the material-balance report (Algorithm 1, Eq. (11)-(12))
  cpr.py      the decoupled, CPR-FPF-preconditioned GMRES solve: Gauss-Jordan
              decoupling, block ILU(0) under a given ordering, pressure
              extraction, classical AMG and its V-cycle, GMRES(m)
              (Sec. 3.2, Eq. (14))

Readings of passages where the paper is silent or inconsistent are listed in
the module docstrings where they are applied.
"""
