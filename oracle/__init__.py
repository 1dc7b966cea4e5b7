"""CPU FP64 oracle for the hierarchical lattice solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything here: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the GPU library; the only thing
both sides use is the seeded input generator in ``workloads``.

Modules
-------
lattice : geometry, bar stiffness and CSR assembly of K (Eq. 1, section 3.1).
solve   : the plain definition the method converges to, u* = K_ff^-1 (f_f -
          K_fc u_c), by dense or banded Cholesky or block-Jacobi PCG; the
          relative residuals of Eq. 19 and the energy of Eq. 2.
method  : the paper's hierarchical iteration (Eqs. 3-14) written out step
          by step with exact local and upper-level solves, used to check
          the GPU's intermediate quantities (modes, upper-level matrix and
          force, coefficients) and the method's invariants.

All arithmetic is float64.  Everything here is slow on purpose.
"""
