"""CPU checker for the variable-density pressure solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the HIP path.

Contents
--------
poisson    -- the discrete problem written out plainly in float64 numpy: mixture
              density, face coefficients, gradient, divergence, operator,
              residual; brute-force dense solve, spectral solve (uniform
              density), and the manufactured solution.
relax      -- plain definitions of the multigrid pieces the GPU kernels are
              checked against one by one: a red-black SOR half-sweep,
              face-sum coarsening, sum restriction, injection prolongation.
cref       -- ctypes binding of ``ppref.c``: the same operator in plain C and a
              float64 OpenMP solver (conjugate gradients preconditioned by a
              damped-Jacobi V-cycle) for reference pressures at full size.
"""
