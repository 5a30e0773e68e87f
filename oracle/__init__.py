"""CPU FP64 oracle for Coordinate Condensation -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product library never calls
into it and shares no code with it (the only common dependency is the seeded
scene generator in ``ccscenes``, which holds no solver arithmetic).

Everything here is float64 NumPy/SciPy and follows the paper's notation:

* implicit Euler as energy minimisation, E(x) = 1/2 (x - x~)^T M (x - x~)
  + h^2 Psi(x) (Background, Optimization-Based Integration);
* the per-vertex perturbation basis U_i = -H_CC^{-1} H_Ci (Background, JGS2
  subsection; Method, Coordinate Condensation);
* the Coordinate Condensation update, Eqs. (displacement)-(schur) and
  Algorithm 1 (Method section).

Parity status per function is recorded in each module's header.  Functions
marked "parity unpinned" have no independent check.
"""
