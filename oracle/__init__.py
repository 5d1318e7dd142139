"""CPU FP64 oracle for the RVE homogenisation path -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the HIP library is checked
against.  It is imported only by the tests, by the smoke check of the entry
module and by the CPU-baseline leg of the benchmark; the product path never
calls it.  It shares no code with the HIP library.

What it computes (all in float64):
  * the plain-weave RVE mesh (Kuhn split of an n^3 grid) and its yarn tagging;
  * the materials: isotropic matrix, transversely isotropic yarns rotated to the
    fibre axis, and the matrix degradation law of the paper (Sec. 4, Eqs.
    Eq_alphaT, Eq_Model_final1);
  * the exact Galerkin solution on the conforming P_p space (Lagrange nodal
    basis, exact barycentric integration) of the RVE problem under linear
    Dirichlet, periodic or uniform-traction constraints, written as the
    Lagrange-multiplier saddle-point system of Sec. 2 (Eqs. eq_RVE_disc_Eqs,
    eq_mat_C_and_D), factorised once and solved for all load cases;
  * homogenised stress from the multipliers (Eq. eq_homo_stress, sign read as
    in the module docs of fem.py) and, as a cross-check, from the volume average
    of the micro stress (Eq. macro_stress).

Parity is pinned by the tests in tests/test_oracle_*.py against closed forms and
invariants; see each function's docstring for the passage it follows.
"""
