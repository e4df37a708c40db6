"""Plain, slow FP64 CPU oracle for the interpolation-based H^2 matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code, tables or constants
with the HIP library; the only common input is the mesh/vector generator
module ``h2_inputs``, which holds none of the method's arithmetic.

The oracle follows the paper (Boerm, "Distributed H^2-matrices for boundary
element methods") section by section:

  quadrature      triangle rules and the Sauter-Schwab rules for the singular
                  Galerkin integrals (Introduction: "suitable quadrature
                  techniques"; experiments: Sauter-Schwab quadrature)
  kernels         Laplace and Helmholtz kernels (Introduction), plus polynomial
                  test kernels for closed-form checks
  galerkin        Galerkin entries g_ij and the dense matrix G (Introduction)
  cluster         cluster tree (Definition 1) by bisection of characteristic
                  points with minimal axis-parallel boxes
  blocks          block tree under the admissibility condition (eq. admissibility)
  interpolation   Chebyshev interpolation, leaf matrices (eq. leafV/leafW),
                  transfer matrices (eq. transfer), coupling (eq. coupling)
  h2              the H^2 matrix: Algorithms 1-3 (forward, backward, interaction),
                  dense G-tilde, and row-sampled products at large sizes
  krylov          CG and GMRES in FP64 for G z = b (Introduction: Krylov methods)

Every floating-point quantity is FP64 (complex128 for Helmholtz).
"""
