"""CPU oracle for the mixed-precision LOBPCG hot path (test infrastructure only).

This package is the plain, slow, obviously correct CPU reference that the GPU
path is checked against.  Only tests, the smoke check and the bench's CPU
baseline leg may import it; the product library never does, and it shares no
code with the HIP path (only the seeded input generators in ``synth`` serve
both).

Contents (each function cites the passage it follows):
  dense     brute-force eigenpairs by a dense symmetric eigensolver (the plain
            definition of the result, section 1)
  precond   the preconditioner T = (L L^T)^{-1} of section 5.1 from an FP64 or
            FP32 Cholesky-type factor, applied in the factor's precision
  mixed_qr  Algorithm 2 (mixed-precision QR) and a Householder reference
  lobpcg    Algorithm 3's working-precision loop (lines 2-17) with the
            convergence test of eq. (stop) and the Hetmaniuk-Lehoucq update
  grad      dense eigen-gradient with respect to a diagonal potential
  pinvit    Algorithm 1 (mixed-precision PINVIT) and the Theorem 1 rate

Every floating-point computation is float64 unless the paper fixes a lower
precision for that step (the lower-precision factor and Algorithm 2 step 1 are
float32, as sections 3.1-3.2 state).
"""
