"""FP64 CPU oracle for finite-temperature CCSD (White & Chan, 2020).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP implementation; the
only common dependency is the seeded input generator package `ftcc_inputs`,
which holds none of the method's arithmetic.

Modules
  grid        imaginary-time grid: composite Gauss-Legendre panels and the
              exponential-propagator weights, by plain quadrature (Section II.C)
  spinorb     spin-orbital FT-CCSD written term by term from Appendix A:
              thermal integrals, the E, S1 and S2 kernels, the imaginary-time
              march, the Lambda adjoint and the response derivatives
  restricted  the same terms summed over spin explicitly for a spin-restricted
              reference (closed-shell amplitudes)
  ed          grand-canonical exact diagonalisation (thermal FCI)
  rk          the differential form (Algorithm alg:diff): explicit RK1/RK2/RK4
              on a uniform grid, Simpson's rule for Omega, reverse-mode
              derivatives
"""
