"""Plain FP64 CPU oracle of the Nyström Lippmann–Schwinger method
(Anand, Pandey, Rathish Kumar, Paul; arXiv:1509.05063).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package.
It shares no code with the GPU library: its own discretisation, its own
near-field quadratures, direct O(N^2) summation for every pair (no
equivalent sources, no FFT) and its own solvers.

Modules:
  quad    one-dimensional rules (Newton–Cotes, Gauss–Legendre, Lagrange, cut-offs)
  geom2d  2-D patches, partition of unity, Nyström nodes and weights
  near2d  2-D kernel, localisation and singular quadratures
  op2d    the discrete operator I + kappa^2 K_h (dense / row by row)
  mie     closed forms: Mie series (2-D, 3-D), volume potential of a constant
  solve   restarted complex GMRES, dense LU
  exterior  scattered field off the scatterer by direct summation
  conv3d  the 3-D face-lattice convolution (monopole + dipole) by direct summation
"""
