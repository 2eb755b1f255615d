"""CPU oracle for the HBS-preconditioned Lippmann-Schwinger solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark may.
It shares no code with the HIP library and never calls it.

Everything here is plain numpy/scipy/mpmath in complex128, written to be read
against Gopal & Martinsson, "An accelerated, high-order accurate direct solver
for the Lippmann-Schwinger equation for acoustic scattering in the plane"
(arXiv 2007.12718):

* ``quadrature`` -- the corrected trapezoidal (Duan-Rokhlin type) weights of
  Sec. 2.2 / eq. (corrected), built by the lattice-zeta moment construction
  (the paper defers the weights to its reference [duan2009high]).
* ``dense``      -- grid, dense Nystrom matrix of eq. (linsys)/(Gmat), LU solve,
  receivers, dense adjoint gradient.
* ``fftop``      -- the coefficient matrix applied by FFT convolution (Sec. 5).
* ``hbs``        -- the tree (Sec. 3.1), proxy-source row IDs (Sec. 3.2,
  eqs. (leafid), (proxy), (parentid), (sibint)), the build of Algorithm 1, the
  apply of Algorithm 2, its exact transpose, and the HBS forward matvec.
* ``gmres``      -- right-preconditioned flexible GMRES (Sec. 5).
* ``disk``       -- textbook transmission series for a constant-b disk
  (Remark 1.1), used only as a pin.
"""
