"""FP64 CPU oracle for band-limited PDE-LDDMM with semi-Lagrangian RK2 integration.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the library and its Python binding
never do.  It shares no code with the HIP path: the truncated Fourier maps are
computed here with complex FFTs plus cropping (the HIP path uses separable real
contractions), the cubic B-spline prefilter by division in Fourier space (the
HIP path uses recursive filtering or folds it into the band-limited basis), and
interpolation by explicit evaluation of the B-spline kernel.

Every routine is written from M. Hernandez, "Combining the band-limited
parameterization and Semi-Lagrangian Runge-Kutta integration for efficient
PDE-constrained LDDMM" (arXiv 2006.06823); each function names the section,
equation or table it follows.  Where the paper is silent or ambiguous the
reading taken is stated in the docstring.

Modules
  spectral     band-limited space: inclusion iota, projection pi, spectral
               gradient / divergence / Jacobian, the operator L~ and its inverse
  bspline      periodic cubic B-spline prefilter and evaluation (value, gradient)
  semilag      characteristics and the Heun (RK2) steps along them
  problem      problem description (grid, band, time steps, alpha, s, sigma^2)
  variant1     original BL PDE-LDDMM (image transport)
  variant2     BL PDE-LDDMM based on the state equation (maps phi, psi, J)
  variant3     BL PDE-LDDMM based on the deformation state equation
  gauss_newton PCG, Armijo line search, Gauss-Newton driver, metrics, Jacobian
  dto          discretise-then-optimise objective for finite-difference pins
"""
