"""Plain FP64 CPU oracle of the S-ADI scheme (arXiv 2312.06206) -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The device library never calls it and shares no code with it.

  coeffs     1D coefficients a_k (printed Gamma closed form) and 2D coefficients
             a_ij (Fourier coefficients of the symbol, via the subordination
             identity and a whole-line trapezoidal rule)
  operators  D = h^-alpha T(a), the BTTB operator L_h (dense double sum, or BCCB
             embedding + library FFT), H = I + kappa tau^2/2 D
  scheme     the S-ADI start-up and three-level schemes in literal and delta form
             (Cholesky line solves), the discrete energy, Error_1 / Error_2

Pins (tests/test_oracle_*.py): closed forms and summation identities of a_k,
brute-force 2D Fourier integrals of a_ij, the far-field constant, the corner and
row-sum identities of the symbol, the operator lemmas of the stability section,
exact energy conservation for g = 0, the alpha = 2 DST closed form, second-order
convergence, and the S-ADI errors printed in the paper's Tables 1, 2 and 4.
Every function is pinned; none is "parity unpinned".
"""
