"""CPU oracle for the accelerated divide-and-conquer (ADC) tridiagonal eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, fp64 numpy restatement
of what the method computes, written from the paper (Li, Liao, Liu, Jiang,
"New fast divide-and-conquer algorithms for the symmetric tridiagonal
eigenvalue problem"), so that the HIP path can be checked against it.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it.
The product path (the HIP library and its Python binding) never imports, links
or calls anything here, and this package never imports the product.

Modules
-------
secular   the secular equation of D + rho z z^T (Theorem 1), solved by bisection
          over the ordered set of representable doubles; Loewner recompute of z
          (eq. ev_z) with the differences of Remark 1 (eq. d-lambda); the
          Cauchy-like eigenvector matrix (eq. Ev-Q).
dc        Cuppen's tear (eqs. T, T2, T3), deflation, and the whole
          divide-and-conquer of Algorithm 1 with a dense or an HSS update.
hss       interpolative decomposition, the randomized HSS construction of
          Algorithm 2, the right HSS multiplication of Algorithm 3, the dense
          expansion of an HSS matrix (eq. new-hss) and the rank estimate of
          eq. (bounds) with the neighbouring-segment rules of Section 4.1.
sturm     Sturm-sequence eigenvalue counts of a tridiagonal matrix (textbook),
          used to check single eigenvalues at any size.
mlp       fp64 forward/backward/Adam of the 16-64-64-1 rank-predictor MLP.
fmm       fast sampling for Algorithm 2: a one-dimensional Chebyshev FMM for
          the off-diagonal Cauchy sums, and the same samples by definition.
"""
