"""FP64 CPU oracle for the reciprocal part of Kroneckerised PME.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and
its Python binding) may import, call or link anything in this package.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code, tables or helpers with the GPU path.

Everything here is plain, slow and written to be checked by eye against the
definitions it follows:

* ``bspline``  -- cardinal B-splines M_p, their derivative and the Euler
  exponential-spline moduli |b(m)|^2 (the SPME interpolation the paper names
  as the alternative to Lagrange interpolation, Sec. 2.2).
* ``ewald``    -- direct Ewald summation: real + reciprocal + self + neutralising
  terms, potentials and forces (Sec. 1.1 Eq. qmutheta_coulomb, Sec. 1.2
  Eqs. tau, hexpr, sumhexpr).
* ``spme``     -- classical FFT-based smooth PME on the same grid (Sec. 1.2).
* ``skp``      -- the Sum-of-Kronecker-Products reciprocal operator: the nested
  SVD of the kernel tensor (Sec. 2.1.1, Eqs. last_decomp_kron, eym,
  estimate_svd), real circulant per-axis factors (Sec. 2.3-2.4, Eq. VtV,
  Eq. formfinale), the three mode products per term (Sec. 3.2-3.3, Alg. 1 and
  Alg. 2) and the constant correction (Sec. 4.1 Eq. termbonsum, Alg. 4).

* ``lagrange`` -- the paper's own discretisation (Sec. 2.2, Sec. 4.1): per-cell
  equispaced Lagrange interpolation and the mode-truncated kernel alpha_M,
  with the direct alpha_M mode sum it approximates.
* ``rect``     -- the rectangular real cos/sin form of the per-axis factors
  (Sec. 2.3 Eq. kronw, Sec. 2.4 Eq. VtV): A = V^T S V, two thin products per
  mode product.
* ``quadrature`` -- the second SKP construction: the sinc quadrature of 1/x
  (Sec. 2.1.2, Eqs. one_over_r_int and quaddecompalpham), one Kronecker term
  per node, with the brute-force choice of the lifting factor h.

Parity status of each function is stated in its module header; every function
here is pinned by a test in ``tests/test_oracle_*.py`` against values the
mathematics fixes (closed forms, textbook constants, identities, brute force).
"""
