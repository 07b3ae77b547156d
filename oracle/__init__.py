"""CPU oracle for the exponential-integrator hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
product path (the HIP library and its Python binding) never calls it, and it
shares no code with that path: the two meet only in the seeded input arrays of
the ``synth`` module and in the results the tests compare.

What it computes (Einkemmer & Ostermann, "Exponential Integrators on Graphic
Processing Units", HPCS 2013):

* ``operators``   - the matrices A of Sec. III-A/III-B assembled as scipy
  sparse matrices straight from their definitions (stencils with the boundary
  conditions folded into A, as Sec. II-C states), the product (alpha A +
  beta I) x of eq. (3), and the Gershgorin field-of-values bound that the
  polynomial interpolation of Sec. II-C needs.
* ``leja``        - Leja points on [-2, 2] and the divided differences of the
  phi functions at those points, in 80-digit mpmath arithmetic.
* ``integrators`` - the Newton-form interpolation at Leja points (Sec. III-C)
  applied to a vector, the action phi_k(tau A) v with substeps, and the
  exponential Euler step of eq. (2).

Everything is float64 (mpmath where noted), unblocked and in the order the
definitions state, so that each function can be checked against the paper by
eye.  The pins that tie it to the mathematics live in ``tests/test_oracle_*``.
"""
