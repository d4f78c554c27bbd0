"""CPU oracle for batched elliptic-curve multi-scalar multiplication and ECDSA
verification.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the GPU library.

Two independent implementations of the same plain definitions:

* ``oracle.ref``  -- Python integers; the field is ``%`` and ``pow(x, -1, p)``,
  points are affine with the full case analysis of the short-Weierstrass
  group law (Section 2.1: Eqn 1 curve, Eqns 2-3 point addition, the PDBL
  tangent slope), scalar multiplication is the double-and-add loop of
  Algorithm 1, and an MSM is literally the sum of the scalar multiples.
* ``oracle.c_oracle`` -- the same definitions in plain C (schoolbook
  products with Barrett reduction, Fermat inversion, Jacobian coordinates),
  multi-threaded, for sizes the Python version cannot reach in seconds.
"""
