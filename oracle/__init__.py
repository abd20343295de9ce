"""Plain FP64 CPU oracle for TT-IGA (test infrastructure, not product code).

This package is the slow, obviously correct reference that the HIP library is
checked against.  Only the test suite, the graft smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP path: the two read the same seeded problem
descriptions (package ``workloads``) and nothing else.

Modules, each following the passage of the paper named in its header:

* ``bspline``    - knot vectors, Cox-de Boor basis and derivative (Section 2.1)
* ``nurbs``      - NURBS curves and solids, homogeneous form (Section 2.3)
* ``quadrature`` - Gauss-Legendre rule per knot span
* ``geometry``   - Jacobian, det J, R = det J J^-1 J^-T, f det J (Section 3.3, eq. Rxi)
* ``sources``    - evaluation of the source term f
* ``sparse_iga`` - full-grid sparse K, F, Dirichlet reduction and direct solve (Section 3.3)
* ``tt``         - TT format, TT-SVD, TT-rounding, TT-matrix algebra (Section 4.1)
* ``tt_iga``     - TT assembly of K and F and the TT solve (Sections 4.2-4.3)
* ``errors``     - relative L2 error (eq. L2norm)

Parity unpinned: nothing in this package.  Every function is pinned by a
``-m "not gpu"`` test against closed forms, identities, library routines or
brute force (the test files named ``test_oracle_*``): the error measures by
integrals with closed forms on the annulus and the identity cube, the
condition estimate by the extreme eigenvalues of the dense K_II.
"""
