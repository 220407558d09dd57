"""Slow, dense, obviously-correct CPU oracle for the high-order boundary condition
deblurring method (Donatelli, "Fast transforms for high order boundary conditions").

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import or run it.
The product path (the HIP library and its Python binding) never calls it and shares no
code, table or constant generator with it.

Everything here is written from the paper's definitions:

* ``bc``          blurring matrices assembled directly from the boundary conditions
                  (periodic / reflective / antireflective, Section 2) and the
                  second-difference stencil (eq. L).  These are the independent
                  brute-force references that pin the spectral constructions.
* ``transforms``  the dense transform matrices T (eq. ART), T_C (eq. Tc), T_F (eq. Tf)
                  and the degree-3 extension, built entry by entry on the extended grids
                  with exactly reduced angles; the eigenvalue vectors (eqs. jcf, Ac, Af,
                  and the smoothing spectra of Section 4); dense inverse by LU with
                  extended-precision iterative refinement.
* ``tikhonov``    the reblurred Tikhonov spectral filter (eq. freg), the dense normal
                  equations it solves (eq. nerebl), the GCV functional the method
                  minimises (eqs. gcv2 / mugcv) and the exact GCV (eq. gcv) diagnostic.
* ``twod``        the tensor-product (Kronecker) 2D case of Section 6.

Parity status of each function is stated in its docstring; see also the tests under
``tests/test_oracle_*.py`` which pin the oracle against closed forms, brute-force
boundary-condition assemblies and invariants.
"""

from . import bc, transforms, tikhonov, twod  # noqa: F401
