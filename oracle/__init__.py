"""Plain FP64 CPU oracle of the explicit octree-SBFEM solver (TEST INFRASTRUCTURE).

This package is the reference the GPU path is checked against.  It is slow
on purpose and written to be read against the paper:

* :mod:`oracle.element`  -- the SBFEM cube cell of Sec. 2 (scaled boundary
  geometry, strain operator, coefficient matrices E0/E1/E2/M0, stiffness from
  the bounded eigen-solution, consistent mass with radial integration) and the
  same-direction mass lumping of Sec. 3.3; computed directly for each cell's
  own node layout, never through canonical patterns or orientations.
* :mod:`oracle.solver`   -- Alg. 1 (explicit solver in serial): element-by-
  element internal force (eq. Rinte), central-difference update with a
  diagonal mass (eq. DnMdiag), start-up point (eq. D0), element stability
  limit (eq. tcr and its scaling, eq. tcr_scale).
* :mod:`oracle.symmetry` -- the 48 cube transformations of Sec. 3.2.2, used
  only by the checks (pattern counts, orientation invariance).
* :mod:`oracle.loads`    -- the load-time functions of Sec. 5 (eq. Ricker,
  eq. Triangle, eq. Lamb).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_2103_09100_amd``) and imports nothing from it; the only common
module is the seeded input generator ``meshgen``, which holds none of the
method's arithmetic.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(closed forms, invariants, brute force, the paper's printed values).  The
absolute stiffness of the hanging-node cells is constrained only through
invariants (rigid modes, linear-field energy, mass conservation, orientation
covariance, convergence of eigenfrequencies): the paper prints no entries of
those matrices.
"""
