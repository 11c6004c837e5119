"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package builds the meshes, boundary conditions, nodal load vectors,
load-time parameters and random states that both sides consume.  It holds
none of the method's arithmetic: no surface discretisation, no SBFEM
matrices, no symmetry group, no time stepping.  Everything here is octree
topology, integer lattice bookkeeping and seeded random numbers.

Mesh format (the "natural" numbering both sides read):

* The domain is ``roots = (nx, ny, nz)`` root cubes of edge ``h0``.  A cell at
  octree level ``l`` has edge ``h0 * 2**-l``.  All nodes lie on the lattice of
  spacing ``h0 * 2**-lmax``.
* Every cell lists its nodes in *natural slot order*: the 8 corners, then the
  present mid-edge nodes in edge order, then the present face-centre nodes in
  face order (see :mod:`meshgen.slots`).  ``cell_slots`` is an 18-bit mask,
  bits 0-11 for the 12 edge midpoints and bits 12-17 for the 6 face centres.
* Degrees of freedom are node-major: dof ``3*node + axis``.
"""

from .slots import CORNERS, EDGES, FACES, SLOT_POS, slot_positions, n_slots  # noqa: F401
from .octree import Mesh, build_mesh  # noqa: F401
from . import configs  # noqa: F401
