"""MI355X-native explicit octree-SBFEM time stepper.

Host set-up (FP64): :mod:`.patterns` (cube-cell patterns and orientations),
:mod:`.sbfem_cell` and :mod:`.library` (master-cell library, mesh
canonicalisation).  Device path: the C-ABI library ``libsbfem.so`` built from
``csrc/`` for gfx950, reached through :mod:`.binding`.
"""
