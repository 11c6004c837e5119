"""Write ``zoo_masks.txt``: the smallest 12-bit edge configuration of each of
the 144 classes of cube cells under the 48 cube transformations.

The classes come from the oracle's enumeration (the only place the symmetry
group lives outside the GPU path's own set-up code).  The list only decides
which test cells the mesh generator places; neither side reads it as data.
Run from the repository root:  python -m meshgen.make_zoo_masks
"""

import os

from oracle import symmetry


def main():
    reps = sorted(o[0] for o in symmetry.orbits())
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zoo_masks.txt")
    with open(path, "w") as f:
        f.write("# one 12-bit edge configuration per class of cube cells (smallest member);\n")
        f.write("# written by meshgen/make_zoo_masks.py\n")
        for r in reps:
            f.write(f"{r}\n")


if __name__ == "__main__":
    main()
