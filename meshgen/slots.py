"""Natural node-slot convention of a cube cell.

A node position is written as an integer vector ``p`` in {-1, 0, 1}^3, in
units of half the cell edge, measured from the cell centre.  A balanced
octree cell (2:1 rule, Sec. 3.2.1) can carry nodes only at the 8 corners,
the 12 edge midpoints and the 6 face centres.

Slot order (fixed; both the oracle and the GPU path read conn in this order):

* slots 0-7   corners, index ``i + 2*j + 4*k`` at ``p = (2i-1, 2j-1, 2k-1)``;
* slots 8-19  edge midpoints, bit ``e`` of the edge mask is slot ``8 + e``;
  edges 0-3 run along x, 4-7 along y, 8-11 along z;
* slots 20-25 face centres, bit ``12 + f`` of the slot mask is slot ``20 + f``;
  faces in the order -x, +x, -y, +y, -z, +z.
"""

import numpy as np

CORNERS = np.array([[2 * i - 1, 2 * j - 1, 2 * k - 1]
                    for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=np.int64)

EDGES = np.array([
    # along x: (0, +-1, +-1)
    [0, -1, -1], [0, 1, -1], [0, -1, 1], [0, 1, 1],
    # along y: (+-1, 0, +-1)
    [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [1, 0, 1],
    # along z: (+-1, +-1, 0)
    [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 1, 0],
], dtype=np.int64)

FACES = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]],
                 dtype=np.int64)

# all 26 slot positions in slot order
SLOT_POS = np.concatenate([CORNERS, EDGES, FACES], axis=0)

EDGE_BITS = 12
FACE_BITS = 6
FULL_SLOT_MASK = (1 << (EDGE_BITS + FACE_BITS)) - 1


def present_slots(slot_mask):
    """Slot indices (0..25) present in a cell with the given 18-bit mask, in order."""
    slot_mask = int(slot_mask)
    out = list(range(8))
    for b in range(EDGE_BITS + FACE_BITS):
        if (slot_mask >> b) & 1:
            out.append(8 + b)
    return out


def slot_positions(slot_mask):
    """Positions (n, 3) of the present nodes, natural order, units of h/2."""
    return SLOT_POS[present_slots(slot_mask)]


def n_slots(slot_mask):
    return 8 + bin(int(slot_mask) & FULL_SLOT_MASK).count("1")


def popcount32(a):
    """Vectorised popcount of a uint32 array."""
    a = a.astype(np.uint32)
    a = a - ((a >> 1) & 0x55555555)
    a = (a & 0x33333333) + ((a >> 2) & 0x33333333)
    a = (a + (a >> 4)) & 0x0F0F0F0F
    return ((a * 0x01010101) & 0xFFFFFFFF) >> 24
