"""Cube-cell patterns and orientations (Sec. 3.2.1-3.2.2), host set-up code.

A balanced octree cell can carry mid-edge nodes on any of its 12 edges
(4096 configurations).  Under the 48 signed axis permutations they fall into
144 patterns; every cell is linked to one master cell per pattern through
an orientation Q with  u_master[k] = Q u_cell[conn[k]]  (Sec. 3.2.2).

Input node order of a cell ("natural" order, the mesh format this package
reads): 8 corners, then present mid-edge nodes in edge order, then present
face centres in face order.  Positions are integer vectors in {-1,0,1}^3
(units of half the cell edge about the centre):
  corners  i + 2j + 4k  at (2i-1, 2j-1, 2k-1);
  edges    x-edges (0,-1,-1) (0,1,-1) (0,-1,1) (0,1,1), y-edges
           (-1,0,-1) (1,0,-1) (-1,0,1) (1,0,1), z-edges (-1,-1,0) (1,-1,0)
           (-1,1,0) (1,1,0)  -> slot mask bits 0..11;
  faces    -x +x -y +y -z +z  -> slot mask bits 12..17.

Orientation codes follow the header: code = 8*perm + signs with the
permutations (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0) and sign bit a
meaning s_a = -1;  Q[a][perm[a]] = s_a.

Face-centre nodes: a face carries one unless it has no mid-edge node or
exactly two on opposite edges (the face discretisation of Fig. OctreeDist
read so that every surface element is a rectangle or an isosceles triangle).
"""

import numpy as np

PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))

_CORNER = [(2 * i - 1, 2 * j - 1, 2 * k - 1) for k in (0, 1) for j in (0, 1) for i in (0, 1)]
_EDGE = [(0, -1, -1), (0, 1, -1), (0, -1, 1), (0, 1, 1),
         (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (1, 0, 1),
         (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 1, 0)]
_FACE = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
POSITIONS = np.array(_CORNER + _EDGE + _FACE, dtype=np.int64)   # slot -> position
_POS_INDEX = {p: s for s, p in enumerate(_CORNER + _EDGE + _FACE)}


def orientation_matrix(code):
    perm, signs = PERMS[code // 8], code % 8
    Q = np.zeros((3, 3), dtype=np.int64)
    for a in range(3):
        Q[a, perm[a]] = -1 if (signs >> a) & 1 else 1
    return Q


ORIENT_Q = np.stack([orientation_matrix(c) for c in range(48)])
ORIENT_PERM = np.array([PERMS[c // 8] for c in range(48)], dtype=np.int64)
ORIENT_SIGN = np.array([[-1 if (c % 8 >> a) & 1 else 1 for a in range(3)] for c in range(48)],
                       dtype=np.int64)


def slot_image(code):
    """slot -> slot under Q (positions p -> Q p), for all 26 slots."""
    Q = ORIENT_Q[code]
    return np.array([_POS_INDEX[tuple(int(v) for v in Q @ p)] for p in POSITIONS], dtype=np.int64)


SLOT_IMAGE = np.stack([slot_image(c) for c in range(48)])        # (48, 26)


def transform_slot_masks(masks, code):
    """Image of 18-bit slot masks (bits = slots 8..25) under orientation ``code``."""
    masks = np.asarray(masks, dtype=np.int64)
    out = np.zeros_like(masks)
    img = SLOT_IMAGE[code]
    for s in range(8, 26):
        out |= ((masks >> (s - 8)) & 1) << (img[s] - 8)
    return out


def face_bits(edge_masks):
    """Face-centre bits (6) implied by 12-bit edge masks."""
    edge_masks = np.asarray(edge_masks, dtype=np.int64)
    out = np.zeros_like(edge_masks)
    for f, fp in enumerate(_FACE):
        a = int(np.flatnonzero(fp)[0])
        es = [e for e, ep in enumerate(_EDGE) if ep[a] == fp[a]]
        bits = [(edge_masks >> e) & 1 for e in es]
        nh = sum(bits)
        axes = [int(np.flatnonzero(np.array(_EDGE[e]) == 0)[0]) for e in es]
        opp = np.zeros(edge_masks.shape, dtype=bool)
        for i in range(4):
            for j in range(i + 1, 4):
                if axes[i] == axes[j]:
                    opp |= (bits[i] == 1) & (bits[j] == 1) & (nh == 2)
        out |= ((nh > 0) & ~opp).astype(np.int64) << f
    return out


def full_mask(edge_masks):
    e = np.asarray(edge_masks, dtype=np.int64)
    return e | (face_bits(e) << 12)


def present(slot_mask):
    """Slots present in a cell (natural order)."""
    return [s for s in range(26) if s < 8 or (int(slot_mask) >> (s - 8)) & 1]


class PatternTable:
    """The 144 patterns and the lookup from any edge configuration to
    (pattern id, valid orientation codes)."""

    def __init__(self):
        all_masks = full_mask(np.arange(4096))
        images = np.stack([transform_slot_masks(all_masks, c) for c in range(48)])   # (48, 4096)
        canon = images.min(axis=0)
        reps = np.unique(canon)
        # ids ordered by node count, then mask value
        counts = np.array([len(present(r)) for r in reps])
        order = np.lexsort((reps, counts))
        self.master_mask = reps[order]                       # pattern id -> master slot mask
        self.n_patterns = len(self.master_mask)
        lut = {int(m): i for i, m in enumerate(self.master_mask)}
        self.pattern_of = np.array([lut[int(c)] for c in canon], dtype=np.int64)   # edge mask -> id
        self.valid = images == canon[None, :]                # (48, 4096) code maps mask onto master
        self.first_code = np.argmax(self.valid, axis=0)
        self.n_nodes = np.array([len(present(m)) for m in self.master_mask], dtype=np.int64)

    def master_positions(self, pid):
        return POSITIONS[present(self.master_mask[pid])]

    def conn_permutation(self, slot_mask, code):
        """perm[k] = index, in the cell's natural order, of the node that master node k reads.

        Master node k sits at position P_k; the cell node mapped onto it sits at
        Q^T P_k (Q orthogonal)."""
        Q = ORIENT_Q[code]
        cell_slots = present(slot_mask)
        pid = self.pattern_of[int(slot_mask) & 0xFFF]
        out = []
        for p in self.master_positions(pid):
            src = _POS_INDEX[tuple(int(v) for v in Q.T @ p)]
            out.append(cell_slots.index(src))
        return np.array(out, dtype=np.int64)


_TABLE = None


def table():
    global _TABLE
    if _TABLE is None:
        _TABLE = PatternTable()
    return _TABLE
