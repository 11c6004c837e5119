"""Pins of the cube symmetry group and the pattern count (Sec. 3.2.2, App. A)."""

import os

import numpy as np

from meshgen.slots import EDGES
from oracle import symmetry

GOLD = os.path.join(os.path.dirname(__file__), "golden", "transforms.txt")


def _golden():
    mats, counts = {}, {}
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if len(tok) == 10:
            mats[tok[0]] = np.array([int(v) for v in tok[1:]]).reshape(3, 3)
        else:
            counts[tok[0]] = int(tok[1])
    return mats, counts


def test_printed_matrices_and_products():
    mats, counts = _golden()
    assert np.array_equal(symmetry.T_X, mats["T_x"])
    assert np.array_equal(symmetry.T_Y, mats["T_y"])
    assert np.array_equal(symmetry.T_Z, mats["T_z"])
    assert np.array_equal(symmetry.R_X, mats["R_x"])
    assert np.array_equal(symmetry.R_Y, mats["R_y"])
    assert np.array_equal(symmetry.R_Z, mats["R_z"])
    # worked example of Fig. OctTrans: Q1 = T_x T_z
    assert np.array_equal(symmetry.T_X @ symmetry.T_Z, mats["Q1"])
    assert np.array_equal(symmetry.R_X, mats["Q2"])


def test_group_size_and_closure():
    _, counts = _golden()
    G = symmetry.all_transforms()
    assert len(G) == counts["n_transforms"] == 48
    keys = {tuple(Q.ravel()) for Q in G}
    assert len(keys) == 48
    for A in G:
        for B in G:
            assert tuple((A @ B).ravel()) in keys
    dets = [round(np.linalg.det(Q)) for Q in G]
    assert dets.count(1) == 24 and dets.count(-1) == 24
    # the printed generators lie in the group
    for M in (symmetry.T_X, symmetry.T_Y, symmetry.T_Z, symmetry.R_X, symmetry.R_Y, symmetry.R_Z):
        assert tuple(M.ravel()) in keys


def _edge_perm(Q):
    idx = {tuple(p): e for e, p in enumerate(EDGES.tolist())}
    return [idx[tuple((Q @ EDGES[e]).tolist())] for e in range(12)]


def _cycle_lengths(perm):
    seen, out = set(), []
    for s in range(len(perm)):
        if s in seen:
            continue
        n, j = 0, s
        while j not in seen:
            seen.add(j)
            j = perm[j]
            n += 1
        out.append(n)
    return out


def _burnside_by_k(G):
    """Orbit counts per number of marked edges by Burnside's lemma (generating function)."""
    total = np.zeros(13, dtype=np.int64)
    for Q in G:
        poly = np.zeros(13, dtype=np.int64)
        poly[0] = 1
        for L in _cycle_lengths(_edge_perm(Q)):
            nxt = poly.copy()
            nxt[L:] += poly[:-L]
            poly = nxt
        total += poly
    assert (total % len(G) == 0).all()
    return total // len(G)


def test_144_patterns_burnside_and_enumeration():
    _, counts = _golden()
    G = symmetry.all_transforms()
    by_k = _burnside_by_k(G)
    assert by_k.sum() == counts["n_unique_patterns"] == 144
    # complement symmetry stated with the pattern listing (App. A)
    assert np.array_equal(by_k, by_k[::-1])
    orbs = symmetry.orbits(G)
    assert len(orbs) == 144
    assert sum(len(o) for o in orbs) == counts["n_configurations"] == 4096
    enum_k = np.zeros(13, dtype=np.int64)
    for o in orbs:
        enum_k[bin(o[0]).count("1")] += 1
    assert np.array_equal(enum_k, by_k)
    assert by_k.tolist() == [1, 1, 4, 9, 18, 24, 30, 24, 18, 9, 4, 1, 1]


def test_rotations_alone_do_not_suffice():
    G = symmetry.all_transforms()
    rot = [Q for Q in G if round(np.linalg.det(Q)) == 1]
    assert _burnside_by_k(rot).sum() == 218
    assert len(symmetry.orbits(rot)) == 218
