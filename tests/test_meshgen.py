"""Checks of the seeded input generator: 2:1 balance, node sharing, conformity, sizes."""

import numpy as np
import pytest

from meshgen import configs
from meshgen.slots import SLOT_POS, present_slots
from oracle import symmetry


def _level_map(m):
    n = np.array(m.roots) * (1 << m.lmax)
    lv = np.full(tuple(n), -1, dtype=np.int64)
    for c in range(m.n_cells):
        s = 1 << (m.lmax - int(m.cell_level[c]))
        x, y, z = m.cell_lat[c]
        assert (lv[x:x + s, y:y + s, z:z + s] == -1).all()
        lv[x:x + s, y:y + s, z:z + s] = m.cell_level[c]
    assert (lv >= 0).all()
    return lv


@pytest.mark.parametrize("mesh_fn", [lambda: configs.cfg2(lcoarse=2, lfine=5, delta=0.1),
                                     lambda: configs.small_zoo(),
                                     lambda: configs.inclusion_mesh(seed=1, lcoarse=3, lfine=5, band=0.2)])
def test_balance_and_conformity(mesh_fn):
    m = mesh_fn()
    lv = _level_map(m)
    for ax in range(3):
        for off in (-1, 1):
            sh = np.roll(lv, off, axis=ax)
            sl = [slice(None)] * 3
            sl[ax] = slice(1, -1)
            assert np.abs(lv[tuple(sl)] - sh[tuple(sl)]).max() <= 1
    # diagonal neighbours too (edge and corner balance)
    for d in [(1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1), (1, -1, 0), (1, -1, 1), (1, 1, -1), (-1, 1, 1)]:
        a = lv[1:-1, 1:-1, 1:-1]
        b = lv[1 + d[0]:lv.shape[0] - 1 + d[0], 1 + d[1]:lv.shape[1] - 1 + d[1], 1 + d[2]:lv.shape[2] - 1 + d[2]]
        assert np.abs(a - b).max() <= 1
    # every node lying at a slot position of a cell belongs to that cell, and the
    # listed nodes sit exactly at their slot positions
    key = {tuple(p): i for i, p in enumerate(m.node_lat.tolist())}
    for c in range(m.n_cells):
        s = 1 << (m.lmax - int(m.cell_level[c]))
        centre2 = 2 * m.cell_lat[c].astype(np.int64) + s
        listed = list(m.cell_nodes(c))
        slots = present_slots(int(m.cell_slots[c]))
        for k, pos in enumerate(SLOT_POS):
            lat2 = centre2 + pos * s
            if (lat2 % 2).any():
                nid = None
            else:
                nid = key.get(tuple((lat2 // 2).tolist()))
            if k in slots:
                assert nid == listed[slots.index(k)]
            else:
                assert nid is None, (c, k)
    assert len(set(m.conn.tolist())) == m.n_nodes


def test_cfg1_shape():
    m = configs.cfg1()
    assert (m.n_cells, m.n_nodes, m.n_dof) == (512, 729, 2187)
    assert int(m.fixed.sum()) == 3 * 81
    assert m.load_val.tolist() == [-1.0]
    assert m.node_lat[m.load_dof[0] // 3].tolist() == [4, 4, 8]


def test_cfg2_size_and_pattern_coverage():
    orbs = symmetry.orbits()
    orbit_of = np.zeros(4096, dtype=np.int64)
    for i, o in enumerate(orbs):
        orbit_of[o] = i
    for m in (configs.cfg2(), configs.small_zoo()):
        present = set(orbit_of[np.unique(m.cell_slots & 0xFFF)].tolist())
        assert len(present) == 144
        assert m.load_dof.size > 0 and np.abs(m.load_val).sum() > 0
    assert 1.8e6 <= configs.cfg2().n_dof <= 2.2e6


def test_zoo_list_is_one_per_class():
    orbs = symmetry.orbits()
    orbit_of = np.zeros(4096, dtype=np.int64)
    for i, o in enumerate(orbs):
        orbit_of[o] = i
    masks = configs.zoo_masks()
    assert sorted(orbit_of[masks].tolist()) == list(range(144))
