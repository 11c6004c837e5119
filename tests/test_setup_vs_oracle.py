"""CPU checks of the GPU path's host set-up against the oracle.

The GPU path builds its master-cell library and its cell-to-master links with
its own code (``paper_2103_09100_amd.patterns / sbfem_cell / library``); here
they are compared with the oracle's direct per-cell SBFEM.  No GPU needed.
"""

import numpy as np
import pytest

from meshgen import configs
from meshgen.slots import SLOT_POS
from oracle import element as el
from oracle.solver import Oracle
from paper_2103_09100_amd import library, patterns as pt


@pytest.fixture(scope="module")
def lib():
    return library.build_library(0.25, workers=4)


def test_slot_convention_matches_input_format():
    assert np.array_equal(pt.POSITIONS, SLOT_POS)


def test_pattern_table_counts():
    tab = pt.table()
    assert tab.n_patterns == 144
    assert tab.valid.any(axis=0).all()
    counts = np.bincount(tab.n_nodes, minlength=27)
    assert counts[8] == 1 and counts[26] == 1 and counts.sum() == 144
    # orientation codes are the 48 signed permutations
    keys = {tuple(q.ravel()) for q in pt.ORIENT_Q}
    assert len(keys) == 48


def test_master_cells_match_oracle(lib):
    tab = pt.table()
    for p in range(lib.n_patterns):
        c = el.Cell(int(tab.master_mask[p]), 0.25)
        assert np.abs(c.K - lib.K[p]).max() <= 1e-12 * np.abs(c.K).max()
        assert np.abs(c.m - lib.m[p]).max() <= 1e-12 * c.m.max()
        assert abs(c.omega_max - lib.omega[p]) <= 1e-12 * c.omega_max


@pytest.mark.parametrize("seed", [None, 4])
def test_linked_cells_reproduce_direct_cells(lib, seed):
    """s R^T K_p R on the cell's global dofs == the oracle's own matrix of that cell."""
    mesh = configs.small_zoo()
    pid, code, conn = library.canonicalise(mesh, seed=seed)
    o = Oracle(mesh, workers=4)
    rng = np.random.default_rng(0)
    cells = np.concatenate([rng.choice(mesh.n_cells, 300, replace=False),
                            np.flatnonzero(mesh.cell_slots != 0)[:300]])
    for c in cells:
        lo, hi = mesh.conn_ptr[c], mesh.conn_ptr[c + 1]
        nat = mesh.conn[lo:hi].astype(np.int64)
        mst = conn[lo:hi].astype(np.int64)
        assert sorted(nat.tolist()) == sorted(mst.tolist())
        K_or = o.cell_of(c).K
        Q = pt.ORIENT_Q[code[c]]
        n = len(nat)
        # R maps cell dofs (natural order) to master dofs: u_master[k] = Q u[mst[k]]
        pos = {v: i for i, v in enumerate(nat.tolist())}
        R = np.zeros((3 * n, 3 * n))
        for k, v in enumerate(mst.tolist()):
            i = pos[v]
            R[3 * k:3 * k + 3, 3 * i:3 * i + 3] = Q
        K_gpu = R.T @ lib.K[pid[c]] @ R
        assert np.abs(K_gpu - K_or).max() <= 1e-11 * np.abs(K_or).max(), c
        m_gpu = np.abs(R.T) @ lib.m[pid[c]]
        assert np.allclose(m_gpu, o.cell_of(c).m, rtol=1e-11)
