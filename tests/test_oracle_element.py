"""Pins of the oracle's SBFEM cell (Sec. 2, Sec. 3.2-3.3) against mechanics and closed forms."""

import numpy as np
import pytest

from meshgen.octree import face_centre_bits
from meshgen.slots import SLOT_POS, present_slots
from oracle import element as el
from oracle import symmetry

NU = 0.25


def slot_mask(edge_mask):
    return int(edge_mask) | (int(face_centre_bits(np.array([edge_mask]))[0]) << 12)


def sample_masks(k=6, seed=0):
    rng = np.random.default_rng(seed)
    masks = [0, 1, 0b11, 0b101, (1 << 12) - 1]
    masks += [int(v) for v in rng.integers(0, 4096, size=k)]
    return [slot_mask(m) for m in masks]


def voigt(A):
    e = 0.5 * (A + A.T)
    return np.array([e[0, 0], e[1, 1], e[2, 2], 2 * e[1, 2], 2 * e[0, 2], 2 * e[0, 1]])


def sym_tensor(v):
    return np.array([[v[0], v[5], v[4]], [v[5], v[1], v[3]], [v[4], v[3], v[2]]])


@pytest.fixture(scope="module")
def cells():
    return {m: el.Cell(m, NU) for m in sample_masks()}


def test_elasticity_matrix_moduli():
    E, nu = 2.0, 0.3
    D = el.elasticity_matrix(E, nu)
    K_bulk = E / (3 * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    s = D @ np.array([1, 1, 1, 0, 0, 0.0])
    assert np.allclose(s, [3 * K_bulk] * 3 + [0, 0, 0], rtol=1e-14)
    s = D @ np.array([0, 0, 0, 0, 0, 1.0])       # engineering shear strain 1
    assert np.isclose(s[5], mu, rtol=1e-14) and np.allclose(s[:5], 0)


def test_surface_elements_tile_each_face():
    """Rectangles and isosceles right triangles covering each face exactly once."""
    for m in sample_masks(40, seed=1):
        subs = el.face_subelements(m)
        P = SLOT_POS[present_slots(m)].astype(float)
        area = 0.0
        for s in subs:
            x = P[s]
            if len(s) == 4:
                e = [x[(i + 1) % 4] - x[i] for i in range(4)]
                for i in range(4):
                    assert abs(e[i] @ e[(i + 1) % 4]) < 1e-14          # right angles
                area += np.linalg.norm(e[0]) * np.linalg.norm(e[1])
            else:
                e = [x[(i + 1) % 3] - x[i] for i in range(3)]
                L = sorted(np.linalg.norm(v) for v in e)
                assert np.isclose(L[0], L[1]) and np.isclose(L[2], np.sqrt(2) * L[0])
                area += 0.5 * np.linalg.norm(np.cross(e[0], e[1]))
            # every surface element lies in one face plane
            assert np.ptp(np.abs(x), axis=0).min() == 0
        assert np.isclose(area, 6 * 4.0)          # 6 faces of edge 2 in units of h/2


def test_quadrature_is_exact():
    m = slot_mask(0b100000100101)
    A = el.coefficient_matrices(m, nu=NU, nq=3)
    B = el.coefficient_matrices(m, nu=NU, nq=6)
    for a, b in zip(A, B):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_rigid_modes_symmetry_psd(cells):
    for m, c in cells.items():
        K = c.K
        assert np.abs(K - K.T).max() == 0.0
        w = np.linalg.eigvalsh(K)
        scale = w.max()
        assert (np.abs(w[:6]) < 1e-12 * scale).all(), (m, w[:8])
        assert w[6] > 1e-3 * scale
        X = SLOT_POS[present_slots(m)] * 0.5
        for a in range(3):                       # translations
            t = np.zeros_like(X)
            t[:, a] = 1.0
            assert np.abs(K @ t.ravel()).max() < 1e-12 * scale
        for a in range(3):                       # rotations
            w_ = np.zeros(3)
            w_[a] = 1.0
            r = np.cross(w_, X)
            assert np.abs(K @ r.ravel()).max() < 1e-12 * scale


def test_linear_fields_energy_and_first_moment(cells):
    """SBFEM reproduces linear fields: v_B^T K u_A = V eps_B:D:eps_A and
    sum_i f_i x_i^T = sigma_A V (divergence theorem)."""
    D = el.elasticity_matrix(1.0, NU)
    rng = np.random.default_rng(3)
    for m, c in cells.items():
        X = SLOT_POS[present_slots(m)] * 0.5
        A = rng.normal(size=(3, 3))
        B = rng.normal(size=(3, 3))
        uA = (X @ A.T).ravel()
        uB = (X @ B.T).ravel()
        ref = voigt(B) @ D @ voigt(A)
        assert np.isclose(uB @ c.K @ uA, ref, rtol=1e-12, atol=1e-13)
        f = (c.K @ uA).reshape(-1, 3)
        sigma = sym_tensor(D @ voigt(A))
        assert np.allclose(f.T @ X, sigma, atol=1e-12)


def test_mass_conservation_and_linear_fields(cells):
    rng = np.random.default_rng(4)
    for m, c in cells.items():
        X = SLOT_POS[present_slots(m)] * 0.5
        for a in range(3):
            t = np.zeros_like(X)
            t[:, a] = 1.0
            assert np.isclose(t.ravel() @ c.M @ t.ravel(), 1.0, rtol=1e-12)
            assert np.isclose(c.m[a::3].sum(), 1.0, rtol=1e-12)
        assert (c.m > 0).all()
        A = rng.normal(size=(3, 3))
        B = rng.normal(size=(3, 3))
        # int_cube (A x).(B x) dV = tr(A^T B) h^5 / 12
        lhs = (X @ A.T).ravel() @ c.M @ (X @ B.T).ravel()
        assert np.isclose(lhs, np.trace(A.T @ B) / 12.0, rtol=1e-12)
    m8 = cells[slot_mask(0)].m
    assert np.allclose(m8, 1.0 / 8.0, rtol=1e-13)


def test_paper_eigen_formulas_agree():
    """K = Phi_q1 Phi_u1^-1 (eq. K) and m_ij = m0_ij/(s_i+s_j+3) via eigenvectors."""
    for m in (slot_mask(0b000100100110), slot_mask(0b011000001011)):
        E0, E1, E2, M0 = el.coefficient_matrices(m, nu=NU)
        n = E0.shape[0]
        Z = el.hamiltonian(E0, E1, E2)
        w, V = np.linalg.eig(Z)
        sel = np.flatnonzero(w.real < 0)
        assert len(sel) == n
        Pu, Pq = V[:n, sel], V[n:, sel]
        Pu_inv = np.linalg.inv(Pu)
        K = (Pq @ Pu_inv).real
        s = -w[sel] - 0.5
        m0 = Pu.T @ M0 @ Pu
        mm = m0 / (s[:, None] + s[None, :] + 3.0)
        M = (Pu_inv.T @ mm @ Pu_inv).real
        c = el.Cell(m, NU)
        assert np.abs(K - c.K).max() < 1e-9 * np.abs(c.K).max()
        assert np.abs(M - c.M).max() < 1e-9 * np.abs(c.M).max()
        # Hamiltonian pairing of the spectrum (lambda, -lambda)
        assert np.allclose(np.sort(w.real), np.sort(-w.real), atol=1e-8)
        assert np.isclose(np.sort(w.real)[-n:].min(), 0.5, atol=1e-9)   # translations


def test_scaling_laws():
    """eq. KM_scale and eq. tcr_scale: K ~ E h, M ~ rho h^3, dt_cr ~ h sqrt(rho/E)."""
    m = slot_mask(0b000001000011)
    c1 = el.Cell(m, NU)
    h, E, rho = 0.37, 5.0, 2.0
    c2 = el.Cell(m, NU, h=h, E=E, rho=rho)
    assert np.abs(c2.K - E * h * c1.K).max() < 1e-12 * np.abs(c2.K).max()
    assert np.abs(c2.M - rho * h ** 3 * c1.M).max() < 1e-12 * np.abs(c2.M).max()
    assert np.isclose(2 / c2.omega_max, np.sqrt(rho / E) * h * 2 / c1.omega_max, rtol=1e-12)


def _transform_cell(m, Q):
    pos = SLOT_POS[present_slots(m)]
    lut = {tuple(p): i for i, p in enumerate(SLOT_POS.tolist())}
    img = [lut[tuple((Q @ p).tolist())] for p in pos]
    mt = 0
    for s in img:
        if s >= 8:
            mt |= 1 << (s - 8)
    slots_t = present_slots(mt)
    sigma = [slots_t.index(s) for s in img]
    return mt, sigma


def test_orientation_covariance():
    """Direct SBFEM of a transformed cell equals the rotated/mirrored matrices (Sec. 3.2.2)."""
    G = symmetry.all_transforms()
    rng = np.random.default_rng(5)
    for trial in range(10):
        m = slot_mask(int(rng.integers(0, 4096)))
        Q = G[int(rng.integers(0, 48))]
        mt, sigma = _transform_cell(m, Q)
        c, ct = el.Cell(m, NU), el.Cell(mt, NU)
        n = len(sigma)
        R = np.zeros((3 * n, 3 * n))
        for i, j in enumerate(sigma):
            R[3 * j:3 * j + 3, 3 * i:3 * i + 3] = Q
        assert np.abs(R.T @ ct.K @ R - c.K).max() < 1e-11 * np.abs(c.K).max()
        assert np.abs(R.T @ ct.M @ R - c.M).max() < 1e-11 * np.abs(c.M).max()
        P = np.abs(Q)
        for i, j in enumerate(sigma):
            assert np.allclose(P @ c.m[3 * i:3 * i + 3], ct.m[3 * j:3 * j + 3], rtol=1e-11)
        assert np.isclose(c.omega_max, ct.omega_max, rtol=1e-10)


def test_stabiliser_invariance():
    """A pattern is unchanged by every transformation that fixes its mask."""
    G = symmetry.all_transforms()
    m = slot_mask(0b000000000011)
    c = el.Cell(m, NU)
    n = c.n_nodes
    hits = 0
    for Q in G:
        mt, sigma = _transform_cell(m, Q)
        if mt != m:
            continue
        hits += 1
        R = np.zeros((3 * n, 3 * n))
        for i, j in enumerate(sigma):
            R[3 * j:3 * j + 3, 3 * i:3 * i + 3] = Q
        assert np.abs(R.T @ c.K @ R - c.K).max() < 1e-11 * np.abs(c.K).max()
    assert hits >= 2
