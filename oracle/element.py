"""SBFEM cube cell, computed directly in the cell's own (natural) node order.

Follows Sec. 2 of the paper:

* boundary geometry and Jacobian (eqs. xyz_hat, J_bd) with the scaling
  centre at the cube centroid;
* strain operator L = b1 d/dxi + (b2 d/deta + b3 d/dzeta)/xi (eq. L), with
  b1, b2, b3 written out from the inverse of the scaled-boundary Jacobian;
* coefficient matrices E0, E1, E2 (eq. E0E1E2) and M0 assembled over the
  surface elements;
* the bounded solution of the scaled boundary equation (eq. SBFE) through
  the invariant subspace of the eigenvalues with negative real part, and the
  stiffness K = Phi_q1 Phi_u1^-1 (eq. K);
* consistent mass M = Phi_u1^-T m Phi_u1^-1 with the radial integral
  m_ij = int_0^1 xi^si m0_ij xi^sj xi^2 dxi (Sec. 2.2);
* mass lumping by summing same-direction entries of each row (Sec. 3.3).

Readings where the paper is silent (all stated again in the design notes):

* Z, the first-order form of eq. SBFE, is derived here:  with
  Y = [u; E0 xi u' + E1^T u]  and  xi dY/dxi = A Y,
  A = [[-E0^-1 E1^T, E0^-1], [E2 - E1 E0^-1 E1^T, E1 E0^-1 - I]], and
  Z = -(A + I/2) has eigenvalues lambda with u ~ xi^(-lambda-1/2).
  The bounded set is Re(lambda) < 0.
* The exponent in the mass integral is the displacement exponent
  s = -lambda - 1/2, not the eigenvalue itself.
* The eigen-solution is taken in ordered real Schur form (same invariant
  subspace as the eigenvectors, robust to the repeated eigenvalues of
  symmetric cells); the radial mass integral with a non-diagonal exponent
  matrix S is the Sylvester equation (S^T + 3/2) m + m (S + 3/2) = m0, which
  reduces to m_ij = m0_ij / (s_i + s_j + 3) when S is diagonal.
* Face discretisation: a face with no mid-edge node is one quadrilateral;
  with two mid-edge nodes on opposite edges it is two rectangles; otherwise a
  face-centre node is added, every corner flanked by two mid-edge nodes gets
  the quarter square [corner, mid, centre, mid], and every remaining
  boundary segment of the face forms a triangle with the centre.  All
  surface elements are rectangles or isosceles right triangles.
"""

import numpy as np
from scipy import linalg

from meshgen.slots import SLOT_POS, present_slots

# Voigt order: eps = [e_xx, e_yy, e_zz, g_yz, g_xz, g_xy]
L_X = np.zeros((6, 3))
L_Y = np.zeros((6, 3))
L_Z = np.zeros((6, 3))
L_X[0, 0] = 1.0
L_X[4, 2] = 1.0
L_X[5, 1] = 1.0
L_Y[1, 1] = 1.0
L_Y[3, 2] = 1.0
L_Y[5, 0] = 1.0
L_Z[2, 2] = 1.0
L_Z[3, 1] = 1.0
L_Z[4, 0] = 1.0


def elasticity_matrix(E, nu):
    """Isotropic linear elasticity in the Voigt order above."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] += 2.0 * mu
    for i in range(3, 6):
        D[i, i] = mu
    return D


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def quad_rule(n=4):
    """n x n Gauss-Legendre points on [-1,1]^2."""
    x, w = np.polynomial.legendre.leggauss(n)
    pts = np.array([[a, b] for a in x for b in x])
    wts = np.array([wa * wb for wa in w for wb in w])
    return pts, wts


def tri_rule(n=4):
    """Collapsed (Duffy) Gauss rule on the unit triangle eta, zeta >= 0, eta + zeta <= 1."""
    x, w = _gauss01(n)
    pts, wts = [], []
    for a, wa in zip(x, w):
        for b, wb in zip(x, w):
            pts.append([a * (1.0 - b), b])
            wts.append(wa * wb * (1.0 - b))
    return np.array(pts), np.array(wts)


def q4_shape(eta, zeta):
    """Bilinear shape functions, nodes at (-1,-1), (1,-1), (1,1), (-1,1)."""
    en = np.array([-1.0, 1.0, 1.0, -1.0])
    zn = np.array([-1.0, -1.0, 1.0, 1.0])
    N = 0.25 * (1 + eta * en) * (1 + zeta * zn)
    dNe = 0.25 * en * (1 + zeta * zn)
    dNz = 0.25 * (1 + eta * en) * zn
    return N, dNe, dNz


def t3_shape(eta, zeta):
    N = np.array([1.0 - eta - zeta, eta, zeta])
    dNe = np.array([-1.0, 1.0, 0.0])
    dNz = np.array([-1.0, 0.0, 1.0])
    return N, dNe, dNz


def face_subelements(slot_mask):
    """Surface elements of the cell boundary as lists of local node indices.

    Node order inside each element is counter-clockwise seen from outside
    (checked through det J > 0 when the matrices are integrated).
    """
    slots = present_slots(slot_mask)
    local = {tuple(int(v) for v in SLOT_POS[s]): i for i, s in enumerate(slots)}
    subs = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in (-1, 1):
            def pt(pb, pc):
                p = [0, 0, 0]
                p[a], p[b], p[c] = side, pb, pc
                return local.get(tuple(p))
            ring_bc = [(-1, -1), (0, -1), (1, -1), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0)]
            ring = [pt(*q) for q in ring_bc]          # c0 m0 c1 m1 c2 m2 c3 m3
            corners = ring[0::2]
            mids = ring[1::2]
            centre = pt(0, 0)
            present = [m is not None for m in mids]
            nh = sum(present)
            if nh == 0:
                if centre is not None:
                    raise ValueError("face centre without mid-edge nodes")
                subs.append(list(corners))
                continue
            if nh == 2 and present[0] and present[2]:
                if centre is not None:
                    raise ValueError("face centre on a two-opposite face")
                subs.append([corners[0], mids[0], mids[2], corners[3]])
                subs.append([mids[0], corners[1], corners[2], mids[2]])
                continue
            if nh == 2 and present[1] and present[3]:
                if centre is not None:
                    raise ValueError("face centre on a two-opposite face")
                subs.append([corners[0], corners[1], mids[1], mids[3]])
                subs.append([mids[3], mids[1], corners[2], corners[3]])
                continue
            if centre is None:
                raise ValueError("face needs a centre node")
            # corner i sits between mid (i-1) and mid i in ring order
            full = [present[(i - 1) % 4] and present[i] for i in range(4)]
            for i in range(4):
                if full[i]:
                    subs.append([corners[i], mids[i], centre, mids[(i - 1) % 4]])
            # boundary segments of the ring not covered by a corner quad
            pts = [p for p in ring if p is not None]
            for k in range(len(pts)):
                p, q = pts[k], pts[(k + 1) % len(pts)]
                covered = False
                for i in range(4):
                    if full[i] and ((p == corners[i] and q == mids[i]) or
                                    (p == mids[(i - 1) % 4] and q == corners[i])):
                        covered = True
                if not covered:
                    subs.append([p, q, centre])
    return subs


def coefficient_matrices(slot_mask, h=1.0, E=1.0, nu=0.25, rho=1.0, nq=4):
    """E0, E1, E2, M0 of the cell (edge h, centred at the scaling centre)."""
    slots = present_slots(slot_mask)
    X = SLOT_POS[slots].astype(np.float64) * (0.5 * h)
    n = len(slots)
    D = elasticity_matrix(E, nu)
    E0 = np.zeros((3 * n, 3 * n))
    E1 = np.zeros((3 * n, 3 * n))
    E2 = np.zeros((3 * n, 3 * n))
    M0 = np.zeros((3 * n, 3 * n))
    qpts, qw = quad_rule(nq)
    tpts, tw = tri_rule(nq)
    I3 = np.eye(3)
    for sub in face_subelements(slot_mask):
        sub = list(sub)
        shape = q4_shape if len(sub) == 4 else t3_shape
        pts, wts = (qpts, qw) if len(sub) == 4 else (tpts, tw)
        # orientation: outward normal <=> det J > 0 at the element centroid
        cen = (0.0, 0.0) if len(sub) == 4 else (1.0 / 3.0, 1.0 / 3.0)
        N, dNe, dNz = shape(*cen)
        xs = X[sub]
        r, re, rz = N @ xs, dNe @ xs, dNz @ xs
        if r @ np.cross(re, rz) < 0:
            sub = sub[::-1]
            xs = X[sub]
        m = len(sub)
        dofs = np.array([3 * i + k for i in sub for k in range(3)])
        # all quadrature points of this surface element at once
        sh = [shape(eta, zeta) for eta, zeta in pts]
        N = np.array([t[0] for t in sh])            # (g, m)
        dNe = np.array([t[1] for t in sh])
        dNz = np.array([t[2] for t in sh])
        r, re, rz = N @ xs, dNe @ xs, dNz @ xs      # (g, 3)
        g1 = np.cross(re, rz)
        g2 = np.cross(rz, r)
        g3 = np.cross(r, re)
        detJ = np.einsum("gi,gi->g", r, g1)
        if (detJ <= 0).any():
            raise ValueError("non-positive boundary Jacobian")
        Lxyz = np.stack([L_X, L_Y, L_Z])            # (3, 6, 3)
        b1 = np.einsum("gk,kij->gij", g1, Lxyz) / detJ[:, None, None]
        b2 = np.einsum("gk,kij->gij", g2, Lxyz) / detJ[:, None, None]
        b3 = np.einsum("gk,kij->gij", g3, Lxyz) / detJ[:, None, None]
        Nu = np.einsum("ga,ij->giaj", N, I3).reshape(len(pts), 3, 3 * m)
        Nue = np.einsum("ga,ij->giaj", dNe, I3).reshape(len(pts), 3, 3 * m)
        Nuz = np.einsum("ga,ij->giaj", dNz, I3).reshape(len(pts), 3, 3 * m)
        B1 = b1 @ Nu                                 # (g, 6, 3m)
        B2 = b2 @ Nue + b3 @ Nuz
        wd = (wts * detJ)[:, None, None]

        def wsum(Bl, Br):
            # sum over quadrature points of w |J| Bl^T Br, as one matrix product
            return (Bl * wd).transpose(2, 0, 1).reshape(3 * m, -1) @ Br.reshape(-1, 3 * m)
        DB1 = np.matmul(D, B1)
        DB2 = np.matmul(D, B2)
        E0[np.ix_(dofs, dofs)] += wsum(B1, DB1)
        E1[np.ix_(dofs, dofs)] += wsum(B2, DB1)
        E2[np.ix_(dofs, dofs)] += wsum(B2, DB2)
        M0[np.ix_(dofs, dofs)] += rho * wsum(Nu, Nu)
    return E0, E1, E2, M0


def hamiltonian(E0, E1, E2):
    """Z of the first-order form; eigenvalue lambda <-> u ~ xi^(-lambda - 1/2)."""
    n = E0.shape[0]
    E0i = np.linalg.inv(E0)
    I = np.eye(n)
    return np.block([[E0i @ E1.T - 0.5 * I, -E0i],
                     [-E2 + E1 @ E0i @ E1.T, -E1 @ E0i + 0.5 * I]])


def stiffness_and_mass(E0, E1, E2, M0, check=True):
    """K (eq. K) and consistent M from the bounded invariant subspace of Z."""
    n = E0.shape[0]
    Z = hamiltonian(E0, E1, E2)
    T, V, sdim = linalg.schur(Z, output="real", sort="lhp")
    if sdim != n:
        raise RuntimeError(f"bounded subspace has dimension {sdim}, expected {n}")
    Vu, Vq = V[:n, :n], V[n:, :n]
    Vu_inv = np.linalg.inv(Vu)
    K = Vq @ Vu_inv
    if check:
        asym = np.abs(K - K.T).max() / np.abs(K).max()
        if asym > 1e-9:
            raise RuntimeError(f"stiffness not symmetric ({asym:.2e})")
    K = 0.5 * (K + K.T)
    S = -T[:n, :n] - 0.5 * np.eye(n)       # u(xi) = Vu xi^S c
    m0 = Vu.T @ M0 @ Vu
    m = linalg.solve_sylvester(S.T + 1.5 * np.eye(n), S + 1.5 * np.eye(n), m0)
    M = Vu_inv.T @ m @ Vu_inv
    M = 0.5 * (M + M.T)
    return K, M


def lump(M):
    """Sum each row over the columns of the same coordinate direction (Sec. 3.3)."""
    n = M.shape[0]
    d = np.arange(n) % 3
    out = np.zeros(n)
    for a in range(3):
        idx = np.flatnonzero(d == a)
        out[idx] = M[np.ix_(idx, idx)].sum(axis=1)
    return out


def max_frequency(K, m_lumped):
    """omega_max of K phi = omega^2 diag(m) phi."""
    s = 1.0 / np.sqrt(m_lumped)
    A = K * s[:, None] * s[None, :]
    return float(np.sqrt(max(np.linalg.eigvalsh(A).max(), 0.0)))


class Cell:
    """SBFEM matrices of one cell layout (slot mask) at edge h, modulus E, density rho."""

    def __init__(self, slot_mask, nu, h=1.0, E=1.0, rho=1.0):
        self.slot_mask = int(slot_mask)
        E0, E1, E2, M0 = coefficient_matrices(slot_mask, h=h, E=E, nu=nu, rho=rho)
        self.K, self.M = stiffness_and_mass(E0, E1, E2, M0)
        self.m = lump(self.M)
        self.omega_max = max_frequency(self.K, self.m)
        self.n_nodes = len(present_slots(slot_mask))
