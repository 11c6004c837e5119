"""Master-cell stiffness and lumped mass by the SBFEM (Sec. 2, Sec. 3.3), FP64 host code.

For a unit cube (edge 1, E = 1, rho = 1, Poisson ratio nu) centred on its
scaling centre:

1. The boundary is split face by face into 4-node rectangles and 3-node
   isosceles triangles (Fig. OctreeDist); the face-centre node, where present,
   is the apex of every triangle.
2. Coefficient matrices E0, E1, E2 (eq. E0E1E2) and M0 are integrated over
   the surface elements: rectangles with 3x3 Gauss points, triangles with the
   3-point interior rule.  Both are exact here because every surface element
   is planar and affinely mapped, so |J| is constant on it.
3. Writing u(xi) = Phi xi^s c, eq. SBFE becomes the linear eigenproblem
   s [phi; q] = A [phi; q] with q = (s E0 + E1^T) phi the boundary force
   (eq. q_E0E1) and A = [[-E0^-1 E1^T, E0^-1], [E2 - E1 E0^-1 E1^T, E1 E0^-1 - I]].
   Bounded solutions have Re(s) >= 0 (the paper's -lambda - 1/2 exponent);
   their invariant subspace is taken by an ordered real Schur form.
   K = Phi_q Phi_u^-1 (eq. K).
4. Consistent mass M = Phi_u^-T m Phi_u^-1 where m solves
   (S^T + 3/2) m + m (S + 3/2) = Phi_u^T M0 Phi_u, the radial integral
   int_0^1 xi^(S^T) m0 xi^S xi^2 dxi for the block-triangular exponent S
   (elementwise m0_ij / (s_i + s_j + 3) when S is diagonal).
5. Lumping: each diagonal entry becomes the sum of its row over the columns
   of the same coordinate direction (Sec. 3.3).
"""

import numpy as np
from scipy import linalg

from .patterns import POSITIONS, present

_GP3 = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GW3 = np.array([5.0, 8.0, 5.0]) / 9.0
QUAD_PTS = np.array([(a, b) for a in _GP3 for b in _GP3])
QUAD_W = np.array([wa * wb for wa in _GW3 for wb in _GW3])
TRI_PTS = np.array([(1 / 6, 1 / 6), (2 / 3, 1 / 6), (1 / 6, 2 / 3)])
TRI_W = np.full(3, 1 / 6)


def _strain_operator_blocks():
    """Selectors so that eps(Voigt xx,yy,zz,yz,zx,xy) = sum_i Lsel[i] du/dx_i."""
    L = np.zeros((3, 6, 3))
    # d/dx
    L[0, 0, 0] = 1
    L[0, 4, 2] = 1
    L[0, 5, 1] = 1
    # d/dy
    L[1, 1, 1] = 1
    L[1, 3, 2] = 1
    L[1, 5, 0] = 1
    # d/dz
    L[2, 2, 2] = 1
    L[2, 3, 1] = 1
    L[2, 4, 0] = 1
    return L


LSEL = _strain_operator_blocks()


def elastic_matrix(nu, E=1.0):
    mu = E / (2.0 * (1.0 + nu))
    lam = 2.0 * mu * nu / (1.0 - 2.0 * nu)
    D = np.diag([2 * mu] * 3 + [mu] * 3).astype(np.float64)
    D[:3, :3] += lam
    return D


def surface_elements(slot_mask):
    """(quads, tris) as arrays of slot-position triples in counter-clockwise order
    seen from outside the cell."""
    slots = present(slot_mask)
    have = {tuple(POSITIONS[s]) for s in slots}
    quads, tris = [], []
    for axis in range(3):
        for side in (-1, 1):
            # face frame: (t1, t2, n) right-handed with n the outward normal
            n = np.zeros(3, dtype=np.int64)
            n[axis] = side
            t1 = np.zeros(3, dtype=np.int64)
            t1[(axis + 1) % 3] = 1
            t2 = np.cross(n, t1)

            def P(a, b):
                return tuple(int(v) for v in n + a * t1 + b * t2)
            ring = [P(-1, -1), P(0, -1), P(1, -1), P(1, 0), P(1, 1), P(0, 1), P(-1, 1), P(-1, 0)]
            mid_on = [ring[i] in have for i in (1, 3, 5, 7)]
            centre = P(0, 0)
            if not any(mid_on):
                quads.append([ring[0], ring[2], ring[4], ring[6]])
            elif mid_on == [True, False, True, False]:
                quads.append([ring[0], ring[1], ring[5], ring[6]])
                quads.append([ring[1], ring[2], ring[4], ring[5]])
            elif mid_on == [False, True, False, True]:
                quads.append([ring[0], ring[2], ring[3], ring[7]])
                quads.append([ring[7], ring[3], ring[4], ring[6]])
            else:
                assert centre in have, "face needs its centre node"
                used = set()
                for c in (0, 2, 4, 6):
                    before, after = ring[(c - 1) % 8], ring[c + 1]
                    if before in have and after in have:
                        quads.append([ring[c], after, centre, before])
                        used.add((before, ring[c]))
                        used.add((ring[c], after))
                pts = [p for p in ring if p in have]
                for i, p in enumerate(pts):
                    q = pts[(i + 1) % len(pts)]
                    if (p, q) not in used:
                        tris.append([p, q, centre])
    return quads, tris


def _shape_q4(pts):
    xi, et = pts[:, 0:1], pts[:, 1:2]
    sx = np.array([-1, 1, 1, -1.0])
    se = np.array([-1, -1, 1, 1.0])
    N = 0.25 * (1 + xi * sx) * (1 + et * se)
    d1 = 0.25 * sx * (1 + et * se)
    d2 = 0.25 * (1 + xi * sx) * se
    return N, d1, d2


def _shape_t3(pts):
    g = pts.shape[0]
    N = np.stack([1 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)
    d1 = np.tile([-1.0, 1.0, 0.0], (g, 1))
    d2 = np.tile([-1.0, 0.0, 1.0], (g, 1))
    return N, d1, d2


def coefficients(slot_mask, nu):
    """E0, E1, E2, M0 of the unit master cell in its node order (FP64)."""
    slots = present(slot_mask)
    index = {tuple(POSITIONS[s]): i for i, s in enumerate(slots)}
    nd = 3 * len(slots)
    D = elastic_matrix(nu)
    mats = [np.zeros((nd, nd)) for _ in range(4)]
    quads, tris = surface_elements(slot_mask)
    for elems, (N, d1, d2), w in ((quads, _shape_q4(QUAD_PTS), QUAD_W),
                                  (tris, _shape_t3(TRI_PTS), TRI_W)):
        if not elems:
            continue
        nodes = np.array([[index[p] for p in e] for e in elems])             # (ne, m)
        X = 0.5 * np.array([[list(p) for p in e] for e in elems], dtype=np.float64)  # (ne, m, 3)
        r = np.einsum("gm,emk->egk", N, X)
        r1 = np.einsum("gm,emk->egk", d1, X)
        r2 = np.einsum("gm,emk->egk", d2, X)
        # rows of J^-1 scaled by |J|: cofactor vectors of J = [r; r1; r2]
        c1 = np.cross(r1, r2)
        c2 = np.cross(r2, r)
        c3 = np.cross(r, r1)
        jac = np.einsum("egk,egk->eg", r, c1)
        assert (jac > 0).all(), "surface element orientation"
        b1 = np.einsum("egk,kij->egij", c1, LSEL) / jac[..., None, None]
        b2 = np.einsum("egk,kij->egij", c2, LSEL) / jac[..., None, None]
        b3 = np.einsum("egk,kij->egij", c3, LSEL) / jac[..., None, None]
        ne, g, m = len(elems), N.shape[0], N.shape[1]
        eye = np.eye(3)
        Nu = np.einsum("gm,ij->gimj", N, eye).reshape(g, 3, 3 * m)
        Nd1 = np.einsum("gm,ij->gimj", d1, eye).reshape(g, 3, 3 * m)
        Nd2 = np.einsum("gm,ij->gimj", d2, eye).reshape(g, 3, 3 * m)
        B1 = np.einsum("egij,gjq->egiq", b1, Nu)
        B2 = np.einsum("egij,gjq->egiq", b2, Nd1) + np.einsum("egij,gjq->egiq", b3, Nd2)
        wj = w[None, :] * jac
        DB1 = np.einsum("ij,egjq->egiq", D, B1)
        DB2 = np.einsum("ij,egjq->egiq", D, B2)
        e0 = np.einsum("eg,egip,egiq->epq", wj, B1, DB1)
        e1 = np.einsum("eg,egip,egiq->epq", wj, B2, DB1)
        e2 = np.einsum("eg,egip,egiq->epq", wj, B2, DB2)
        m0 = np.einsum("eg,gip,giq->epq", wj, Nu, Nu)
        dofs = (3 * nodes[:, :, None] + np.arange(3)).reshape(ne, 3 * m)
        for target, blk in zip(mats, (e0, e1, e2, m0)):
            for e in range(ne):
                target[np.ix_(dofs[e], dofs[e])] += blk[e]
    return mats


def solve_cell(E0, E1, E2, M0):
    """(K, M) from the bounded solution of the scaled boundary equation."""
    nd = E0.shape[0]
    cho = linalg.cho_factor(E0)
    E0i_E1T = linalg.cho_solve(cho, E1.T)
    E0i = linalg.cho_solve(cho, np.eye(nd))
    A = np.block([[-E0i_E1T, E0i], [E2 - E1 @ E0i_E1T, E1 @ E0i - np.eye(nd)]])
    T, Y, k = linalg.schur(A, output="real", sort=lambda re, im: re > -0.5)
    if k != nd:
        raise RuntimeError(f"bounded subspace of size {k}, expected {nd}")
    Yu, Yq = Y[:nd, :nd], Y[nd:, :nd]
    K = linalg.solve(Yu.T, Yq.T).T
    K = 0.5 * (K + K.T)
    S = T[:nd, :nd]
    I = np.eye(nd)
    mm = linalg.solve_sylvester(S.T + 1.5 * I, S + 1.5 * I, Yu.T @ M0 @ Yu)
    Yi = linalg.inv(Yu)
    M = Yi.T @ mm @ Yi
    return K, 0.5 * (M + M.T)


def lumped(M):
    nd = M.shape[0]
    out = np.empty(nd)
    for i in range(nd):
        out[i] = M[i, i % 3::3].sum()
    return out


def master_cell(slot_mask, nu):
    """K (unit cell), lumped diagonal mass, and the largest circular frequency."""
    K, M = solve_cell(*coefficients(slot_mask, nu))
    m = lumped(M)
    w2 = linalg.eigh(K, np.diag(m), eigvals_only=True)
    return K, m, float(np.sqrt(max(w2.max(), 0.0)))
