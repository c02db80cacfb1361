"""Voxel finite elements for periodic linear elasticity (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Sec. 4.1 (K_e = beta_e K_0, one shared element matrix for a fully
solid voxel) and Eq. (8) (six unit-strain load cases, test displacements
chi^k, periodic system K u^(k) = f^(k), energy form of C^H).

Conventions (pinned by tests):
* Voigt order (11, 22, 33, 23, 13, 12) with engineering shear strains.
* Element corners a = (ax, ay, az) in {0,1}^3, local corner index
  ax + 2 ay + 4 az; element dof 3 * corner + component.
* Grid nodes (i, j, k), 0 <= i, j, k < n, global node (k n + j) n + i, global
  dof 3 * node + component.  Element (i, j, k) joins nodes
  ((i + ax) mod n, (j + ay) mod n, (k + az) mod n) -- periodic wrap.
* Everything is in unit-element coordinates (element edge 1, cell volume n^3);
  the element matrix of edge h is h K_0, so C^H needs no rescaling.
"""
import numpy as np
import scipy.sparse as sp


def lame(E, nu):
    """Lame parameters (lambda, mu) of an isotropic material."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic_D(E, nu):
    """6x6 isotropic elasticity matrix in Voigt (11,22,33,23,13,12), engineering shear."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] = lam + 2.0 * mu
    for i in range(3, 6):
        D[i, i] = mu
    return D


CORNERS = np.array([(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)], dtype=np.int64)


def _shape_gradients(xi):
    """Gradients of the 8 trilinear shape functions N_a(x) = prod_d phi_{a_d}(x_d),
    phi_0(s) = 1 - s, phi_1(s) = s, at a point xi of the unit cube. Shape (8, 3)."""
    g = np.zeros((8, 3))
    for a, (ax, ay, az) in enumerate(CORNERS):
        phi = [xi[d] if c else 1.0 - xi[d] for d, c in enumerate((ax, ay, az))]
        dphi = [1.0 if c else -1.0 for c in (ax, ay, az)]
        g[a, 0] = dphi[0] * phi[1] * phi[2]
        g[a, 1] = phi[0] * dphi[1] * phi[2]
        g[a, 2] = phi[0] * phi[1] * dphi[2]
    return g


def strain_displacement(xi):
    """B (6 x 24) with engineering shear: strain = B u_e at point xi."""
    g = _shape_gradients(xi)
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = g[a]
        B[0, 3 * a + 0] = gx
        B[1, 3 * a + 1] = gy
        B[2, 3 * a + 2] = gz
        B[3, 3 * a + 1] = gz
        B[3, 3 * a + 2] = gy
        B[4, 3 * a + 0] = gz
        B[4, 3 * a + 2] = gx
        B[5, 3 * a + 0] = gy
        B[5, 3 * a + 1] = gx
    return B


def element_stiffness(nu, E=1.0):
    """K_0: stiffness of a fully solid unit-cube voxel, int B^T D B over the cube
    by 2x2x2 Gauss-Legendre quadrature (exact for the trilinear element)."""
    D = isotropic_D(E, nu)
    pts = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    K0 = np.zeros((24, 24))
    for x in pts:
        for y in pts:
            for z in pts:
                B = strain_displacement((x, y, z))
                K0 += 0.125 * (B.T @ D @ B)
    return K0


def unit_strains():
    """The six symmetric unit strain tensors of Voigt (11,22,33,23,13,12);
    a unit engineering shear puts 1/2 in each off-diagonal slot."""
    eps = np.zeros((6, 3, 3))
    eps[0, 0, 0] = eps[1, 1, 1] = eps[2, 2, 2] = 1.0
    for k, (i, j) in zip((3, 4, 5), ((1, 2), (0, 2), (0, 1))):
        eps[k, i, j] = eps[k, j, i] = 0.5
    return eps


def test_displacements():
    """chi^k (24 x 6): corner a of the unit element displaced by eps^k a (Eq. (8))."""
    eps = unit_strains()
    chi = np.zeros((24, 6))
    for k in range(6):
        for a, corner in enumerate(CORNERS):
            chi[3 * a:3 * a + 3, k] = eps[k] @ corner
    return chi


def element_dofs(n):
    """Global dof indices (n^3, 24) of every element, periodic wrap, element
    index (k n + j) n + i."""
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    kk = kk.ravel()
    dofs = np.zeros((n ** 3, 24), dtype=np.int64)
    for a, (ax, ay, az) in enumerate(CORNERS):
        node = (((kk + az) % n) * n + (jj + ay) % n) * n + (ii + ax) % n
        for c in range(3):
            dofs[:, 3 * a + c] = 3 * node + c
    return dofs


def assemble(Ee, nu, n):
    """Periodic global stiffness K = sum_e E_e P_e^T K_0 P_e as a CSR matrix."""
    K0 = element_stiffness(nu)
    dofs = element_dofs(n)
    e = np.asarray(Ee, dtype=np.float64).ravel()
    ndof = 3 * n ** 3
    rows = np.repeat(dofs, 24, axis=1).ravel()
    cols = np.tile(dofs, (1, 24)).ravel()
    vals = (e[:, None] * K0.ravel()[None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def load_vectors(Ee, nu, n):
    """f^(k) = - sum_e E_e P_e^T K_0 chi^k for the six load cases, shape (3 n^3, 6)."""
    K0 = element_stiffness(nu)
    chi = test_displacements()
    dofs = element_dofs(n)
    e = np.asarray(Ee, dtype=np.float64).ravel()
    g = K0 @ chi  # (24, 6)
    f = np.zeros((3 * n ** 3, 6))
    for k in range(6):
        np.add.at(f[:, k], dofs.ravel(), -(e[:, None] * g[None, :, k]).ravel())
    return f


def stiffness_rows(Ee, nu, n, u_at, nodes):
    """Rows of K u at selected nodes, straight from K = sum_e E_e P_e^T K_0 P_e
    (Sec. 4.1): node v is corner a of exactly one element per corner a, the
    element (v - a) mod n, which contributes E_e times the three rows of K_0
    for corner a applied to that element's 24 displacements.

    u_at(node_ids) returns the displacements of the given global nodes as an
    array (len, 3, m); nodes are global node ids.  Returns (len(nodes), 3, m).
    For sampling K u on grids too large to assemble."""
    K0 = element_stiffness(nu)
    E = np.asarray(Ee, dtype=np.float64).ravel()
    v = np.asarray(nodes, dtype=np.int64)
    vx, vy, vz = v % n, (v // n) % n, v // (n * n)
    out = None
    for a, (ax, ay, az) in enumerate(CORNERS):
        ex, ey, ez = (vx - ax) % n, (vy - ay) % n, (vz - az) % n
        ue = []
        for bx, by, bz in CORNERS:
            ue.append(u_at((((ez + bz) % n) * n + (ey + by) % n) * n + (ex + bx) % n))
        ue = np.concatenate(ue, axis=1)  # (len, 24, m), dof 3 * corner + component
        part = E[(ez * n + ey) * n + ex][:, None, None] * np.einsum("ij,pjm->pim", K0[3 * a:3 * a + 3], ue)
        out = part if out is None else out + part
    return out
