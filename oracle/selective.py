"""Selective (culled) voxel homogenization of Sec. 4.2 (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Sec. 4.2 restricts the cell problems to an active set of voxels,
A = {e | beta_e > eps} with eps = 1e-3 (Sec. 4.2.3: culling removes the
stiffness floor that a dense grid needs), and to the active nodes, the
vertices of at least one active voxel.  Here:

* an active voxel carries K_e = E beta_e K_0 (Sec. 4.1's K_e = beta_e K_0 for
  a solid of modulus E); a culled voxel carries nothing -- no stiffness floor;
* the unknowns are the three displacement components of the active nodes;
  culled nodes hold u = 0 and enter neither K nor f;
* C^H is the energy form of Eq. (8) summed over the active voxels, with |Y|
  the whole cell (n^3 voxels);
* a right-hand side whose norm is at rounding level (at most 1e-12 E sqrt(3 n^3))
  is a zero load with u = 0, as in the dense path;
* the gradient (Eq. (9)) follows the culled model: E_e = E beta_e on an
  active voxel has dE_e/dbeta_e = E, a culled voxel contributes nothing, and
  the jump of a voxel crossing eps is not differentiated.

The restricted K is singular beyond the three rigid translations whenever the
active voxels fall apart into several pieces (every piece floats freely), but
each f^(k) is a sum of element terms K_e chi^k, which are orthogonal to every
rigid motion of every piece, so the system is consistent: Jacobi-PCG from
u = 0 converges to a solution, and C^H does not depend on which one (a rigid
motion of a piece carries no strain energy).  The oracle therefore solves
with the plain Jacobi-PCG of ``solve.py``, without pinning a node.
"""
import numpy as np
import scipy.sparse as sp

from . import adjoint as adj
from . import fem
from . import field as fld
from . import homogenize as hom
from . import solve as slv

EPS_ACTIVE = 1e-3  # Sec. 4.2.3


def active_voxels(beta, eps=EPS_ACTIVE):
    """A = {e | beta_e > eps} as a boolean (n, n, n) grid."""
    return np.asarray(beta, dtype=np.float64) > eps


def active_nodes(act):
    """Nodes incident to at least one active voxel.  Node (i, j, k) is corner
    (ax, ay, az) of voxel (i - ax, j - ay, k - az) (periodic), so it is active
    if any of those eight voxels is."""
    act = np.asarray(act, dtype=bool)
    out = np.zeros_like(act)
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                out |= np.roll(act, shift=(az, ay, ax), axis=(0, 1, 2))
    return out


def culled_moduli(beta, E=1.0, eps=EPS_ACTIVE):
    """E_e = E beta_e on the active voxels, 0 on the culled ones."""
    beta = np.asarray(beta, dtype=np.float64)
    return np.where(active_voxels(beta, eps), E * beta, 0.0)


def active_dofs(node_mask):
    """Global dof indices (3 * node + component) of the active nodes, ascending."""
    nodes = np.flatnonzero(np.asarray(node_mask, dtype=bool).ravel())
    return (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()


def solve_selective(Ec, nu, rtol=1e-12, maxiter=200000):
    """The six cell problems on the active nodes for culled moduli Ec (n,n,n)
    (zero on culled voxels).  Returns (U (3 n^3, 6) with zeros at culled
    nodes, info with iterations, residuals and the active counts)."""
    Ec = np.asarray(Ec, dtype=np.float64)
    n = Ec.shape[0]
    act = Ec > 0.0
    nodes = active_nodes(act)
    idx = active_dofs(nodes)
    K = fem.assemble(Ec, nu, n)
    f = fem.load_vectors(Ec, nu, n)
    Ka = K[idx][:, idx].tocsr()
    fa = f[idx].copy()
    # a load that is zero up to rounding (||f|| <= 1e-12 E sqrt(3 n^3), E the
    # largest modulus) is a zero load, u = 0: e.g. in-plane strains of free
    # plates, whose element forces cancel exactly.  Rounding is not orthogonal
    # to the floating pieces' rigid motions, so CG must not chase it.
    emax = float(Ec.max()) if Ec.size else 0.0
    zero = np.linalg.norm(fa, axis=0) <= 1e-12 * emax * np.sqrt(3.0 * n ** 3)
    fa[:, zero] = 0.0
    U = np.zeros((3 * n ** 3, 6))
    if idx.size:
        Ua, iters, res = slv.pcg_jacobi(Ka, fa, rtol=rtol, maxiter=maxiter)
        U[idx] = Ua
    else:
        iters, res = np.zeros(6, dtype=np.int64), np.zeros(6)
    return U, {"iters": iters, "rel_res": res, "n_active_voxels": int(act.sum()),
               "n_active_nodes": int(nodes.sum()), "active_node_mask": nodes}


def homogenize_selective_stiffness(Ec, nu, rtol=1e-12, maxiter=200000):
    """C^H (Eq. (8)) of culled moduli Ec: the solve on the active nodes, then
    the energy form over the voxels (culled ones contribute zero)."""
    Ec = np.asarray(Ec, dtype=np.float64)
    n = Ec.shape[0]
    U, info = solve_selective(Ec, nu, rtol=rtol, maxiter=maxiter)
    C = hom.energy_tensor(Ec, U, nu, n)
    info["U"] = U
    return C, info


def homogenize_design_selective(pos, q, n, *, K=3, alpha=None, iso=0.0, thickness=None,
                                target_vf=None, kappa=0.0, dist_mode=0, E=1.0, nu=0.3,
                                eps=EPS_ACTIVE, rtol=1e-12, maxiter=200000):
    """The forward path with the selective solve: field (Eq. (6)) -> distance
    (Eq. (7)) -> t (given, or for target_vf over all voxels, as in the dense
    path) -> beta -> culled moduli -> solve on the active nodes -> C^H."""
    F, G = fld.field_and_gradient(pos, q, n, K=K, alpha=alpha)
    d = fld.distance(F, G, iso=iso, dist_mode=dist_mode)
    if thickness is None or thickness < 0:
        thickness = fld.thickness_for_volume(d, target_vf, kappa)
    beta = fld.occupancy(d, thickness, kappa)
    Ec = culled_moduli(beta, E, eps)
    C, info = homogenize_selective_stiffness(Ec, nu, rtol=rtol, maxiter=maxiter)
    info.update({"t": thickness, "beta": beta, "V": beta.mean(), "Ec": Ec})
    return C, info


def components(node_mask, Ec):
    """Connected pieces of the active nodes (two nodes are joined when they
    share an active voxel): (count, label per active node in ascending node
    order).  Used by the tests to pin one node per piece for a direct solve."""
    from scipy.sparse.csgraph import connected_components
    n = Ec.shape[0]
    act = (np.asarray(Ec) > 0.0).ravel()
    dofs = fem.element_dofs(n)[act][:, ::3] // 3          # (n_act, 8) node ids
    nodes = np.flatnonzero(np.asarray(node_mask).ravel())
    where = -np.ones(n ** 3, dtype=np.int64)
    where[nodes] = np.arange(nodes.size)
    loc = where[dofs]
    rows = np.repeat(loc[:, :1], 7, axis=1).ravel()
    cols = loc[:, 1:].ravel()
    g = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(nodes.size, nodes.size))
    return connected_components(g, directed=False)


def design_gradient_selective(pos, q, n, dL_dC, dL_dV, *, thickness, kappa, K=3, alpha=None, iso=0.0,
                              dist_mode=0, E=1.0, nu=0.3, eps=EPS_ACTIVE, rtol=1e-13):
    """Eq. (9) through the culled system for a logistic shell (kappa > 0)
    with t given: returns (C^H, V, dL/dpos (N, 3), dL/dq (N,)) for the
    upstream gradients dL/dC (6x6) and dL/dV.  The element weights
    s_e = dL/dC : dC/dE_e come from the culled solution (zero on culled
    voxels), then the chain of the dense path with dE_e/dbeta_e = E."""
    F, G = fld.field_and_gradient(pos, q, n, K=K, alpha=alpha)
    d = fld.distance(F, G, iso=iso, dist_mode=dist_mode)
    beta = fld.occupancy(d, thickness, kappa)
    Ec = culled_moduli(beta, E, eps)
    C, info = homogenize_selective_stiffness(Ec, nu, rtol=rtol)
    s_e = adj.element_energy_weights(Ec, info["U"], nu, n, dL_dC) * (Ec > 0.0)
    gF, gG = adj.voxel_sensitivities(F, G, d, beta, thickness, kappa, E, 0.0, s_e, dL_dV, iso=iso,
                                     dist_mode=dist_mode)
    dpos, dq = adj.charge_gradients(gF, gG, pos, q, n, K=K, alpha=alpha)
    return C, float(beta.mean()), dpos, dq
