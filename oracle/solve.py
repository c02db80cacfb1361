"""Linear solves of the six periodic cell problems K u^(k) = f^(k) (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The periodic stiffness matrix is singular (three rigid translations).  Like the
coarsest level of the paper's solver (Sec. 4.2, Fig. "Active voxels across
multigrid levels": one node carries a Dirichlet constraint to remove the null
space), the oracle fixes the three dofs of node 0; C^H is unchanged by that
choice because a rigid translation carries no strain.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def pin_node0(K, f):
    """Replace the rows and columns of dofs 0, 1, 2 by the identity and zero
    their right-hand side: u at node 0 is fixed to zero."""
    ndof = K.shape[0]
    keep = np.ones(ndof)
    keep[:3] = 0.0
    P = sp.diags(keep)
    Kp = (P @ K @ P + sp.diags(1.0 - keep)).tocsr()
    fp = f.copy()
    fp[:3] = 0.0
    return Kp, fp


def pcg_jacobi(K, f, rtol=1e-12, maxiter=200000):
    """Jacobi-preconditioned CG, run independently on each column of f.

    Stops a column when ||r||_2 <= rtol ||f||_2 (a zero right-hand side stops at
    once with u = 0).  Returns (u, iterations per column, true relative
    residual per column).
    """
    f = np.asarray(f, dtype=np.float64)
    nrhs = f.shape[1]
    dinv = 1.0 / K.diagonal()
    u = np.zeros_like(f)
    r = f.copy()
    fnorm = np.linalg.norm(f, axis=0)
    z = dinv[:, None] * r
    p = z.copy()
    rho = np.einsum("ij,ij->j", r, z)
    active = fnorm > 0
    iters = np.zeros(nrhs, dtype=np.int64)
    for _ in range(maxiter):
        rn = np.linalg.norm(r, axis=0)
        active &= rn > rtol * fnorm
        if not active.any():
            break
        # finished columns keep their state: their step lengths are set to zero
        q = K @ p
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        u += alpha * p
        r -= alpha * q
        z = dinv[:, None] * r
        rho_new = np.einsum("ij,ij->j", r, z)
        beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        p = np.where(active, z + beta * p, p)
        rho = np.where(active, rho_new, rho)
        iters += active
    true_res = np.linalg.norm(f - K @ u, axis=0) / np.where(fnorm > 0, fnorm, 1.0)
    return u, iters, true_res


def direct_solve(K, f):
    """Sparse LU (SuperLU) solve of each column: the cross-check for pcg_jacobi."""
    lu = spla.splu(K.tocsc())
    return lu.solve(np.asarray(f, dtype=np.float64))
