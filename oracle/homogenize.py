"""Homogenized elasticity tensor C^H (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Implements the energy form of Eq. (8):
    C^H_ij = (1/|Y|) sum_e (chi^i + u^(i)_e)^T K_e (chi^j + u^(j)_e),
with K_e = E_e K_0 (Sec. 4.1) and |Y| = n^3 in unit-element coordinates, and the
whole forward path field -> distance -> occupancy -> solve -> C^H.
"""
import time

import numpy as np

from . import fem
from . import field as fld
from . import solve as slv


def element_vectors(U, n):
    """chi^k + u^(k)_e for every element: shape (n^3, 24, 6)."""
    dofs = fem.element_dofs(n)
    chi = fem.test_displacements()
    return U[dofs, :] + chi[None, :, :]


def energy_tensor(Ee, U, nu, n):
    """C^H_ij = (1/n^3) sum_e E_e (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)  (Eq. (8))."""
    K0 = fem.element_stiffness(nu)
    V = element_vectors(U, n)
    W = np.einsum("ab,ebj->eaj", K0, V)
    e = np.asarray(Ee, dtype=np.float64).ravel()
    return np.einsum("e,eai,eaj->ij", e, V, W) / n ** 3


def mixed_form_tensor(Ee, U, nu, n):
    """The alternative form (1/n^3) sum_e E_e chi^i^T K_0 (chi^j + u^j_e); equal to
    the energy form when each u^j is at equilibrium (used as a cross-check)."""
    K0 = fem.element_stiffness(nu)
    chi = fem.test_displacements()
    V = element_vectors(U, n)
    W = np.einsum("ab,ebj->eaj", K0, V)
    e = np.asarray(Ee, dtype=np.float64).ravel()
    return np.einsum("e,ai,eaj->ij", e, chi, W) / n ** 3


def solve_cell(Ee, nu, n, rtol=1e-12, solver="cg", maxiter=200000):
    """Solve the six periodic cell problems for a stiffness field E_e (n,n,n).

    Returns (U (3 n^3, 6), info dict)."""
    t0 = time.perf_counter()
    K = fem.assemble(Ee, nu, n)
    f = fem.load_vectors(Ee, nu, n)
    t1 = time.perf_counter()
    Kp, fp = slv.pin_node0(K, f)
    if solver == "cg":
        U, iters, res = slv.pcg_jacobi(Kp, fp, rtol=rtol, maxiter=maxiter)
    else:
        U = slv.direct_solve(Kp, fp)
        iters = np.zeros(6, dtype=np.int64)
        fn = np.linalg.norm(fp, axis=0)
        res = np.linalg.norm(fp - Kp @ U, axis=0) / np.where(fn > 0, fn, 1.0)
    t2 = time.perf_counter()
    return U, {"iters": iters, "rel_res": res, "t_assemble": t1 - t0, "t_solve": t2 - t1}


def homogenize_stiffness(Ee, nu, rtol=1e-12, solver="cg", maxiter=200000):
    """C^H for a given voxel stiffness field E_e (n,n,n) and Poisson ratio nu."""
    Ee = np.asarray(Ee, dtype=np.float64)
    n = Ee.shape[0]
    U, info = solve_cell(Ee, nu, n, rtol=rtol, solver=solver, maxiter=maxiter)
    t0 = time.perf_counter()
    C = energy_tensor(Ee, U, nu, n)
    info["t_C"] = time.perf_counter() - t0
    info["U"] = U
    return C, info


def homogenize_design(pos, q, n, *, K=3, alpha=None, iso=0.0, thickness=None,
                      target_vf=None, kappa=0.0, dist_mode=0, E=1.0, nu=0.3,
                      E_void=1e-3, rtol=1e-12, solver="cg", maxiter=200000):
    """The whole forward path for one design.

    Field (Eq. (6)) -> distance (Eq. (7)) -> thickness t (given, or chosen for
    target_vf) -> occupancy beta -> E_e = E_void + (E - E_void) beta -> six cell
    problems -> C^H (Eq. (8)).  Returns (C, info) with info holding V = mean beta,
    t, beta, F, G, U, iteration counts and stage times.
    """
    t0 = time.perf_counter()
    F, G = fld.field_and_gradient(pos, q, n, K=K, alpha=alpha)
    d = fld.distance(F, G, iso=iso, dist_mode=dist_mode)
    if thickness is None or thickness < 0:
        thickness = fld.thickness_for_volume(d, target_vf, kappa)
    beta = fld.occupancy(d, thickness, kappa)
    Ee = fld.stiffness_field(beta, E, E_void)
    t1 = time.perf_counter()
    C, info = homogenize_stiffness(Ee, nu, rtol=rtol, solver=solver, maxiter=maxiter)
    info.update({"t_field": t1 - t0, "t": thickness, "beta": beta, "F": F, "G": G,
                 "d": d, "V": beta.mean(), "Ee": Ee})
    return C, info
