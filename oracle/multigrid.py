"""Coarse grids of the geometric multigrid hierarchy (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Sec. 4.2 builds a 2x2x2 voxel hierarchy with coarse-grid operators formed from
the fine one.  Written here from the plain definitions:

* ``prolongation(nc)``: the periodic trilinear interpolation P from a coarse
  grid of nc^3 nodes to the fine grid of (2 nc)^3 nodes (a fine node halfway
  between coarse nodes takes their mean, per axis), as a sparse matrix on the
  fem module's dof numbering (dof 3 node + component, node (k n + j) n + i).
* ``galerkin(K, n)``: the Galerkin coarse operator P^T K P of an operator on
  the n^3 grid (n even).
"""
import numpy as np
import scipy.sparse as sp


def _prolong_1d(nc):
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for i in range(nf):
        if i % 2 == 0:
            rows.append(i)
            cols.append(i // 2)
            vals.append(1.0)
        else:
            rows += [i, i]
            cols += [(i - 1) // 2, ((i + 1) // 2) % nc]
            vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation(nc):
    """P: coarse nc^3 -> fine (2 nc)^3, dofs 3 node + c, node (k n + j) n + i."""
    P1 = _prolong_1d(nc)
    # node index (k, j, i) with i fastest is the Kronecker order z (x) y (x) x
    P3 = sp.kron(sp.kron(P1, P1), P1, format="csr")
    return sp.kron(P3, sp.identity(3), format="csr")


def galerkin(K, n):
    """P^T K P for K on the n^3 grid."""
    if n % 2:
        raise ValueError("the grid must have an even number of nodes per axis")
    P = prolongation(n // 2)
    return (P.T @ K @ P).tocsr()
