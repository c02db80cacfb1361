"""Shared helpers of the GPU tests: layout conversion between the oracle's
(3 n^3, 6) dof vectors and the library's (6, 3, n, n, n) nodal fields, and the
per-entry C^H comparison rule."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


def oracle_to_nodal(U, n):
    """(3 n^3, 6) with dof 3 * node + c  ->  (6, 3, n, n, n)."""
    return np.ascontiguousarray(U.reshape(n ** 3, 3, 6).transpose(2, 1, 0).reshape(6, 3, n, n, n))


def nodal_to_oracle(u, n):
    return np.ascontiguousarray(np.asarray(u).reshape(6, 3, n ** 3).transpose(2, 1, 0).reshape(3 * n ** 3, 6))


def ch_errors(C, Cref):
    """Per-entry error rule: relative error for |Cref_ij| >= 1e-3 max|Cref|,
    else absolute error scaled by max|Cref|.  Returns (max rel, max small-abs,
    relative Frobenius error)."""
    s = np.abs(Cref).max()
    big = np.abs(Cref) >= 1e-3 * s
    rel = np.max(np.abs(C - Cref)[big] / np.abs(Cref)[big]) if big.any() else 0.0
    small = np.max(np.abs(C - Cref)[~big]) / s if (~big).any() else 0.0
    frob = np.linalg.norm(C - Cref) / np.linalg.norm(Cref)
    return rel, small, frob


def assert_ch_close(C, Cref, rel_tol, abs_tol=None):
    if abs_tol is None:
        abs_tol = rel_tol * 1e-3
    rel, small, frob = ch_errors(C, Cref)
    assert rel <= rel_tol and small <= abs_tol, (rel, small, frob)
    return rel, small, frob
