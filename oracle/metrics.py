"""Material metrics, bounds and objectives on C^H (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Sec. 5.2 (random structure generation) names: directional Young's moduli
E_k = 1 / (C^-1)_kk, the average normal stiffness C_avg, Hill's bulk and shear
moduli, the universal anisotropy index, the off-diagonal (normal-shear) block
sum, the Hashin-Shtrikman upper bounds and the Voigt bound v E for E_x.
The bulk-modulus / Poisson-ratio objective of the differentiable design step is
defined here in the same terms (Voigt bulk modulus and Hill Poisson ratio).
"""
import numpy as np


def _normal_block_sums(M):
    """(trace of the 3x3 normal block, sum of its off-diagonal entries, trace of
    the shear block).  Written over all entries so that no symmetry is assumed."""
    tr_n = M[0, 0] + M[1, 1] + M[2, 2]
    off_n = M[:3, :3].sum() - tr_n
    tr_s = M[3, 3] + M[4, 4] + M[5, 5]
    return tr_n, off_n, tr_s


def voigt_bulk_shear(C):
    """Voigt averages K_V = (sum_{i,j<=3} C_ij) / 9 and
    G_V = (tr_n - off_n / 2 + 3 tr_s) / 15 of a 6x6 stiffness (engineering shear)."""
    tr_n, off_n, tr_s = _normal_block_sums(C)
    return (tr_n + off_n) / 9.0, (tr_n - 0.5 * off_n + 3.0 * tr_s) / 15.0


def reuss_bulk_shear(C):
    """Reuss averages K_R = 1 / sum_{i,j<=3} S_ij and
    G_R = 15 / (4 tr_n S - 2 off_n S + 3 tr_s S), S = C^-1."""
    tr_n, off_n, tr_s = _normal_block_sums(np.linalg.inv(C))
    return 1.0 / (tr_n + off_n), 15.0 / (4.0 * tr_n - 2.0 * off_n + 3.0 * tr_s)


def hill_bulk_shear(C):
    """Hill's approximation: the mean of the Voigt and Reuss averages."""
    KV, GV = voigt_bulk_shear(C)
    KR, GR = reuss_bulk_shear(C)
    return 0.5 * (KV + KR), 0.5 * (GV + GR)


def poisson_from_bulk_shear(K, G):
    """Isotropic Poisson ratio nu = (3K - 2G) / (2 (3K + G))."""
    return (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G))


def young_moduli(C):
    """Directional Young's moduli E_k = 1 / (C^-1)_kk, k = x, y, z."""
    S = np.linalg.inv(C)
    return 1.0 / np.diag(S)[:3]


def c_avg(C):
    """Average normal stiffness (C11 + C22 + C33) / 3."""
    return (C[0, 0] + C[1, 1] + C[2, 2]) / 3.0


def universal_anisotropy(C):
    """Universal anisotropy index A^U = 5 G_V/G_R + K_V/K_R - 6."""
    KV, GV = voigt_bulk_shear(C)
    KR, GR = reuss_bulk_shear(C)
    return 5.0 * GV / GR + KV / KR - 6.0


def off_diagonal_sum(C):
    """Sum of |C_ij| over the upper-right 3x3 (normal-shear) block."""
    return np.abs(C[:3, 3:]).sum()


def hashin_shtrikman_upper(f1, K1, G1, K2, G2):
    """Two-phase Hashin-Shtrikman upper bounds on the bulk and shear moduli, with
    phase 1 the stiffer phase at volume fraction f1 and phase 2 at 1 - f1."""
    f2 = 1.0 - f1
    # equal phase moduli: the correction term vanishes (1 / (K2 - K1) -> infinity)
    KU = K1 if K2 == K1 else K1 + f2 / (1.0 / (K2 - K1) + 3.0 * f1 / (3.0 * K1 + 4.0 * G1))
    GU = G1 if G2 == G1 else G1 + f2 / (1.0 / (G2 - G1) + 6.0 * f1 * (K1 + 2.0 * G1) /
                                       (5.0 * G1 * (3.0 * K1 + 4.0 * G1)))
    return KU, GU


def bulk_poisson_loss(C, K_target, nu_target, w_K=1.0, w_nu=1.0):
    """Weighted bulk-modulus / Poisson-ratio objective on one C^H:
    w_K (K_V / K_target - 1)^2 + w_nu (nu_H - nu_target)^2, with K_V the Voigt
    bulk modulus and nu_H the Poisson ratio of Hill's K and G."""
    KV, _ = voigt_bulk_shear(C)
    KH, GH = hill_bulk_shear(C)
    nuH = poisson_from_bulk_shear(KH, GH)
    return w_K * (KV / K_target - 1.0) ** 2 + w_nu * (nuH - nu_target) ** 2
