"""Pins of the oracle's material metrics: an isotropic tensor must give back its
own moduli, and a cubic tensor the textbook Voigt/Reuss shear averages."""
import numpy as np

from oracle import fem, metrics


def test_isotropic_metrics():
    E, nu = 2.0, 0.27
    D = fem.isotropic_D(E, nu)
    lam, mu = fem.lame(E, nu)
    K = lam + 2.0 * mu / 3.0
    for f in (metrics.voigt_bulk_shear, metrics.reuss_bulk_shear, metrics.hill_bulk_shear):
        k, g = f(D)
        assert abs(k - K) < 1e-14 and abs(g - mu) < 1e-14
    assert abs(metrics.poisson_from_bulk_shear(K, mu) - nu) < 1e-14
    assert np.max(np.abs(metrics.young_moduli(D) - E)) < 1e-14
    assert abs(metrics.universal_anisotropy(D)) < 1e-13
    assert metrics.off_diagonal_sum(D) == 0.0
    assert abs(metrics.c_avg(D) - (lam + 2 * mu)) < 1e-15


def test_cubic_shear_averages():
    c11, c12, c44 = 3.0, 1.2, 0.5
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    for i in range(3):
        C[i, i] = c11
        C[i + 3, i + 3] = c44
    kv, gv = metrics.voigt_bulk_shear(C)
    kr, gr = metrics.reuss_bulk_shear(C)
    assert abs(kv - (c11 + 2 * c12) / 3) < 1e-14 and abs(kr - kv) < 1e-14
    assert abs(gv - (c11 - c12 + 3 * c44) / 5) < 1e-14
    assert abs(gr - 5 * (c11 - c12) * c44 / (4 * c44 + 3 * (c11 - c12))) < 1e-14
    A = 2 * c44 / (c11 - c12)
    # for cubic symmetry A^U = 6/5 (sqrt(A) - 1/sqrt(A))^2
    assert abs(metrics.universal_anisotropy(C) - 1.2 * (np.sqrt(A) - 1 / np.sqrt(A)) ** 2) < 1e-13


def test_hashin_shtrikman_limits():
    K1, G1, K2, G2 = 5.0, 3.0, 1.0, 0.5
    assert np.allclose(metrics.hashin_shtrikman_upper(1.0, K1, G1, K2, G2), (K1, G1))
    assert np.allclose(metrics.hashin_shtrikman_upper(0.0, K1, G1, K2, G2), (K2, G2))
    ku, gu = metrics.hashin_shtrikman_upper(0.4, K1, G1, K2, G2)
    assert 0.4 * K1 + 0.6 * K2 >= ku >= 1 / (0.4 / K1 + 0.6 / K2)
