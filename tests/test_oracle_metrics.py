"""Pins of the oracle's material metrics: an isotropic tensor must give back its
own moduli, a cubic tensor the textbook Voigt/Reuss shear averages, and the
Hashin-Shtrikman bounds their limits, Walpole's form, Hill's equal-shear result
and the porous closed form."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("f1", [0.13, 0.4, 0.77])
def test_hashin_shtrikman_walpole_form(f1):
    """The upper bounds in Walpole's harmonic-mean form: with the stiffer phase's
    K1, G1, K* = [sum_i f_i / (K_i + 4 G1 / 3)]^-1 - 4 G1 / 3 and
    G* = [sum_i f_i / (G_i + z)]^-1 - z, z = G1 (9 K1 + 8 G1) / (6 (K1 + 2 G1)).
    A different algebraic arrangement of the same bound, so a wrong coefficient
    in either form shows up at interior volume fractions."""
    for (K1, G1, K2, G2) in ((5.0, 3.0, 1.0, 0.5), (0.833, 0.385, 0.02, 0.011), (2.0, 0.7, 1.9, 0.69)):
        f2 = 1.0 - f1
        a = 4.0 * G1 / 3.0
        k_ref = 1.0 / (f1 / (K1 + a) + f2 / (K2 + a)) - a
        z = G1 * (9.0 * K1 + 8.0 * G1) / (6.0 * (K1 + 2.0 * G1))
        g_ref = 1.0 / (f1 / (G1 + z) + f2 / (G2 + z)) - z
        ku, gu = metrics.hashin_shtrikman_upper(f1, K1, G1, K2, G2)
        assert abs(ku - k_ref) <= 1e-13 * K1
        assert abs(gu - g_ref) <= 1e-13 * G1


def test_hashin_shtrikman_equal_shear_and_porous():
    """Hill's exact result: for equal shear moduli every composite has
    K = [f1 / (K1 + 4G/3) + f2 / (K2 + 4G/3)]^-1 - 4G/3, so the upper bound
    equals it.  With a void phase the bulk bound reduces to the porous closed
    form 4 K1 G1 f1 / (3 K1 f2 + 4 G1)."""
    K1, K2, G = 3.0, 0.8, 1.1
    for f1 in (0.2, 0.5, 0.9):
        exact = 1.0 / (f1 / (K1 + 4 * G / 3) + (1 - f1) / (K2 + 4 * G / 3)) - 4 * G / 3
        ku, _ = metrics.hashin_shtrikman_upper(f1, K1, G, K2, G)
        assert abs(ku - exact) <= 1e-13
    K1, G1 = 0.8333333333333334, 0.38461538461538464
    for f1 in (0.05, 0.1, 0.3):
        ku, _ = metrics.hashin_shtrikman_upper(f1, K1, G1, 0.0, 0.0)
        assert abs(ku - 4 * K1 * G1 * f1 / (3 * K1 * (1 - f1) + 4 * G1)) <= 1e-14
