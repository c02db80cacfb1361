"""Host logic of the surface fit (Sec. 5.3): the target surfaces' gradients
against central differences, and the samplers' contracts (points on the
surface to 1e-12, off-surface points at least the requested distance away
to first order).  No GPU."""
import numpy as np
import pytest

from paper_2511_04025_amd import tpms


@pytest.mark.parametrize("name", ["P", "G", "D"])
def test_target_gradients_match_differences(name):
    f = tpms.TARGETS[name]
    x = np.random.default_rng(0).random((50, 3))
    _, g = f(x)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (f(x + e)[0] - f(x - e)[0]) / (2 * h)
        assert np.max(np.abs(fd - g[:, d])) < 1e-7 * np.abs(g).max()


def test_schwarz_p_is_the_charge_series_leading_term():
    # the +1 / -1 charge pair at the cell corner and center: the single-axis
    # modes of Eq. (6) sum to (cos 2 pi x + cos 2 pi y + cos 2 pi z) / 2 (the
    # P surface); the mode (1, 1, 1) adds (2/3) cos cos cos
    from oracle import field as fld
    x = np.random.default_rng(1).random((40, 3))
    pos, q = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]), np.array([1.0, -1.0])
    alpha = np.zeros((2, 2, 2))
    alpha[1, 0, 0] = alpha[0, 1, 0] = alpha[0, 0, 1] = 1.0
    F = fld.field_at_points(x, pos, q, K=1, alpha=alpha)
    assert np.max(np.abs(F - 0.5 * tpms.schwarz_p(x)[0])) < 1e-13
    F1 = fld.field_at_points(x, pos, q, K=1)
    c = np.cos(2 * np.pi * x)
    assert np.max(np.abs(F1 - 0.5 * tpms.schwarz_p(x)[0] - (2 / 3) * c.prod(axis=1))) < 1e-13


@pytest.mark.parametrize("name", ["P", "G", "D"])
def test_samplers(name):
    f = tpms.TARGETS[name]
    on = tpms.sample_surface(f, 300, seed=2)
    assert on.shape == (300, 3) and np.all((on >= 0) & (on < 1))
    assert np.max(np.abs(f(on)[0])) <= 1e-12
    off = tpms.sample_off_surface(f, 300, dist=0.05, seed=3)
    phi, g = f(off)
    assert np.min(np.abs(phi) / np.linalg.norm(g, axis=1)) >= 0.05
