"""Host logic of the inverse-design pipeline (Sec. 4.3, Sec. 5.4): the six
objectives against the oracle's metric definitions, and the CMA-ES
optimizer on functions with known minima.  No GPU."""
import numpy as np
import pytest
import torch

from oracle import metrics
from paper_2511_04025_amd import inverse as inv


def _random_spd(rng):
    A = rng.standard_normal((6, 6))
    return A @ A.T + 6.0 * np.eye(6)


def test_objectives_match_the_metric_definitions():
    rng = np.random.default_rng(0)
    for _ in range(5):
        C = _random_spd(rng)
        V = float(rng.uniform(0.05, 0.3))
        Ct = torch.tensor(C[None])
        Vt = torch.tensor([V], dtype=torch.float64)
        KH, GH = metrics.hill_bulk_shear(C)
        Ex = metrics.young_moduli(C)[0]
        assert np.isclose(float(inv.objective("ex")(Ct, Vt)), -Ex / V, rtol=1e-11)
        assert np.isclose(float(inv.objective("cavg")(Ct, Vt)), -metrics.c_avg(C) / V, rtol=1e-11)
        assert np.isclose(float(inv.objective("keff")(Ct, Vt)), -KH / V, rtol=1e-11)
        assert np.isclose(float(inv.objective("geff")(Ct, Vt)), -GH / V, rtol=1e-11)
        assert np.isclose(float(inv.objective("offdiag")(Ct, Vt)), -metrics.off_diagonal_sum(C), rtol=1e-11)
        f = inv.objective("force", k=3, target=0.25)
        assert np.isclose(float(f(Ct, Vt)), abs(C[3, 3] - 0.25), rtol=1e-11)


def test_objectives_are_differentiable():
    # gradients through torch agree with central differences
    rng = np.random.default_rng(1)
    C = _random_spd(rng)
    for name in ("ex", "keff", "geff"):
        f = inv.objective(name)
        Ct = torch.tensor(C[None], requires_grad=True)
        f(Ct, torch.tensor([0.2], dtype=torch.float64)).sum().backward()
        g = Ct.grad.numpy()[0]
        h = 1e-6
        for (i, j) in ((0, 0), (1, 2), (4, 4)):
            Cp, Cm = C.copy(), C.copy()
            Cp[i, j] += h
            Cm[i, j] -= h
            fd = (float(f(torch.tensor(Cp[None]), torch.tensor([0.2], dtype=torch.float64)))
                  - float(f(torch.tensor(Cm[None]), torch.tensor([0.2], dtype=torch.float64)))) / (2 * h)
            assert abs(fd - g[i, j]) < 1e-6 * max(1.0, abs(fd)), (name, i, j, fd, g[i, j])


def _run(es, f, gens):
    for _ in range(gens):
        X = es.ask()
        es.tell(X, [f(x) for x in X])
    return es


def test_cmaes_converges_on_a_sphere():
    es = _run(inv.CMAES(np.full(8, 3.0), 1.0, seed=3), lambda x: float(np.sum(x * x)), 250)
    assert np.sum(es.m ** 2) < 1e-12


def test_cmaes_learns_an_ill_conditioned_ellipsoid():
    # condition number 1e6: needs the covariance adaptation, not only the step size
    d = 6
    scale = 10.0 ** (3.0 * np.arange(d) / (d - 1))
    f = lambda x: float(np.sum((scale * x) ** 2))
    es = _run(inv.CMAES(np.ones(d), 0.5, seed=4), f, 600)
    assert f(es.m) < 1e-10
    # the learned covariance lines up with the inverse Hessian's axes
    ev = np.sort(np.linalg.eigvalsh(es.C))
    assert ev[-1] / ev[0] > 1e4


def test_cmaes_on_rosenbrock():
    f = lambda x: float(np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1.0 - x[:-1]) ** 2))
    es = _run(inv.CMAES(np.zeros(4), 0.5, seed=5), f, 800)
    assert np.max(np.abs(es.m - 1.0)) < 1e-5


def test_cmaes_is_deterministic_and_sizes_its_population():
    a = inv.CMAES(np.zeros(12), 0.3, seed=7)
    b = inv.CMAES(np.zeros(12), 0.3, seed=7)
    assert a.lam == 4 + int(3 * np.log(12)) and a.mu == a.lam // 2
    assert np.isclose(a.w.sum(), 1.0) and np.all(np.diff(a.w) < 0)
    Xa, Xb = a.ask(), b.ask()
    assert np.array_equal(Xa, Xb)
    fa = np.sum(Xa ** 2, axis=1)
    a.tell(Xa, fa)
    b.tell(Xb, fa)
    assert np.array_equal(a.m, b.m) and a.sigma == b.sigma
