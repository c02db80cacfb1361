"""Fundamental bounding volumes as a design input (Sec. 3.2): charges given
in a one-eighth-cell or tetrahedral volume are mirrored over the cell by the
library.  The result equals the design with the images spelled out, carries
the symmetry the group implies (orthotropic / cubic C^H), matches the oracle
on the expanded charges, and the gradient with respect to the given charges
is the fold of the expanded design's gradient."""
import numpy as np
import pytest

from oracle import homogenize as hom
from paper_2511_04025_amd import workloads as wl

pytestmark = pytest.mark.gpu

PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def images(pos, q, sym):
    """The group's images, charge by charge: axes permuted (cubic only), then
    x_d -> 1 - x_d for the bits of g % 8."""
    G = {1: 8, 2: 48}[sym]
    P, Q, maps = [], [], []
    for p, qq in zip(pos, q):
        for g in range(G):
            perm = PERMS[g // 8]
            v = np.array([p[perm[d]] for d in range(3)])
            sgn = np.ones(3)
            for d in range(3):
                if (g >> d) & 1:
                    v[d] = 1.0 - v[d]
                    sgn[d] = -1.0
            P.append(v)
            Q.append(qq)
            maps.append((perm, sgn))
    return np.array(P), np.array(Q), maps


def fbv_design(seed, n, N, sym, kappa=0.0, vf=0.2):
    rng = np.random.default_rng(seed)
    # points in the fundamental volume: 0 <= x <= y <= z <= 1/2 for the cubic group
    pos = 0.5 * rng.random((N, 3))
    if sym == 2:
        pos = np.sort(pos, axis=1)
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    return wl.Design(pos=pos, q=q, n=n, target_vf=vf, E_void=1e-3, kappa=kappa, seed=seed, symmetry=sym)


def _off_orthotropic(C):
    m = np.zeros((6, 6), bool)
    m[:3, 3:] = m[3:, :3] = True
    for i in range(3, 6):
        for j in range(3, 6):
            m[i, j] = i != j
    return np.abs(C[m]).max()


@pytest.mark.parametrize("sym", [1, 2])
def test_fbv_equals_explicit_images_and_has_the_group_symmetry(sym):
    from paper_2511_04025_amd import api
    n = 24
    d = fbv_design(400 + sym, n, 2, sym, kappa=4.0 * n)
    r = api.homogenize(d, precision="fp64", rtol=1e-11)
    P, Q, _ = images(d.pos, d.q, sym)
    e = api.homogenize(d.with_(pos=P, q=Q, symmetry=0), precision="fp64", rtol=1e-11)
    assert r["status"] == 0 and np.array_equal(r["C"], e["C"]) and r["V"] == e["V"]
    C = r["C"]
    s = np.abs(C).max()
    print("fbv", sym, "off-orthotropic", _off_orthotropic(C) / s, flush=True)
    assert _off_orthotropic(C) <= 1e-9 * s
    if sym == 2:
        assert abs(C[0, 0] - C[1, 1]) <= 1e-9 * s and abs(C[0, 0] - C[2, 2]) <= 1e-9 * s
        assert abs(C[0, 1] - C[0, 2]) <= 1e-9 * s and abs(C[3, 3] - C[5, 5]) <= 1e-9 * s


def test_fbv_matches_the_oracle_on_the_expanded_charges():
    from paper_2511_04025_amd import api
    n = 12
    d = fbv_design(410, n, 1, 2, kappa=4.0 * n, vf=0.3)
    r = api.homogenize(d, precision="fp64", rtol=1e-11)
    P, Q, _ = images(d.pos, d.q, 2)
    C, info = hom.homogenize_design(P, Q, n, thickness=r["t"], kappa=d.kappa, E_void=d.E_void, solver="direct")
    assert abs(r["V"] - info["V"]) <= 1e-13
    assert np.max(np.abs(r["C"] - C)) <= 1e-8 * np.abs(C).max()


@pytest.mark.parametrize("sym", [1, 2])
def test_fbv_gradient_is_the_fold_of_the_expanded_gradient(sym):
    from paper_2511_04025_amd import api
    n = 16
    d = fbv_design(420 + sym, n, 2, sym, kappa=4.0 * n).with_(thickness=None)
    r = api.homogenize(d, precision="fp64", rtol=1e-12, save_for_backward=True, return_workspace=True)
    g = np.random.default_rng(5).standard_normal((6, 6))
    gp, gq, ga, gt = api.grad(d, r["opts"], r["workspace"], g, 0.3, full=True)
    P, Q, maps = images(d.pos, d.q, sym)
    de = d.with_(pos=P, q=Q, symmetry=0, thickness=r["t"], target_vf=None)
    re = api.homogenize(de, precision="fp64", rtol=1e-12, save_for_backward=True, return_workspace=True)
    ep, eq, ea, et = api.grad(de, re["opts"], re["workspace"], g, 0.3, full=True)
    G = len(maps) // len(d.q)
    fp = np.zeros_like(d.pos)
    fq = np.zeros_like(d.q)
    for k, (perm, sgn) in enumerate(maps):
        j = k // G
        for dd in range(3):
            fp[j, perm[dd]] += sgn[dd] * ep[k, dd]
        fq[j] += eq[k]
    scale = max(np.abs(fp).max(), np.abs(fq).max())
    assert np.max(np.abs(gp - fp)) <= 1e-9 * scale and np.max(np.abs(gq - fq)) <= 1e-9 * scale
    assert np.max(np.abs(ga - ea)) <= 1e-9 * np.abs(ea).max() and abs(gt - et) <= 1e-9 * abs(et)
