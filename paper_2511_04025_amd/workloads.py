"""Seeded synthetic workloads (charges, volume fractions, material) for tests,
the smoke run and the benchmark.

This module only draws inputs: it holds none of the method's arithmetic and is
the one piece shared by the HIP path and the CPU oracle.  Imports nothing from
the rest of the package.

The paper's timing set (86 shells) and random-structure set are not available;
these generators stand in for them with the paper's shapes: uniform charge
positions in the unit cell, +-1 charges in equal numbers (Eq. (6)) or real
magnitudes shifted to zero net charge, K = 3 (Sec. 5), thin shells of a few to
twenty percent solid volume (Table 3 active fractions 9-17%).
"""
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np


@dataclass
class Design:
    """One homogenization request.

    pos: (N, 3) charge positions in [0, 1)^3.   q: (N,) charge values.
    n: voxels per axis.  thickness: shell half-thickness t (cell units) or None
    to choose t for target_vf.  kappa: 0 for the hard step d < t, > 0 for the
    logistic occupancy.  alpha: (K+1)^3 spectral weights or None for all ones.
    """
    pos: np.ndarray
    q: np.ndarray
    n: int
    K: int = 3
    alpha: Optional[np.ndarray] = None
    iso: float = 0.0
    thickness: Optional[float] = None
    target_vf: Optional[float] = None
    kappa: float = 0.0
    dist_mode: int = 0
    E: float = 1.0
    nu: float = 0.3
    E_void: float = 1e-3
    seed: Optional[int] = None
    tag: str = ""
    symmetry: object = 0  # 0/'none', 1/'mirror' (8 images), 2/'cubic' (48 images): pos, q lie in the FBV

    def with_(self, **kw):
        return replace(self, **kw)


def plus_minus_charges(N):
    """q_j = +1 for the first half, -1 for the second (Eq. (6) sign pattern)."""
    return np.concatenate([np.ones(N // 2), -np.ones(N - N // 2)])


def small_shell_24(seed=1):
    """24^3, 16 charges of +-1 at uniform positions, hard shell at V = 0.12,
    E = 1, nu = 0.3, void E = 1e-3 (solved in FP64 to 1e-10)."""
    rng = np.random.default_rng(seed)
    pos = rng.random((16, 3))
    return Design(pos=pos, q=plus_minus_charges(16), n=24, target_vf=0.12,
                  E_void=1e-3, seed=seed, tag="c1")


def shell_128(seed, n=128):
    """128^3 (or n^3), 48 charges with magnitudes U[-1, 1] shifted to zero net
    charge, volume fraction U[0.05, 0.15], void E = 1e-6."""
    rng = np.random.default_rng(seed)
    pos = rng.random((48, 3))
    q = rng.uniform(-1.0, 1.0, 48)
    q = q - q.mean()
    vf = rng.uniform(0.05, 0.15)
    return Design(pos=pos, q=q, n=n, target_vf=float(vf), E_void=1e-6, seed=seed, tag="c2")


def shell_128_designs(n=128, count=8):
    return [shell_128(2000 + i, n=n) for i in range(count)]


def large_shell_256(seed=3000, n=256):
    """256^3, 64 charges of +-1, volume fraction 0.05, void E = 1e-6."""
    rng = np.random.default_rng(seed)
    pos = rng.random((64, 3))
    return Design(pos=pos, q=plus_minus_charges(64), n=n, target_vf=0.05,
                  E_void=1e-6, seed=seed, tag="c3")


def serving_trace(count=512, seed=4000, resolutions=(64, 96, 128)):
    """Serving trace: resolution uniform over `resolutions`, charge count
    U{16..64}, magnitudes as shell_128, volume fraction U[0.03, 0.2], void
    E = 1e-6.  Arrival times are drawn separately (poisson_arrivals)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(resolutions))
        N = int(rng.integers(16, 65))
        pos = rng.random((N, 3))
        q = rng.uniform(-1.0, 1.0, N)
        q = q - q.mean()
        vf = float(rng.uniform(0.03, 0.2))
        out.append(Design(pos=pos, q=q, n=n, target_vf=vf, E_void=1e-6, seed=seed * 1000 + i, tag="c4"))
    return out


def poisson_arrivals(count, rate, seed=4001):
    """Arrival times (s) of a Poisson process of the given rate (requests/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def smooth_shell_96(seed, n=96):
    """Differentiable design step: 32 charges of +-1, logistic occupancy whose
    transition spans one voxel (kappa = 4 n, see the transition-width reading),
    void E = 1e-6; t is set from V = 0.10 at the initial design."""
    rng = np.random.default_rng(seed)
    pos = rng.random((32, 3))
    return Design(pos=pos, q=plus_minus_charges(32), n=n, target_vf=0.10,
                  kappa=4.0 * n, E_void=1e-6, seed=seed, tag="c5")


def smooth_shell_96_batch(n=96, count=32):
    return [smooth_shell_96(5000 + i, n=n) for i in range(count)]


def random_design(seed, n, N=16, vf=0.12, E_void=1e-3, kappa=0.0, pm=True):
    """A small generic design for unit tests."""
    rng = np.random.default_rng(seed)
    pos = rng.random((N, 3))
    if pm:
        q = plus_minus_charges(N)
    else:
        q = rng.uniform(-1.0, 1.0, N)
        q = q - q.mean()
    return Design(pos=pos, q=q, n=n, target_vf=vf, E_void=E_void, kappa=kappa, seed=seed, tag="rand")


def octahedral_orbit(points, q, tol=1e-12):
    """Images of each charge under the 48 symmetries of the cube about the cell
    center (reflections x -> 1 - x per axis and axis permutations), with
    coincident images merged.  Returns (pos, q)."""
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    out_p, out_q = [], []
    for p, qq in zip(np.asarray(points, float), np.asarray(q, float)):
        for perm in perms:
            for m in range(8):
                v = p[list(perm)].copy()
                for ax in range(3):
                    if (m >> ax) & 1:
                        v[ax] = 1.0 - v[ax]
                v = np.mod(v, 1.0)
                dup = False
                for w in out_p:
                    dd = np.abs(w - v)
                    dd = np.minimum(dd, 1.0 - dd)
                    if dd.max() < tol:
                        dup = True
                        break
                if not dup:
                    out_p.append(v)
                    out_q.append(qq)
    return np.array(out_p), np.array(out_q)


def mirror_orbit(points, q, tol=1e-12):
    """Images under the 8 reflections x -> 1 - x per axis (the one-eighth-cell
    fundamental volume of Sec. 3.2), coincident images merged."""
    out_p, out_q = [], []
    for p, qq in zip(np.asarray(points, float), np.asarray(q, float)):
        for m in range(8):
            v = p.copy()
            for ax in range(3):
                if (m >> ax) & 1:
                    v[ax] = 1.0 - v[ax]
            v = np.mod(v, 1.0)
            dup = any(np.max(np.minimum(np.abs(w - v), 1.0 - np.abs(w - v))) < tol for w in out_p)
            if not dup:
                out_p.append(v)
                out_q.append(qq)
    return np.array(out_p), np.array(out_q)
