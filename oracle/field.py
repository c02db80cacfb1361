"""Charge field, distance, occupancy and thickness selection (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Array convention: a voxel grid of resolution n is an array of shape (n, n, n)
indexed [k, j, i] with i along x, j along y, k along z; voxel (i, j, k) has its
center at ((i + 1/2)/n, (j + 1/2)/n, (k + 1/2)/n) (Sec. 4.1: the field is
sampled at voxel centers p_e).

Readings of the paper taken here (each pinned by a test):
* w_hkl = 1 when no index is zero (Eq. (5) only states the one-zero and
  two-zero cases; folding the lattice sum over Z^3 minus the origin into the
  first octant gives weight 1/2^(number of zero indices)).
* Eq. (6) is used as printed: no 8/pi prefactor, B_000 = 0, cubic truncation
  0 <= h, k, l <= K.
* Charges may carry any real value (Eq. (6) uses +-1; B_000 = 0 makes the net
  charge irrelevant).
* The distance floor: ||grad F|| is clamped below at 1e-12 * max ||grad F||;
  a zero numerator gives d = 0.
"""
import numpy as np
from scipy.special import expit


def mode_weight(h, k, l):
    """w_hkl of Eq. (5): 1/2 for one zero index, 1/4 for two, 1 for none."""
    zeros = int(h == 0) + int(k == 0) + int(l == 0)
    return 0.5 ** zeros


def modes(K):
    """All (h, k, l) with 0 <= h, k, l <= K except (0, 0, 0) (Eq. (6), B_000 = 0)."""
    out = []
    for h in range(K + 1):
        for k in range(K + 1):
            for l in range(K + 1):
                if h == 0 and k == 0 and l == 0:
                    continue
                out.append((h, k, l))
    return out


def voxel_centers(n):
    """1D voxel-center coordinates (i + 1/2)/n, i = 0..n-1 (Sec. 4.1)."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _alpha(alpha, K):
    if alpha is None:
        return np.ones((K + 1, K + 1, K + 1))
    a = np.asarray(alpha, dtype=np.float64).reshape(K + 1, K + 1, K + 1)
    return a


def field_and_gradient(pos, q, n, K=3, alpha=None):
    """F and grad F of Eq. (6) at the n^3 voxel centers, by direct summation.

    F(x) = sum_{(h,k,l) != 0} alpha_hkl w_hkl / (h^2+k^2+l^2)
               * sum_j q_j cos(2 pi h (x - x_j)) cos(2 pi k (y - y_j)) cos(2 pi l (z - z_j))

    Loops over every (charge, mode) term; each term is evaluated on the whole
    grid as an outer product of its three 1D cosine factors.
    Returns F with shape (n, n, n) and G with shape (3, n, n, n) = (dF/dx, dF/dy, dF/dz).
    """
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    a = _alpha(alpha, K)
    c = voxel_centers(n)
    F = np.zeros((n, n, n))
    G = np.zeros((3, n, n, n))
    two_pi = 2.0 * np.pi
    for j in range(len(q)):
        xj, yj, zj = pos[j]
        for (h, k, l) in modes(K):
            coef = a[h, k, l] * mode_weight(h, k, l) / (h * h + k * k + l * l) * q[j]
            if coef == 0.0:
                continue
            cx = np.cos(two_pi * h * (c - xj))
            cy = np.cos(two_pi * k * (c - yj))
            cz = np.cos(two_pi * l * (c - zj))
            sx = -two_pi * h * np.sin(two_pi * h * (c - xj))
            sy = -two_pi * k * np.sin(two_pi * k * (c - yj))
            sz = -two_pi * l * np.sin(two_pi * l * (c - zj))
            # grid index order [k(z), j(y), i(x)]
            F += coef * cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
            G[0] += coef * cz[:, None, None] * cy[None, :, None] * sx[None, None, :]
            G[1] += coef * cz[:, None, None] * sy[None, :, None] * cx[None, None, :]
            G[2] += coef * sz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    return F, G


def field_at_points(pts, pos, q, K=3, alpha=None):
    """F of Eq. (6) at arbitrary points pts (m, 3), by direct summation."""
    pts = np.asarray(pts, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    a = _alpha(alpha, K)
    F = np.zeros(len(pts))
    for j in range(len(q)):
        for (h, k, l) in modes(K):
            coef = a[h, k, l] * mode_weight(h, k, l) / (h * h + k * k + l * l) * q[j]
            F += coef * (np.cos(2 * np.pi * h * (pts[:, 0] - pos[j, 0]))
                         * np.cos(2 * np.pi * k * (pts[:, 1] - pos[j, 1]))
                         * np.cos(2 * np.pi * l * (pts[:, 2] - pos[j, 2])))
    return F


def field_and_gradient_at_points(pts, pos, q, K=3, alpha=None):
    """F and grad F of Eq. (6) at arbitrary points pts (m, 3), by direct
    summation over every (charge, mode) term.  Returns (F (m,), G (m, 3))."""
    pts = np.asarray(pts, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    a = _alpha(alpha, K)
    F = np.zeros(len(pts))
    G = np.zeros((len(pts), 3))
    tp = 2.0 * np.pi
    for j in range(len(q)):
        for (h, k, l) in modes(K):
            coef = a[h, k, l] * mode_weight(h, k, l) / (h * h + k * k + l * l) * q[j]
            if coef == 0.0:
                continue
            ax = tp * h * (pts[:, 0] - pos[j, 0])
            ay = tp * k * (pts[:, 1] - pos[j, 1])
            az = tp * l * (pts[:, 2] - pos[j, 2])
            cx, cy, cz = np.cos(ax), np.cos(ay), np.cos(az)
            F += coef * cx * cy * cz
            G[:, 0] += coef * (-tp * h * np.sin(ax)) * cy * cz
            G[:, 1] += coef * cx * (-tp * k * np.sin(ay)) * cz
            G[:, 2] += coef * cx * cy * (-tp * l * np.sin(az))
    return F, G


def distance(F, G, iso=0.0, dist_mode=0):
    """d_e of Eq. (7): |F - c| / ||grad F|| (dist_mode 0) or |F - c| (dist_mode 1).

    The gradient norm is floored at 1e-12 * max ||grad F||; where the numerator
    is zero the distance is zero, and where both vanish (a constant field) too.
    """
    num = np.abs(F - iso)
    if dist_mode == 1:
        return num
    gn = np.sqrt(G[0] ** 2 + G[1] ** 2 + G[2] ** 2)
    gmin = 1e-12 * gn.max()
    den = np.maximum(gn, gmin)
    d = np.zeros_like(num)
    nz = num > 0
    with np.errstate(divide="ignore"):
        d[nz] = num[nz] / den[nz]
    return d


def occupancy(d, t, kappa):
    """beta_e = h(d_e) (Eq. (7)): the hard step [d < t] for kappa = 0, else the
    logistic 1 / (1 + exp(-kappa (t - d))) of Sec. 4.1."""
    if kappa == 0:
        return (d < t).astype(np.float64)
    return expit(kappa * (t - d))


def thickness_for_volume(d, target_vf, kappa):
    """Half-thickness t giving volume fraction target_vf (Sec. 4.3 volume constraint).

    Hard step: with m voxels and k = round(target_vf * m), t is the midpoint of
    the k-th and (k+1)-th smallest distances, so exactly k voxels (absent ties)
    satisfy d < t.  Logistic: bisection on t until |V(t) - target| <= 1e-12.
    """
    s = np.sort(np.asarray(d, dtype=np.float64).ravel())
    m = s.size
    if kappa == 0:
        k = int(np.floor(target_vf * m + 0.5))
        if k <= 0:
            return 0.5 * s[0]
        if k >= m:
            return 2.0 * s[-1] + 1.0
        return 0.5 * (s[k - 1] + s[k])
    lo = s[0] - 40.0 / kappa
    hi = s[-1] + 40.0 / kappa
    t = 0.5 * (lo + hi)
    for _ in range(200):
        t = 0.5 * (lo + hi)
        v = occupancy(s, t, kappa).mean()
        if abs(v - target_vf) <= 1e-12:
            break
        if v < target_vf:
            lo = t
        else:
            hi = t
    return t


def stiffness_field(beta, E, E_void):
    """E_e = E_void + (E - E_void) beta_e: the per-voxel Young's modulus, with a
    stiffness floor for void voxels (Sec. 4.2 notes that a dense grid needs one)."""
    return E_void + (E - E_void) * beta
