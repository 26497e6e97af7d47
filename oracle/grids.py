"""Angular grid, scattering-angle table and the cubic-spline basis (oracle).

* Angular quadrature (Sect. 4.2): tensor product of two Gauss-Legendre sets in
  mu = cos(theta), one per hemisphere [-1,0] and [0,1], and a trapezoidal rule
  in the azimuth chi on [0, 2pi).  Weights are normalised to the measure
  dOmega/(4 pi).
* Scattering angles (Sects. 2.3 and 4.2): Theta = arccos(Omega . Omega'); the
  comoving redistribution function depends on the pair only through Theta, so
  the distinct values are tabulated once.
* Interpolation (Sect. 6.2): all observer/comoving frequency interpolations are
  cubic splines.  Reading: not-a-knot end conditions and flat (edge-value)
  extension outside the grid.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline


def angular_grid(n_mu: int, n_chi: int, los_mu=None):
    """Directions ordered mu-major (mu ascending from -1 to 1), chi-minor.

    Returns dict with mu, chi, w (sum 1), dirs [N,3], e_a, e_b [N,3].
    e_a is the positive-Q reference direction: perpendicular to the vertical
    plane that contains the ray, i.e. parallel to the limb (Sect. 6.3, Fig. 2
    caption); (e_a, e_b, Omega) is right-handed.

    ``los_mu`` (optional, each in (0, 1]): lines of sight off the quadrature
    (the emergent profiles of Sect. 6 are shown at such mu values).  Each
    adds a ring of the n_chi azimuths after the quadrature directions with
    zero weight: the rays are solved like any other but take no part in the
    angular integrals.  "n_grid" counts the quadrature directions.
    """
    if n_mu < 2 or n_mu % 2:
        raise ValueError("n_mu must be even and >= 2 (double Gauss-Legendre)")
    if n_chi < 1:
        raise ValueError("n_chi must be >= 1")
    h = n_mu // 2
    t, wt = np.polynomial.legendre.leggauss(h)
    mu_p = 0.5 * (t + 1.0)
    w_p = 0.5 * wt
    mu1 = np.concatenate([-mu_p[::-1], mu_p])
    wmu = np.concatenate([w_p[::-1], w_p])
    los = np.zeros(0) if los_mu is None else np.asarray(los_mu, float).ravel()
    if np.any(~(los > 0.0)) or np.any(los > 1.0):
        raise ValueError("line-of-sight mu must lie in (0, 1]")
    mu1 = np.concatenate([mu1, los])
    wmu = np.concatenate([wmu, np.zeros_like(los)])
    chi1 = 2.0 * np.pi * np.arange(n_chi) / n_chi
    n_ring = mu1.size
    mu = np.repeat(mu1, n_chi)
    chi = np.tile(chi1, n_ring)
    w = np.repeat(wmu, n_chi) / (2.0 * n_chi)
    st = np.sqrt(1.0 - mu * mu)
    dirs = np.stack([st * np.cos(chi), st * np.sin(chi), mu], axis=1)
    e_a = np.stack([-np.sin(chi), np.cos(chi), np.zeros_like(chi)], axis=1)
    e_b = np.cross(dirs, e_a)
    return {"mu": mu, "chi": chi, "w": w, "dirs": dirs, "e_a": e_a, "e_b": e_b,
            "n_mu": n_mu, "n_chi": n_chi, "n_grid": n_mu * n_chi, "n_los": los.size}


def theta_table(dirs: np.ndarray, tol: float = 1e-10):
    """Distinct scattering angles over all ordered direction pairs.

    Returns (theta_values ascending, pair_index[N_out, N_in]) with
    pair_index[o, i] the table index of the angle between outgoing direction o
    and incoming direction i.  cos(Theta) within 1e-12 of +-1 is snapped to
    exactly 0 or pi (forward and backward scattering).
    """
    c = np.clip(dirs @ dirs.T, -1.0, 1.0)
    c[np.abs(c - 1.0) < 1e-12] = 1.0
    c[np.abs(c + 1.0) < 1e-12] = -1.0
    flat = np.sort(c.ravel())[::-1]          # descending cos -> ascending Theta
    reps = [flat[0]]
    for v in flat[1:]:
        if reps[-1] - v > tol:
            reps.append(v)
    reps = np.array(reps)
    idx = np.empty(c.shape, dtype=np.int64)
    for k in range(c.shape[0]):
        for j in range(c.shape[1]):
            idx[k, j] = int(np.argmin(np.abs(reps - c[k, j])))
    theta = np.arccos(reps)
    theta[reps == 1.0] = 0.0
    theta[reps == -1.0] = np.pi
    return theta, idx


class SplineBasis:
    """Cardinal not-a-knot cubic-spline basis on nodes x with flat extension.

    ``coef`` has SciPy's layout [4, n-1, n]: on interval k the basis function
    S_m(y) = sum_p coef[p, k, m] (y - x_k)^(3-p).
    """

    def __init__(self, x: np.ndarray):
        self.x = np.asarray(x, float)
        n = self.x.size
        if n < 4:
            raise ValueError("need >= 4 frequency nodes for a not-a-knot cubic spline")
        self.cs = CubicSpline(self.x, np.eye(n), bc_type="not-a-knot")
        self.coef = self.cs.c

    def matrix(self, y: np.ndarray) -> np.ndarray:
        """Rows S_m(y_i) for every m (flat extension beyond the end nodes)."""
        yc = np.clip(np.asarray(y, float), self.x[0], self.x[-1])
        return self.cs(yc)

    def interpolate(self, values: np.ndarray, y: np.ndarray, axis: int = 0) -> np.ndarray:
        """Spline of ``values`` (nodes along ``axis``) evaluated at y."""
        S = self.matrix(y)
        v = np.moveaxis(values, axis, 0)
        out = np.tensordot(S, v, axes=([1], [0]))
        return np.moveaxis(out, 0, axis)
