"""Angular grid, scattering-angle table and the cubic-spline basis (oracle).

* Angular quadrature (Sect. 4.2): tensor product of two Gauss-Legendre sets in
  mu = cos(theta), one per hemisphere [-1,0] and [0,1], and a trapezoidal rule
  in the azimuth chi on [0, 2pi).  Weights are normalised to the measure
  dOmega/(4 pi).
* Scattering angles (Sects. 2.4 and 4.2): Theta = arccos(Omega . Omega'); the
  comoving redistribution function depends on the pair only through Theta, so
  the distinct values are tabulated once.
* Interpolation (Sect. 6.2): all observer/comoving frequency interpolations are
  cubic splines.  Reading: not-a-knot end conditions and flat (edge-value)
  extension outside the grid.
* Non-oscillatory interpolation (Sect. 4.1 names high-order non-oscillatory
  interpolation as the remedy for oscillations under strong velocities and
  points to a weighted essentially non-oscillatory scheme; it gives no
  formulas, so the scheme below is a reading): weno4_interpolate.
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


def weno4_interpolate(x: np.ndarray, values: np.ndarray, y: np.ndarray, axis: int = 0,
                      eps_rel: float = 1e-12) -> np.ndarray:
    """Fourth-order weighted essentially non-oscillatory interpolation of
    ``values`` (nodes x along ``axis``, each trailing column separately) at y,
    flat (edge-value) extension outside [x_0, x_{n-1}].

    Reading of the remedy named in Sect. 4.1.  On the interval [x_i, x_{i+1}]
    holding y, the two quadratics through the three-node stencils
    {x_{i-1}, x_i, x_{i+1}} and {x_i, x_{i+1}, x_{i+2}} share the line through
    the interval's end values:
        q_k(y) = v_i + d (y - x_i) + D_k (y - x_i)(y - x_{i+1}),
    d the first divided difference on the interval, D_k the second divided
    difference of stencil k.  With the linear weights
        g_1 = (x_{i+2} - y) / (x_{i+2} - x_{i-1}),  g_2 = 1 - g_1
    (Neville's recursion) g_1 q_1 + g_2 q_2 is the cubic through the four
    nodes.  The nonlinear weights replace them:
        b_k = (h_i^2 D_k)^2            (h_i = x_{i+1} - x_i)
        e   = eps_rel * mean(v_{i-1}^2, v_i^2, v_{i+1}^2, v_{i+2}^2)
        a_k = g_k / (e + b_k)^2,   w_k = a_k / (a_1 + a_2),
    so a stencil that straddles a jump (large b) loses its weight and the
    result follows the smooth side.  e keeps the scheme invariant under a
    scaling of the data and gives the linear weights on flat data (a floor of
    1e-150, whose square is still a normal number, covers all-zero data).  The first
    and last intervals have one stencil only and take its quadratic.
    Any weights reproduce a quadratic exactly (q_1 = q_2 there); a very large
    eps_rel gives the linear weights and so the four-node cubic.
    """
    x = np.asarray(x, float)
    n = x.size
    if n < 4:
        raise ValueError("need >= 4 frequency nodes")
    v = np.moveaxis(np.asarray(values, float), axis, 0)
    yy = np.clip(np.asarray(y, float), x[0], x[-1])
    out = np.empty((yy.size,) + v.shape[1:])
    for j, t in enumerate(yy.ravel()):
        i = int(np.searchsorted(x, t, side="right")) - 1
        i = min(max(i, 0), n - 2)
        h = x[i + 1] - x[i]
        d = (v[i + 1] - v[i]) / h
        lin = v[i] + d * (t - x[i])
        bub = (t - x[i]) * (t - x[i + 1])
        if i == 0 or i == n - 2:
            # one stencil: the one that stays on the grid
            a, b, c = (i, i + 1, i + 2) if i == 0 else (i - 1, i, i + 1)
            D = ((v[c] - v[b]) / (x[c] - x[b]) - (v[b] - v[a]) / (x[b] - x[a])) / (x[c] - x[a])
            out[j] = lin + D * bub
            continue
        D1 = (d - (v[i] - v[i - 1]) / (x[i] - x[i - 1])) / (x[i + 1] - x[i - 1])
        D2 = ((v[i + 2] - v[i + 1]) / (x[i + 2] - x[i + 1]) - d) / (x[i + 2] - x[i])
        g1 = (x[i + 2] - t) / (x[i + 2] - x[i - 1])
        g2 = 1.0 - g1
        b1 = (h * h * D1) ** 2
        b2 = (h * h * D2) ** 2
        e = eps_rel * (v[i - 1] ** 2 + v[i] ** 2 + v[i + 1] ** 2 + v[i + 2] ** 2) / 4.0 + 1e-150
        a1 = g1 / (e + b1) ** 2
        a2 = g2 / (e + b2) ** 2
        w1 = a1 / (a1 + a2)
        out[j] = lin + (w1 * D1 + (1.0 - w1) * D2) * bub
    out = out.reshape(np.shape(yy) + v.shape[1:])
    return np.moveaxis(out, 0, axis) if np.ndim(yy) == 1 else out
