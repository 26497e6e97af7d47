"""Redistribution functions and their frequency integrals (oracle).

* Faddeeva function W(a, v) = w(v + i a) (reading of Sect. 2.4: Re W is the
  Voigt function H with integral sqrt(pi), which makes the Theta = 0 identity
  of Sect. 4.3 consistent).  Evaluated with scipy.special.wofz.
* F(Theta, u', u) (Sect. 2.4, below Eq. G):
      F = exp(-((u - u')/(2 sin(Theta/2)))^2)
          * W(a / cos(Theta/2), (u + u')/(2 cos(Theta/2))) / sin(Theta).
  Theta = 0 is the distribution sqrt(pi) delta(u - u') W(a, u') (Sect. 4.3);
  Theta = pi uses the limit (reading; the paper only warns of sharp peaks):
      F(pi, u', u) = exp(-((u - u')/2)^2) * i / (2 sqrt(pi) ((u + u')/2 + i a)).
* The R_II kernel matrix of one (height, Theta, transition):
      M[n, m] = int_R F(Theta, u' + s, u_n + s) S_m(u') du'
  so that the intermediate of App. D (Eq. Wkukl, per unit Doppler width) is
  W(u_n) = sum_m M[n, m] Ibar_m.  S_m is the cardinal cubic spline of the
  comoving frequency grid with flat extension, so the integral is exact
  product integration of F against the interpolated field (Sect. 4.3 asks
  for a quadrature of the field interpolated to the nodes; with the field
  written as a spline the exact integral is the limit of any such rule).
* R_III absorption weights (Eq. RIIIQKKp, incoming factor):
      r[m] = int_R W(a, u' + s) S_m(u') du'
  with the 1/u' tail of Im W subtracted on both tails (it cancels between
  the W and W* halves of each incoming factor, so every sum the method forms
  is unchanged).

The quadrature here is composite Gauss-Legendre on panels that follow the
features of the integrand (spline knots, the Gaussian envelope of width
2 sin(Theta/2), the Voigt/Lorentz structure of width 2 max(cos(Theta/2), a)
at u' = -u - 2s).  It is pinned against adaptive Gauss-Kronrod (scipy quad)
and against the closed form int F du' = sqrt(pi) W(a, u) in tests.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad
from scipy.special import wofz

SQRT_PI = np.sqrt(np.pi)
_GL_CACHE = {}


def _gl(n: int):
    if n not in _GL_CACHE:
        _GL_CACHE[n] = np.polynomial.legendre.leggauss(n)
    return _GL_CACHE[n]


def faddeeva(a, v):
    """W(a, v) = w(v + i a)."""
    return wofz(np.asarray(v) + 1j * np.asarray(a))


def F_function(theta: float, up, u, a: float):
    """F(Theta, u', u) for 0 < Theta <= pi (vectorised over u', u)."""
    up = np.asarray(up, float)
    u = np.asarray(u, float)
    if theta <= 0.0:
        raise ValueError("Theta = 0 is a distribution; use the diagonal form")
    if theta >= np.pi:
        m = 0.5 * (u + up)
        return np.exp(-(0.5 * (u - up)) ** 2) * 1j / (2.0 * SQRT_PI * (m + 1j * a))
    s = np.sin(0.5 * theta)
    c = np.cos(0.5 * theta)
    g = np.exp(-((u - up) / (2.0 * s)) ** 2)
    return g * faddeeva(a / c, (u + up) / (2.0 * c)) / np.sin(theta)


def _panels(lo, hi, knots, centre, wc, gauss_len):
    """Breakpoints on [lo, hi]: knots, the Voigt centre with geometric grading,
    then splitting so that every panel is at most gauss_len and at most the
    larger of wc and its distance to the centre."""
    pts = [lo, hi]
    pts.extend(knots[(knots > lo) & (knots < hi)].tolist())
    if lo < centre < hi:
        pts.append(centre)
        step = wc
        span = hi - lo
        while step < span:
            for sgn in (-1.0, 1.0):
                q = centre + sgn * step
                if lo < q < hi:
                    pts.append(q)
            step *= 1.5
    pts = np.unique(np.asarray(pts))
    out = [pts[0]]
    for p, q in zip(pts[:-1], pts[1:]):
        d = 0.0 if p <= centre <= q else min(abs(p - centre), abs(q - centre))
        lmax = min(gauss_len, max(wc, d))
        k = max(1, int(np.ceil((q - p) / lmax)))
        out.extend((p + (q - p) * np.arange(1, k + 1) / k).tolist())
    return np.asarray(out)


def _nodes(breaks, n_gl):
    t, w = _gl(n_gl)
    a = breaks[:-1, None]
    b = breaks[1:, None]
    x = 0.5 * (b - a) * t[None, :] + 0.5 * (a + b)
    wx = 0.5 * (b - a) * w[None, :]
    return x.ravel(), wx.ravel()


def _moments_to_row(basis, xq, fq):
    """Given nodes xq and weighted integrand values fq (complex), return the
    row sum_m int f S_m via interval moments and the spline coefficients."""
    x = basis.x
    n = x.size
    k = np.searchsorted(x, xq, side="right") - 1       # -1: left tail, n-1: right tail
    row = np.zeros(n, complex)
    left = k < 0
    right = k >= n - 1
    row[0] += fq[left].sum()
    row[n - 1] += fq[right].sum()
    inner = ~(left | right)
    ki = k[inner]
    dx = xq[inner] - x[ki]
    fi = fq[inner]
    mom = np.zeros((n - 1, 4), complex)
    for p in range(4):
        np.add.at(mom[:, p], ki, fi * dx ** p)
    # coef[p, k, m] multiplies (y - x_k)^(3-p)
    row += np.einsum("pkm,kp->m", basis.coef, mom[:, ::-1])
    return row


def kernel_matrix(theta: float, s: float, a: float, lam: float, basis, n_gl: int = 20):
    """R_II kernel M[n, m] for one (height, Theta, transition).

    theta: scattering angle; s: reduced transition shift u_{k_u,k_l} at this
    height; a: damping; lam: dnu_D_ref / dnu_D(z) (u = lam * x); basis: the
    SplineBasis of the reference grid x.
    """
    x = basis.x
    n = x.size
    M = np.zeros((n, n), complex)
    if theta == 0.0:
        M[np.arange(n), np.arange(n)] = SQRT_PI * faddeeva(a, lam * x + s)
        return M
    sG = np.sin(0.5 * theta)
    cG = np.cos(0.5 * theta) if theta < np.pi else 0.0
    sigma = 2.0 * sG / lam
    R = 6.6 * sigma
    wc = 2.0 * max(cG, a) / lam
    for i in range(n):
        xn = x[i]
        centre = -xn - 2.0 * s / lam
        br = _panels(xn - R, xn + R, x, centre, wc, 0.5 * sigma)
        xq, wq = _nodes(br, n_gl)
        fq = wq * lam * F_function(theta, lam * xq + s, lam * xn + s, a)
        M[i] = _moments_to_row(basis, xq, fq)
    return M


def kernel_matrix_aa(s: float, a: float, lam: float, basis, n_theta: int = 25):
    """Angle-averaged R_II kernel (Sect. 5.2, Eq. R_AA): the scattering-angle
    average (1/2) int_0^pi sin(Theta) M(Theta) dTheta of the kernel matrix, with
    the Gauss-Legendre rule of n_theta nodes on [0, pi] that App. C uses for it."""
    t, w = np.polynomial.legendre.leggauss(n_theta)
    th = 0.5 * np.pi * (t + 1.0)
    wt = 0.5 * np.pi * w * 0.5 * np.sin(th)
    M = np.zeros((basis.x.size, basis.x.size), complex)
    for thk, wk in zip(th, wt):
        M += wk * kernel_matrix(float(thk), s, a, lam, basis)
    return M


def _tail_integral(fun, start, direction):
    """int from start to +-inf of a complex function, with scipy quad."""
    if direction > 0:
        lo, hi = start, np.inf
    else:
        lo, hi = -np.inf, start
    re = quad(lambda t: fun(t).real, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    im = quad(lambda t: fun(t).imag, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    return re + 1j * im


def r3_weights(s: float, a: float, lam: float, basis, n_gl: int = 20):
    """R_III incoming weights r[m] = int W(a, u'+s) S_m(u') du' (tails
    regularised by subtracting i/(sqrt(pi) u'), see module docstring)."""
    x = basis.x
    n = x.size
    centre = -s / lam
    br = _panels(x[0], x[-1], x, centre, 0.25 / lam, 0.25 / lam)
    xq, wq = _nodes(br, n_gl)
    fq = wq * lam * faddeeva(a, lam * xq + s)
    row = _moments_to_row(basis, xq, fq)
    u0, u1 = lam * x[0], lam * x[-1]
    if not (u0 < 0.0 < u1):
        raise ValueError("frequency grid must bracket the line centre")

    def reg(u):
        return faddeeva(a, u + s) - 1j / (SQRT_PI * u)
    row[0] += _tail_integral(reg, u0, -1)
    row[n - 1] += _tail_integral(reg, u1, +1)
    return row
