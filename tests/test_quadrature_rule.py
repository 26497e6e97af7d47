"""The node count of the kernel precompute's graded rule (R_II rows, Sect. 4.3
product integration).  Panels are graded towards the Voigt core: width at
most Lg = 1.5 sigma (sigma = 2 sin(Theta/2) / lambda, the Gaussian's width)
and at most max(wc, distance to the core) (wc = 2 max(cos(Theta/2), a) /
lambda, the core's width).  A panel takes 16 Gauss-Legendre nodes, or 8 when
it spans at most 0.15 of that natural width (it is cut short by a knot
interval).  Pinned here: on such panels the 8-node rule integrates F t^q
(q = 0..3, the spline moments) to within 1e-12 of the panel's integral of
|F|, measured against a 40-node rule, over random angles, damping, Doppler
ratios, frequencies and panel positions (including panels at the core and
Theta = pi); and the 16-node rule does so on panels of the full natural
width, which is what keeps the 8-node shortcut to short panels."""
import numpy as np

from oracle.redistribution import F_function

_G = {n: np.polynomial.legendre.leggauss(n) for n in (8, 16, 40)}


def _gl(f, a, b, n):
    t, w = _G[n]
    x = 0.5 * (b - a) * t + 0.5 * (a + b)
    return 0.5 * (b - a) * np.sum(w * f(x))


def _panels(seed, ratios, trials):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < trials:
        Th = np.pi if rng.uniform() < 0.15 else rng.uniform(0.02, np.pi)
        a = 10 ** rng.uniform(-3, -1)
        lam = rng.uniform(0.5, 1.2)
        sG, cG = (1.0, 0.0) if Th >= np.pi else (np.sin(Th / 2), np.cos(Th / 2))
        sigma = 2 * sG / lam
        Lg, wc = 1.5 * sigma, 2 * max(cG, a) / lam
        xn = rng.uniform(-15, 15)
        xc = -xn                                    # the core of F(x', xn) in x' (zero shift)
        d = abs(rng.normal(0, 3 * sigma)) * (rng.uniform() < 0.8) + 1e-4
        w = rng.choice(ratios) * min(Lg, max(wc, d))
        pa = xc + d if rng.uniform() < 0.5 else xc - d - w
        if pa > xn + 6.6 * sigma or pa + w < xn - 6.6 * sigma:
            continue                                # outside the row's support
        out.append((Th, a, lam, xn, pa, pa + w))
    return out


def _worst(panels, n):
    worst = 0.0
    for Th, a, lam, xn, pa, pb in panels:
        F = lambda xp: lam * F_function(Th, lam * xp, lam * xn, a)
        scale = _gl(lambda xp: np.abs(F(xp)), pa, pb, 40) + 1e-300
        for q in range(4):
            f = lambda xp: F(xp) * ((xp - pa) / (pb - pa)) ** q
            worst = max(worst, abs(_gl(f, pa, pb, n) - _gl(f, pa, pb, 40)) / scale)
    return worst


def test_eight_nodes_suffice_on_short_panels():
    assert _worst(_panels(1, [0.02, 0.05, 0.1, 0.15], 600), 8) < 1e-12


def test_sixteen_nodes_on_full_panels_and_eight_do_not():
    full = _panels(2, [0.5, 1.0], 300)
    assert _worst(full, 16) < 1e-12
    assert _worst(full, 8) > 1e-9                  # the shortcut must stay on short panels
