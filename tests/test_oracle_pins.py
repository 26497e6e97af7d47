"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle
with itself: the references are closed forms, independent library routines
(scipy quad, wofz, CubicSpline), classical textbook special cases written
here in their own variables, and values the paper prints.
"""
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erfc, wofz

from workloads import tiny, two_level_atom, two_term_atom
from oracle import transfer as T
from oracle.grids import angular_grid, theta_table, SplineBasis
from oracle.redistribution import F_function, kernel_matrix, r3_weights, faddeeva

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SQPI = np.sqrt(np.pi)


# ---------------------------------------------------------------- grids (Sect. 4.2, 6.2)

def test_theta_count_matches_paper():
    """Sect. 6.2: 6+6 Gauss-Legendre mu x 9 azimuths -> N_Theta = 205."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "theta_count.txt"))
            if l.strip() and not l.startswith("#")]
    for n_mu, n_chi, n_theta in rows:
        ang = angular_grid(int(n_mu), int(n_chi))
        theta, pair = theta_table(ang["dirs"])
        assert len(theta) == int(n_theta)
        c = ang["dirs"] @ ang["dirs"].T
        assert np.allclose(np.cos(theta[pair]), c, atol=1e-9)


def test_angular_weights_integrate_low_degree_exactly():
    """Sect. 4.2: double GL in mu x trapezoid in chi integrates the degree <= 2
    direction tensors exactly (needed by the Kirchhoff pin)."""
    ang = angular_grid(4, 4)
    d, w = ang["dirs"], ang["w"]
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("o,oi,oj->ij", w, d, d), np.eye(3) / 3.0, atol=1e-15)
    assert np.allclose(w @ d, 0.0, atol=1e-15)
    assert np.all(np.abs(ang["mu"]) > 0)          # no horizontal rays (Sect. 4.2)


def test_spline_reproduces_cubics_and_flat_extension():
    """Sect. 6.2 (cubic splines) with the not-a-knot reading: cubics are exact."""
    x = np.sort(np.random.default_rng(1).uniform(-5, 5, 17))
    b = SplineBasis(x)
    y = np.linspace(-5, 5, 301)
    y = y[(y >= x[0]) & (y <= x[-1])]
    p = lambda t: 0.3 * t ** 3 - t ** 2 + 2 * t - 1
    assert np.allclose(b.matrix(y) @ p(x), p(y), atol=1e-11)
    S = b.matrix(np.array([x[0] - 3.0, x[-1] + 7.0]))
    assert np.allclose(S[0], np.eye(x.size)[0]) and np.allclose(S[1], np.eye(x.size)[-1])
    assert np.allclose(b.matrix(x), np.eye(x.size), atol=1e-13)


# ---------------------------------------------------------------- Faddeeva and F (Sect. 2.4, 4.3)

def test_faddeeva_reading():
    """Reading of W(a, v): Re W(a, 0) = e^{a^2} erfc(a) and int Re W dv = sqrt(pi)."""
    for a in (1e-3, 0.1, 2.0):
        assert abs(faddeeva(a, 0.0).real - np.exp(a * a) * erfc(a)) < 1e-14
        val = quad(lambda v: faddeeva(a, v).real, -np.inf, np.inf, epsabs=1e-14, limit=500)[0]
        assert abs(val - SQPI) < 1e-9


@pytest.mark.parametrize("theta", [0.05, np.pi / 3, 0.9 * np.pi, np.pi - 1e-3, np.pi])
@pytest.mark.parametrize("a", [1e-3, 1e-2])
def test_F_integrates_to_faddeeva(theta, a):
    """int F(Theta, u', u) du' = sqrt(pi) W(a, u) (App. C Theta = 0 identity
    extended to all Theta), checked with adaptive Gauss-Kronrod."""
    for u in (-3.0, 0.4, 2.5):
        pts = [u, -u]
        f = lambda up, part: getattr(F_function(theta, up, u, a), part)
        lo, hi = u - 40, u + 40
        re = quad(f, lo, hi, args=("real",), points=pts, epsabs=1e-14, epsrel=1e-12, limit=2000)[0]
        im = quad(f, lo, hi, args=("imag",), points=pts, epsabs=1e-14, epsrel=1e-12, limit=2000)[0]
        exact = SQPI * faddeeva(a, u)
        # the Gaussian factor vanishes outside [u-40, u+40] to far below 1e-14
        assert abs(re - exact.real) < 2e-9 * abs(exact)
        assert abs(im - exact.imag) < 2e-9 * abs(exact)


def test_F_symmetry_and_backscatter_limit():
    """F(Theta, u', u) = F(Theta, u, u') (Sect. 4.3 property) and the Theta -> pi
    limit used for exact backscattering converges as O(delta^2) once
    cos(Theta/2) ~ delta/2 is well below the damping a."""
    up = np.linspace(-4, 4, 9)
    u = np.linspace(-3.3, 2.9, 9)[::-1]
    for th in (0.3, 2.0, 3.0):
        assert np.allclose(F_function(th, up, u, 0.01), F_function(th, u, up, 0.01), rtol=1e-13)
    lim = F_function(np.pi, up, u, 0.01)
    e1 = np.abs(F_function(np.pi - 2e-4, up, u, 0.01) - lim).max()
    e2 = np.abs(F_function(np.pi - 1e-4, up, u, 0.01) - lim).max()
    assert e2 < e1 / 3.5 and e2 < 1e-4 * np.abs(lim).max()


@pytest.mark.parametrize("theta,s,a,lam", [(0.7, 0.0, 1e-3, 1.0), (2.3, 0.37, 1e-2, 0.8),
                                           (np.pi, -0.2, 1e-3, 1.1), (np.pi - 0.02, 0.0, 1e-3, 1.0)])
def test_kernel_rows_against_adaptive_quadrature(theta, s, a, lam):
    """Sect. 4.3: the R_II frequency integral to < 1e-8 relative (the paper's
    claim for its own rule); product integration against an adaptive
    Gauss-Kronrod reference of int F(Theta, u'+s, u_n+s) S_m(u') du'."""
    x = np.linspace(-6, 6, 13)
    b = SplineBasis(x)
    M = kernel_matrix(theta, s, a, lam, b)
    rng = np.random.default_rng(3)
    for n in (0, 6, 10):
        un = lam * x[n] + s
        for m in rng.choice(x.size, 3, replace=False):
            def f(xp, part):
                return getattr(lam * F_function(theta, lam * xp + s, un, a) * b.matrix(np.array([xp]))[0, m], part)
            pts = sorted({*x.tolist(), -x[n] - 2 * s / lam})
            lo, hi = x[n] - 30 / lam, x[n] + 30 / lam
            pts = [p for p in pts if lo < p < hi]
            ref = (quad(f, lo, hi, args=("real",), points=pts, epsabs=1e-15, epsrel=1e-12, limit=4000)[0]
                   + 1j * quad(f, lo, hi, args=("imag",), points=pts, epsabs=1e-15, epsrel=1e-12, limit=4000)[0])
            scale = abs(SQPI * faddeeva(a, un))
            assert abs(M[n, m] - ref) < 1e-9 * scale, (n, m, M[n, m], ref)
    # row sums: with flat extension sum_m S_m = 1, so rows sum to sqrt(pi) W(a, u_n + s)
    assert np.allclose(M.sum(axis=1), SQPI * faddeeva(a, lam * x + s), rtol=1e-11, atol=1e-14)


def test_r3_weights_sum():
    """Eq. RIIIQKKp incoming factor: with flat extension the weights of
    W(u'+s') + conj W(u'+s) sum to 2 sqrt(pi) (the subtracted 1/u' tails cancel)."""
    x = np.linspace(-8, 8, 21)
    b = SplineBasis(x)
    r1 = r3_weights(0.3, 1e-2, 1.0, b)
    r2 = r3_weights(-0.1, 1e-2, 1.0, b)
    assert abs((r1 + np.conj(r2)).sum() - 2 * SQPI) < 1e-9


# ---------------------------------------------------------------- propagation matrix (Sect. 2.2, LL04 ch. 7)

def test_propagation_matrix_closed_form_zeeman():
    """J 0->1 propagation matrix against the closed-form Zeeman expressions in
    terms of the field inclination/azimuth in the ray frame (pi, sigma_b with
    M_u - M_l = +1, sigma_r), with dispersion profiles psi = Im W/sqrt(pi)."""
    p = tiny(n_z=2, n_nu=21, x_max=5, n_mu=4, n_chi=4, B=(3000.0, 0.6, 0.9), a=3e-2,
             eps=1e-2, v_z=1.5)
    op = T.setup(p, {"normalize": False})
    for z in range(p.n_z):
        nuL = 1.39962449361e6 * p.B[z, 0]
        th, ch = p.B[z, 1], p.B[z, 2]
        bh = np.array([np.sin(th) * np.cos(ch), np.sin(th) * np.sin(ch), np.cos(th)])
        for o in range(p.n_dir):
            ba, bb, ct = bh @ op.ang["e_a"][o], bh @ op.ang["e_b"][o], bh @ op.ang["dirs"][o]
            c2, s2, st2 = ba * ba - bb * bb, 2 * ba * bb, 1 - ct * ct
            u = op.lam[z] * p.x + op.ub[z, o]
            Wq = {q: wofz(u + nuL * q / op.dnuD[z] + 1j * p.a[z]) / SQPI for q in (-1, 0, 1)}
            ph = {q: Wq[q].real for q in Wq}
            ps = {q: Wq[q].imag for q in Wq}
            eI = 0.5 * (ph[0] * st2 + (ph[1] + ph[-1]) * (1 + ct * ct) / 2)
            eQ = 0.5 * (ph[0] - (ph[1] + ph[-1]) / 2) * c2
            eU = 0.5 * (ph[0] - (ph[1] + ph[-1]) / 2) * s2
            eV = 0.5 * (ph[-1] - ph[1]) * ct
            rQ = 0.5 * (ps[0] - (ps[1] + ps[-1]) / 2) * c2
            rU = 0.5 * (ps[0] - (ps[1] + ps[-1]) / 2) * s2
            rV = 0.5 * (ps[-1] - ps[1]) * ct
            K = np.stack([np.stack([eI, eQ, eU, eV], -1), np.stack([eQ, eI, rV, -rU], -1),
                          np.stack([eU, -rV, eI, rQ], -1), np.stack([eV, rU, -rQ, eI], -1)], -2)
            assert np.abs(K - op.K[z, o]).max() < 1e-14


def test_weak_field_stokes_v_sign():
    """Convention pin: for a field along the ray the sigma_b (M_u - M_l = +1,
    higher frequency, u < 0) component gives eta_V < 0 on the blue side."""
    p = tiny(n_z=1, n_nu=41, x_max=4, n_mu=4, n_chi=4, B=(1000.0, 0.0, 0.0), a=1e-2)
    op = T.setup(p, {"normalize": False})
    o = int(np.argmax(op.ang["mu"]))
    etaV = op.K[0, o, :, 0, 3]
    assert etaV[p.x < -0.3].min() < 0 and etaV[(p.x > -2) & (p.x < 0)].max() <= 0
    assert etaV[(p.x > 0) & (p.x < 2)].min() >= 0


# ---------------------------------------------------------------- emissivity pins (App. E, App. B)

def _flat(p):
    I = np.zeros((p.n_z, p.n_dir, p.n_nu, 4))
    I[..., 0] = p.W_T[:, None, None]
    return I


@pytest.mark.parametrize("B", [(0.0, 0.0, 0.0), (20.0, np.pi / 2, 0.0), (300.0, 0.7, 1.1)])
def test_kirchhoff_flat_field_two_level(B):
    """App. E, Eq. analytical_eps_sc: for a flat, unpolarised, isotropic field
    I = (W_T, 0, 0, 0), eps^sc = (1 - eps) W_T eta for all four Stokes
    components (unnormalised Sigma; static, no lower-level splitting)."""
    p = tiny(n_z=2, n_nu=13, n_mu=4, n_chi=4, B=B, a=1e-2, eps=3e-2)
    op = T.setup(p, {"normalize": False})
    e = T.sigma_apply(op, _flat(p), normalize=False)
    ref = ((1 - p.eps) * p.W_T)[:, None, None, None] * op.K[:, :, :, 0, :]
    assert np.abs(e - ref).max() < 1e-12


def test_kirchhoff_flat_field_two_term_zero_field():
    """App. E for the two-term atom at B = 0 (no lower-term splitting)."""
    p = tiny(n_z=1, n_nu=15, x_max=14, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2,
             eps=1e-2, atom=two_term_atom(2800.0, 24.305, 20.0))
    op = T.setup(p, {"normalize": False})
    e = T.sigma_apply(op, _flat(p), normalize=False)
    ref = ((1 - p.eps) * p.W_T)[:, None, None, None] * op.K[:, :, :, 0, :]
    assert np.abs(e - ref).max() < 1e-12


def test_branching_ratios_zero_field():
    """App. B normalisation: with a flat field at B = 0, the R_II part alone is
    alpha W_T eta_I and the R_III part alone is (beta - alpha) W_T eta_I."""
    p = tiny(n_z=1, n_nu=13, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=0.1)
    opII = T.setup(p, {"normalize": False, "no_RIII": True})
    opIII = T.setup(p, {"normalize": False, "no_RII": True})
    eII = T.sigma_apply(opII, _flat(p), normalize=False)
    eIII = T.sigma_apply(opIII, _flat(p), normalize=False)
    alpha = (1 - p.eps[0]) / (1 + p.atom.r_E)
    beta = 1 - p.eps[0]
    assert np.allclose(eII[..., 0], alpha * opII.K[..., 0, 0], rtol=1e-12, atol=1e-15)
    assert np.allclose(eIII[..., 0], (beta - alpha) * opII.K[..., 0, 0], rtol=1e-12, atol=1e-15)


def _axisymmetric_field(p, rng, aniso=0.5):
    """Flat-in-frequency, chi-independent (I, Q) field, |Q| < I."""
    ang = angular_grid(p.n_mu, p.n_chi)
    mu_vals = np.unique(ang["mu"])
    Iv = 1.0 + aniso * mu_vals ** 2 + 0.1 * rng.random(mu_vals.size)
    Qv = 0.2 * (rng.random(mu_vals.size) - 0.5)
    idx = np.searchsorted(mu_vals, ang["mu"])
    I = np.zeros((p.n_z, p.n_dir, p.n_nu, 4))
    I[..., 0] = Iv[idx][None, :, None]
    I[..., 1] = Qv[idx][None, :, None]
    return I, mu_vals, Iv, Qv


def _rayleigh_reference(mu_out, mu_vals, w_mu, Iv, Qv, W2):
    """Azimuth-averaged dipole (Rayleigh) phase matrix in Chandrasekhar's
    (I_l, I_r) basis, I_l in the vertical plane; W2 mixes with isotropic
    unpolarised emission.  The paper's Q (positive parallel to the limb) is
    I_r - I_l."""
    Il_in = 0.5 * (Iv - Qv)
    Ir_in = 0.5 * (Iv + Qv)
    m2, mp2 = mu_out[:, None] ** 2, mu_vals[None, :] ** 2
    Pll = 0.75 * (2 * (1 - m2) * (1 - mp2) + m2 * mp2)
    Plr = 0.75 * m2 * np.ones_like(mp2)
    Prl = 0.75 * mp2 * np.ones_like(m2)
    Prr = 0.75 * np.ones_like(m2 * mp2)
    iso = 0.5 * (Il_in + Ir_in)
    Il = W2 * (Pll * Il_in + Plr * Ir_in) + (1 - W2) * iso[None, :]
    Ir = W2 * (Prl * Il_in + Prr * Ir_in) + (1 - W2) * iso[None, :]
    Il = (Il * w_mu[None, :]).sum(1)
    Ir = (Ir * w_mu[None, :]).sum(1)
    return Il + Ir, Ir - Il


def test_rayleigh_scattering_zero_field_crd():
    """Field-free J 0->1 line in complete redistribution (alpha = 0, so only
    the R_III term of Eq. RIIIQKKp with beta = 1 - eps): for an axisymmetric
    flat-in-frequency field, eps^sc = (1 - eps) phi(u) x Rayleigh phase
    matrix (W2 = 1), with positive Q parallel to the limb."""
    rng = np.random.default_rng(5)
    p = tiny(n_z=1, n_nu=11, n_mu=6, n_chi=5, B=(0.0, 0.0, 0.0), a=1e-2, eps=0.05)
    op = T.setup(p, {"normalize": False, "alpha_zero": True})
    I, mu_vals, Iv, Qv = _axisymmetric_field(p, rng)
    e = T.sigma_apply(op, I, normalize=False)[0]
    t, wt = np.polynomial.legendre.leggauss(p.n_mu // 2)
    w_mu = np.concatenate([wt[::-1], wt]) / 4.0
    refI, refQ = _rayleigh_reference(op.ang["mu"], mu_vals, w_mu, Iv, Qv, 1.0)
    phi = op.K[0, :, :, 0, 0]
    assert np.allclose(e[..., 0], (1 - p.eps[0]) * phi * refI[:, None], rtol=1e-12, atol=1e-15)
    assert np.allclose(e[..., 1], (1 - p.eps[0]) * phi * refQ[:, None], rtol=1e-11, atol=1e-15)
    assert np.abs(e[..., 2:]).max() < 1e-15
    # limb-darkened field: emission towards the horizon is polarised parallel to the limb
    p2 = tiny(n_z=1, n_nu=11, n_mu=6, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=0.05)
    op2 = T.setup(p2, {"normalize": False, "alpha_zero": True})
    I2 = np.zeros((1, p2.n_dir, p2.n_nu, 4))
    I2[..., 0] = (0.3 + np.abs(op2.ang["mu"]))[None, :, None]
    e2 = T.sigma_apply(op2, I2, normalize=False)[0]
    horiz = np.argmin(np.abs(op2.ang["mu"]))
    assert e2[horiz, :, 1].min() > 0


def test_hanle_vertical_field_invariance():
    """Hanle effect (App. B beta with 2 pi i nu_{u,u'}): an axisymmetric
    field about a vertical B excites no Zeeman coherences, so the CRD
    emissivity equals the zero-field one for any field strength."""
    rng = np.random.default_rng(6)
    base = dict(n_z=1, n_nu=11, n_mu=4, n_chi=4, a=1e-2, eps=0.05)
    p0 = tiny(B=(0.0, 0.0, 0.0), **base)
    p1 = tiny(B=(500.0, 0.0, 0.0), **base)
    o = {"normalize": False, "alpha_zero": True, "zero_profile_shifts": True}
    op0, op1 = T.setup(p0, o), T.setup(p1, o)
    I, *_ = _axisymmetric_field(p0, rng)
    e0 = T.sigma_apply(op0, I, normalize=False)
    e1 = T.sigma_apply(op1, I, normalize=False)
    assert np.abs(e1 - e0).max() < 1e-13


def _sigma_factors(ct, c2, s2):
    """Angular factors of the pi (q=0) and sigma (q=+-1) components for
    (I, Q, U, V): field inclination cos = ct, sin^2 cos 2chi = c2, sin^2 sin 2chi = s2."""
    st2 = 1 - ct * ct
    return {0: np.array([st2, c2, s2, 0 * ct]),
            1: np.array([(1 + ct * ct) / 2, -c2 / 2, -s2 / 2, -ct]),
            -1: np.array([(1 + ct * ct) / 2, -c2 / 2, -s2 / 2, ct])}


def test_hanle_saturation_population_limit():
    """Hanle saturation (|nu_{u,u'}| >> Gamma in beta of App. B): coherences
    vanish and each Zeeman sublevel is fed and emits independently; written
    here with the pi/sigma angular factors only (no dipole vectors)."""
    rng = np.random.default_rng(7)
    p = tiny(n_z=1, n_nu=11, n_mu=4, n_chi=5, B=(3e8, 1.1, 0.4), a=1e-2, eps=0.05)
    op = T.setup(p, {"normalize": False, "alpha_zero": True, "zero_profile_shifts": True})
    I = np.zeros((1, p.n_dir, p.n_nu, 4))
    base = 1.0 + rng.random(p.n_dir)
    I[..., 0] = base[None, :, None]
    for j in (1, 2, 3):
        I[..., j] = (0.3 * (rng.random(p.n_dir) - 0.5) * base)[None, :, None]
    e = T.sigma_apply(op, I, normalize=False)[0]
    th, ch = p.B[0, 1], p.B[0, 2]
    bh = np.array([np.sin(th) * np.cos(ch), np.sin(th) * np.sin(ch), np.cos(th)])
    ea, eb, dd = op.ang["e_a"], op.ang["e_b"], op.ang["dirs"]
    ba, bb, ct = ea @ bh, eb @ bh, dd @ bh
    g = _sigma_factors(ct, ba * ba - bb * bb, 2 * ba * bb)          # each [4, n_dir]
    pop = {q: (op.ang["w"] * (g[q] * I[0, :, 0, :].T).sum(0)).sum() / 2 for q in g}
    ref = 1.5 * (1 - p.eps[0]) * sum(pop[q] * g[q] for q in g)      # [4, n_dir]
    phi = op.K[0, :, :, 0, 0]
    expect = phi[:, :, None] * ref.T[:, None, :]
    assert np.abs(e - expect).max() < 2e-6 * np.abs(expect).max()


def test_two_term_fine_structure_limit():
    """Two-term atom with fine structure >> Doppler width, B = 0, CRD: the
    2S1/2 - 2P1/2 component is unpolarisable and 2S1/2 - 2P3/2 scatters with
    W2 = 1/2 (residual J-state interference ~ a/splitting)."""
    rng = np.random.default_rng(8)
    atom = two_term_atom(2800.0, 24.305, 20.0)
    p = tiny(n_z=1, n_nu=41, x_max=20, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2,
             eps=0.05, atom=atom)
    op = T.setup(p, {"normalize": False, "alpha_zero": True})
    I, mu_vals, Iv, Qv = _axisymmetric_field(p, rng, aniso=6.0)
    e = T.sigma_apply(op, I, normalize=False)[0]
    t, wt = np.polynomial.legendre.leggauss(p.n_mu // 2)
    w_mu = np.concatenate([wt[::-1], wt]) / 4.0
    rI, rQ = _rayleigh_reference(op.ang["mu"], mu_vals, w_mu, Iv, Qv, 0.5)
    k32 = int(np.argmin(np.abs(p.x + 10.0)))    # J=3/2 (higher energy) at u = -10
    k12 = int(np.argmin(np.abs(p.x - 10.0)))
    assert np.abs(e[:, k32, 1] / e[:, k32, 0] - rQ / rI).max() < 2e-3
    assert np.abs(e[:, k12, 1] / e[:, k12, 0]).max() < 2e-3
    assert np.abs(rQ / rI).max() > 0.05          # the test field is anisotropic enough


# ---------------------------------------------------------------- operator properties

def test_sigma_linearity_and_azimuthal_equivariance():
    """Sigma is linear in I (Sect. 2.5); rotating the field azimuth by one
    grid step permutes the chi index of the emissivity (Sect. 4.2 grid)."""
    rng = np.random.default_rng(9)
    kw = dict(n_z=2, n_nu=13, n_mu=4, n_chi=4, a=2e-2, eps=0.03, v_z=0.0)
    p = tiny(B=(40.0, 1.0, 0.3), **kw)
    pr = tiny(B=(40.0, 1.0, 0.3 + 2 * np.pi / 4), **kw)
    op, opr = T.setup(p), T.setup(pr)
    I1 = rng.random((p.n_z, p.n_dir, p.n_nu, 4))
    I2 = rng.random((p.n_z, p.n_dir, p.n_nu, 4))
    s1, s2 = T.sigma_apply(op, I1), T.sigma_apply(op, I2)
    assert np.allclose(T.sigma_apply(op, 2.0 * I1 - 0.5 * I2), 2.0 * s1 - 0.5 * s2,
                       rtol=1e-12, atol=1e-14)

    def rot(A):
        B = A.reshape(A.shape[0], p.n_mu, p.n_chi, *A.shape[2:])
        return np.roll(B, 1, axis=2).reshape(A.shape)
    assert np.allclose(T.sigma_apply(opr, rot(I1)), rot(s1), rtol=1e-11, atol=1e-14)


def test_delo_weights_series_and_identity():
    """Sect. 3 DELO-linear weights: the small-x series joins the closed form,
    and psi_u + psi_c = 1 - e^{-x} (integral of the linear interpolant)."""
    x = np.array([1e-9, 1e-4, 9.99e-3, 0.0999, 0.1001, 0.3, 2.0, 30.0])
    pu, pc, ex = T._psi(x)
    assert np.allclose(pu + pc, -np.expm1(-x), rtol=1e-14)
    for xv, a, b in zip(x, pu, pc):
        ru = quad(lambda s: np.exp(-s) * s / xv, 0, xv, epsabs=0, epsrel=2e-14)[0]
        rc = quad(lambda s: np.exp(-s) * (1 - s / xv), 0, xv, epsabs=0, epsrel=2e-14)[0]
        assert abs(a - ru) < 1e-12 * ru
        assert abs(b - rc) < 1e-12 * rc


def test_formal_solver_milne_eddington_exact():
    """Unno-Rachkovsky / Milne-Eddington: K/eta_I constant along the ray and a
    source W = B0 + B1 tau_line in LTE (eps = W K e0).  The exact solution is
    I = W e0 + (B1 mu/r) (K/eta_I)^-1 e0, r = eta_I/eta_0; DELO-linear is exact
    for it (linear effective source) when entered at the bottom boundary."""
    p = tiny(n_z=9, n_nu=15, x_max=5, n_mu=4, n_chi=4, B=(800.0, 0.8, 0.4), a=2e-2, eps=0.1,
             tau_top=1e-2, tau_bot=30.0)
    op = T.setup(p, {"normalize": False})
    B0, B1 = 0.7, 0.35
    Wt = B0 + B1 * p.tau_line
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    ratio = op.K[..., 0, 0] / op.eta0[:, None, None]
    Khat = op.K / op.K[..., 0:1, 0:1]
    e0 = np.array([1.0, 0, 0, 0])
    mu = op.ang["mu"]
    part = np.einsum("zonij,j->zoni", np.linalg.inv(Khat), e0)
    Iex = Wt[:, None, None, None] * e0 + (B1 * mu[None, :, None, None] / ratio[..., None]) * part
    I = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0])
    up = mu > 0
    assert np.abs(I[:, up] - Iex[:, up]).max() < 1e-12


def test_formal_solver_pure_absorption():
    """Sect. 3: with no emissivity the bottom radiation is attenuated as
    exp(-tau) along each upward ray (field-free line, diagonal K)."""
    p = tiny(n_z=6, n_nu=9, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=0.1)
    op = T.setup(p, {"normalize": False})
    I = T.formal_solve(op, np.zeros((p.n_z, p.n_dir, p.n_nu, 4)), boundary=True)
    mu = op.ang["mu"]
    r = op.K[..., 0, 0] / op.eta0[:, None, None]
    for o in np.where(mu > 0)[0]:
        tau = np.vstack([np.zeros(p.n_nu), np.cumsum(0.5 * (r[1:, o] + r[:-1, o])
                         * np.abs(np.diff(p.tau_line))[:, None] / mu[o], axis=0)])
        assert np.allclose(I[:, o, :, 0], np.exp(-tau), rtol=1e-13)
    assert np.abs(I[:, mu < 0]).max() == 0.0


def test_gmres_matches_dense_solve():
    """The linear system (Id - Lambda Sigma) I = Lambda eps_th + t
    (Eq. linear_system) has one solution: FP64 GMRES equals dense LU."""
    p = tiny(n_z=3, n_nu=9, x_max=5, n_mu=4, n_chi=3, B=(25.0, 1.2, 0.3), a=2e-2, eps=0.05,
             v_z=1.0, seed=11)
    op = T.setup(p)
    Ig = T.solve(op, tol=1e-13)
    Id = T.solve(op, method="dense")
    assert np.abs(Ig - Id).max() < 1e-11 * np.abs(Id).max()
    r = T.rhs(op) - T.apply_operator(op, Id)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(T.rhs(op))


# ---------------------------------------------------------------- angle-averaged PRD (Sect. 5.2, Eq. R_AA)

def test_aa_kernel_theta_rule_matches_adaptive_integral():
    """The angle-averaged kernel (1/2) int_0^pi sin(Theta) M(Theta) dTheta,
    evaluated with the 25-node Gauss-Legendre rule of App. C, equals an
    adaptive Theta integral of the angle-dependent kernel."""
    from scipy.integrate import quad_vec
    from oracle.redistribution import kernel_matrix_aa
    b = SplineBasis(np.linspace(-4.0, 4.0, 9))
    for a, s in ((1e-2, 0.3), (5e-2, -1.0)):
        Mg = kernel_matrix_aa(s, a, 1.1, b)
        Mq, _ = quad_vec(lambda th: (0.5 * np.sin(th) * kernel_matrix(th, s, a, 1.1, b)).ravel(),
                         0.0, np.pi, epsrel=1e-10, epsabs=1e-13)
        assert np.abs(Mg - Mq.reshape(Mg.shape)).max() < 1e-8 * np.abs(Mg).max()


def test_aa_and_ad_agree_on_a_flat_field():
    """For a flat incident field every kernel row integrates to sqrt(pi) W
    whatever Theta is, so the angle-averaged and angle-dependent emissivities
    coincide (moving, magnetised, seeded atmosphere; unnormalised Sigma)."""
    p = tiny(n_z=3, n_nu=13, x_max=6, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.4), a=2e-2, eps=3e-2,
             v_z=1.5, seed=5)
    ad = T.sigma_apply(T.setup(p, {"normalize": False}), _flat(p), normalize=False)
    aa = T.sigma_apply(T.setup(p, {"normalize": False, "aa": True}), _flat(p), normalize=False)
    assert np.abs(aa - ad).max() < 1e-10 * np.abs(ad).max()


def test_aa_and_ad_solutions_identical_without_rII():
    """With alpha = 0 only R_III scatters, which does not depend on Theta:
    angle-averaged and angle-dependent solutions are the same."""
    p = tiny(n_z=3, n_nu=9, x_max=5, n_mu=4, n_chi=3, B=(25.0, 1.2, 0.3), a=2e-2, eps=0.05, seed=11)
    s_ad = T.solve(T.setup(p, {"alpha_zero": True}), tol=1e-13)
    s_aa = T.solve(T.setup(p, {"alpha_zero": True, "aa": True}), tol=1e-13)
    assert np.abs(s_aa - s_ad).max() < 1e-12 * np.abs(s_ad).max()


def test_aa_differs_from_ad_for_an_anisotropic_field():
    """Guard against an AA switch that changes nothing: for a strongly
    anisotropic, frequency-structured field the two kernels give different
    emissivities."""
    p = tiny(n_z=2, n_nu=13, x_max=6, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=3e-2)
    rng = np.random.default_rng(3)
    I = rng.random((p.n_z, p.n_dir, p.n_nu, 4))
    ad = T.sigma_apply(T.setup(p, {"normalize": False}), I, normalize=False)
    aa = T.sigma_apply(T.setup(p, {"normalize": False, "aa": True}), I, normalize=False)
    assert np.abs(aa - ad).max() > 1e-3 * np.abs(ad).max()


# ---------------------------------------------------------------- limits the transfer problem fixes

def _unpolarisable_atom():
    """J_l = 1/2 -> J_u = 1/2: no alignment can be carried (W_2 = 0)."""
    import dataclasses
    return dataclasses.replace(two_level_atom(), J_l=0.5, J_u=0.5, g_l=2.0, g_u=2.0 / 3.0)


def test_unpolarisable_line_scatters_no_polarisation():
    """Unpolarised limit: for a J 1/2 -> 1/2 line without a magnetic field the
    scattered radiation from any unpolarised, anisotropic, frequency-dependent
    field has Q = U = V = 0, and so has the solution."""
    p = tiny(n_z=3, n_nu=11, x_max=5, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=3e-2,
             atom=_unpolarisable_atom())
    op = T.setup(p)
    rng = np.random.default_rng(1)
    I = np.zeros((p.n_z, p.n_dir, p.n_nu, 4))
    I[..., 0] = rng.random(I.shape[:-1])
    e = T.sigma_apply(op, I)
    assert np.abs(e[..., 1:]).max() < 1e-14 * np.abs(e[..., 0]).max()
    sol = T.solve(op, tol=1e-12)
    assert np.abs(sol[..., 1:]).max() < 1e-13 * np.abs(sol[..., 0]).max()


def _flux_above(nz, nn):
    p = tiny(n_z=nz, n_nu=nn, x_max=8, n_mu=4, n_chi=2, B=(0.0, 0.0, 0.0), a=1e-3, eps=1e-9,
             tau_top=1e-3, tau_bot=1e2, atom=_unpolarisable_atom())
    op = T.setup(p)
    I = T.solve(op, tol=1e-12)
    wx = np.full(p.n_nu, p.x[1] - p.x[0])
    wx[[0, -1]] *= 0.5
    F = np.einsum("o,o,zon,n->z", op.ang["w"], op.ang["mu"], I[..., 0], wx)
    top = nz // 2                                   # heights above the bottom boundary layer
    return np.abs(F[top:] / F[-1] - 1.0).max()


def test_pure_scattering_conserves_flux():
    """Energy conservation: with no photon destruction and no thermal source
    the frequency- and angle-integrated net flux is constant in height up to
    discretisation error, which falls when the grids are refined (above the
    boundary layer at the illuminated bottom)."""
    coarse, fine = _flux_above(8, 21), _flux_above(16, 41)
    assert fine < 1e-4
    assert fine < 0.5 * coarse


def test_sqrt_eps_law_for_complete_redistribution():
    """Semi-infinite isothermal atmosphere, constant destruction probability,
    complete redistribution (alpha = 0, an unpolarisable line): the surface
    source function tends to sqrt(eps) B; the error falls under depth-grid
    refinement."""
    errs = []
    for nz in (24, 40):
        p = tiny(n_z=nz, n_nu=13, x_max=4.0, n_mu=4, n_chi=1, B=(0.0, 0.0, 0.0), a=1e-3, eps=0.04,
                 tau_top=1e-4, tau_bot=1e4, atom=_unpolarisable_atom())
        op = T.setup(p, {"alpha_zero": True})
        I = T.solve(op, tol=1e-12)
        e = T.sigma_apply(op, I) + op.eps_th
        S = e[-1, :, :, 0] / op.K[-1, :, :, 0, 0]
        assert np.ptp(S) < 1e-10 * S.mean()          # CRD: frequency- and angle-independent
        errs.append(abs(S.mean() / np.sqrt(0.04) - 1.0))
    assert errs[1] < 0.05
    assert errs[1] < errs[0] / 1.8


def test_delopar_weights_reproduce_the_exponential_moments():
    """The parabolic weights integrate e^{-t} times 1, t and t^2 exactly over
    [0, m] with the nodes t = m (upwind), 0 (current), -p (downwind)."""
    from scipy.integrate import quad
    for m, p in ((1e-4, 2e-4), (0.05, 0.3), (0.49, 0.51), (0.7, 0.2), (3.0, 5.0), (40.0, 1.0)):
        wM, wO, wP = T._psi_parabolic(np.array([m]), np.array([p]))
        for k, nodes in ((0, (1.0, 1.0, 1.0)), (1, (m, 0.0, -p)), (2, (m * m, 0.0, p * p))):
            ref = quad(lambda t: t ** k * np.exp(-t), 0.0, m, epsabs=0.0, epsrel=1e-13)[0]
            got = wM[0] * nodes[0] + wO[0] * nodes[1] + wP[0] * nodes[2]
            assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-18


def test_delopar_exact_for_a_quadratic_source():
    """Static, field-free atmosphere (K' = 0) with eta_I / eta_0 constant in
    height and the source W = B0 + B1 tau + B2 tau^2: the emerging intensity of
    a semi-infinite medium is S + mu dS/dtau_v + mu^2 d2S/dtau_v^2.  Entered at
    the bottom with that value, DELOPAR reproduces it at every point that has a
    downwind neighbour (the last point takes the linear step); DELO-linear does
    not."""
    p = tiny(n_z=12, n_nu=9, x_max=4, n_mu=4, n_chi=2, B=(0.0, 0.0, 0.0), a=2e-2, eps=0.1,
             tau_top=1e-2, tau_bot=20.0)
    op = T.setup(p, {"normalize": False})
    B0, B1, B2 = 0.4, 0.3, 0.05
    tl = p.tau_line
    Wt = B0 + B1 * tl + B2 * tl * tl
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    r = op.K[..., 0, 0] / op.eta0[:, None, None]
    assert np.abs(r - r[0:1]).max() < 1e-12 * np.abs(r).max()
    mu = op.ang["mu"]
    Iex = np.zeros_like(eps)
    Iex[..., 0] = (Wt[:, None, None] + mu[None, :, None] * (B1 + 2 * B2 * tl)[:, None, None] / r
                   + 2 * B2 * (mu[None, :, None] / r) ** 2)
    up = mu > 0
    Ip = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0], scheme="delopar")
    Il = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0], scheme="linear")
    rel_p = np.abs(Ip[:-1, up, :, 0] - Iex[:-1, up, :, 0]) / np.abs(Iex[:-1, up, :, 0])
    rel_l = np.abs(Il[:-1, up, :, 0] - Iex[:-1, up, :, 0]) / np.abs(Iex[:-1, up, :, 0])
    assert rel_p.max() < 1e-12
    assert rel_l.max() > 1e-4
    assert np.abs(Ip[..., 1:]).max() < 1e-12 * np.abs(Ip[..., 0]).max()


def test_delopar_exact_for_milne_eddington():
    """The Milne-Eddington case above (constant K/eta_I with dichroism and
    dispersion, linear source) is integrated exactly by DELOPAR too: the
    parabola through a linear source is the line, and K'I is linear along the
    ray."""
    p = tiny(n_z=9, n_nu=15, x_max=5, n_mu=4, n_chi=4, B=(800.0, 0.8, 0.4), a=2e-2, eps=0.1,
             tau_top=1e-2, tau_bot=30.0)
    op = T.setup(p, {"normalize": False})
    B0, B1 = 0.7, 0.35
    Wt = B0 + B1 * p.tau_line
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    ratio = op.K[..., 0, 0] / op.eta0[:, None, None]
    Khat = op.K / op.K[..., 0:1, 0:1]
    e0 = np.array([1.0, 0, 0, 0])
    mu = op.ang["mu"]
    part = np.einsum("zonij,j->zoni", np.linalg.inv(Khat), e0)
    Iex = Wt[:, None, None, None] * e0 + (B1 * mu[None, :, None, None] / ratio[..., None]) * part
    I = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0], scheme="delopar")
    up = mu > 0
    assert np.abs(I[:, up] - Iex[:, up]).max() < 1e-12


def test_rayleigh_phase_matrix_closed_forms():
    """The continuum scattering matrix R = (3/4) Re Tr(Acart_i Acart_j) is the
    dipole (Rayleigh) phase matrix: R_II = 3/4 (1 + cos^2 Theta), linear
    polarisation sqrt(R_QI^2 + R_UI^2) = 3/4 sin^2 Theta, no circular
    polarisation from linear and back, R_VV = 3/2 cos Theta, and an isotropic
    unpolarised field scatters into itself (sum_x w_x R_II = 1)."""
    ang = angular_grid(6, 5)
    acart = T._acart(ang)
    dirs, w = ang["dirs"], ang["w"]
    for o in range(dirs.shape[0]):
        tot = 0.0
        for x in range(dirs.shape[0]):
            R = T.rayleigh_matrix(acart, o, x)
            c = float(dirs[o] @ dirs[x])
            assert abs(R[0, 0] - 0.75 * (1 + c * c)) < 1e-14
            assert abs(np.hypot(R[1, 0], R[2, 0]) - 0.75 * (1 - c * c)) < 1e-14
            assert abs(R[3, 0]) < 1e-14 and abs(R[0, 3]) < 1e-14
            assert abs(R[3, 1]) < 1e-14 and abs(R[3, 2]) < 1e-14
            assert abs(R[3, 3] - 1.5 * c) < 1e-14
            tot += w[x] * R[0, 0]
        assert abs(tot - 1.0) < 1e-14


def test_continuum_flat_field():
    """With a continuum, the normalised Sigma of the flat field (W_T, 0, 0, 0)
    is the line's (1 - eps) W_T eta (App. E) plus sigma_c W_T on Stokes I: the
    continuum scatters an isotropic unpolarised field into itself."""
    p = tiny(n_z=3, n_nu=13, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=3e-2, cont=(0.2, 0.4))
    op = T.setup(p)
    e = T.sigma_apply(op, _flat(p))
    kc = p.kappa_c * op.eta0[:, None]
    sc = p.sigma_c * op.eta0[:, None]
    eta_line = op.K[:, :, :, 0, :].copy()
    eta_line[..., 0] -= (kc + sc)[:, None, :]
    ref = ((1 - p.eps) * p.W_T)[:, None, None, None] * eta_line
    ref[..., 0] += (sc * p.W_T[:, None])[:, None, :]
    assert np.abs(e - ref).max() < 1e-12 * np.abs(ref).max()


def test_continuum_lte_column_keeps_the_planck_value():
    """A pure-absorption line (eps = 1) with continuum absorption and a
    constant W_T: the emissivity W_T (eta_line + kappa_c e_0) is K W_T e_0, so
    the exact solution on upward rays is I = W_T e_0, which the right-hand side
    (the formal solution of the thermal emissivity with the bottom boundary)
    reproduces for every field geometry."""
    p = tiny(n_z=7, n_nu=11, n_mu=4, n_chi=3, B=(300.0, 0.7, 1.1), a=1e-2, eps=1.0, cont=(0.5, 0.0))
    op = T.setup(p)
    b = T.rhs(op)
    up = op.ang["mu"] > 0
    ref = np.zeros_like(b[:, up])
    ref[..., 0] = p.W_T[:, None, None]
    assert np.abs(b[:, up] - ref).max() < 1e-12


def test_kernel_rows_mirror_symmetry():
    """The comoving kernel rows of shift s and -s on a grid symmetric about 0
    are conjugate mirror images, M_s[n][m] = conj(M_-s[N-1-n][N-1-m]): the
    redistribution function is even under reversing both frequencies except
    for its dispersion part, which is odd (w(-x + ia) = conj w(x + ia)), and the
    spline basis of a symmetric grid is mirror symmetric.  A wrong sign of the
    shift or of the dispersion part breaks it."""
    from oracle.redistribution import kernel_matrix
    x = np.linspace(-6.0, 6.0, 21)
    basis = SplineBasis(x)
    for th in (0.0, 0.4, 1.7, np.pi):
        for s in (0.0, 0.45):
            Mp = kernel_matrix(th, s, 0.03, 1.2, basis)
            Mm = kernel_matrix(th, -s, 0.03, 1.2, basis)
            scale = np.abs(Mp).max()
            assert np.abs(Mp - np.conj(Mm[::-1, ::-1])).max() < 1e-12 * scale
            if s and th:
                assert np.abs(Mp - Mm[::-1, ::-1]).max() > 1e-3 * scale     # not without the conjugate
