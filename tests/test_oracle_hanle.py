"""Pins of the oracle's magnetic and unpolarised limits at general parameters.

* Hanle effect at intermediate field strengths (App. B: the branching ratio
  beta carries the Zeeman coherence term 2 pi i nu_{u,u'}).  For a J 0 -> 1
  line in complete redistribution (alpha = 0, so only the R_III term of
  Eq. RIIIQKKp with weight beta), with every Zeeman component at the
  zero-field frequency in the profiles, the atom is the classical isotropic
  oscillator: the radiation excites the dipole tensor rho_0 = J (the
  coherency tensor of the incident field averaged over directions), the
  pattern precesses right-handedly about +B at 2 pi nu_L g_u (a positive
  Lande factor means a magnetic moment opposite to the angular momentum) and
  decays at Gamma = Gamma_R + Gamma_I, so the emitting tensor is
      rho = Gamma int_0^inf e^{-Gamma t} R(t) J R(t)^T dt,
  and each direction emits the transverse projection of rho.  In the frame of
  B the components A_Q = T_xx - T_yy + 2i T_xy (Q = 2) and T_xz + i T_yz
  (Q = 1) are multiplied by 1/(1 - i Q H), H = 2 pi nu_L g_u / Gamma, and
  T_zz is unchanged: the K = 2 Hanle closed form.  Everything below is built
  from physical constants, the direction grid and this picture; none of it
  uses the oracle's dipole vectors, spherical-tensor conventions or beta.
* Unpolarised limit: a J 1/2 -> 1/2 line at B = 0 carries no alignment, so
  Stokes I obeys the scalar angle-dependent PRD scattering integral
      eps_I(Omega, u) = sum_{Omega'} w' int du' [alpha Re F(Theta, u', u)/pi
                        + (beta - alpha) phi(u) phi(u')] S[I(Omega', .)](u'),
  written here with the paper's F (Sect. 2.4), scipy's spline and adaptive
  quadrature: a scalar solver of its own.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.interpolate import CubicSpline
from scipy.special import wofz

from workloads import tiny, two_level_atom
from oracle import transfer as T

C_CGS = 2.99792458e10          # cm/s
K_BOLTZ = 1.380649e-16         # erg/K
AMU_G = 1.66053906660e-24      # g
MUB_OVER_H = 1.39962449361e6   # Bohr magneton / Planck constant, Hz per gauss


def _grid(n_mu, n_chi):
    """Double Gauss-Legendre mu (ascending) x trapezoid chi, weights over dOmega/4pi,
    and the Stokes basis: e1 horizontal (parallel to the limb), e2 = Omega x e1."""
    t, wt = np.polynomial.legendre.leggauss(n_mu // 2)
    mp = 0.5 * (t + 1.0)
    mu1 = np.concatenate([-mp[::-1], mp])
    w1 = np.concatenate([wt[::-1], wt]) / 4.0
    chi1 = 2.0 * np.pi * np.arange(n_chi) / n_chi
    mu = np.repeat(mu1, n_chi)
    chi = np.tile(chi1, mu1.size)
    w = np.repeat(w1, n_chi) / n_chi
    st = np.sqrt(1.0 - mu * mu)
    om = np.stack([st * np.cos(chi), st * np.sin(chi), mu], axis=1)
    e1 = np.stack([-np.sin(chi), np.cos(chi), 0 * chi], axis=1)
    e2 = np.cross(om, e1)
    return om, w, e1, e2


def _coherency(I, Q, U, e1, e2):
    """3x3 coherency tensor of a beam with Stokes (I, Q, U) (V = 0)."""
    return 0.5 * ((I + Q) * np.outer(e1, e1) + (I - Q) * np.outer(e2, e2)
                  + U * (np.outer(e1, e2) + np.outer(e2, e1)))


def _stokes(rho, e1, e2):
    """(I, Q, U, V) emitted along e1 x e2 by a real symmetric dipole tensor."""
    a, b, c = e1 @ rho @ e1, e2 @ rho @ e2, e1 @ rho @ e2
    return np.array([a + b, a - b, 2.0 * c, 0.0])


def _precession_average(J, bhat, H):
    """Gamma int e^{-Gamma t} R J R^T dt for right-handed rotation about bhat at
    angular speed H Gamma: the resolvent (Id - H L)^{-1} of the generator
    L(rho) = G rho - rho G, G the cross-product matrix of bhat."""
    G = np.array([[0.0, -bhat[2], bhat[1]], [bhat[2], 0.0, -bhat[0]], [-bhat[1], bhat[0], 0.0]])
    L = np.kron(G, np.eye(3)) - np.kron(np.eye(3), G.T)       # row-major vec(G rho - rho G)
    v = np.linalg.solve(np.eye(9) - H * L, J.reshape(9))
    return v.reshape(3, 3)


def _hanle_case(H, theta_B, chi_B, seed):
    """Problem with a J 0 -> 1 line whose field gives Hanle parameter H, a
    smooth anisotropic, linearly polarised incident field, the oracle's
    emissivity and this module's expectation."""
    atom = two_level_atom()
    a, eps, T0 = 1e-2, 0.05, 6000.0
    nu0 = C_CGS / (atom.lambda0_A * 1e-8)
    dnuD = nu0 / C_CGS * np.sqrt(2.0 * K_BOLTZ * T0 / (atom.mass_amu * AMU_G))
    gamma = 4.0 * np.pi * a * dnuD / (1.0 + atom.r_E)            # Gamma_R + Gamma_I
    B = H * gamma / (2.0 * np.pi * MUB_OVER_H * atom.g_u)
    p = tiny(n_z=1, n_nu=9, x_max=4.0, n_mu=4, n_chi=5, B=(B, theta_B, chi_B), a=a, eps=eps, T=T0)
    op = T.setup(p, {"normalize": False, "alpha_zero": True, "zero_profile_shifts": True})
    om, w, e1, e2 = _grid(p.n_mu, p.n_chi)
    assert np.allclose(om, op.ang["dirs"], atol=1e-15)
    rng = np.random.default_rng(seed)
    Iv = 1.0 + 0.6 * om[:, 2] ** 2 + 0.2 * rng.random(len(w))
    Qv = 0.3 * (rng.random(len(w)) - 0.5) * Iv
    Uv = 0.3 * (rng.random(len(w)) - 0.5) * Iv
    I = np.zeros((1, p.n_dir, p.n_nu, 4))
    I[0, :, :, 0] = Iv[:, None]
    I[0, :, :, 1] = Qv[:, None]
    I[0, :, :, 2] = Uv[:, None]
    e = T.sigma_apply(op, I, normalize=False)[0]
    J = sum(w[k] * _coherency(Iv[k], Qv[k], Uv[k], e1[k], e2[k]) for k in range(len(w)))
    bhat = np.array([np.sin(theta_B) * np.cos(chi_B), np.sin(theta_B) * np.sin(chi_B), np.cos(theta_B)])
    rho = _precession_average(J, bhat, H)
    phi = wofz(p.x + 1j * a).real / np.sqrt(np.pi)              # T = T_ref: u = x
    expect = 1.5 * (1.0 - eps) * phi[None, :, None] * np.array(
        [_stokes(rho, e1[k], e2[k]) for k in range(len(w))])[:, None, :]
    return op, e, expect, J, rho, bhat, (om, e1, e2)


@pytest.mark.parametrize("H", [0.3, 1.0, 3.0])
def test_hanle_intermediate_fields_precessing_oscillator(H):
    """App. B beta at H = 0.3, 1, 3 on an inclined field: the oracle's CRD
    emissivity equals the precessing-oscillator emission in all four Stokes
    parameters, at every direction and frequency."""
    op, e, expect, *_ = _hanle_case(H, 1.1, 0.4, seed=11)
    assert np.abs(e - expect).max() < 1e-12 * np.abs(expect).max()
    # the field matters: against the zero-field (Rayleigh) emission the change is large
    _, _, zero, *_ = _hanle_case(0.0, 1.1, 0.4, seed=11)
    assert np.abs(expect - zero).max() > 0.02 * np.abs(expect[..., 0]).max()


def _bframe_components(T3, bhat):
    """A_0 = T_zz, A_1 = T_xz + i T_yz, A_2 = T_xx - T_yy + 2i T_xy in a frame
    with z along bhat."""
    z = bhat
    x = np.cross([0.0, 0.0, 1.0], z) if abs(z[2]) < 0.9 else np.cross([1.0, 0.0, 0.0], z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    Tb = R @ T3 @ R.T
    return Tb[2, 2], Tb[0, 2] + 1j * Tb[1, 2], Tb[0, 0] - Tb[1, 1] + 2j * Tb[0, 1]


@pytest.mark.parametrize("H", [0.3, 1.0, 3.0])
def test_hanle_bframe_multipoles_closed_form(H):
    """The K = 2 Hanle closed form read off the oracle's output: the emitting
    dipole tensor is recovered from the emitted (I, Q, U) over all directions
    by least squares, and its components in the frame of B are those of the
    radiation tensor times 1/(1 - i Q H) for Q = 0, 1, 2 (a sign error in
    the coherence term of beta turns this into 1/(1 + i Q H); nu for omega
    rescales H by 2 pi)."""
    op, e, expect, J, rho, bhat, (om, e1, e2) = _hanle_case(H, 0.8, 2.0, seed=12)
    n0 = 4                                      # line centre
    eps, phi0 = 0.05, wofz(0.0 + 1j * 1e-2).real / np.sqrt(np.pi)
    rows, rhs = [], []
    basis = []
    for i in range(3):
        for j in range(i, 3):
            Bm = np.zeros((3, 3))
            Bm[i, j] = Bm[j, i] = 1.0
            basis.append(Bm)
    for k in range(len(om)):
        s = np.array([_stokes(Bm, e1[k], e2[k])[:3] for Bm in basis]).T   # [3 Stokes, 6]
        rows.append(s)
        rhs.append(e[k, n0, :3] / (1.5 * (1.0 - eps) * phi0))
    coef, *_ = np.linalg.lstsq(np.concatenate(rows), np.concatenate(rhs), rcond=None)
    rho_fit = sum(c * Bm for c, Bm in zip(coef, basis))
    A_rho = _bframe_components(rho_fit, bhat)
    A_J = _bframe_components(J, bhat)
    for q in range(3):
        assert abs(A_rho[q] - A_J[q] / (1.0 - 1j * q * H)) < 1e-11 * abs(J).max()
    # the closed form is not trivially met: each Q component carries weight here
    assert min(abs(A_J[1]), abs(A_J[2])) > 1e-3 * abs(J).max()


def test_hanle_rotation_sense_of_u():
    """Sign of the Hanle rotation: a vertical field and a field-free emission
    with U = 0 at every direction of one azimuth ring (a chi-symmetric,
    Q-only incident field), so any U comes from the rotation; with B along
    +z the emission direction's linear polarisation turns right-handedly
    about +z, which flips the sign of U with the field direction."""
    op_up, e_up, ex_up, *_ = _hanle_case(1.0, 0.3, 0.0, seed=13)
    op_dn, e_dn, ex_dn, *_ = _hanle_case(1.0, np.pi - 0.3, np.pi, seed=13)
    assert np.abs(e_up - ex_up).max() < 1e-12 * np.abs(ex_up).max()
    assert np.abs(e_dn - ex_dn).max() < 1e-12 * np.abs(ex_dn).max()
    # reversing B reverses the precession: U of the two emissions differ
    assert np.abs(e_up[..., 2] - e_dn[..., 2]).max() > 1e-3 * np.abs(e_up[..., 0]).max()


# ---------------------------------------------------------------- unpolarised limit (scalar PRD)

def _F(theta, up, u, a):
    """R_II angle-dependent redistribution function of Sect. 2.4 (0 < Theta < pi)."""
    s, c = np.sin(theta / 2.0), np.cos(theta / 2.0)
    return np.exp(-((u - up) / (2.0 * s)) ** 2) * wofz((u + up) / (2.0 * c) + 1j * a / c) / np.sin(theta)


def test_unpolarised_limit_matches_a_scalar_prd_integral():
    """J 1/2 -> 1/2 at B = 0, R_II (angle-dependent) + R_III, no velocity: the
    oracle's Stokes-I emissivity equals the scalar scattering integral above,
    evaluated with adaptive quadrature against scipy's not-a-knot spline of
    each incident direction's profile (flat outside the grid), and Q = U = V
    stay zero."""
    import dataclasses
    atom = dataclasses.replace(two_level_atom(), J_l=0.5, J_u=0.5, g_l=2.0, g_u=2.0 / 3.0)
    a, eps = 5e-2, 0.1
    p = tiny(n_z=1, n_nu=9, x_max=3.0, n_mu=2, n_chi=3, B=(0.0, 0.0, 0.0), a=a, eps=eps, atom=atom)
    op = T.setup(p, {"normalize": False})
    rng = np.random.default_rng(21)
    I = np.zeros((1, p.n_dir, p.n_nu, 4))
    I[0, :, :, 0] = 1.0 + rng.random((p.n_dir, p.n_nu))
    e = T.sigma_apply(op, I, normalize=False)[0]
    om, w, _, _ = _grid(p.n_mu, p.n_chi)
    r_E = atom.r_E
    alpha = (1.0 - eps) / (1.0 + r_E)            # Gamma_R / (Gamma_R + Gamma_I + Gamma_E)
    beta = 1.0 - eps                             # Gamma_R / (Gamma_R + Gamma_I)
    x = p.x
    phi = lambda u: wofz(u + 1j * a).real / np.sqrt(np.pi)
    splines = [CubicSpline(x, I[0, k, :, 0], bc_type="not-a-knot") for k in range(p.n_dir)]
    Sflat = lambda k, u: splines[k](np.clip(u, x[0], x[-1]))
    lo, hi = x[0] - 40.0, x[-1] + 40.0
    brk = list(x)
    # R_III incoming integral over the whole line: spline on the grid, the edge
    # values times the profile's Lorentzian tails beyond it
    tail_lo = quad(phi, -np.inf, x[0], epsabs=0, epsrel=1e-13, limit=400)[0]
    tail_hi = quad(phi, x[-1], np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    r3 = [quad(lambda u, k=k: phi(u) * Sflat(k, u), x[0], x[-1], points=brk[1:-1], limit=400,
               epsabs=0, epsrel=1e-13)[0] + I[0, k, 0, 0] * tail_lo + I[0, k, -1, 0] * tail_hi
          for k in range(p.n_dir)]
    ref = np.zeros((p.n_dir, p.n_nu))
    for o in range(p.n_dir):
        for n in range(p.n_nu):
            un = x[n]
            tot = 0.0
            for k in range(p.n_dir):
                cth = np.clip(om[o] @ om[k], -1.0, 1.0)
                if cth > 1.0 - 1e-12:                # Theta = 0: sqrt(pi) delta(u - u') W(a, u)
                    rII = wofz(un + 1j * a).real / np.sqrt(np.pi) * Sflat(k, un)
                else:
                    th = np.arccos(cth)
                    rII = quad(lambda u: _F(th, u, un, a).real * Sflat(k, u), lo, hi,
                               points=sorted(brk + [un, -un]), limit=800, epsabs=0,
                               epsrel=1e-13)[0] / np.pi
                tot += w[k] * (alpha * rII + (beta - alpha) * phi(un) * r3[k])
            ref[o, n] = tot
    assert np.abs(e[..., 0] - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.abs(e[..., 1:]).max() < 1e-14 * np.abs(ref).max()
