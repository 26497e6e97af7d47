"""Physics-based preconditioner (Sect. 5.2) with the block-diagonal
preconditioner of App. F (oracle, FP64).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Left preconditioning replaces (Id - Lambda Sigma) I = b by
M (Id - Lambda Sigma) I = M b with M ~ P^-1 and P = Id - Lambda* Sigma*, the
operator of a simplified physical setting (Sect. 5.2).  The setting taken
here is the one App. F builds its local blocks from:

* Sigma*: unmagnetised, unpolarised, angle-averaged R_II (Eq. R_AA) plus
  R_III, multipole component K = Q = 0 only.  It maps the Stokes-I field to
  a Stokes-I emissivity through
      Sigma*_z = Ups^{nubar->nu}_z  Phi_z  Phi^Omega  Ups^{nu->nubar}_z:
  interpolation to the comoving grid per direction, the angular mean
  J(u_m) = sum_Omega w_Omega Ibar(Omega, u_m), the comoving frequency
  coupling Phi_z (N_nu x N_nu) and interpolation back to each direction's
  observer grid.  Phi_z is the response of the comoving Stokes-I emissivity
  to an isotropic unpolarised field, so it is read off this oracle's own
  Sigma (``transfer.sigma_height``) on a copy of the problem with B = 0,
  v = 0 and the angle-averaged kernel, one unit field per column, without
  the App. E factor.
* Lambda*: the DELO-linear formal solution of Stokes I with the problem's
  own eta_I (continuum opacity included) and no dichroism or dispersion
  (K' = 0), no incoming radiation, whatever formal solver the problem uses.
  Sigma* leaves the continuum scattering out, as App. F does.
* App. F: the local blocks P^_z = Id - Lambda_zz Sigma*_z with Lambda_zz the
  diagonal of Lambda* at height z (the response of I at z to the emissivity
  at z on the same ray) are inverted in closed form,
      P^_z^-1 = Id + Lambda_zz Ups^{nubar->nu} Phi_z (Id - A_z)^-1 Phi^Omega Ups^{nu->nubar},
      A_z = Phi^Omega Ups^{nu->nubar} Lambda_zz Ups^{nubar->nu} Phi_z,
  reading the interpolation next to Lambda_zz as the one back to the
  observer grid (the index is printed the other way round in App. F).
* P^-1 is approximated by ``sweeps`` steps of the block-Jacobi iteration of
  App. F (Eq. Block_Jacobi) from a zero start,
      x_1 = P^^-1 y,   x_{k+1} = x_k + P^^-1 (y - P x_k),
  a fixed linear map, so plain GMRES applies to the preconditioned system.
Stokes Q, U, V pass through unchanged (P is the identity on them).
"""
from __future__ import annotations

import numpy as np

from . import transfer as T


def comoving_coupling(op) -> np.ndarray:
    """Phi[z] (N_nu x N_nu): comoving Stokes-I emissivity per unit isotropic
    unpolarised comoving field, unmagnetised, angle-averaged R_II + R_III."""
    prob = op.prob
    nz, nd, nn = prob.n_z, prob.n_dir, prob.n_nu
    plain = prob.with_(B=np.zeros_like(prob.B), v=np.zeros_like(prob.v), kappa_c=None, sigma_c=None)
    opts = {k: v for k, v in op.opts.items() if k not in ("aa", "normalize")}
    op0 = T.setup(plain, dict(opts, aa=True, normalize=False))
    Phi = np.zeros((nz, nn, nn))
    for z in range(nz):
        for m in range(nn):
            Iz = np.zeros((nd, nn, 4))
            Iz[:, m, 0] = 1.0
            out = T.sigma_height(op0, z, Iz, normalize=False)[..., 0]
            # an isotropic unpolarised field scatters isotropically at B = 0
            scale = max(np.abs(out).max(), 1e-300)
            if np.abs(out - out[0:1]).max() > 1e-9 * scale:
                raise AssertionError("unmagnetised response is not isotropic")
            Phi[z, :, m] = out[0]
    return Phi


def local_lambda(op) -> np.ndarray:
    """Lambda_zz[z, Omega, n]: dI(z)/d eps_I(z) along each ray of the
    unpolarised DELO-linear solution, psi_c / eta_I of the step that ends at
    z; zero at the first point of a sweep (the boundary value does not depend
    on the emissivity)."""
    prob = op.prob
    nz, nd, nn = prob.n_z, prob.n_dir, prob.n_nu
    etaI = op.K[..., 0, 0]
    ratio = etaI / op.eta0[:, None, None]
    mu = op.ang["mu"]
    dtl = np.abs(np.diff(prob.tau_line))
    L = np.zeros((nz, nd, nn))
    for o in range(nd):
        order = list(range(nz)) if mu[o] > 0 else list(range(nz - 1, -1, -1))
        for k in range(1, nz):
            zu, zc = order[k - 1], order[k]
            x = 0.5 * (ratio[zu, o] + ratio[zc, o]) * dtl[min(zu, zc)] / abs(mu[o])
            _, psi_c, _ = T._psi(x)
            L[zc, o] = psi_c / etaI[zc, o]
    return L


def interpolation_maps(op):
    """U[z, Omega] (observer -> comoving, Ibar(u_m) = S[I](x_m - u_b/lam)) and
    V[z, Omega] (comoving -> observer, eps(x_n) = S[eps_bar](x_n + u_b/lam)),
    dense N_nu x N_nu matrices of the not-a-knot spline with flat extension."""
    prob = op.prob
    nz, nd, nn = prob.n_z, prob.n_dir, prob.n_nu
    x = prob.x
    U = np.zeros((nz, nd, nn, nn))
    V = np.zeros((nz, nd, nn, nn))
    for z in range(nz):
        for o in range(nd):
            sh = op.ub[z, o] / op.lam[z]
            U[z, o] = op.basis.matrix(x - sh)
            V[z, o] = op.basis.matrix(x + sh)
    return U, V


def tables(op) -> dict:
    """Everything the preconditioner needs, per height."""
    Phi = comoving_coupling(op)
    L = local_lambda(op)
    U, V = interpolation_maps(op)
    w = op.ang["w"]
    nz, nd, nn = Phi.shape[0], U.shape[1], Phi.shape[1]
    A = np.zeros((nz, nn, nn))
    C = np.zeros((nz, nn, nn))
    for z in range(nz):
        for o in range(nd):
            A[z] += w[o] * U[z, o] @ (L[z, o][:, None] * (V[z, o] @ Phi[z]))
        C[z] = Phi[z] @ np.linalg.inv(np.eye(nn) - A[z])
    return {"Phi": Phi, "L": L, "U": U, "V": V, "A": A, "C": C, "w": w}


def _mean(tab, z, f):
    """Phi^Omega Ups^{nu->nubar} f for the Stokes-I field f[Omega, n] at z."""
    return sum(tab["w"][o] * tab["U"][z, o] @ f[o] for o in range(f.shape[0]))


def sigma_star(tab, x):
    """Sigma* x for the Stokes-I field x[z, Omega, n]."""
    out = np.zeros_like(x)
    for z in range(x.shape[0]):
        h = tab["Phi"][z] @ _mean(tab, z, x[z])
        for o in range(x.shape[1]):
            out[z, o] = tab["V"][z, o] @ h
    return out


def lambda_star(op, eps):
    """Lambda* eps for the Stokes-I emissivity eps[z, Omega, n] (no boundary)."""
    K = np.zeros_like(op.K)
    for s in range(4):
        K[..., s, s] = op.K[..., 0, 0]
    op_ = T.OracleProblem(**{**op.__dict__, "K": K})
    e4 = np.zeros(eps.shape + (4,))
    e4[..., 0] = eps
    return T.formal_solve(op_, e4, boundary=False, scheme="linear")[..., 0]


def p_apply(op, tab, x):
    """P x = x - Lambda* Sigma* x on the Stokes-I field."""
    return x - lambda_star(op, sigma_star(tab, x))


def block_inverse(tab, r):
    """P^^-1 r on the Stokes-I field r[z, Omega, n] (App. F closed form)."""
    out = r.copy()
    for z in range(r.shape[0]):
        h = tab["C"][z] @ _mean(tab, z, r[z])
        for o in range(r.shape[1]):
            out[z, o] += tab["L"][z, o] * (tab["V"][z, o] @ h)
    return out


def precondition(op, tab, r, sweeps: int):
    """M r for the full vector r[z, Omega, n, 4]: ``sweeps`` block-Jacobi
    steps on P x = r_I from x = 0; Q, U, V unchanged."""
    if sweeps < 1:
        raise ValueError("sweeps must be >= 1")
    y = r[..., 0]
    x = block_inverse(tab, y)
    for _ in range(sweeps - 1):
        x = x + block_inverse(tab, y - p_apply(op, tab, x))
    out = r.copy()
    out[..., 0] = x
    return out
