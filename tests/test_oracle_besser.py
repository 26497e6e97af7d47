"""Pins of the oracle's BESSER formal solver and of its alternating
Anderson-Richardson (AAR) solver (Sects. 3, 5.1, 6.1), each against
something other than the oracle's own result:

* the Bezier weights integrate e^{-t} times each Bernstein factor exactly
  (adaptive quadrature);
* a source linear in optical depth is integrated as DELO-linear does, and
  exactly (semi-infinite closed form S + mu S');
* a monotone quadratic source is integrated exactly (S + mu S' + mu^2 S'')
  at every point with a downwind neighbour, which DELO-linear misses;
* no overshoot: for a source with a jump, every BESSER intensity stays
  inside the range of the source and the boundary value, where DELOPAR
  leaves it on both sides; a non-negative source with ramps into jumps gives
  a non-negative intensity (DELOPAR's goes negative);
* AAR reaches the solution of the linear (DELO-linear) system that GMRES
  reaches, with and without the physics-based preconditioner, in far fewer
  steps than plain Richardson (depth 0);
* with BESSER, AAR reaches a fixed point of the nonlinear map
  I = Lambda (Sigma I + eps_th) + t."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import transfer as T
from workloads import tiny


def test_bezier_weights_integrate_the_bernstein_factors():
    for m in (1e-4, 0.03, 0.49, 0.51, 2.0, 35.0):
        wM, wC, wO = (float(v[0]) for v in T._bezier_weights(np.array([m])))
        for w, f in ((wM, lambda t: (t / m) ** 2), (wC, lambda t: 2 * (t / m) * (1 - t / m)),
                     (wO, lambda t: (1 - t / m) ** 2)):
            ref = quad(lambda t: f(t) * np.exp(-t), 0.0, m, epsabs=0.0, epsrel=1e-13)[0]
            assert abs(w - ref) <= 1e-12 * ref


def _field_free(n_z=12, tau_top=1e-2, tau_bot=20.0):
    p = tiny(n_z=n_z, n_nu=9, x_max=4, n_mu=4, n_chi=2, B=(0.0, 0.0, 0.0), a=2e-2, eps=0.1,
             tau_top=tau_top, tau_bot=tau_bot)
    op = T.setup(p, {"normalize": False})
    r = op.K[..., 0, 0] / op.eta0[:, None, None]
    assert np.abs(r - r[0:1]).max() < 1e-12 * np.abs(r).max()
    return p, op, r


def test_linear_source_as_delo_linear_and_exact():
    p, op, r = _field_free()
    B0, B1 = 0.4, 0.3
    tl = p.tau_line
    Wt = B0 + B1 * tl
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    mu = op.ang["mu"]
    Iex = Wt[:, None, None] + mu[None, :, None] * B1 / r
    up = mu > 0
    Ib = T.formal_solve(op, eps, boundary=True, I_bottom=np.stack([Iex[0], 0 * Iex[0], 0 * Iex[0], 0 * Iex[0]], -1),
                        scheme="besser")
    Il = T.formal_solve(op, eps, boundary=True, I_bottom=np.stack([Iex[0], 0 * Iex[0], 0 * Iex[0], 0 * Iex[0]], -1),
                        scheme="linear")
    assert np.abs(Ib - Il).max() < 1e-13 * np.abs(Il).max()
    assert (np.abs(Ib[..., 0][:, up] - Iex[:, up]) / Iex[:, up]).max() < 1e-12


def test_monotone_quadratic_source_exact():
    p, op, r = _field_free()
    B0, B1, B2 = 0.4, 0.3, 0.05
    tl = p.tau_line
    Wt = B0 + B1 * tl + B2 * tl * tl
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    mu = op.ang["mu"]
    Iex = np.zeros_like(eps)
    Iex[..., 0] = (Wt[:, None, None] + mu[None, :, None] * (B1 + 2 * B2 * tl)[:, None, None] / r
                   + 2 * B2 * (mu[None, :, None] / r) ** 2)
    up = mu > 0
    Ib = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0], scheme="besser")
    Il = T.formal_solve(op, eps, boundary=True, I_bottom=Iex[0], scheme="linear")
    rel_b = np.abs(Ib[:-1, up, :, 0] - Iex[:-1, up, :, 0]) / np.abs(Iex[:-1, up, :, 0])
    rel_l = np.abs(Il[:-1, up, :, 0] - Iex[:-1, up, :, 0]) / np.abs(Iex[:-1, up, :, 0])
    assert rel_b.max() < 1e-12 and rel_l.max() > 1e-4


def test_no_overshoot_at_a_jump():
    p, op, r = _field_free(n_z=16, tau_bot=50.0)
    Wt = np.where(p.tau_line > 2.0, 1.0, 0.0) + 0.01
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    Ib = T.formal_solve(op, eps, boundary=True, scheme="besser")[..., 0]
    Ip = T.formal_solve(op, eps, boundary=True, scheme="delopar")[..., 0]
    lo, hi = 0.0, max(Wt.max(), p.W_T[0])
    assert Ib.min() >= lo and Ib.max() <= hi * (1 + 1e-14)
    assert Ip.min() < lo - 1e-3 and Ip.max() > hi + 1e-2


def test_positive_source_gives_positive_intensity():
    """With K' = 0 every BESSER weight is positive and the control point stays
    between its end values, so a non-negative source and boundary give a
    non-negative intensity everywhere; the source here has gentle ramps into
    jumps and back to zero, where a tangent control point without the range
    limit falls below zero.  DELOPAR goes negative on it."""
    p, op, r = _field_free(n_z=24, tau_top=1e-3, tau_bot=80.0)
    Wt = np.zeros(p.n_z)
    Wt[5:8] = [1e-3, 2e-3, 1.0]
    Wt[8:11] = [1.0, 2e-3, 0.0]
    Wt[15:18] = [5e-4, 1e-3, 2.0]
    p = p.with_(W_T=np.full(p.n_z, 1.0))
    eps = Wt[:, None, None, None] * op.K[:, :, :, :, 0]
    Ib = T.formal_solve(op, eps, boundary=True, I_bottom=np.zeros((p.n_dir, p.n_nu, 4)), scheme="besser")
    Ip = T.formal_solve(op, eps, boundary=True, I_bottom=np.zeros((p.n_dir, p.n_nu, 4)), scheme="delopar")
    assert Ib[..., 0].min() >= 0.0
    assert Ip[..., 0].min() < -1e-4


CASE = dict(n_z=5, n_nu=13, x_max=6.0, n_mu=4, n_chi=3, B=(30.0, 1.0, 0.4), a=2e-2, eps=5e-2, v_z=2.0, seed=13)


@pytest.fixture(scope="module")
def linear_case():
    op = T.setup(tiny(**CASE))
    return op, T.solve(op, tol=1e-13)


def test_aar_reaches_the_gmres_solution(linear_case):
    op, ref = linear_case
    x, k = T.solve_aar(op, tol=1e-12)
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()
    _, k_rich = T.solve_aar(op, tol=1e-12, depth=0)
    assert k < 0.4 * k_rich


def test_preconditioned_aar(linear_case):
    from oracle import precond as PC
    op, ref = linear_case
    tab = PC.tables(op)
    x, k = T.solve_aar(op, tol=1e-12, precond=lambda r: PC.precondition(op, tab, r, 2))
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()
    _, k0 = T.solve_aar(op, tol=1e-12)
    assert k < k0


def test_besser_fixed_point():
    op = T.setup(tiny(**CASE), {"formal": "besser"})
    x, k = T.solve_aar(op, tol=1e-12)
    g0 = T.fixed_point_map(op, np.zeros_like(x))
    assert np.linalg.norm(T.fixed_point_map(op, x) - x) < 1e-12 * np.linalg.norm(g0)
    # a different scheme gives a different solution on this coarse column
    lin = T.solve(T.setup(tiny(**CASE)), tol=1e-13)
    assert np.abs(x - lin).max() > 1e-3 * np.abs(lin).max()
