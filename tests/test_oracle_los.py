"""Pins of the oracle's off-grid lines of sight (the emergent profiles of
Sect. 6 at mu values off the quadrature), none of which goes through the
oracle's own line-of-sight result:

* zero weight: the operator restricted to the quadrature directions does not
  change when line-of-sight rings are added, whatever the field on them;
* a line of sight on a quadrature mu reproduces the converged solution there
  (the solution is the fixed point I = Lambda (Sigma I + eps_th) + t);
* LTE closed form: with no scattering (eps = 1), an isothermal column and a
  continuum, I = (W_T, 0, 0, 0) solves the transfer equation for any field,
  so every line of sight, the limb and disc centre included, gives it;
* disc-centre symmetry: unmagnetised and static, the four-fold azimuthal
  symmetry of the grid forces Q = U = 0 at mu = 1, with I the same for
  every azimuth."""
import numpy as np
import pytest

from oracle import transfer as T
from workloads import tiny


def test_grid_block_unchanged_by_zero_weight_rings():
    base = dict(n_z=5, n_nu=11, x_max=6.0, n_mu=4, n_chi=3, B=(30.0, 1.0, 0.4), a=2e-2, eps=5e-2, v_z=2.0,
                seed=13, cont=(0.05, 0.2))
    p0 = tiny(**base)
    p1 = tiny(**base, los_mu=[0.1, 0.77])
    op0, op1 = T.setup(p0), T.setup(p1)
    assert op1.ang["w"][p0.n_dir:].sum() == 0.0 and p1.n_dir == p0.n_dir + 2 * p0.n_chi
    rng = np.random.default_rng(3)
    x = rng.standard_normal((p1.n_z, p1.n_dir, p1.n_nu, 4))
    y1 = T.apply_operator(op1, x)
    ring1 = x[:, p0.n_dir:].copy()
    x[:, p0.n_dir:] = rng.standard_normal(x[:, p0.n_dir:].shape)   # another field on the rings
    y2 = T.apply_operator(op1, x)
    y0 = T.apply_operator(op0, x[:, :p0.n_dir])
    scale = np.abs(y0).max()
    assert np.abs(y1[:, :p0.n_dir] - y0).max() < 1e-13 * scale
    assert np.abs(y2[:, :p0.n_dir] - y0).max() < 1e-13 * scale
    # the rings' own rows change with their own values only through the identity
    d = (y2 - y1)[:, p0.n_dir:]
    assert np.abs(d - (x[:, p0.n_dir:] - ring1)).max() < 1e-13 * scale
    assert np.abs(T.rhs(op1)[:, :p0.n_dir] - T.rhs(op0)).max() < 1e-13 * np.abs(T.rhs(op0)).max()


@pytest.mark.parametrize("atom", ["two_level", "two_term"])
def test_line_of_sight_on_a_quadrature_mu_reproduces_the_solution(atom):
    from workloads import two_term_atom
    kw = dict(n_z=5, n_nu=13, x_max=6.0, n_mu=4, n_chi=3, B=(30.0, 1.0, 0.4), a=2e-2, eps=5e-2, v_z=2.0,
              seed=13)
    if atom == "two_term":
        kw.update(n_z=4, n_nu=15, x_max=14.0, atom=two_term_atom(2800.0, 24.305, 20.0))
    p0 = tiny(**kw)
    op0 = T.setup(p0)
    mu_q = op0.ang["mu"][op0.ang["mu"] > 0][::p0.n_chi]           # the two positive quadrature mu
    p1 = tiny(**kw, los_mu=mu_q)
    op1 = T.setup(p1)
    sol = T.solve(op0, tol=1e-13)
    got = T.los_emergent(op1, sol)                                   # [los, chi, n, 4]
    want = T.emergent(op0, sol).reshape(2, p0.n_chi, p0.n_nu, 4)
    err = np.abs(got - want).max() / np.abs(want[..., 0]).max()
    assert err < 1e-10
    # and it differs from a line of sight a little off that mu
    p2 = tiny(**kw, los_mu=mu_q * 0.97)
    other = T.los_emergent(T.setup(p2), sol)
    assert np.abs(other - want).max() / np.abs(want[..., 0]).max() > 1e-4


@pytest.mark.parametrize("B", [(0.0, 0.0, 0.0), (80.0, 1.1, 0.7)])
def test_lte_isothermal_column_gives_the_planck_value_on_every_line_of_sight(B):
    los = [0.05, 0.1, 0.5, 1.0]
    p = tiny(n_z=7, n_nu=13, x_max=6.0, n_mu=4, n_chi=4, B=B, a=2e-2, eps=1.0, v_z=0.0, cont=(0.1, 0.4),
             los_mu=los)
    p = p.with_(W_T=np.full(p.n_z, 1.0))
    op = T.setup(p)
    I = np.zeros((p.n_z, p.n_dir_grid, p.n_nu, 4))
    I[..., 0] = 1.0
    got = T.los_emergent(op, I)
    assert np.abs(got[..., 0] - 1.0).max() < 1e-12
    assert np.abs(got[..., 1:]).max() < 1e-12


def test_disc_centre_is_azimuth_symmetric_and_unpolarised():
    p = tiny(n_z=6, n_nu=13, x_max=6.0, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=2e-2, eps=5e-2, los_mu=[1.0, 0.3])
    op = T.setup(p)
    sol = T.solve(op, tol=1e-13)
    got = T.los_emergent(op, sol[:, :p.n_dir_grid])
    centre, off = got[0], got[1]
    I0 = np.abs(centre[..., 0]).max()
    assert np.abs(centre[..., 0] - centre[:1, :, 0]).max() < 1e-11 * I0
    assert np.abs(centre[..., 1:3]).max() < 1e-11 * I0
    # off the centre the scattering polarisation is there (Q != 0), V is not
    assert np.abs(off[..., 1]).max() > 1e-4 * I0
    assert np.abs(off[..., 3]).max() < 1e-11 * I0
