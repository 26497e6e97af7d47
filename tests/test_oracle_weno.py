"""Pins of the oracle's non-oscillatory interpolation (the remedy that Sect. 4.1
names for oscillations under strong velocities) against what the construction
fixes by itself: exactness on quadratics for any weights, the four-node cubic
when the weights are the linear ones (and so fourth order on smooth data), no
overshoot at a jump and no negative lobes around a spike where the cubic
spline of Sect. 6.2 rings, invariance under scaling and mirroring, and the flat
extension.  At zero velocity and zero lower-level splitting every transform is
the identity, so Sigma is the same with either interpolant."""
import numpy as np
import pytest
from scipy.interpolate import BarycentricInterpolator, CubicSpline

from oracle.grids import weno4_interpolate


def _grid(n, seed, lo=-4.0, hi=4.0):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(lo, hi, n))
    x[0], x[-1] = lo, hi
    return x


def _spline(x, v, y):
    return CubicSpline(x, v, bc_type="not-a-knot")(np.clip(y, x[0], x[-1]))


def test_quadratics_are_exact_on_a_nonuniform_grid():
    x = _grid(17, 1)
    y = np.random.default_rng(2).uniform(x[0], x[-1], 400)
    for a, b, c in [(0.3, -1.2, 0.7), (-2.0, 0.0, 5.0), (0.0, 1.5, -0.25)]:
        q = lambda t: a * t * t + b * t + c
        got = weno4_interpolate(x, q(x), y)
        assert np.abs(got - q(y)).max() < 1e-12 * max(1.0, np.abs(q(y)).max())


def test_linear_weights_give_the_four_node_cubic():
    """eps_rel huge: w_k = g_k, the Neville combination of the two quadratics,
    i.e. the cubic through x_{i-1}..x_{i+2} (interior intervals)."""
    x = _grid(14, 3)
    rng = np.random.default_rng(4)
    v = rng.normal(size=x.size)
    for i in range(1, x.size - 2):
        y = rng.uniform(x[i], x[i + 1], 7)
        got = weno4_interpolate(x, v, y, eps_rel=1e30)
        ref = BarycentricInterpolator(x[i - 1:i + 3], v[i - 1:i + 3])(y)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(v).max(), i
    cub = lambda t: 0.2 * t ** 3 - t ** 2 + 0.5 * t - 2.0
    y = np.linspace(x[1], x[-2], 300)
    assert np.abs(weno4_interpolate(x, cub(x), y, eps_rel=1e30) - cub(y)).max() < 1e-11


def test_fourth_order_on_a_smooth_line_profile():
    """exp(-t^2) on uniform grids of step h, h/2, ... (away from the first and
    last intervals): the nonlinear weights differ from the linear ones by
    O(h) and the two quadratics from the cubic by O(h^3), so the error falls
    as h^4 where the curvature does not vanish.  Around the inflection points
    |t| = 1/sqrt(2) the second differences change sign, the weights leave the
    linear ones and the order drops to three: the maximum error over the whole
    profile converges at third order."""
    far, whole = [], []
    y = np.linspace(-6.0, 6.0, 4001)
    away = np.abs(np.abs(y) - 1.0 / np.sqrt(2.0)) > 0.4
    for n in (41, 81, 161, 321, 641):
        x = np.linspace(-8.0, 8.0, n)
        e = np.abs(weno4_interpolate(x, np.exp(-x * x), y) - np.exp(-y * y))
        far.append(e[away].max())
        whole.append(e.max())
    o_far = np.log2(np.array(far[:-1]) / np.array(far[1:]))
    o_all = np.log2(np.array(whole[:-1]) / np.array(whole[1:]))
    assert o_far[1:].min() > 3.5, o_far
    assert o_all[1:].min() > 2.9, o_all


def test_no_overshoot_at_a_jump_where_the_spline_rings():
    x = _grid(40, 5)
    v = np.where(x < 0.3, 0.0, 1.0)
    y = np.linspace(x[0], x[-1], 5001)
    got = weno4_interpolate(x, v, y)
    assert got.min() >= -1e-12 and got.max() <= 1.0 + 1e-12
    assert np.all(np.diff(got) >= -1e-12)                  # monotone, like the data
    sp = _spline(x, v, y)
    assert sp.min() < -0.02 or sp.max() > 1.02              # the spline does ring here


def test_no_negative_lobes_around_a_spike():
    x = np.linspace(-5.0, 5.0, 21)
    v = np.zeros_like(x)
    v[10] = 1.0
    y = np.linspace(-5.0, 5.0, 4001)
    got = weno4_interpolate(x, v, y)
    assert got.min() >= -1e-12 and got.max() <= 1.0 + 1e-12
    assert np.abs(got[np.abs(y) >= 1.0]).max() < 1e-12     # zero beyond the neighbouring nodes
    assert _spline(x, v, y).min() < -0.05


def test_sharp_line_shifted_by_a_velocity_jump_stays_positive():
    """A line narrower than the grid step (a chromospheric profile under a
    strong velocity): the comoving transform I(x - u_b) of a positive profile
    stays positive and keeps one maximum, while the spline goes negative."""
    x = np.linspace(-10.0, 10.0, 41)
    prof = np.exp(-(x / 0.35) ** 2) + 1e-3 / (1.0 + x * x)
    for ub in (2.3, -3.71, 5.25):
        y = np.linspace(-10.0, 10.0, 8001) - ub
        got = weno4_interpolate(x, prof, y)
        assert got.min() > 0.0
        inner = (got[1:-1] > got[:-2]) & (got[1:-1] > got[2:])
        assert inner.sum() == 1
        assert _spline(x, prof, y).min() < 0.0


def test_scaling_sign_and_mirror_invariance():
    x = _grid(23, 6)
    rng = np.random.default_rng(7)
    v = np.exp(-x ** 2) + 0.1 * rng.normal(size=x.size)
    y = rng.uniform(x[0], x[-1], 300)
    base = weno4_interpolate(x, v, y)
    for c in (-3.7, 1e-8, 2.5e6):
        assert np.abs(weno4_interpolate(x, c * v, y) - c * base).max() < 1e-12 * abs(c) * np.abs(base).max()
    mir = weno4_interpolate(-x[::-1], v[::-1], -y)
    assert np.abs(mir - base).max() < 1e-12 * np.abs(base).max()


def test_flat_extension_and_nodes():
    x = _grid(9, 8)
    v = np.random.default_rng(9).normal(size=(x.size, 4))
    got = weno4_interpolate(x, v, np.array([x[0] - 3.0, x[-1] + 7.0]))
    assert np.array_equal(got[0], v[0]) and np.array_equal(got[1], v[-1])
    assert np.abs(weno4_interpolate(x, v, x) - v).max() < 1e-14   # nodes reproduced


def test_sigma_at_zero_velocity_is_the_same_with_either_interpolant():
    from oracle import transfer as T
    from workloads import tiny
    prob = tiny(n_z=3, n_nu=13, seed=3)
    I = np.random.default_rng(1).uniform(0.5, 1.5, (prob.n_z, prob.n_dir, prob.n_nu, 4))
    a = T.sigma_apply(T.setup(prob, {"normalize": False}), I, normalize=False)
    b = T.sigma_apply(T.setup(prob, {"normalize": False, "interp": "weno4"}), I, normalize=False)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def test_comoving_field_under_a_strong_velocity_has_no_negative_intensity():
    """Sigma's first step with the non-oscillatory reading: a sharp positive
    Stokes-I profile on a coarse grid, vertical velocity of several Doppler
    widths; the comoving field keeps I > 0, which the spline does not."""
    from oracle import transfer as T
    from workloads import tiny
    prob = tiny(n_z=2, n_nu=21, x_max=10.0, v_z=25.0)
    opw = T.setup(prob, {"normalize": False, "interp": "weno4"})
    ops = T.setup(prob, {"normalize": False})
    prof = np.exp(-(prob.x / 0.4) ** 2) + 1e-3
    I = np.zeros((prob.n_z, prob.n_dir, prob.n_nu, 4))
    I[..., 0] = prof[None, None, :]
    shifts = opw.ub[0] / opw.lam[0]
    assert np.abs(shifts).max() > 2.0
    wen = np.stack([T.comoving_field(opw, 0, I[0], o) for o in range(prob.n_dir)])
    spl = np.stack([T.comoving_field(ops, 0, I[0], o) for o in range(prob.n_dir)])
    assert wen[..., 0].min() > 0.0
    assert spl[..., 0].min() < 0.0


def test_fixed_point_with_the_nonoscillatory_transforms():
    """With WENO transforms Sigma is nonlinear, so the oracle's solution is the
    fixed point of G (AAR) and the linear solver refuses the map.  On a coarse
    grid under a strong velocity (shifts of ~4 grid steps) the spline's
    back-transform makes the App. E normalisation factor change sign and the
    solution carries a spurious Q of the size of I; the non-oscillatory
    transforms keep f positive and I >= 0.  On grids that resolve the shifts
    the two readings converge to the same solution as the grid is refined."""
    from oracle import transfer as T
    from workloads import tiny
    prob = tiny(n_z=5, n_nu=15, x_max=8.0, v_z=12.0, seed=4)
    opw = T.setup(prob, {"interp": "weno4"})
    with pytest.raises(ValueError):
        T.solve(opw)
    xw, steps = T.solve_aar(opw, tol=1e-11)
    r = T.fixed_point_map(opw, xw) - xw
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(xw)
    assert opw.f.min() > 0.0 and xw[..., 0].min() >= 0.0
    ops = T.setup(prob)
    assert ops.f.min() < 0.0
    d = []
    for n_nu in (41, 81):
        mild = tiny(n_z=5, n_nu=n_nu, x_max=8.0, v_z=2.0, seed=4)
        xw, _ = T.solve_aar(T.setup(mild, {"interp": "weno4"}), tol=1e-11)
        xs = T.solve(T.setup(mild), tol=1e-12)
        d.append(np.abs(xw - xs).max() / np.abs(xs[..., 0]).max())
    # both converge to the same solution: the gap falls faster than h^2
    assert d[1] < 2e-3 and d[0] / d[1] > 4.0, d
