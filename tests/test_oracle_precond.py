"""Pins of the oracle's preconditioner (Sect. 5.2, App. F) against routes that
do not go through its closed forms: brute-force inverses and diagonals, the
flat-field identity of App. E, and the linear solve it must not change."""
import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, gmres

from workloads import tiny, two_term_atom
from oracle import transfer as T
from oracle import precond as PC


def _problem(**kw):
    base = dict(n_z=5, n_nu=13, x_max=6.0, n_mu=4, n_chi=3, B=(30.0, 1.0, 0.4), a=2e-2, eps=5e-2,
                v_z=2.0, seed=13)
    base.update(kw)
    return tiny(**base)


@pytest.fixture(scope="module")
def setup_tab():
    p = _problem()
    op = T.setup(p)
    return p, op, PC.tables(op)


def test_local_lambda_is_the_diagonal_of_the_unpolarised_formal_solution(setup_tab):
    """Lambda_zz from psi_c / eta_I equals, entry by entry, the response of the
    scalar formal solution at (z, Omega, n) to a unit emissivity there."""
    p, op, tab = setup_tab
    nz, nd, nn = p.n_z, p.n_dir, p.n_nu
    diag = np.zeros((nz, nd, nn))
    for z in range(nz):
        for n in range(nn):
            e = np.zeros((nz, nd, nn))
            e[z, :, n] = 1.0          # rays do not couple, so one column per (z, n) serves all Omega
            diag[z, :, n] = PC.lambda_star(op, e)[z, :, n]
    assert np.abs(tab["L"] - diag).max() <= 1e-13 * np.abs(diag).max()
    assert np.all(diag >= 0.0)


def test_block_inverse_equals_dense_inverse(setup_tab):
    """App. F closed form of P^_z^-1 against the inverse of
    Id - Lambda_zz Sigma*_z assembled column by column (moving atmosphere,
    so the two interpolations do not commute with Lambda_zz)."""
    p, op, tab = setup_tab
    nz, nd, nn = p.n_z, p.n_dir, p.n_nu
    n = nd * nn
    for z in (1, nz - 2):
        Pz = np.eye(n)
        for k in range(n):
            x = np.zeros((nz, nd, nn))
            x.reshape(nz, n)[z, k] = 1.0
            col = (tab["L"] * PC.sigma_star(tab, x))[z].reshape(n)
            Pz[:, k] -= col
        rng = np.random.default_rng(z)
        r = rng.standard_normal((nz, nd, nn))
        got = PC.block_inverse(tab, r)[z].reshape(n)
        ref = np.linalg.solve(Pz, r[z].reshape(n))
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("atom", ["two_level", "two_term"])
def test_comoving_coupling_flat_field(atom):
    """App. E identity on the unmagnetised static problem: a flat unit field
    gives the emissivity (1 - eps) eta_I, so Phi_z 1 = (1 - eps_z) eta_I(z, u);
    this checks the redistribution coupling against the absorption profile."""
    kw = {}
    if atom == "two_term":
        kw = dict(atom=two_term_atom(2800.0, 24.305, 20.0), x_max=14.0, n_nu=15)
    p = _problem(**kw)
    op = T.setup(p)
    Phi = PC.comoving_coupling(op)
    plain = p.with_(B=np.zeros_like(p.B), v=np.zeros_like(p.v))
    op0 = T.setup(plain, {"normalize": False})
    ref = (1.0 - p.eps)[:, None] * op0.K[:, 0, :, 0, 0]
    got = Phi.sum(axis=2)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_sweeps_converge_to_the_inverse_of_P(setup_tab):
    """k block-Jacobi sweeps tend to P^-1 y (P assembled column by column and
    solved densely); one sweep is P^^-1 itself."""
    p, op, tab = setup_tab
    nz, nd, nn = p.n_z, p.n_dir, p.n_nu
    N = nz * nd * nn
    Pm = np.empty((N, N))
    for k in range(N):
        x = np.zeros(N)
        x[k] = 1.0
        Pm[:, k] = PC.p_apply(op, tab, x.reshape(nz, nd, nn)).ravel()
    rng = np.random.default_rng(3)
    r = rng.standard_normal((nz, nd, nn, 4))
    exact = np.linalg.solve(Pm, r[..., 0].ravel())
    errs = []
    for k in (1, 2, 4, 8, 30):
        got = PC.precondition(op, tab, r, k)
        assert np.array_equal(got[..., 1:], r[..., 1:])
        errs.append(np.abs(got[..., 0].ravel() - exact).max() / np.abs(exact).max())
    assert np.allclose(PC.precondition(op, tab, r, 1)[..., 0], PC.block_inverse(tab, r[..., 0]), rtol=0, atol=0)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-9


def test_preconditioned_solve_same_solution_fewer_iterations():
    """Left preconditioning leaves the solution of (Id - Lambda Sigma) I = b
    unchanged (dense LU) and needs fewer GMRES iterations."""
    p = _problem(n_z=6, n_nu=11, n_mu=2, n_chi=4, eps=1e-3, tau_bot=1e3)
    op = T.setup(p)
    tab = PC.tables(op)
    ref = T.solve(op, method="dense")
    b = T.rhs(op)
    shape = b.shape
    N = b.size
    A = LinearOperator((N, N), matvec=lambda v: T.apply_operator(op, v.reshape(shape)).ravel(), dtype=float)
    M = lambda v: PC.precondition(op, tab, v.reshape(shape), 3).ravel()
    MA = LinearOperator((N, N), matvec=lambda v: M(A @ v), dtype=float)
    counts = []
    sols = []
    for Aop, rhs in ((A, b.ravel()), (MA, M(b.ravel()))):
        n = [0]
        x, info = gmres(Aop, rhs, rtol=1e-12, atol=0.0, restart=200, maxiter=400,
                        callback=lambda _r: n.__setitem__(0, n[0] + 1), callback_type="pr_norm")
        assert info == 0
        counts.append(n[0])
        sols.append(x)
    for x in sols:
        assert np.abs(x - ref.ravel()).max() <= 1e-9 * np.abs(ref).max()
    assert counts[1] < counts[0]
