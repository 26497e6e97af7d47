"""GPU parity of the BESSER formal solver and of the alternating
Anderson-Richardson (AAR) solver (Sects. 3, 5.1, 6.1) against the oracle:
the BESSER formal solution per field (FP64 1e-12, FP32 1e-6 relative), AAR
on a linear (DELO-linear) problem against the GMRES solution (solution 1e-9,
with and without the preconditioner), AAR on BESSER problems against the
oracle's own AAR fixed point (parity contract on the emergent profiles, and
the fixed-point residual through the C ABI), the mixed-precision defect
correction reaching the same fixed points, and the error paths."""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu

CASES = {
    "two_level_moving_seeded": dict(n_z=6, n_nu=25, x_max=7, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0), a=2e-2,
                                    eps=3e-2, v_z=2.0, seed=21),
    "two_term_doublet_continuum": dict(n_z=4, n_nu=33, x_max=16, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2,
                                       eps=5e-2, atom=two_term_atom(2800.0, 24.305, 20.0), cont=(0.02, 0.1)),
}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(prob, scheme):
    from paper_2505_20968_amd import Context
    c = Context(0)
    c.set_formal_scheme(scheme)
    c.set_problem(prob)
    c.precompute(3)
    return c


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FORMAL_BESSER
    torch = _torch()
    prob = tiny(**CASES[request.param])
    print(f"\n[besser case {request.param}] N={prob.n_unknowns}", flush=True)
    op = T.setup(prob, {"formal": "besser"})
    ctx = _ctx(prob, TRAP_FORMAL_BESSER)
    yield request.param, prob, op, ctx, torch
    ctx.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_besser_formal_solve(case):
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    rng = np.random.default_rng(5)
    eps = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
    eps[..., 1:] = 0.2 * (eps[..., 1:] - 0.5) * eps[..., :1]
    for bnd in (True, False):
        ref = T.formal_solve(op, eps, boundary=bnd)
        assert _rel(T.formal_solve(op, eps, boundary=bnd, scheme="delopar"), ref) > 1e-6
        for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-6)):
            et = torch.tensor(eps, dtype=dt, device="cuda")
            out = torch.empty_like(et)
            ctx.formal_solve(et, out, with_boundary=bnd)
            torch.cuda.synchronize()
            r = _rel(out.double().cpu().numpy(), ref)
            print(f"[{name}] BESSER formal bnd={bnd} {dt} rel {r:.3e}", flush=True)
            assert r < tol


def test_besser_aar_matches_oracle(case):
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    ref, k = T.solve_aar(op, tol=1e-12)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.aar_solve(x, tol=1e-11, max_iters=500, zero_guess=True)
    print(f"[{name}] BESSER AAR: {st} (oracle {k} steps)", flush=True)
    assert st["final_rel_res"] < 1e-11 and st["anderson_steps"] > 0
    xs = x.cpu().numpy()
    assert np.abs(xs - ref).max() < 1e-8 * np.abs(ref).max()
    em = ctx.emergent(x)
    emr = ref[-1][op.ang["mu"] > 0]
    assert (np.abs(em[..., 0] - emr[..., 0]) / np.abs(emr[..., 0])).max() < 1e-6
    for s in (1, 2, 3):
        assert np.abs(em[..., s] / em[..., 0] - emr[..., s] / emr[..., 0]).max() < 1e-4
    # the fixed-point residual through the C ABI: G(x) = formal_from_field(x)
    g = torch.empty_like(x)
    ctx.formal_from_field(x, g)
    b = torch.empty_like(x)
    ctx.rhs(b)
    torch.cuda.synchronize()
    assert (torch.linalg.norm(g - x) / torch.linalg.norm(b)).item() < 1e-11


@pytest.mark.parametrize("sweeps", [0, 2])
def test_besser_mixed_aar_matches_oracle(case, sweeps):
    """FP64 defect correction around FP32 inner iterations reaches the same
    fixed point (the FP64 residual meets the tolerance)."""
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FP32
    ref, _ = T.solve_aar(op, tol=1e-12)
    if sweeps:
        ctx.precompute_preconditioner()
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.aar_solve(x, tol=1e-11, max_iters=800, zero_guess=True, inner=TRAP_FP32, inner_tol=1e-4,
                       max_outer=12, precond_sweeps=sweeps)
    print(f"[{name}] BESSER mixed AAR, {sweeps} sweeps: {st}", flush=True)
    assert st["final_rel_res"] < 1e-11 and st["applies_fp32"] > 0 and st["applies_fp64"] >= 1
    assert np.abs(x.cpu().numpy() - ref).max() < 1e-8 * np.abs(ref).max()


def test_gmres_refuses_besser(case):
    name, prob, op, ctx, torch = case
    from paper_2505_20968_amd import TrapError
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(TrapError, match="EINVAL"):
        ctx.gmres_solve(x, tol=1e-8, zero_guess=True)


@pytest.mark.parametrize("sweeps", [0, 2])
def test_aar_on_a_linear_problem_matches_gmres(sweeps):
    torch = _torch()
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FORMAL_DELO_LINEAR
    prob = tiny(**CASES["two_level_moving_seeded"])
    op = T.setup(prob)
    ref = T.solve(op, tol=1e-13)
    c = _ctx(prob, TRAP_FORMAL_DELO_LINEAR)
    try:
        if sweeps:
            c.precompute_preconditioner()
        x = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
        st = c.aar_solve(x, tol=1e-11, max_iters=500, zero_guess=True, precond_sweeps=sweeps)
        print(f"[linear AAR, {sweeps} sweeps] {st}", flush=True)
        assert st["final_rel_res"] < 1e-11
        assert (st["applies_precond"] > 0) == (sweeps > 0)
        from paper_2505_20968_amd import TRAP_FP32
        xm = torch.zeros_like(x)
        sm = c.aar_solve(xm, tol=1e-11, max_iters=800, zero_guess=True, precond_sweeps=sweeps, inner=TRAP_FP32,
                         inner_tol=1e-4, max_outer=12)
        print(f"[linear mixed AAR, {sweeps} sweeps] {sm}", flush=True)
        assert sm["final_rel_res"] < 1e-11 and np.abs(xm.cpu().numpy() - ref).max() < 1e-9 * np.abs(ref).max()
        xg = torch.zeros_like(x)
        sg = c.gmres_solve(xg, tol=1e-11, restart=30, max_iters=600, zero_guess=True)
        assert np.abs(x.cpu().numpy() - ref).max() < 1e-9 * np.abs(ref).max()
        assert np.abs(x.cpu().numpy() - xg.cpu().numpy()).max() < 1e-9 * np.abs(ref).max()
        # Richardson alone (depth 0) needs more residuals to get there
        if not sweeps:
            xr = torch.zeros_like(x)
            sr = c.aar_solve(xr, tol=1e-11, max_iters=2000, depth=0, zero_guess=True)
            assert sr["residuals"] > st["residuals"] and sr["anderson_steps"] == 0
        print(f"[linear AAR] GMRES took {sg['inner_iters']} iterations", flush=True)
    finally:
        c.close()


def test_aar_errors():
    torch = _torch()
    from paper_2505_20968_amd import TrapError, TRAP_FORMAL_BESSER
    prob = tiny(**CASES["two_level_moving_seeded"])
    c = _ctx(prob, TRAP_FORMAL_BESSER)
    try:
        x = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
        for bad in (dict(depth=17), dict(depth=-1), dict(period=0), dict(omega=0.0), dict(beta=-1.0),
                    dict(tol=0.0), dict(precond_sweeps=65)):
            with pytest.raises(TrapError, match="EINVAL"):
                c.aar_solve(x, **bad)
        from paper_2505_20968_amd import TRAP_FP32
        for bad in (dict(inner=5), dict(inner=TRAP_FP32, inner_tol=0.0), dict(inner=TRAP_FP32, inner_tol=1.0),
                    dict(inner=TRAP_FP32, max_outer=0)):
            with pytest.raises(TrapError, match="EINVAL"):
                c.aar_solve(x, **bad)
        with pytest.raises(TrapError, match="ESTATE"):
            c.aar_solve(x, precond_sweeps=2)
        with pytest.raises(TrapError, match="ENOCONV"):
            c.aar_solve(x, tol=1e-14, max_iters=3, zero_guess=True)
        st = c.aar_solve(x, tol=1e-9, zero_guess=True)          # usable afterwards
        assert st["final_rel_res"] < 1e-9
    finally:
        c.close()
