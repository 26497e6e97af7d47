"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 path 1e-10 relative (quadrature and summation-order level);
FP32 operator 2e-5 relative; emergent profiles of full solves 1e-6 relative
on I and 1e-4 absolute on Q/I, U/I, V/I (the stated parity contract).
"""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(prob, store=3):
    from paper_2505_20968_amd import Context
    c = Context(0)
    c.set_problem(prob)
    c.precompute(store)
    return c


CASES = {
    "two_level_static": dict(n_z=5, n_nu=21, x_max=6, n_mu=4, n_chi=4, B=(30.0, 1.1, 0.4), a=1e-2,
                             eps=5e-2),
    "two_level_moving_seeded": dict(n_z=6, n_nu=25, x_max=7, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0),
                                    a=2e-2, eps=3e-2, v_z=2.0, seed=21),
    "two_term_doublet": dict(n_z=4, n_nu=33, x_max=16, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2,
                             eps=5e-2, atom=two_term_atom(2800.0, 24.305, 20.0)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from oracle import transfer as T
    torch = _torch()
    kw = dict(CASES[request.param])
    prob = tiny(**kw)
    print(f"\n[parity case {request.param}] N={prob.n_unknowns}", flush=True)
    op = T.setup(prob)
    ctx = _ctx(prob)
    rng = np.random.default_rng(123)
    I = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
    I[..., 1:] = 0.2 * (I[..., 1:] - 0.5) * I[..., :1]
    yield request.param, prob, op, ctx, I, torch
    ctx.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


PATHS = {"auto": 0, "fused": 1, "chunked": 2}


@pytest.mark.parametrize("path", ["auto", "chunked"])
def test_sigma_apply_fp64(case, path):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    ref = T.sigma_apply(op, I)
    It = torch.tensor(I, dtype=torch.float64, device="cuda")
    e = torch.empty_like(It)
    ctx.set_path(PATHS[path])
    try:
        ctx.apply_sigma(It, e)
        torch.cuda.synchronize()
    finally:
        ctx.set_path(0)
    got = e.cpu().numpy()
    r = _rel(got, ref)
    print(f"[{name}] sigma fp64 {path} rel {r:.3e} maxabs {np.abs(got - ref).max():.3e}", flush=True)
    assert r < 1e-10


def test_fused_path_is_fp32_only(case):
    """The FP64 operator keeps the height-chunked path; forcing the fused
    kernel for it is an error, not a silent fallback."""
    name, prob, op, ctx, I, torch = case
    from paper_2505_20968_amd import TrapError
    It = torch.tensor(I, dtype=torch.float64, device="cuda")
    e = torch.empty_like(It)
    ctx.set_path(PATHS["fused"])
    try:
        with pytest.raises(TrapError):
            ctx.apply_sigma(It, e)
    finally:
        ctx.set_path(0)


@pytest.mark.parametrize("path", ["fused", "chunked"])
def test_sigma_apply_fp32(case, path):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    ref = T.sigma_apply(op, I)
    It = torch.tensor(I, dtype=torch.float32, device="cuda")
    e = torch.empty_like(It)
    ctx.set_path(PATHS[path])
    try:
        ctx.apply_sigma(It, e)
        torch.cuda.synchronize()
    finally:
        ctx.set_path(0)
    r = _rel(e.double().cpu().numpy(), ref)
    print(f"[{name}] sigma fp32 {path} rel {r:.3e}", flush=True)
    assert r < 2e-5


def test_sigma_thermal_term(case):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    ref = T.sigma_apply(op, I) + op.eps_th
    It = torch.tensor(I, dtype=torch.float64, device="cuda")
    e = torch.empty_like(It)
    ctx.apply_sigma(It, e, add_thermal=True)
    torch.cuda.synchronize()
    assert _rel(e.cpu().numpy(), ref) < 1e-10


def test_formal_solve(case):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    eps = np.abs(I) * 0.3
    for bnd in (True, False):
        ref = T.formal_solve(op, eps, boundary=bnd)
        for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-6)):
            et = torch.tensor(eps, dtype=dt, device="cuda")
            out = torch.empty_like(et)
            ctx.formal_solve(et, out, with_boundary=bnd)
            torch.cuda.synchronize()
            r = _rel(out.double().cpu().numpy(), ref)
            print(f"[{name}] formal bnd={bnd} {dt} rel {r:.3e}", flush=True)
            assert r < tol


def test_operator_and_rhs(case):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    ref = T.apply_operator(op, I)
    It = torch.tensor(I, dtype=torch.float64, device="cuda")
    y = torch.empty_like(It)
    ctx.apply_operator(It, y)
    b = torch.empty_like(It)
    ctx.rhs(b)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), ref) < 1e-10
    assert _rel(b.cpu().numpy(), T.rhs(op)) < 1e-10


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_full_solve_matches_oracle(case, inner):
    name, prob, op, ctx, I, torch = case
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FP32, TRAP_FP64
    ref = T.solve(op, tol=1e-12)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=1e-10, restart=30, max_iters=600,
                         inner=TRAP_FP64 if inner == "fp64" else TRAP_FP32, inner_tol=1e-4)
    print(f"[{name}] solve {inner}: {st}", flush=True)
    assert st["final_rel_res"] < 1e-10
    em = ctx.emergent(x)
    up = op.ang["mu"] > 0
    emr = ref[-1][up]
    relI = np.abs(em[..., 0] - emr[..., 0]) / np.abs(emr[..., 0])
    assert relI.max() < 1e-6
    for s in (1, 2, 3):
        assert np.abs(em[..., s] / em[..., 0] - emr[..., s] / emr[..., 0]).max() < 1e-4
    assert _rel(x.cpu().numpy(), ref) < 1e-8
