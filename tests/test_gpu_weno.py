"""GPU parity of the non-oscillatory frame transforms (Sect. 4.1, the remedy
for oscillations under strong velocities; trap_set_interpolation) against the
oracle: Sigma applied element by element (FP64 1e-12, FP32 1e-5 of the
largest value, per Stokes component), the identity at rest, the fixed point
of the nonlinear map by AAR in FP64 and by the mixed-precision defect
corrections (GMRES and AAR around linear spline inner applies), and the
setter's error paths.  The strong case (shifts of up to four grid steps on a
15-point grid) is one where the spline's normalisation factor changes sign."""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu

CASES = {
    "two_level_strong_velocity": dict(n_z=5, n_nu=15, x_max=8.0, v_z=12.0, seed=4),
    "two_term_doublet_moving": dict(n_z=4, n_nu=33, x_max=16, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2,
                                    eps=5e-2, atom=two_term_atom(2800.0, 24.305, 20.0), v_z=6.0, seed=8),
}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(prob, mode):
    from paper_2505_20968_amd import Context
    c = Context(0)
    c.set_interpolation(mode)
    c.set_problem(prob)
    c.precompute(3)
    return c


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_INTERP_WENO4
    torch = _torch()
    prob = tiny(**CASES[request.param])
    print(f"\n[weno case {request.param}] N={prob.n_unknowns}", flush=True)
    op = T.setup(prob, {"interp": "weno4"})
    ctx = _ctx(prob, TRAP_INTERP_WENO4)
    yield request.param, prob, op, ctx, torch
    ctx.close()


def _field(prob, seed):
    rng = np.random.default_rng(seed)
    I = rng.uniform(0.2, 1.0, (prob.n_z, prob.n_dir, prob.n_nu, 4))
    # a sharp positive line core in I, signed Q, U, V a tenth of it
    core = np.exp(-(prob.x / 0.5) ** 2)[None, None, :]
    I[..., 0] += 3.0 * core
    I[..., 1:] = 0.1 * (I[..., 1:] - 0.6) * I[..., :1]
    return I


def test_weno_sigma_matches_oracle(case):
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    I = _field(prob, 3)
    ref = T.sigma_apply(op, I)
    scale = np.abs(ref).max(axis=(0, 1, 2))
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        x = torch.tensor(I, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        ctx.apply_sigma(x, y)
        torch.cuda.synchronize()
        err = (np.abs(y.double().cpu().numpy() - ref).max(axis=(0, 1, 2)) / scale).max()
        print(f"[{name}] WENO Sigma {dt}: max |diff| / max |ref| per Stokes {err:.2e}", flush=True)
        assert err < tol


def test_weno_at_rest_is_the_spline():
    """At zero velocity and zero lower-level splitting the transforms are the
    identity, so both interpolants give the same Sigma."""
    torch = _torch()
    from paper_2505_20968_amd import TRAP_INTERP_SPLINE, TRAP_INTERP_WENO4
    prob = tiny(n_z=4, n_nu=21, seed=2)
    I = torch.tensor(_field(prob, 4), dtype=torch.float64, device="cuda")
    out = []
    for mode in (TRAP_INTERP_SPLINE, TRAP_INTERP_WENO4):
        ctx = _ctx(prob, mode)
        y = torch.empty_like(I)
        ctx.apply_sigma(I, y)
        torch.cuda.synchronize()
        out.append(y.cpu().numpy())
        ctx.close()
    assert np.abs(out[0] - out[1]).max() <= 1e-15 * np.abs(out[0]).max()


def _contract(name, em, emr):
    ri = (np.abs(em[..., 0] - emr[..., 0]) / np.abs(emr[..., 0])).max()
    rq = max(np.abs(em[..., s] / em[..., 0] - emr[..., s] / emr[..., 0]).max() for s in (1, 2, 3))
    print(f"[{name}] emergent: max rel I {ri:.2e}, max |dQ/I|,|dU/I|,|dV/I| {rq:.2e}", flush=True)
    assert ri < 1e-6 and rq < 1e-4


def test_weno_aar_fp64_matches_oracle_fixed_point(case):
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    ref, k = T.solve_aar(op, tol=1e-12)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.aar_solve(x, tol=1e-11, max_iters=600, zero_guess=True)
    print(f"[{name}] WENO AAR FP64: {st} (oracle {k} steps)", flush=True)
    assert st["final_rel_res"] < 1e-11
    xs = x.cpu().numpy()
    assert np.abs(xs - ref).max() < 1e-8 * np.abs(ref[..., 0]).max()
    _contract(name, ctx.emergent(x), ref[-1][op.ang["mu"] > 0])


def test_weno_mixed_defect_corrections_reach_the_fixed_point(case):
    """GMRES and AAR with FP32 inner applies on the linear spline transforms and
    FP64 residuals with the WENO ones: the outer refinement converges to the
    nonlinear fixed point on the case whose grid resolves the shifts; on the
    strong case it either converges there too or stops with TRAP_ENOCONV (or
    TRAP_ENAN if the correction diverges)."""
    name, prob, op, ctx, torch = case
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FP32, TrapError
    ref, _ = T.solve_aar(op, tol=1e-12)
    for solver in ("gmres", "aar"):
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        try:
            if solver == "gmres":
                st = ctx.gmres_solve(x, tol=1e-10, restart=30, max_iters=3000, inner=TRAP_FP32, max_outer=25,
                                     inner_tol=1e-5, zero_guess=True)
            else:
                st = ctx.aar_solve(x, tol=1e-10, max_iters=3000, zero_guess=True, inner=TRAP_FP32, inner_tol=1e-4,
                                   max_outer=25)
        except TrapError as e:
            print(f"[{name}] WENO mixed {solver}: {e}", flush=True)
            assert name == "two_level_strong_velocity" and ("ENOCONV" in str(e) or "ENAN" in str(e))
            continue
        print(f"[{name}] WENO mixed {solver}: {st}", flush=True)
        assert st["final_rel_res"] < 1e-10 and st["applies_fp32"] > 0
        assert np.abs(x.cpu().numpy() - ref).max() < 1e-7 * np.abs(ref[..., 0]).max()


def test_interpolation_setter_errors():
    torch = _torch()
    from paper_2505_20968_amd import Context, TrapError, TRAP_INTERP_SPLINE, TRAP_INTERP_WENO4
    prob = tiny(n_z=3, n_nu=13)
    c = Context(0)
    try:
        with pytest.raises(TrapError, match="EINVAL"):
            c.set_interpolation(7)
        c.set_interpolation(TRAP_INTERP_WENO4)
        c.set_problem(prob)
        c.precompute(1)
        c.set_interpolation(TRAP_INTERP_WENO4)                  # unchanged: fine
        with pytest.raises(TrapError, match="ESTATE"):
            c.set_interpolation(TRAP_INTERP_SPLINE)
        c.set_problem(prob)                                      # a new problem frees it again
        c.set_interpolation(TRAP_INTERP_SPLINE)
    finally:
        c.close()
