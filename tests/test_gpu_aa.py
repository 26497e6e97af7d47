"""Angle-averaged PRD on the device against the oracle's AA mode (Sect. 5.2,
Eq. R_AA with the 25-node Gauss-Legendre rule in Theta of App. C), and the
AA/AD consistency that the paper fixes: identical emissivities for a flat
incident field."""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu

CASES = {
    "two_level_moving_seeded": dict(n_z=5, n_nu=21, x_max=6, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0), a=2e-2,
                                    eps=3e-2, v_z=2.0, seed=21),
    "two_term_doublet": dict(n_z=3, n_nu=29, x_max=14, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2,
                             eps=5e-2, atom=two_term_atom(2800.0, 24.305, 20.0)),
}


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _ctx(prob, mode):
    from paper_2505_20968_amd import Context
    c = Context(0)
    c.set_prd_mode(mode)
    c.set_problem(prob)
    c.precompute(3)
    return c


@pytest.mark.parametrize("name", list(CASES))
def test_aa_operator_and_solve_match_oracle(name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import transfer as T
    from paper_2505_20968_amd import TRAP_FP32, TRAP_FP64, TRAP_PRD_AA
    prob = tiny(**CASES[name])
    op = T.setup(prob, {"aa": True})
    ctx = _ctx(prob, TRAP_PRD_AA)
    rng = np.random.default_rng(5)
    I = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
    ref = T.sigma_apply(op, I)
    for dt, tol in ((torch.float64, 1e-10), (torch.float32, 2e-5)):
        It = torch.tensor(I, dtype=dt, device="cuda")
        e = torch.empty_like(It)
        ctx.apply_sigma(It, e)
        torch.cuda.synchronize()
        r = _rel(e.double().cpu().numpy(), ref)
        print(f"[{name} AA] sigma {dt} rel {r:.2e}", flush=True)
        assert r < tol
    sol = T.solve(op, tol=1e-12)
    up = op.ang["mu"] > 0
    for inner in (TRAP_FP64, TRAP_FP32):
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        st = ctx.gmres_solve(x, tol=1e-11, restart=30, max_iters=600, inner=inner, inner_tol=1e-4)
        em, emr = ctx.emergent(x), sol[-1][up]
        relI = (np.abs(em[..., 0] - emr[..., 0]) / np.abs(emr[..., 0])).max()
        print(f"[{name} AA] solve inner {inner}: {st['inner_iters']} iters, emergent I rel {relI:.2e}", flush=True)
        assert relI < 1e-6
        for s in (1, 2, 3):
            assert np.abs(em[..., s] / em[..., 0] - emr[..., s] / emr[..., 0]).max() < 1e-4
    ctx.close()


def test_aa_and_ad_agree_on_flat_field_on_device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20968_amd import TRAP_PRD_AA, TRAP_PRD_AD
    prob = tiny(**CASES["two_level_moving_seeded"])
    flat = np.zeros((prob.n_z, prob.n_dir, prob.n_nu, 4))
    flat[..., 0] = prob.W_T[:, None, None]
    out = {}
    for mode in (TRAP_PRD_AD, TRAP_PRD_AA):
        ctx = _ctx(prob, mode)
        It = torch.tensor(flat, device="cuda")
        e = torch.empty_like(It)
        ctx.apply_sigma(It, e)
        torch.cuda.synchronize()
        out[mode] = e.cpu().numpy()
        ctx.close()
    assert _rel(out[TRAP_PRD_AA], out[TRAP_PRD_AD]) < 1e-10
