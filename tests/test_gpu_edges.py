"""Edge cases through the C ABI: the degenerate field-free static atmosphere
(all Zeeman components coincide, no Doppler shifts), the smallest grids the
library accepts (two heights, four frequencies, one azimuth, one mu per
hemisphere; a ragged frequency count), the largest azimuth count, and invalid
descriptions, which must fail with TRAP_EINVAL and leave the context usable."""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "field_free_static": dict(n_z=5, n_nu=19, x_max=6, n_mu=4, n_chi=4, B=(0.0, 0.0, 0.0), a=1e-2, eps=5e-2),
    "field_free_two_term": dict(n_z=4, n_nu=29, x_max=14, n_mu=4, n_chi=3, B=(0.0, 0.0, 0.0), a=1e-2,
                                eps=5e-2, atom=two_term_atom(2800.0, 24.305, 20.0)),
    "smallest_grids": dict(n_z=2, n_nu=4, x_max=3, n_mu=2, n_chi=1, B=(15.0, 0.7, 0.2), a=2e-2, eps=1e-1),
    "ragged_odd_chi": dict(n_z=3, n_nu=11, x_max=5, n_mu=2, n_chi=7, B=(50.0, 1.3, 2.2), a=1e-2, eps=3e-2,
                           v_z=3.0, seed=4),
    "sixteen_azimuths": dict(n_z=2, n_nu=9, x_max=5, n_mu=2, n_chi=16, B=(30.0, 0.5, 1.0), a=1e-2, eps=5e-2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_edge_case_matches_oracle(name):
    torch = _torch()
    from oracle import transfer as T
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64
    prob = tiny(**CASES[name])
    op = T.setup(prob)
    ctx = Context(0)
    ctx.set_problem(prob)
    ctx.precompute(3)
    rng = np.random.default_rng(11)
    I = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
    It = torch.tensor(I, device="cuda")
    e = torch.empty_like(It)
    ctx.apply_sigma(It, e)
    torch.cuda.synchronize()
    r = _rel(e.cpu().numpy(), T.sigma_apply(op, I))
    ref = T.solve(op, tol=1e-12)
    up = op.ang["mu"] > 0
    for inner in (TRAP_FP64, TRAP_FP32):
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        st = ctx.gmres_solve(x, tol=1e-11, restart=30, max_iters=600, inner=inner, inner_tol=1e-4)
        em, emr = ctx.emergent(x), ref[-1][up]
        relI = (np.abs(em[..., 0] - emr[..., 0]) / np.abs(emr[..., 0])).max()
        print(f"[{name}] sigma rel {r:.2e}; inner {inner}: {st['inner_iters']} iters, emergent I rel {relI:.2e}",
              flush=True)
        assert relI < 1e-6
        for s in (1, 2, 3):
            assert np.abs(em[..., s] / em[..., 0] - emr[..., s] / emr[..., 0]).max() < 1e-4
    ctx.close()
    assert r < 1e-10


def test_invalid_descriptions_fail_cleanly():
    torch = _torch()
    from paper_2505_20968_amd import Context, TrapError
    good = tiny(n_z=3, n_nu=9, x_max=4, n_mu=2, n_chi=2)
    ctx = Context(0)
    bad = [
        good.with_(x=good.x[::-1].copy()),                         # frequencies must increase
        good.with_(x=np.linspace(0.5, 4.0, 9)),                     # grid must bracket 0
        good.with_(x=np.linspace(-1.0, 1.0, 3)),                    # fewer than 4 nodes
        good.with_(n_mu=3),                                         # odd mu count
        good.with_(n_chi=17),                                       # more than 16 azimuths
        good.with_(tau_line=np.array([1.0, -1.0, 1e-3])),           # optical depth must be positive
    ]
    for p in bad:
        with pytest.raises(TrapError) as ei:
            ctx.set_problem(p)
        assert ei.value.code == -1, ei.value
    # the context still works after the failures
    ctx.set_problem(good)
    ctx.precompute(3)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=1e-9, restart=20, max_iters=300, inner=0)
    assert st["final_rel_res"] < 1e-9
    # calls out of order are state errors (TRAP_ESTATE)
    ctx2 = Context(0)
    ctx2.set_problem(good)
    v = torch.zeros(ctx2.shape, device="cuda", dtype=torch.float64)
    with pytest.raises(TrapError) as ei:
        ctx2.apply_sigma(v, torch.empty_like(v))
    assert ei.value.code == -5
    ctx2.close()
    ctx.close()


@pytest.mark.parametrize("store", [1, 3])
def test_footprint_bounds_what_a_solve_allocates(store):
    """Admission sizing: trap_footprint (host arithmetic) is at least what a
    context holds on the device after set-up, precompute and a solve, and
    not wildly more."""
    torch = _torch()
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64, footprint
    from workloads import cfg1
    for prob in (cfg1(), tiny(n_z=6, n_nu=25, x_max=7, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0), a=2e-2,
                              eps=3e-2, v_z=2.0, seed=21),
                 tiny(n_z=4, n_nu=33, x_max=16, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2, eps=5e-2,
                      atom=two_term_atom(2800.0, 24.305, 20.0))):
        est = footprint(prob, store)
        ctx = Context(0)
        ctx.set_problem(prob)
        ctx.precompute(store)
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        ctx.gmres_solve(x, tol=1e-9, restart=40, inner=TRAP_FP32 if store == 3 else TRAP_FP64,
                        inner_tol=1e-4, max_outer=10)
        used = ctx.info()["bytes_device_total"]
        ctx.close()
        print(f"store {store}: footprint {est} B, held {used} B", flush=True)
        assert used <= est <= 1.5 * used + (1 << 20)


@pytest.mark.parametrize("store", [1, 3])
def test_footprint_with_preconditioner(store):
    """With store_mask bit 2 the footprint also covers the preconditioner's
    tables, scratch and sweep vectors: exactly what a context holds after a
    preconditioned solve when both kernel stores are kept."""
    torch = _torch()
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64, footprint
    for prob in (tiny(n_z=6, n_nu=25, x_max=7, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0), a=2e-2, eps=3e-2, v_z=2.0,
                      seed=21),
                 tiny(n_z=4, n_nu=33, x_max=16, n_mu=4, n_chi=4, B=(40.0, 1.0, 0.3), a=1e-2, eps=5e-2,
                      atom=two_term_atom(2800.0, 24.305, 20.0))):
        est = footprint(prob, store | 4)
        ctx = Context(0)
        ctx.set_problem(prob)
        ctx.precompute(store)
        ctx.precompute_preconditioner()
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        ctx.gmres_solve(x, tol=1e-9, restart=40, inner=TRAP_FP32 if store == 3 else TRAP_FP64,
                        inner_tol=1e-4, max_outer=10, precond_sweeps=2, zero_guess=True)
        used = ctx.info()["bytes_device_total"]
        ctx.close()
        print(f"store {store} + preconditioner: footprint {est} B, held {used} B", flush=True)
        assert used <= est <= 1.5 * used + (1 << 20)
        if store == 3:
            assert est == used


@pytest.mark.parametrize("inner", ["fp64", "mixed"])
def test_zero_guess_skips_the_first_apply_and_changes_nothing(inner):
    """Declaring the initial guess zero replaces the first residual's operator
    apply by r = b (A 0 = 0 exactly): same iterations, same solution bitwise,
    one FP64 apply fewer; a nonzero guess declared zero is rejected."""
    torch = _torch()
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64, TrapError
    prob = tiny(n_z=6, n_nu=25, x_max=7, n_mu=4, n_chi=5, B=(60.0, 0.8, 2.0), a=2e-2, eps=3e-2, v_z=2.0, seed=21)
    ctx = Context(0)
    ctx.set_problem(prob)
    ctx.precompute(3)
    opts = dict(tol=1e-10, restart=30, max_iters=500, inner=TRAP_FP32 if inner == "mixed" else TRAP_FP64,
                inner_tol=1e-7, max_outer=10)
    xa = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    sa = ctx.gmres_solve(xa, **opts)
    xb = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    sb = ctx.gmres_solve(xb, zero_guess=True, **opts)
    print(f"[{inner}] applies fp64 {sa['applies_fp64']} -> {sb['applies_fp64']}", flush=True)
    assert torch.equal(xa, xb)
    assert sb["inner_iters"] == sa["inner_iters"]
    assert sb["applies_fp64"] == sa["applies_fp64"] - 1
    xc = torch.full(ctx.shape, 1e-3, dtype=torch.float64, device="cuda")
    with pytest.raises(TrapError):
        ctx.gmres_solve(xc, zero_guess=True, **opts)
    ctx.close()


def test_kernel_rows_by_mirror_symmetry():
    """On a frequency grid symmetric about 0, the kernel rows of the shift +s
    transition (and half of those of the unshifted one) are taken from mirror
    images; Sigma still matches the oracle (1e-10), and an asymmetric grid,
    which computes every row, does too."""
    torch = _torch()
    from oracle import transfer as T
    from paper_2505_20968_amd import Context
    base = tiny(n_z=4, n_nu=17, x_max=6.0, n_mu=4, n_chi=3, B=(40.0, 1.0, 0.4), a=2e-2, eps=5e-2, v_z=1.5, seed=9)
    for prob, mirrored in ((base, 17 + 8), (base.with_(x=np.linspace(-6.0, 6.5, 17)), 0),
                           (base.with_(B=np.zeros_like(base.B)), 3 * 8)):
        c = Context(0)
        try:
            c.set_problem(prob)
            c.precompute(3)
            assert c.info()["kernel_rows_mirrored"] == mirrored
            rng = np.random.default_rng(3)
            I = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
            ref = T.sigma_apply(T.setup(prob), I)
            for dt, tol in ((torch.float64, 1e-10), (torch.float32, 2e-5)):
                It = torch.tensor(I, dtype=dt, device="cuda")
                e = torch.empty_like(It)
                c.apply_sigma(It, e)
                torch.cuda.synchronize()
                r = np.linalg.norm(e.double().cpu().numpy() - ref) / np.linalg.norm(ref)
                print(f"mirrored rows {mirrored}: sigma {dt} rel {r:.2e}", flush=True)
                assert r < tol
        finally:
            c.close()
