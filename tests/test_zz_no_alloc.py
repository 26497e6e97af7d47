"""The allocation-free preconditioner apply (trap_apply_preconditioner_noalloc)
against the allocating one (trap_apply_preconditioner), through the C ABI.

Both run the same kernels on the same tables, so the results must agree to the
last bit; checked on two calls in a row, the second on a smaller problem (the
shared device scratch keeps the first call's contents), then on the first
problem again, in place, and with the scalar sweeps in FP32.  A problem whose
scratch would exceed the fixed array is rejected with TRAP_ENOMEM and leaves
the context usable; a call before the tables is TRAP_ESTATE.
"""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu

BIG = dict(n_z=8, n_nu=41, x_max=8.0, n_mu=6, n_chi=5, B=(30.0, 1.0, 0.4), a=2e-2, eps=5e-2, v_z=2.0, seed=13)
SMALL = dict(n_z=3, n_nu=15, x_max=14.0, n_mu=4, n_chi=3, B=(40.0, 1.0, 0.3), a=1e-2, eps=5e-2, v_z=1.0, seed=5,
             atom=two_term_atom(2800.0, 24.305, 20.0))


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ready(prob):
    from paper_2505_20968_amd import Context
    ctx = Context(0)
    ctx.set_problem(prob)
    ctx.precompute(1)
    ctx.precompute_preconditioner()
    return ctx


def _pair(ctx, torch, seed, sweeps, prec):
    rng = np.random.default_rng(seed)
    r = torch.tensor(rng.standard_normal(ctx.shape), device="cuda")
    a = torch.empty_like(r)
    b = torch.full_like(r, np.nan)            # stale contents must not matter
    ctx.apply_preconditioner(r, a, sweeps, prec)
    ctx.apply_preconditioner_noalloc(r, b, sweeps, prec)
    torch.cuda.synchronize()
    return r, a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_the_allocating_apply_on_two_calls():
    torch = _torch()
    from paper_2505_20968_amd import TRAP_FP32, TRAP_FP64
    big = _ready(tiny(**BIG))
    small = _ready(tiny(**SMALL))
    try:
        print("\n[noalloc] big problem, 3 sweeps FP64", flush=True)
        _, a, b = _pair(big, torch, 1, 3, TRAP_FP64)
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        assert np.array_equal(a, b)
        print("[noalloc] smaller problem, 2 sweeps FP64", flush=True)
        _, a, b = _pair(small, torch, 2, 2, TRAP_FP64)
        assert np.array_equal(a, b)
        print("[noalloc] big problem again, 4 sweeps FP32 sweeps", flush=True)
        _, a, b = _pair(big, torch, 3, 4, TRAP_FP32)
        assert np.array_equal(a, b)
        print("[noalloc] one sweep, in place", flush=True)
        r, a, _ = _pair(small, torch, 4, 1, TRAP_FP64)
        big_r = r.clone()
        small.apply_preconditioner_noalloc(big_r, big_r, 1, TRAP_FP64)
        torch.cuda.synchronize()
        assert np.array_equal(big_r.cpu().numpy(), a)
    finally:
        big.close()
        small.close()


def test_noalloc_rejects_problems_beyond_its_scratch_and_calls_out_of_order():
    torch = _torch()
    from paper_2505_20968_amd import Context, TrapError, TRAP_FP64
    # three n_z n_dir N_nu vectors of doubles: 3 x 8 x 60 x 128 x 801 B = 148 MB > 128 MiB
    huge = tiny(n_z=60, n_nu=801, x_max=12.0, n_mu=16, n_chi=8, a=1e-2, eps=1e-2)
    ctx = Context(0)
    try:
        ctx.set_problem(huge)
        # rejected from the sizes alone, before any vector is read (a one-element
        # placeholder is passed straight through the C ABI)
        import ctypes
        r = torch.zeros((1,), dtype=torch.float64, device="cuda")
        p = ctypes.c_void_p(r.data_ptr())
        code = ctx.lib.trap_apply_preconditioner_noalloc(ctx.h, p, p, 2, TRAP_FP64)
        msg = ctx.lib.trap_last_error().decode()
        print(f"[noalloc] oversized problem: {code} {msg}", flush=True)
        assert code == -2 and "scratch" in msg
    finally:
        ctx.close()
    c2 = Context(0)
    try:
        prob = tiny(**SMALL)
        c2.set_problem(prob)
        c2.precompute(1)
        r = torch.zeros(c2.shape, dtype=torch.float64, device="cuda")
        with pytest.raises(TrapError) as e:
            c2.apply_preconditioner_noalloc(r, r, 2, TRAP_FP64)
        assert e.value.code == -5                 # tables not computed
        c2.precompute_preconditioner()
        with pytest.raises(TrapError) as e:
            c2.apply_preconditioner_noalloc(r, r, 65, TRAP_FP64)
        assert e.value.code == -1
        out = torch.empty_like(r)
        c2.apply_preconditioner_noalloc(r, out, 2, TRAP_FP64)      # still usable
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0
    finally:
        c2.close()
