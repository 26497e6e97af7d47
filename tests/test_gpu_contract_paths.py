"""The two FP32 R_II contractions (Sect. 4.3 banded store; the mixed precision
of Sect. 5.1).  Up to 312 frequencies one column group's comoving field over
every frequency fits in LDS and the resident-field kernel runs; past that the
chunked, pipelined kernel does.  Each is checked against the FP64 apply (which
is pinned to the oracle elsewhere) to FP32 rounding, 1e-6 of the largest
Stokes-I value in every component, on problems with both column classes
(theta bins of more than 16 and of at most 16 incoming directions), ragged
frequency counts and two heights."""
import numpy as np
import pytest

from workloads import tiny, two_term_atom

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n_nu,atom", [(97, "two_level"), (311, "two_level"), (305, "two_term"),
                                       (337, "two_level"), (409, "two_term")])
def test_fp32_contraction_matches_fp64(n_nu, atom):
    torch = _torch()
    from paper_2505_20968_amd import Context
    at = two_term_atom(1215.67, 1.008, 0.3) if atom == "two_term" else None
    prob = tiny(n_z=2, n_nu=n_nu, x_max=30.0, n_mu=8, n_chi=8, atom=at, seed=11, a=3e-2, v_z=2.0)
    ctx = Context(0)
    try:
        ctx.set_problem(prob)
        ctx.precompute(3)
        info = ctx.info()
        print(f"[contract paths] n_nu={n_nu}: {info['n_slots']} slots over {info['n_theta']} theta bins", flush=True)
        rng = np.random.default_rng(n_nu)
        I = rng.uniform(0.2, 1.0, (prob.n_z, prob.n_dir, prob.n_nu, 4))
        I[..., 0] += 4.0 * np.exp(-(prob.x / 3.0) ** 2)[None, None, :]
        I[..., 1:] = 0.1 * (I[..., 1:] - 0.6) * I[..., :1]
        out = {}
        for dt in (torch.float64, torch.float32):
            x = torch.tensor(I, dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ctx.apply_sigma(x, y)
            torch.cuda.synchronize()
            out[dt] = y.double().cpu().numpy()
        ref = out[torch.float64]
        assert np.isfinite(out[torch.float32]).all()
        err = np.abs(out[torch.float32] - ref).max(axis=(0, 1, 2)) / np.abs(ref[..., 0]).max()
        print(f"[contract paths] n_nu={n_nu} {atom}: FP32 vs FP64 per Stokes over max |eps_I| {err}", flush=True)
        assert err.max() < 1e-6
        assert np.abs(ref[..., 0]).max() > 0
    finally:
        ctx.close()
