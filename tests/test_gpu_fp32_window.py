"""The FP32 operator's column windows (Sect. 4.3 banded store; the mixed
precision of Sect. 5.1): the FP32 contraction steps through narrower windows
of the stored tiles (4.6 Gaussian widths, spline reach to 1e-9) than the FP64
one (6.6, reach to 1e-13).  On the Ly-alpha-like grid (sinh grid to +-1000
Doppler widths, 301 frequencies, two heights): the windows are narrower and
nested in the bands, and the FP32 Sigma apply agrees with the FP64 one to
FP32 rounding (1e-6 of the largest Stokes-I value, in every component; the
same build without the windows gives the same differences to three digits),
which a window that cut entries of the FP32 sum's size would break.  The FP64 apply
is pinned to the oracle elsewhere."""
import numpy as np
import pytest

from workloads import cfg4

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_fp32_windows_are_narrower_and_lose_nothing_at_fp32_resolution():
    torch = _torch()
    from paper_2505_20968_amd import Context
    prob = cfg4(n_z=2)
    ctx = Context(0)
    try:
        ctx.set_problem(prob)
        ctx.precompute(3)
        info = ctx.info()
        print(f"[fp32 windows] entries {info['kernel_entries']:.4e} -> {info['kernel_entries_fp32']:.4e}, "
              f"reach {info['band_reach']} -> {info['band_reach_fp32']}, flops "
              f"{info['flops_contraction']:.4e} -> {info['flops_contraction_fp32']:.4e}", flush=True)
        assert 0 < info["kernel_entries_fp32"] < info["kernel_entries"]
        assert 0 < info["band_reach_fp32"] < info["band_reach"]
        assert 0.4 * info["flops_contraction"] < info["flops_contraction_fp32"] < info["flops_contraction"]
        assert info["bytes_contraction_fp32"] < 0.5 * info["bytes_contraction_fp64"]
        rng = np.random.default_rng(7)
        I = rng.uniform(0.2, 1.0, (prob.n_z, prob.n_dir, prob.n_nu, 4))
        core = np.exp(-(prob.x / 3.0) ** 2)[None, None, :]
        I[..., 0] += 5.0 * core
        I[..., 1:] = 0.1 * (I[..., 1:] - 0.6) * I[..., :1]
        out = {}
        for dt in (torch.float64, torch.float32):
            x = torch.tensor(I, dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ctx.apply_sigma(x, y)
            torch.cuda.synchronize()
            out[dt] = y.double().cpu().numpy()
        ref = out[torch.float64]
        # against the Stokes-I scale: Q, U, V are about 1e-3 of I here, and the
        # FP32 sums carry rounding of the I-sized terms they are made of
        err = np.abs(out[torch.float32] - ref).max(axis=(0, 1, 2)) / np.abs(ref[..., 0]).max()
        print(f"[fp32 windows] FP32 vs FP64 Sigma per Stokes, over max |eps_I|: {err}", flush=True)
        assert err.max() < 1e-6
    finally:
        ctx.close()
