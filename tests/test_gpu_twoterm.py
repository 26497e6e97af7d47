"""Two-term workloads on their full frequency and angular grids, against the
oracle's emergent profiles at a reduced number of heights (the oracle's set-up
cost grows with the heights; the GPU path is the same at any height count).

* The Mg II-like doublet (2S_1/2 -> 2P_1/2,3/2, fine-structure splitting of 20
  Doppler widths, J-state interference): 200 frequencies spanning both
  components and the +-40 Doppler-width wings, 12 mu x 8 azimuths, 3 heights
  of the chromosphere-like generator.  Reference: tests/golden/cfg3_nz3_emergent.txt
  (every 4th frequency), written by tests/golden/make_reduced_emergent.py from
  the oracle alone, solved to 1e-11.
* The Ly-alpha-like line (fine-structure splitting of 0.3 Doppler width,
  damping 1e-2 - 1e-1, B up to 300 G): 301 frequencies on a sinh-spaced grid
  to +-1000 Doppler widths, 16 mu x 8 azimuths, 2 heights.  Reference:
  tests/golden/cfg4_nz2_emergent.txt (every 4th frequency), same script; its
  angle-averaged solve against tests/golden/cfg4_nz2_aa_emergent.txt, and the
  AD - AA difference of the two GPU solves against that of the goldens.
Both the plain FP64 GMRES and the mixed-precision solve (FP32 operator inside
FP64 iterative refinement) are checked to the parity contract: 1e-6 relative
on I, 1e-4 absolute on Q/I, U/I, V/I; the FP64 solve also on every Stokes
component to 1e-8 of the largest I (the U and V signals here are ~1e-5 of I,
below what the 1e-4 gate on U/I and V/I can see).  The Ly-alpha-like case is
also solved exactly as bench.py times it (tolerance 1e-8, restart 40, inner
tolerance 1e-7, 32 block-Jacobi steps of the preconditioner, zero initial
guess) and checked to the parity contract.
"""
import os

import numpy as np
import pytest

from workloads import cfg3, cfg4

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name, shape):
    g = np.loadtxt(os.path.join(HERE, "golden", name))
    ref = np.full(shape, np.nan)
    ref[g[:, 0].astype(int), g[:, 1].astype(int)] = g[:, 2:]
    return ref, g[:, 0].astype(int), g[:, 1].astype(int)


CASES = {"doublet": (lambda: cfg3(n_z=3), "cfg3_nz3_emergent.txt"),
         "lyman_alpha": (lambda: cfg4(n_z=2), "cfg4_nz2_emergent.txt")}


@pytest.mark.parametrize("inner", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_two_term_reduced_heights_matches_oracle(case, inner):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64
    make, golden = CASES[case]
    prob = make()
    ctx = Context(0)
    ctx.set_problem(prob)
    ctx.precompute(3 if inner == "mixed" else 1)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=1e-10, restart=40, max_iters=2000,
                         inner=TRAP_FP32 if inner == "mixed" else TRAP_FP64, inner_tol=1e-4, max_outer=10)
    em = ctx.emergent(x)
    ctx.close()
    ref, o, n = _golden(golden, em.shape)
    got, want = em[o, n], ref[o, n]
    relI = np.abs(got[:, 0] - want[:, 0]) / np.abs(want[:, 0])
    pol = max(np.abs(got[:, s] / got[:, 0] - want[:, s] / want[:, 0]).max() for s in (1, 2, 3))
    print(f"[{case} {inner}] {st['inner_iters']} iters, res {st['final_rel_res']:.2e}, "
          f"max rel I {relI.max():.2e}, max pol {pol:.2e}", flush=True)
    assert st["final_rel_res"] < 1e-10
    assert relI.max() < (1e-8 if inner == "fp64" else 1e-6)
    assert pol < 1e-4
    if inner == "fp64":
        full = np.abs(got - want).max(axis=0) / np.abs(want[:, 0]).max()
        print(f"[{case} fp64] max |diff| / max I per Stokes {full}", flush=True)
        assert full.max() < 1e-8


def _check_contract(tag, em, golden):
    ref, o, n = _golden(golden, em.shape)
    got, want = em[o, n], ref[o, n]
    relI = np.abs(got[:, 0] - want[:, 0]) / np.abs(want[:, 0])
    pol = max(np.abs(got[:, s] / got[:, 0] - want[:, s] / want[:, 0]).max() for s in (1, 2, 3))
    print(f"[{tag}] max rel I {relI.max():.2e}, max pol {pol:.2e}", flush=True)
    assert relI.max() < 1e-6
    assert pol < 1e-4


def test_lyman_alpha_solved_as_the_bench_times_it():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20968_amd import Context, TRAP_FP32
    ctx = Context(0)
    ctx.set_problem(cfg4(n_z=2))
    ctx.precompute(3)
    ctx.precompute_preconditioner()
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=1e-8, restart=40, max_iters=2000, inner=TRAP_FP32, max_outer=10, inner_tol=1e-7,
                         zero_guess=True, precond_sweeps=32)
    em = ctx.emergent(x)
    ctx.close()
    print(f"[lyman_alpha bench settings] {st}", flush=True)
    assert st["final_rel_res"] < 1e-8
    _check_contract("lyman_alpha bench settings", em, "cfg4_nz2_emergent.txt")


def _lyman_alpha_solve(mode, inner):
    import torch
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64
    ctx = Context(0)
    ctx.set_prd_mode(mode)
    ctx.set_problem(cfg4(n_z=2))
    ctx.precompute(3)
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=1e-10, restart=40, max_iters=2000,
                         inner=TRAP_FP32 if inner == "mixed" else TRAP_FP64, inner_tol=1e-7, max_outer=10,
                         zero_guess=True)
    em = ctx.emergent(x)
    ctx.close()
    return st, em


@pytest.mark.parametrize("inner", ["fp64", "mixed"])
def test_lyman_alpha_angle_averaged_matches_oracle(inner):
    """The angle-averaged redistribution (Sect. 5.2, Eq. R_AA) on the Ly-alpha-like
    grid, against tests/golden/cfg4_nz2_aa_emergent.txt (same script, 'aa')."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20968_amd import TRAP_PRD_AA
    st, em = _lyman_alpha_solve(TRAP_PRD_AA, inner)
    print(f"[lyman_alpha AA {inner}] {st}", flush=True)
    assert st["final_rel_res"] < 1e-10
    _check_contract(f"lyman_alpha AA {inner}", em, "cfg4_nz2_aa_emergent.txt")
    if inner == "fp64":
        ref, o, n = _golden("cfg4_nz2_aa_emergent.txt", em.shape)
        full = np.abs(em[o, n] - ref[o, n]).max(axis=0) / np.abs(ref[o, n][:, 0]).max()
        print(f"[lyman_alpha AA fp64] max |diff| / max I per Stokes {full}", flush=True)
        assert full.max() < 1e-8


def test_lyman_alpha_ad_versus_aa():
    """Sect. 6.6 compares the angle-dependent and angle-averaged redistribution
    on Ly-alpha.  Both solved on the GPU (mixed precision): their difference in
    I and Q/I is the oracle's difference (the two goldens) to the sum of the
    two solves' contract errors, and it is well above those errors (about 1 %
    in I and 1e-3 in Q/I here), so the GPU resolves the AD/AA effect."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20968_amd import TRAP_PRD_AA, TRAP_PRD_AD
    _, ad = _lyman_alpha_solve(TRAP_PRD_AD, "mixed")
    _, aa = _lyman_alpha_solve(TRAP_PRD_AA, "mixed")
    r_ad, o, n = _golden("cfg4_nz2_emergent.txt", ad.shape)
    r_aa, _, _ = _golden("cfg4_nz2_aa_emergent.txt", aa.shape)
    g_ad, g_aa, w_ad, w_aa = ad[o, n], aa[o, n], r_ad[o, n], r_aa[o, n]
    dI_gpu = (g_ad[:, 0] - g_aa[:, 0]) / g_ad[:, 0]
    dI_ref = (w_ad[:, 0] - w_aa[:, 0]) / w_ad[:, 0]
    dQ_gpu = g_ad[:, 1] / g_ad[:, 0] - g_aa[:, 1] / g_aa[:, 0]
    dQ_ref = w_ad[:, 1] / w_ad[:, 0] - w_aa[:, 1] / w_aa[:, 0]
    print(f"[lyman_alpha AD-AA] max |dI/I| {np.abs(dI_ref).max():.2e} (GPU off by {np.abs(dI_gpu - dI_ref).max():.1e}),"
          f" max |dQ/I| {np.abs(dQ_ref).max():.2e} (GPU off by {np.abs(dQ_gpu - dQ_ref).max():.1e})", flush=True)
    assert np.abs(dI_ref).max() > 5e-3 and np.abs(dQ_ref).max() > 5e-4
    assert np.abs(dI_gpu - dI_ref).max() < 3e-6
    assert np.abs(dQ_gpu - dQ_ref).max() < 2e-4
