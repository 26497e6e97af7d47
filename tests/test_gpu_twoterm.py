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
  tests/golden/cfg4_nz2_emergent.txt (every 4th frequency), same script.
Both the plain FP64 GMRES and the mixed-precision solve (FP32 operator inside
FP64 iterative refinement) are checked to the parity contract: 1e-6 relative
on I, 1e-4 absolute on Q/I, U/I, V/I; the FP64 solve also on every Stokes
component to 1e-8 of the largest I (the U and V signals here are ~1e-5 of I,
below what the 1e-4 gate on U/I and V/I can see).  The Ly-alpha-like case is
also solved exactly as bench.py times it (tolerance 1e-8, restart 40, inner
tolerance 1e-7, four block-Jacobi steps of the preconditioner, zero initial
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
                         zero_guess=True, precond_sweeps=4)
    em = ctx.emergent(x)
    ctx.close()
    print(f"[lyman_alpha bench settings] {st}", flush=True)
    assert st["final_rel_res"] < 1e-8
    _check_contract("lyman_alpha bench settings", em, "cfg4_nz2_emergent.txt")
