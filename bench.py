#!/usr/bin/env python3
"""Benchmark of the GPU hot path: full Stokes solves of the polarised PRD
transfer problem on seeded chromosphere-like columns, by default the largest
configuration that fits one GPU: the two-term Ly-alpha-like line (N_z = 100,
N_nu = 301 on a sinh grid to +-1000 Doppler widths, 8+8 Gauss-Legendre mu x
8 azimuths, angle-dependent PRD; N = 15.4 M unknowns), tolerance 1e-8.
--config cfg2 / cfg3 selects the two-level column or the Mg II-like doublet.

One step = one whole pass of the method on a fresh seeded atmosphere:
per-height setup, device precompute (R_II kernels by product integration into
the banded store, R_III weights, propagation matrix, normalisation,
right-hand side), the tables of the physics-based preconditioner (Sect. 5.2,
App. F) and the left-preconditioned GMRES solve to tolerance (mixed
precision: FP32 inner operator, FP64 Arnoldi, residual and iterative
refinement; or plain FP64 with --precision fp64; --precond-sweeps 0 solves
without the preconditioner).

Prints one JSON line.  `value` is solves/s; `roofline` covers the emissivity
apply's dominant kernel (the FP32 R_II contraction), timed with HIP events on
the library's stream over the timed region, with its algorithmic flops (16
per in-band kernel entry and incoming slot); `sigma_apply` the whole FP32
Sigma apply against the same flops; `accuracy` the timed solve's emergent
profiles against a tight FP64 solve of the same atmosphere; `ad_vs_aa` solves
that atmosphere again with angle-averaged PRD (Sect. 5.2) and reports its
time and the emergent AD - AA differences (the comparison of Sect. 6.6);
`serving` a bounded request stream (mixed precision against FP64);
`cpu_baseline` times the FP64 oracle on a bounded sample of the same workload.
Everything after the timed steps runs outside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = ("Stokes solves/s + emissivity-apply GB/s or TFLOP/s at 1e-6 rel; "
          "p50/p99 latency")
PEAK = {"fp32": 157.3, "fp64": 78.6}     # dense TFLOP/s, MI355X published figures
HBM_PEAK = 8000.0                        # GB/s
COPY_PROBE_BYTES = 256 << 20
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_contract_f32_{}_traffic.txt")


def _gen(name):
    def make(seed):
        import workloads
        return getattr(workloads, name)(seed)
    return make


# workload generator, description, default timed steps, default preconditioner
# steps (a block-Jacobi step costs about 1 % of an operator apply at the
# Ly-alpha-like size, where 32 steps cut the iterations from 10 to 7, and
# about 6 % at cfg2, where 4 steps do best)
CONFIGS = {
    "cfg2": (_gen("cfg2"), "two-level J0->1 PRD-AD chromosphere-like column: N_z=70, N_nu=101 on [-12,12], "
                           "4+4 GL mu x 8 chi, seeded B/v/a/eps, tol 1e-8", 5, 4),
    "cfg3": (_gen("cfg3"), "two-term 2S1/2 -> 2P1/2,3/2 Mg II h&k-like doublet (fine structure 20 Doppler "
                           "widths, J-state interference), PRD-AD: N_z=80, N_nu=200 to +-50, 6+6 GL mu x 8 chi, "
                           "seeded chromosphere-like column, tol 1e-8", 3, 4),
    "cfg4": (_gen("cfg4"), "two-term H I Ly-alpha-like line (fine structure 0.3 Doppler width, a 1e-2..1e-1, "
                           "|B| 1-300 G), PRD-AD: N_z=100, N_nu=301 on a sinh grid to +-1000 Doppler widths, "
                           "8+8 GL mu x 8 chi, seeded chromosphere-like column, tol 1e-8", 3, 32),
}


def _pct(v, q):
    s = sorted(v)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def measured_traffic(config):
    """HBM bytes per launch of the FP32 contraction from the committed counter
    summary of this workload, or None when the contraction's source changed
    since the counters were taken."""
    from paper_2505_20968_amd.profile_summary import contraction_source_hash
    path = TRAFFIC_FILE.format(config)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("contraction_source_sha256") != contraction_source_hash():
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _subcolumn(prob, zs):
    """The same atmosphere restricted to the heights zs (bottom to top)."""
    import numpy as np
    import dataclasses
    zs = np.asarray(zs)
    kw = {}
    for f in ("tau_line", "T", "xi", "a", "eps", "W_T", "v", "B"):
        kw[f] = np.asarray(getattr(prob, f))[zs]
    for f in ("kappa_c", "sigma_c"):
        v = getattr(prob, f, None)
        kw[f] = None if v is None else np.asarray(v)[zs]
    return dataclasses.replace(prob, **kw)


def _oracle_sample(prob, n_applies: float, threads: int, heights: int = 4, kernels_per_height: int = 2):
    """Seconds of one oracle solve of `prob`, estimated from a bounded sample of
    the oracle's own work at the workload's full frequency and angle grids:
    its per-height set-up and formal solution on `heights` heights of the
    column (scaled by N_z / heights; both are height-local), its kernel
    matrices (kernels_per_height per sampled height, at angles spread over the
    Theta table; scaled by N_z N_Theta N_t, the kernels the apply builds), and
    the kernel-times-field products of the Sigma apply (scaled by their count
    N_z n_up n_lo N_dir^2).  The apply's angular and sublevel sums and its
    interpolations are not timed, so the estimate is a lower bound on the
    oracle's time."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import transfer as T
    from oracle.redistribution import kernel_matrix
    nz = prob.n_z
    zs = np.unique(np.linspace(0, nz - 1, heights).round().astype(int))
    sub = _subcolumn(prob, zs)
    rng = np.random.default_rng(0)
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        op = T.setup(sub, {"normalize": False})
        t_setup = (time.perf_counter() - t0) * nz / len(zs)
        I = rng.random((sub.n_z, sub.n_dir, sub.n_nu, 4))
        t0 = time.perf_counter()
        T.formal_solve(op, I)
        t_formal = (time.perf_counter() - t0) * nz / len(zs)
        nth = len(op.theta)
        th_pick = [k for k in np.linspace(1, nth - 1, kernels_per_height).round().astype(int)]
        nU, nL = op.atoms[0].E_u.size, op.atoms[0].E_l.size
        t0 = time.perf_counter()
        nk = 0
        for zi in range(len(zs)):
            for j, th in enumerate(th_pick):
                u, l = (zi + j) % nU, (zi * 3 + j) % nL
                kernel_matrix(op.theta[th], op.s_ul[zi, u, l], sub.a[zi], op.lam[zi], op.basis)
                nk += 1
        t_kernels = (time.perf_counter() - t0) / nk * nz * nth * nU * nL
        M = rng.random((sub.n_nu, sub.n_nu)) + 1j * rng.random((sub.n_nu, sub.n_nu))
        Ib = rng.random((sub.n_nu, 4))
        reps = 256
        t0 = time.perf_counter()
        for _ in range(reps):
            M @ Ib
        t_prod = (time.perf_counter() - t0) / reps * nz * nU * nL * prob.n_dir ** 2
    # one Sigma for the normalisation factor and one Lambda for the right-hand side
    t_solve = t_setup + t_kernels + (n_applies + 1) * (t_prod + t_formal)
    return t_solve, {"setup_s": t_setup, "kernels_s": t_kernels, "apply_products_s": t_prod,
                     "formal_s": t_formal, "kernels_sampled": nk, "heights_sampled": int(len(zs))}


def cpu_baseline(prob, n_applies: float):
    """The oracle on the host's cores (all of this process's affinity set, BLAS
    threads pinned to it) and on one core, from the bounded sample of
    _oracle_sample; solves/s of the full workload, scaled and labelled."""
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    t_all, parts = _oracle_sample(prob, n_applies, cores)
    t_one, _ = _oracle_sample(prob, n_applies, 1)
    measured = time.perf_counter() - t0
    return {"value": 1.0 / t_all, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "value_1_core": 1.0 / t_one,
            "sample": (f"FP64 oracle on the same workload ({prob.name}, full frequency and angle grids): "
                       f"set-up and formal solution on {parts['heights_sampled']} of {prob.n_z} heights, "
                       f"{parts['kernels_sampled']} kernel matrices at those heights, 256 kernel-times-field "
                       f"products; scaled to one solve with {n_applies:.1f} operator applies (the GPU solve's "
                       f"count) by N_z, the kernel count and the product count; the apply's angular sums and "
                       f"interpolations are not timed (a lower bound on the oracle's time, so an upper bound on "
                       f"its solves/s); scaled estimate, not a measured full solve"),
            "estimate_s": {"all_cores": t_all, "one_core": t_one, **parts},
            "seconds_measured": measured}


# a bounded stream over the serving configuration's full ranges: N_z 40-100,
# N_nu 31-301, N_dir 16-128, all four generators
SERVE_STREAM = dict(n_z_range=(40, 100), nu_choices=tuple(range(31, 302, 30)),
                    angle_sets=[(4, 4), (8, 4), (8, 8), (12, 8), (16, 8)])


def serving_bench(n_requests: int, seed: int, precond_sweeps: int):
    """Continuous-batching serving of a bounded request stream (all four atom/grid
    generators over the full serving ranges): saturated runs (all requests at
    t = 0) in mixed precision and in plain FP64, both to the same FP64 residual
    tolerance; the mixed one fixes the arrival rate, then Poisson arrivals at
    0.8 x that rate are served in both precisions."""
    from workloads import serving_stream
    from paper_2505_20968_amd.serving import Request, serve
    base = serving_stream(n_requests, seed=seed, rate_hz=1.0, **SERVE_STREAM)
    solver = dict(tol=1e-8, restart=40, inner_tol=1e-7, max_outer=10, max_iters=2000,
                  precond_sweeps=precond_sweeps)

    def summary(res):
        return {"solves_per_s": res["solves_per_s"], "p50_ms": 1e3 * res["p50_s"], "p99_ms": 1e3 * res["p99_s"],
                "n_ok": res["n_ok"], "n_rejected": res["n_rejected"], "n_failed": res["n_failed"],
                "peak_active": res["peak_active"], "wall_s": res["wall_s"]}

    sat = serve([Request(i, 0.0, p) for i, (_, p) in enumerate(base)], "mixed", max_active=16, **solver)
    _progress(f"serving: saturated mixed run done, {sat['solves_per_s']:.3f} solves/s")
    sat64 = serve([Request(i, 0.0, p) for i, (_, p) in enumerate(base)], "fp64", max_active=16, **solver)
    _progress(f"serving: saturated FP64 run done, {sat64['solves_per_s']:.3f} solves/s")
    lam = 0.8 * sat["solves_per_s"]
    runs = {}
    for prec in ("mixed", "fp64"):
        reqs = [Request(i, t / lam, p) for i, (t, p) in enumerate(base)]
        runs[prec] = summary(serve(reqs, prec, max_active=16, **solver))
        _progress(f"serving: paced {prec} run done")
    return {"requests": n_requests, "stream": "seeded mix of the four generators over the full serving ranges "
                                              "(N_z 40-100, N_nu 31-301, N_dir 16-128), tol 1e-8; "
                                              f"{n_requests} requests instead of 1024 to bound the run",
            "sizes": [[p.n_z, p.n_nu, p.n_dir] for _, p in base],
            "saturated_solves_per_s": {"mixed": sat["solves_per_s"], "fp64": sat64["solves_per_s"]},
            "arrival_rate_hz": lam, "precond_sweeps": precond_sweeps,
            "mixed": runs["mixed"], "fp64": runs["fp64"],
            "mixed_over_fp64_throughput": runs["mixed"]["solves_per_s"] / max(runs["fp64"]["solves_per_s"], 1e-30)}


def ad_versus_aa(prob, em_ad, tol, restart, sweeps, mixed):
    """Sect. 6.6 on the GPU at the bench's size: the same atmosphere solved with
    the angle-averaged redistribution (Sect. 5.2, Eq. R_AA) and the same solver
    settings, its wall time (set-up, precompute and solve) and the emergent
    differences from the timed angle-dependent solve."""
    import numpy as np
    import torch
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64, TRAP_PRD_AA
    ctx = Context(0)
    ctx.set_prd_mode(TRAP_PRD_AA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_problem(prob)
    ctx.precompute(3 if mixed else 1)
    if sweeps:
        ctx.precompute_preconditioner()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    st = ctx.gmres_solve(x, tol=tol, restart=restart, max_iters=2000, inner=TRAP_FP32 if mixed else TRAP_FP64,
                         max_outer=10, inner_tol=1e-7, zero_guess=True, precond_sweeps=sweeps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    em = ctx.emergent(x)
    info = ctx.info()
    ctx.close()
    d_rel_I = np.abs(em_ad[..., 0] - em[..., 0]) / np.abs(em_ad[..., 0])
    return {"what": "the timed atmosphere solved with angle-averaged PRD (same solver settings); "
                    "differences of the emergent profiles, AD minus AA",
            "aa_seconds": t2 - t0, "aa_precompute_s": t1 - t0, "aa_solve_s": t2 - t1,
            "aa_inner_iters": st["inner_iters"], "aa_final_rel_res": st["final_rel_res"],
            "aa_kernel_store_bytes": info["bytes_kernel_fp64"],
            "max_rel_dI": float(d_rel_I.max()),
            "max_abs_d_Q_over_I": float(np.abs(em_ad[..., 1] / em_ad[..., 0] - em[..., 1] / em[..., 0]).max()),
            "max_abs_d_U_over_I": float(np.abs(em_ad[..., 2] / em_ad[..., 0] - em[..., 2] / em[..., 0]).max()),
            "max_abs_d_V_over_I": float(np.abs(em_ad[..., 3] / em_ad[..., 0] - em[..., 3] / em[..., 0]).max()),
            "max_abs_Q_over_I_ad": float(np.abs(em_ad[..., 1] / em_ad[..., 0]).max())}


def _progress(msg: str) -> None:
    """One line on stderr per finished phase, so a long run shows where it is."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="cfg4",
                    help="workload (default: the largest configuration that fits one GPU)")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: per configuration)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--precond-sweeps", type=int, default=None,
                    help="block-Jacobi steps of the physics-based preconditioner (0: none)")
    ap.add_argument("--serve-precond-sweeps", type=int, default=1,
                    help="the same for the serving measurement (its requests are smaller and its host "
                         "loop issues every request's preconditioner launches, so fewer steps pay)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--no-aa", action="store_true",
                    help="skip the angle-averaged solve of the timed atmosphere (outside the timed region)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="before the timed region, run one elementwise kernel over a known byte "
                         "count (reads and writes 256 MiB) to calibrate HBM traffic counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "this build has no multi-GPU path: heights shard with zero communication for Sigma "
              "and one all-to-all per apply for Lambda", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64
    gen, workload, default_steps, default_sweeps = CONFIGS[args.config]
    if args.precond_sweeps is None:
        args.precond_sweeps = default_sweeps
    if args.steps is None:
        args.steps = default_steps

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    mixed = args.precision == "mixed"
    ctx = Context(0)

    phases = {"set_problem": [], "precompute": [], "solve": []}
    sweeps = args.precond_sweeps

    last = {}

    def one_step(seed, sw=None, record=True):
        sw = sweeps if sw is None else sw
        prob = gen(seed)
        t0 = time.perf_counter()
        ctx.set_problem(prob)
        t1 = time.perf_counter()
        ctx.precompute(3 if mixed else 1)
        if sw:
            # the tables overlap the precompute on the library's side stream
            ctx.precompute_preconditioner()
        torch.cuda.synchronize()         # both are asynchronous: attribute their time here
        t3 = t2 = time.perf_counter()
        x = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
        st = ctx.gmres_solve(x, tol=args.tol, restart=args.restart, max_iters=2000,
                             inner=TRAP_FP32 if mixed else TRAP_FP64, max_outer=10, inner_tol=1e-7,
                             zero_guess=True, precond_sweeps=sw)
        t4 = time.perf_counter()
        last.update(prob=prob, x=x, seed=seed)
        if not record:
            return st
        phases["set_problem"].append(t1 - t0)
        phases["precompute"].append(t2 - t1)     # with the preconditioner tables
        phases["solve"].append(t4 - t3)
        return st

    if args.copy_probe:
        xs = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        ys = torch.empty_like(xs)
        torch.neg(xs, out=ys)
        torch.cuda.synchronize()
        del xs, ys
    for i in range(args.warmup):
        one_step(1000 + i)
        _progress(f"warmup step {i} done")
    for v in phases.values():
        v.clear()
    torch.cuda.synchronize()
    ctx.profile(True)
    lat, stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st = one_step(2 + i)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        stats.append(st)
        _progress(f"timed step {i} done: {lat[-1]:.2f} s, {st['inner_iters']} inner iterations")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage = ctx.stage_times()
    ctx.profile(False)
    info = ctx.info()
    # outside the timed region: (1) the timed solve's emergent profiles against
    # a tight FP64 solve of the same atmosphere (the parity contract: 1e-6
    # relative on I, 1e-4 absolute on Q/I, U/I, V/I); (2) whole FP32 Sigma
    # applies timed with events, against the contraction's algorithmic flops
    em = ctx.emergent(last["x"])
    xt = torch.zeros(ctx.shape, dtype=torch.float64, device="cuda")
    stt = ctx.gmres_solve(xt, tol=1e-12, restart=args.restart, max_iters=4000, inner=TRAP_FP64, max_outer=20,
                          inner_tol=1e-7, zero_guess=True, precond_sweeps=sweeps)
    ref = ctx.emergent(xt)
    accuracy = {"reference": "FP64 GMRES to 1e-12 of the last timed atmosphere",
                "reference_final_rel_res": stt["final_rel_res"],
                "max_rel_I": float((np.abs(em[..., 0] - ref[..., 0]) / np.abs(ref[..., 0])).max()),
                "max_rel_I_over_max": float(np.abs(em[..., 0] - ref[..., 0]).max() / np.abs(ref[..., 0]).max()),
                "max_abs_QUV_over_I": float(max(np.abs(em[..., s] / em[..., 0] - ref[..., s] / ref[..., 0]).max()
                                                for s in (1, 2, 3)))}
    accuracy["within_contract"] = accuracy["max_rel_I"] < 1e-6 and accuracy["max_abs_QUV_over_I"] < 1e-4
    _progress(f"accuracy check done: {accuracy}")
    del xt
    xs = torch.rand(ctx.shape, dtype=torch.float32, device="cuda")
    ys = torch.empty_like(xs)
    ctx.apply_sigma(xs, ys)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_sig = 5
    ev0.record(ctx.stream)
    for _ in range(n_sig):
        ctx.apply_sigma(xs, ys)
    ev1.record(ctx.stream)
    ev1.synchronize()
    sigma_ms = ev0.elapsed_time(ev1) / n_sig
    _progress(f"Sigma apply timing done: {sigma_ms:.2f} ms")
    del xs, ys
    ctx.close()

    key = "fp32" if mixed else "fp64"
    cstage = stage["contract_fp32" if mixed else "contract_fp64"]
    flops = stage["flops_contraction"][key]
    cbytes = stage["bytes_contraction"][key]
    ms_c = cstage["ms"]
    achieved = flops / (ms_c * 1e-3) / 1e12 if ms_c > 0 else 0.0
    n_applies = sum(s["applies_fp32"] + s["applies_fp64"] for s in stats) / len(stats)
    apply_ms = {k: v["ms"] / max(v["launches"], 1) for k, v in stage.items() if isinstance(v, dict) and "ms" in v}
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "name": args.config, "tol": args.tol,
                   "precision": ("FP32 inner operator, FP64 Arnoldi/residual/refinement" if mixed
                                 else "FP64 throughout"),
                   "n_unknowns": info["n_unknowns"], "n_theta": info["n_theta"],
                   "n_slots": info["n_slots"], "restart": args.restart,
                   "kernel_entries_in_band": info["kernel_entries"],
                   "kernel_entries_in_fp32_windows": info["kernel_entries_fp32"],
                   "kernel_store_bytes": info["bytes_kernel_fp64"],
                   "device_bytes": info["bytes_device_total"],
                   "preconditioner": (f"physics-based P = Id - Lambda* Sigma* (unmagnetised, unpolarised, "
                                      f"angle-averaged), {sweeps} block-Jacobi steps with the App. F "
                                      f"local inverse" if sweeps else "none")},
        "latency_ms": {"p50": 1e3 * _pct(lat, 0.5), "p99": 1e3 * _pct(lat, 0.99)},
        "phase_ms": {k: 1e3 * sum(v) / len(v) for k, v in phases.items()},
        "solver": {"inner_iters_mean": sum(s["inner_iters"] for s in stats) / len(stats),
                   "outer_steps_mean": sum(s["outer_steps"] for s in stats) / len(stats),
                   "applies_mean": n_applies,
                   "precond_applies_mean": sum(s["applies_precond"] for s in stats) / len(stats),
                   "max_final_rel_res": max(s["final_rel_res"] for s in stats)},
        "emissivity_apply": {"contraction_tflops": achieved,
                             "contraction_ms_per_launch": ms_c / max(cstage["launches"], 1),
                             "contraction_launches": cstage["launches"],
                             "stage_ms_per_launch": apply_ms},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[key], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[key],
                     "traffic": measured_traffic(args.config) if mixed else None,
                     "algorithmic_bytes_per_launch": cbytes / max(cstage["launches"], 1),
                     "algorithmic_flops_per_launch": flops / max(cstage["launches"], 1),
                     "kernel": ("k_contract_res (resident-field FP32 contraction, both column classes)"
                                if mixed else "k_contract<double, NH>")},
        "sigma_apply": {"ms": sigma_ms, "flops": info["flops_contraction_fp32"],
                        "tflops": info["flops_contraction_fp32"] / (sigma_ms * 1e-3) / 1e12,
                        "frac_fp32_peak": info["flops_contraction_fp32"] / (sigma_ms * 1e-3) / 1e12 / PEAK["fp32"],
                        "what": "whole FP32 Sigma apply (comoving interpolation, contraction, R_III, angular "
                                "sum, back-interpolation) timed with events, against the FP32 contraction's "
                                "algorithmic flops (its column windows)"},
        "accuracy": accuracy,
    }
    if not args.no_aa:
        torch.cuda.empty_cache()
        out["ad_vs_aa"] = ad_versus_aa(last["prob"], em, args.tol, args.restart, sweeps, mixed)
        _progress(f"AD versus AA done: {out['ad_vs_aa']}")
    if args.serve_requests > 0:
        torch.cuda.empty_cache()
        out["serving"] = serving_bench(args.serve_requests, seed=5, precond_sweeps=args.serve_precond_sweeps)
        _progress("serving measurement done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(last["prob"], n_applies)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
