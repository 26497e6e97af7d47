#!/usr/bin/env python3
"""Benchmark of the GPU hot path: full Stokes solves of the two-level,
chromosphere-like PRD problem (N_z = 70, N_nu = 101 on [-12, 12] Doppler
widths, 4+4 Gauss-Legendre mu x 8 azimuths, seeded atmosphere, tolerance 1e-8).

One step = one whole pass of the method on a fresh seeded atmosphere:
per-height setup, device precompute (R_II kernels by product integration,
R_III weights, propagation matrix, normalisation, right-hand side), the
tables of the physics-based preconditioner (Sect. 5.3, App. F) and the
left-preconditioned GMRES solve to tolerance (mixed precision: FP32 inner
operator, FP64 Arnoldi, residual and iterative refinement; or plain FP64 with
--precision fp64; --precond-sweeps 0 solves without the preconditioner).

Prints one JSON line.  `value` is solves/s; `roofline` covers the dominant
kernel (the FP32 R_II contraction), timed with HIP events on the library's
stream over the timed region; `cpu_baseline` times the FP64 oracle on a
bounded sample of the same workload.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_contract_f32_cfg2_traffic.txt")


def _pct(v, q):
    s = sorted(v)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def measured_traffic():
    """HBM bytes per launch of the FP32 contraction from the committed counter
    summary, or None when the contraction's source changed since the counters
    were taken."""
    from paper_2505_20968_amd.profile_summary import contraction_source_hash
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as f:
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


def cpu_baseline(n_applies: float, seed: int, budget_heights: int = 1):
    """Time the FP64 oracle on a bounded sample of the workload and scale it to
    one full solve: setup + kernels and one Sigma per sampled height (scaled by
    N_z, Sigma being height-local) + the full Lambda, times the apply count
    the GPU solve needed."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from workloads import cfg2
    from oracle import transfer as T
    with threadpool_limits(limits=1):
        prob = cfg2(seed)
        t0 = time.perf_counter()
        op = T.setup(prob, {"normalize": False})
        t_setup = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        I = rng.random((prob.n_z, prob.n_dir, prob.n_nu, 4))
        zs = list(range(0, prob.n_z, max(1, prob.n_z // budget_heights)))[:budget_heights]
        t_first = t_second = 0.0
        for z in zs:
            t0 = time.perf_counter()
            T.sigma_height(op, z, I[z], normalize=False)      # builds this height's kernels
            t_first += time.perf_counter() - t0
            t0 = time.perf_counter()
            T.sigma_height(op, z, I[z], normalize=False)
            t_second += time.perf_counter() - t0
        t0 = time.perf_counter()
        T.formal_solve(op, I)
        t_formal = time.perf_counter() - t0
    k = len(zs)
    t_kernels = (t_first - t_second) / k * prob.n_z
    t_sigma = t_second / k * prob.n_z
    # +1 Sigma for the normalisation factor, +1 Lambda for the right-hand side
    t_solve = t_setup + t_kernels + (n_applies + 1) * t_sigma + (n_applies + 1) * t_formal
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on seed {seed}: setup, R_II/R_III kernels and one Sigma apply "
                       f"at {k} of {prob.n_z} heights (scaled by N_z; Sigma is height-local), "
                       f"one full Lambda; scaled to {n_applies:.1f} operator applies per solve "
                       f"(the oracle's unpreconditioned GMRES; apply count of an unpreconditioned "
                       f"GPU solve of the same atmosphere); single BLAS thread"),
            "seconds_measured": t_setup + t_first + t_second + t_formal,
            "seconds_per_solve_est": t_solve}


SERVE_STREAM = dict(n_z_range=(40, 70), nu_choices=(51, 71, 101), angle_sets=[(8, 4), (8, 8)])


def serving_bench(n_requests: int, seed: int, precond_sweeps: int):
    """Continuous-batching serving of a bounded request stream (all four atom/grid
    generators, N_z 40-70, N_nu 51-101, N_dir 32-64): saturated runs (all
    requests at t = 0) in mixed precision and in plain FP64; the mixed one fixes
    the arrival rate, then Poisson arrivals at 0.8 x that rate are served in
    both precisions."""
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
    sat64 = serve([Request(i, 0.0, p) for i, (_, p) in enumerate(base)], "fp64", max_active=16, **solver)
    lam = 0.8 * sat["solves_per_s"]
    runs = {}
    for prec in ("mixed", "fp64"):
        reqs = [Request(i, t / lam, p) for i, (t, p) in enumerate(base)]
        runs[prec] = summary(serve(reqs, prec, max_active=16, **solver))
    return {"requests": n_requests, "stream": "seeded mix of the four generators, N_z 40-70, N_nu 51-101, "
                                              "N_dir 32-64, tol 1e-8",
            "saturated_solves_per_s": {"mixed": sat["solves_per_s"], "fp64": sat64["solves_per_s"]},
            "arrival_rate_hz": lam, "precond_sweeps": precond_sweeps,
            "mixed": runs["mixed"], "fp64": runs["fp64"],
            "mixed_over_fp64_throughput": runs["mixed"]["solves_per_s"] / max(runs["fp64"]["solves_per_s"], 1e-30)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--precond-sweeps", type=int, default=4,
                    help="block-Jacobi steps of the physics-based preconditioner (0: none)")
    ap.add_argument("--serve-precond-sweeps", type=int, default=1,
                    help="the same for the serving measurement (its requests are smaller and its host "
                         "loop issues every request's preconditioner launches, so fewer steps pay)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests in the serving measurement (0 skips it)")
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

    import torch
    from paper_2505_20968_amd import Context, TRAP_FP32, TRAP_FP64
    from workloads import cfg2

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    mixed = args.precision == "mixed"
    ctx = Context(0)

    phases = {"set_problem": [], "precompute": [], "solve": []}
    sweeps = args.precond_sweeps

    def one_step(seed, sw=None, record=True):
        sw = sweeps if sw is None else sw
        prob = cfg2(seed)
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
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage = ctx.stage_times()
    ctx.profile(False)
    info = ctx.info()
    # the oracle solves without a preconditioner: its CPU estimate is scaled
    # to the applies of an unpreconditioned solve of the same atmosphere
    # (outside the timed region)
    plain = stats[0]
    if sweeps and not args.no_cpu_baseline:
        plain = one_step(2, sw=0, record=False)
    ctx.close()

    key = "fp32" if mixed else "fp64"
    cstage = stage["contract_fp32" if mixed else "contract_fp64"]
    flops = stage["flops_contraction"][key]
    cbytes = stage["bytes_contraction"][key]
    ms_c = cstage["ms"]
    achieved = flops / (ms_c * 1e-3) / 1e12 if ms_c > 0 else 0.0
    n_applies = sum(s["applies_fp32"] + s["applies_fp64"] for s in stats) / len(stats)
    plain_applies = plain["applies_fp32"] + plain["applies_fp64"]
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
        "config": {"workload": "two-level J0->1 PRD-AD chromosphere-like column: N_z=70, "
                               "N_nu=101 on [-12,12], 4+4 GL mu x 8 chi, seeded B/v/a/eps, tol 1e-8",
                   "precision": ("FP32 inner operator, FP64 Arnoldi/residual/refinement" if mixed
                                 else "FP64 throughout"),
                   "n_unknowns": info["n_unknowns"], "n_theta": info["n_theta"],
                   "n_slots": info["n_slots"], "restart": args.restart,
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
                     "frac": achieved / PEAK[key], "traffic": measured_traffic() if mixed else None,
                     "algorithmic_bytes_per_launch": cbytes / max(cstage["launches"], 1),
                     "algorithmic_flops_per_launch": flops / max(cstage["launches"], 1),
                     "kernel": ("k_contract_pipe<NH> (persistent FP32 contraction, both column classes)"
                                if mixed else "k_contract<double, NH>")},
    }
    if args.serve_requests > 0:
        out["serving"] = serving_bench(args.serve_requests, seed=5, precond_sweeps=args.serve_precond_sweeps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(plain_applies, seed=2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
