"""Reduce rocprofv3 CSV output to the short text summaries kept in profiles/.

    python -m paper_2505_20968_amd.profile_summary stats KERNEL_STATS_CSV OUT --command "..."
    python -m paper_2505_20968_amd.profile_summary traffic FETCH_CSV WRITE_CSV OUT --command "..."
    python -m paper_2505_20968_amd.profile_summary counters PASS_CSV [PASS_CSV ...] OUT --command "..."

`stats` keeps the per-kernel table of a `--kernel-trace --stats` run.
`counters` sums `--pmc` passes per kernel and derives matrix-core busy time,
executed matrix-core flops, VALU and wait fractions of the wave cycles.
`traffic` takes two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a command
that also launched the calibration kernel (an elementwise negation reading and
writing COPY_BYTES), scales both counters by what they read for that kernel,
and records HBM bytes per launch of the FP32 contraction together with a hash
of the source file that holds the kernel and its launch configuration, so that
a stale figure is not reported after either changes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
SIGMA_SRC = os.path.join(HERE, "csrc", "sigma.hip")
COPY_BYTES = 256 << 20
CONTRACT_NAME = "k_contract_res"      # the resident-field FP32 contraction (one dispatch per height chunk)
COPY_NAME = "neg"


def contraction_source_hash() -> str:
    """Hash of the file holding the contraction kernel and its launch
    configuration (height chunking, column groups): any change there makes a
    stored traffic figure stale."""
    with open(SIGMA_SRC) as f:
        src = f.read()
    return hashlib.sha256(src.encode()).hexdigest()


def _short(name: str, width: int = 72) -> str:
    name = name.split("(")[0] if "(" in name and not name.startswith("void at::") else name
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(path: str, out: str, command: str, top: int = 25) -> None:
    with open(path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"command: {command}", f"source: {os.path.basename(path)}",
             f"total kernel time: {total / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} dispatches",
             "",
             f"{'kernel':72s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{_short(r['Name']):72s} {int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                     f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['MinNs']) / 1e3:9.1f} "
                     f"{float(r['MaxNs']) / 1e3:9.1f} {100 * float(r['TotalDurationNs']) / total:6.1f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_by_kernel(path: str, counter: str):
    vals: dict[str, list[float]] = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _pick(vals, needle):
    hits = {k: v for k, v in vals.items() if needle in k}
    if not hits:
        raise SystemExit(f"no dispatch of a kernel named like {needle!r}")
    return [x for v in hits.values() for x in v]


def _names_kernel(name: str, needle: str) -> bool:
    """True when the kernel's name is `needle` itself, or a template instance
    of it (`needle<...>`): not a kernel whose name only starts like it."""
    base = name.split("(")[0].replace("void ", "").strip()
    base = base.split("::")[-1] if "::" in base and not base.split("::")[-1].startswith("<") else base
    return base == needle or base.startswith(needle + "<")


def _per_launch(vals, needle):
    """Mean counter value of one launch of the stage: the stage issues one
    dispatch of each matching kernel, so the per-kernel means add up."""
    hits = {k: v for k, v in vals.items() if _names_kernel(k, needle)}
    if not hits:
        raise SystemExit(f"no dispatch of a kernel named like {needle!r}")
    return sum(statistics.mean(v) for v in hits.values()), {k.split("(")[0]: len(v) for k, v in hits.items()}


def traffic(fetch_csv: str, write_csv: str, out: str, command: str) -> None:
    fv = _counter_by_kernel(fetch_csv, "FETCH_SIZE")
    wv = _counter_by_kernel(write_csv, "WRITE_SIZE")
    copy_kib = COPY_BYTES / 1024.0
    f_copy, w_copy = statistics.mean(_pick(fv, COPY_NAME)), statistics.mean(_pick(wv, COPY_NAME))
    f_scale, w_scale = copy_kib / f_copy, copy_kib / w_copy
    fmean, fn = _per_launch(fv, CONTRACT_NAME)
    wmean, wn = _per_launch(wv, CONTRACT_NAME)
    f_bytes = fmean * f_scale * 1024.0
    w_bytes = wmean * w_scale * 1024.0
    lines = [f"command: {command}",
             f"calibration kernel: elementwise negation over {COPY_BYTES} bytes "
             f"(FETCH_SIZE {f_copy:.0f} KiB -> scale {f_scale:.4f}; WRITE_SIZE {w_copy:.0f} KiB -> scale {w_scale:.4f})",
             f"kernels of one contraction launch (dispatch counts, FETCH_SIZE pass): {fn}; WRITE_SIZE pass: {wn}",
             f"fetch_bytes_per_launch: {f_bytes:.6e}",
             f"write_bytes_per_launch: {w_bytes:.6e}",
             f"traffic_bytes_per_launch: {f_bytes + w_bytes:.6e}",
             f"contraction_source_sha256: {contraction_source_hash()}"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(paths, out: str, command: str, xcds: int = 8, simds: int = 1024) -> None:
    """Per kernel: counters summed over dispatches (each pass divided by its
    own dispatch count), then
      mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / xcds * simds)
    (GRBM_GUI_ACTIVE adds the active cycles of every XCD; the busy cycles add
    over every SIMD), executed matrix-core flops = 512 x the MOPS counters,
    and SQ_ACTIVE_INST_VALU, SQ_WAIT_ANY, SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES."""
    tot: dict[str, dict[str, float]] = {}
    for path in paths:
        per: dict[str, dict[str, float]] = {}
        disp: dict[str, set] = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                k = r["Kernel_Name"].split("(")[0].replace("void ", "")
                per.setdefault(k, {}).setdefault(r["Counter_Name"], 0.0)
                per[k][r["Counter_Name"]] += float(r["Counter_Value"])
                disp.setdefault(k, set()).add(r["Dispatch_Id"])
        for k, v in per.items():
            d = tot.setdefault(k, {"dispatches": float(len(disp[k]))})
            for c, x in v.items():
                d[c] = x / len(disp[k])           # per dispatch
    lines = [f"command: {command}",
             f"per dispatch, averaged; mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {xcds} x {simds} SIMDs)",
             "",
             f"{'kernel':44s} {'disp':>6s} {'mfma_busy':>9s} {'mfma_GF':>9s} {'valu_act':>8s} {'wait_any':>8s} "
             f"{'wait_dep':>8s} {'valu/wave':>9s}"]
    for k, d in sorted(tot.items(), key=lambda kv: -kv[1].get("GRBM_GUI_ACTIVE", 0.0) * kv[1]["dispatches"]):
        g = d.get("GRBM_GUI_ACTIVE", 0.0)
        busy = d.get("SQ_VALU_MFMA_BUSY_CYCLES")
        mb = f"{100 * busy / (g / xcds * simds):8.1f}%" if busy is not None and g else f"{'-':>9s}"
        gf = sum(d.get(c, 0.0) for c in ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64",
                                          "SQ_INSTS_VALU_MFMA_MOPS_F16", "SQ_INSTS_VALU_MFMA_MOPS_BF16")) * 512 / 1e9
        wc = d.get("SQ_WAVE_CYCLES")

        def frac(c):
            return f"{d[c] / wc:8.3f}" if wc and c in d else f"{'-':>8s}"
        vpw = f"{d['SQ_INSTS_VALU'] / d['SQ_WAVES']:9.0f}" if "SQ_INSTS_VALU" in d and d.get("SQ_WAVES") else f"{'-':>9s}"
        lines.append(f"{_short(k, 44):44s} {int(d['dispatches']):6d} {mb} {gf:9.2f} {frac('SQ_ACTIVE_INST_VALU')} "
                     f"{frac('SQ_WAIT_ANY')} {frac('SQ_WAIT_INST_ANY')} {vpw}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("out")
    b.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csvs", nargs="+")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    args = ap.parse_args()
    if args.mode == "stats":
        stats(args.csv, args.out, args.command)
    elif args.mode == "counters":
        counters(args.csvs, args.out, args.command)
    else:
        traffic(args.fetch_csv, args.write_csv, args.out, args.command)


if __name__ == "__main__":
    main()
