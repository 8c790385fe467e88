"""Summaries of rocprofv3 output for the batched solve.

    python -m paper_2503_13075_amd.rocprof_summary trace <dir>
    python -m paper_2503_13075_amd.rocprof_summary traffic <fetch dir> <write dir> <solves> <copy MiB> \
        <algorithmic bytes per solve> [json out] [launch tuning as JSON] [bench variant]
    python -m paper_2503_13075_amd.rocprof_summary valu <solves> <ms per solve> <dir> [<dir> ...]

``trace`` prints the kernel statistics of a ``--kernel-trace --stats`` run as
a markdown table.  ``traffic`` turns two ``--pmc FETCH_SIZE`` / ``--pmc
WRITE_SIZE`` runs of ``bench.py --calibrate-copy MiB`` into HBM bytes per
solve: the counters of every dispatch of the solve kernels are summed and
divided by the number of solves, and each counter is scaled by what it reads
for the plain device copy of known size that bench.py runs first (the
largest ``__amd_rocclr_copyBuffer`` dispatch).  ``valu`` sums the SQ / GRBM
counters of the solve kernels' dispatches in one or more ``--pmc`` runs per
solve and derives the FP64 / FP32 VALU flop rates (at the solve's duration,
against MI355X's vector peaks) and the fraction of SIMD cycles issuing VALU
work.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys

SOLVE_KERNELS = ("solve_kernel", "reset_counters", "copy_free_atoms")


def _csv(path_glob):
    files = sorted(glob.glob(path_glob, recursive=True))
    if not files:
        raise FileNotFoundError(path_glob)
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def trace_table(d: str) -> str:
    rows = _csv(os.path.join(d, "**", "*kernel_stats.csv"))
    out = ["| kernel | calls | total us | average us | min us | max us |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "")
        name = name.split("(")[0] if "solve_kernel" not in name else name.split(")(")[0] + ")"
        out.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} |")
    return "\n".join(out)


def solve_spans(d: str) -> list:
    """Per solve, the span from its queue-counter reset to the end of its
    last solve-kernel dispatch (ns), from a ``--kernel-trace`` run.  The
    launch groups of one solve run concurrently on several streams, so this
    span -- not any single dispatch -- is the solve's duration."""
    rows = _csv(os.path.join(d, "**", "*kernel_trace.csv"))
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    spans, start, end = [], None, None
    for t0, t1, name in ev:
        if "reset_counters" in name:
            if start is not None and end is not None:
                spans.append(end - start)
            start, end = t0, None
        elif start is not None and ("solve_kernel" in name or "small_kernel" in name):
            end = t1 if end is None else max(end, t1)
    if start is not None and end is not None:
        spans.append(end - start)
    return spans


def span_table(d: str) -> str:
    sp = solve_spans(d)
    if not sp:
        return "(no solves found)"
    us = [x / 1e3 for x in sp]
    return ("| solves | average span us | min us | max us |\n|---|---|---|---|\n"
            f"| {len(us)} | {sum(us) / len(us):.1f} | {min(us):.1f} | {max(us):.1f} |\n\n"
            "spans in order (us): " + ", ".join(f"{x:.1f}" for x in us))


def _counter(d: str, name: str):
    rows = _csv(os.path.join(d, "**", "*counter_collection.csv"))
    solve, copies = 0.0, []
    for r in rows:
        if r["Counter_Name"] != name:
            continue
        v = float(r["Counter_Value"])
        if any(k in r["Kernel_Name"] for k in SOLVE_KERNELS):
            solve += v
        elif "copyBuffer" in r["Kernel_Name"]:
            copies.append(v)
    return solve, (max(copies) if copies else None)


def traffic(fetch_dir: str, write_dir: str, solves: int, copy_mib: int, algorithmic: float) -> dict:
    copy_bytes = copy_mib * (1 << 20)
    f_sum, f_copy = _counter(fetch_dir, "FETCH_SIZE")
    w_sum, w_copy = _counter(write_dir, "WRITE_SIZE")
    ff = copy_bytes / (f_copy * 1024.0)
    fw = copy_bytes / (w_copy * 1024.0)
    fetch = f_sum / solves * 1024.0 * ff
    write = w_sum / solves * 1024.0 * fw
    return {"fetch_bytes_per_solve": fetch, "write_bytes_per_solve": write,
            "traffic_bytes_per_solve": fetch + write, "fetch_calibration_factor": ff,
            "write_calibration_factor": fw, "raw_fetch_kib_per_solve": f_sum / solves,
            "raw_write_kib_per_solve": w_sum / solves, "algorithmic_bytes_per_solve": algorithmic,
            "traffic_over_algorithmic": (fetch + write) / algorithmic}


N_SIMD = 4 * 256                       # MI355X: 256 CUs of 4 SIMDs
PEAK_F64_VEC_TFLOPS = 78.6             # published vector FP64 peak
PEAK_F32_VEC_TFLOPS = 157.3            # published vector FP32 peak (packed)
CLOCK_HZ = 2.4e9                       # MI355X peak engine clock


def valu(dirs, solves: int, ms_per_solve: float) -> dict:
    """Per-solve counter sums of the solve kernels and derived rates.  Flops
    count every lane of a wave64 instruction (64 per add / mul /
    transcendental, 128 per fma), an upper bound when lanes are masked.  The
    rates use ``ms_per_solve``, the solve's duration measured outside the
    profiler (counter collection serialises the dispatches).  The VALU issue
    fraction is the share of the SIMDs' cycles over that duration that the
    solve's VALU instructions would occupy at 4 cycles each (a wave64
    instruction on a 16-lane SIMD): SQ_INSTS_VALU x 4 / (SIMDs x clock x
    duration)."""
    tot = {}
    for d in dirs:
        for r in _csv(os.path.join(d, "**", "*counter_collection.csv")):
            if any(k in r["Kernel_Name"] for k in SOLVE_KERNELS):
                tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    per = {k: v / solves for k, v in tot.items()}
    out = {"counters_per_solve": per, "ms_per_solve": ms_per_solve}
    sec = ms_per_solve / 1e3

    def flops(kind):
        keys = [f"SQ_INSTS_VALU_{op}_{kind}" for op in ("ADD", "MUL", "TRANS", "FMA")]
        if not all(k in per for k in keys):
            return None
        return 64.0 * (per[keys[0]] + per[keys[1]] + per[keys[2]] + 2.0 * per[keys[3]])

    for kind, peak in (("F64", PEAK_F64_VEC_TFLOPS), ("F32", PEAK_F32_VEC_TFLOPS)):
        f = flops(kind)
        if f is not None:
            out[f"{kind.lower()}_flops_per_solve"] = f
            out[f"{kind.lower()}_tflops"] = f / sec / 1e12
            out[f"{kind.lower()}_frac_of_peak"] = f / sec / 1e12 / peak
    if "SQ_INSTS_VALU" in per:
        out["valu_issue_fraction"] = per["SQ_INSTS_VALU"] * 4.0 / (N_SIMD * CLOCK_HZ * sec)
    return out


def main(argv=None):
    a = sys.argv[1:] if argv is None else argv
    if a and a[0] == "trace":
        print(trace_table(a[1]))
        print()
        print(span_table(a[1]))
    elif a and a[0] == "traffic":
        res = traffic(a[1], a[2], int(a[3]), int(a[4]), float(a[5]))
        from .build import kernel_source_hash
        res["kernel_source_sha256_16"] = kernel_source_hash()
        if len(a) > 7:
            res["tuning"] = json.loads(a[7])
        if len(a) > 8:
            res["variant"] = a[8]
        text = json.dumps(res, indent=1)
        if len(a) > 6:
            with open(a[6], "w") as f:
                f.write(text + "\n")
        print(text)
    elif a and a[0] == "valu":
        res = valu(a[3:], int(a[1]), float(a[2]))
        from .build import kernel_source_hash
        res["kernel_source_sha256_16"] = kernel_source_hash()
        print(json.dumps(res, indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main())
