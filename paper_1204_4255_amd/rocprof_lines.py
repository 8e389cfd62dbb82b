"""Summary of rocprofv3 runs of ``bench.py --forms-only``: the whole-line kernels (1D
steps, adaptive integrator) and the other kernels of the forms.

Reads from one directory the CSV output of
  kt_kernel_stats.csv           --kernel-trace --stats   (per-kernel durations)
  valu_counter_collection.csv   --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES
and writes ``line_kernels_bench_forms.md`` plus ``counters_line_kernels.json`` (read by
bench.py for the VALU issue of the batched-path kernel while the kernel sources still hash to
the recorded value).

VALU issue of a dispatch = SQ_INSTS_VALU / (256 CUs x 2.4 GHz x its duration in the counter
run): the fraction of the chip's wave64 VALU issue slots it used (one per CU per clock
without packed FP32). Per kernel, the dispatches are weighted by duration.

    python -m paper_1204_4255_amd.rocprof_lines <csv dir> <out dir>
"""
from __future__ import annotations

import csv
import json
import os
import sys
from collections import defaultdict

from .build import source_hash

CUS, CLOCK = 256, 2.4e9

COMMANDS = """    cd /tmp && export TMPDIR=/tmp
    R=<repository root>; OUT=<a writable output directory>
    rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_forms -o kt -- python3 $R/bench.py --forms-only
    rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES --output-format csv -d $OUT/prof_forms -o valu -- python3 $R/bench.py --forms-only --forms other_workloads,batched_paths,uneven_batch,fp64_transforms,semi_implicit,ark45,potential_terms,bases
    cd $R && python3 -m paper_1204_4255_amd.rocprof_lines $OUT/prof_forms profiles"""

# the forms of the counter run (the adjoint form's torch.autograd comparison is left out)
# template arguments of the whole-line kernels, for the table
LEGEND = {
    "k_line_kstep": "(length, lines per workgroup, noise, values per thread, semi-implicit): the step with "
                    "the line's state in k-space",
    "k_line_step": "(length, lines per workgroup, noise, FP64 transforms, values per thread, semi-implicit, "
                   "noisy / non-local potential): the step in x-space (the FP64-transform form, the potential's "
                   "extra terms, the cosine / sine extension)",
    "k_line_basis": "(length, lines per workgroup, noise, values per thread, semi-implicit): cosine / sine "
                    "lines through the reordered n-point transform",
    "k_line_ark45": "(length, lines per workgroup, non-local potential, explicit method): the adaptive "
                    "Cash-Karp integrator",
}


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("rk4ip::", "").strip()


def summarise(src: str) -> dict:
    stats = {}
    with open(os.path.join(src, "kt_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            stats[_short(r["Name"])] = {"calls": int(r["Calls"]), "average_us": float(r["AverageNs"]) / 1e3,
                                        "total_ms": float(r["TotalDurationNs"]) / 1e6,
                                        "percent": float(r["Percentage"])}
    disp = defaultdict(dict)
    path = os.path.join(src, "valu_counter_collection.csv")
    if os.path.exists(path):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                d = disp[r["Dispatch_Id"]]
                d["name"] = _short(r["Kernel_Name"])
                d[r["Counter_Name"]] = float(r["Counter_Value"])
                d["dur"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e9
    agg = defaultdict(lambda: defaultdict(float))
    for d in disp.values():
        if d.get("dur", 0) <= 0 or "SQ_INSTS_VALU" not in d:
            continue
        a = agg[d["name"]]
        a["dur"] += d["dur"]
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAVES"):
            a[c] += d.get(c, 0.0)
        a["n"] += 1
        if d["dur"] > a["longest_dur"]:
            a["longest_dur"] = d["dur"]
            a["longest_issue"] = d["SQ_INSTS_VALU"] / (CUS * CLOCK * d["dur"])
    kernels = {}
    for name, st in stats.items():
        rec = dict(st)
        a = agg.get(name)
        if a and a["dur"] > 0:
            rec["valu_issue_frac"] = a["SQ_INSTS_VALU"] / (CUS * CLOCK * a["dur"])
            rec["lds_per_valu"] = a["SQ_INSTS_LDS"] / a["SQ_INSTS_VALU"] if a["SQ_INSTS_VALU"] else None
            rec["lds_bank_conflict_cycles_per_dispatch"] = a["SQ_LDS_BANK_CONFLICT"] / a["n"]
            rec["counter_dispatches"] = int(a["n"])
            rec["valu_issue_longest_dispatch"] = a["longest_issue"]
            rec["longest_dispatch_us"] = a["longest_dur"] * 1e6
        kernels[name] = rec
    return {"source_hash": source_hash(), "kernels": kernels}


def report(out: dict) -> str:
    lines = [
        "# Kernels of the benchmark's forms: rocprofv3 kernel trace and VALU counters",
        "",
        "The kernels behind `bench.py --forms-only` (the batched paths, semi-implicit, adaptive,",
        "potential-term, basis, uneven-batch and adjoint forms and the other workloads). Commands",
        "(one MI355X, repository root):",
        "",
        COMMANDS,
        "",
        f"The last command writes this file and `counters_line_kernels.json`, which `bench.py` reads",
        f"while the kernel sources still hash to `{out['source_hash']}`.",
        "",
        "The counter run leaves out the adjoint form: under counter collection the profiler ended",
        "with a host-side segmentation fault inside the form's torch.autograd comparison.",
        "",
        "Columns: calls and durations from the kernel trace (they mix every form that launches a",
        "kernel, and several steps run per launch where a form fuses them, so a launch is not a",
        "step; the forms' own event timings are in `bench.py`'s JSON). VALU issue = SQ_INSTS_VALU /",
        "(256 CUs x 2.4 GHz x duration) over the counter run's dispatches, weighted by duration;",
        "that average mixes full launches with the forms' small ones (a plan of one line, a",
        "conversion-only launch), so the issue of each kernel's longest dispatch (for the line",
        "kernels, a launch of many steps over the whole batch) is given beside it. Integer",
        "multiplies (Philox) and transcendentals issue at a quarter of the rate and count once.",
        "Rows: the 30 kernels of most GPU time, then every other whole-line and merged kernel.",
        "",
        "| kernel | calls | average us | total ms | % GPU time | VALU issue | VALU issue, longest dispatch (us) | LDS / VALU instr | bank-conflict cycles per dispatch |",
        "|---|---|---|---|---|---|---|---|---|",
    ]
    rows = sorted(out["kernels"].items(), key=lambda kv: -kv[1]["total_ms"])
    for i, (name, r) in enumerate(rows):
        if i >= 30 and not name.startswith(("k_line", "k_axis_merged")):
            continue
        iss = r.get("valu_issue_frac")
        lpv = r.get("lds_per_valu")
        bc = r.get("lds_bank_conflict_cycles_per_dispatch")
        li, ld = r.get("valu_issue_longest_dispatch"), r.get("longest_dispatch_us")
        lines.append(f"| `{name}` | {r['calls']} | {r['average_us']:.1f} | {r['total_ms']:.2f} | {r['percent']:.2f} | "
                     f"{'' if iss is None else f'{iss:.2f}'} | {'' if li is None else f'{li:.2f} ({ld:.0f})'} | "
                     f"{'' if lpv is None else f'{lpv:.3f}'} | {'' if bc is None else f'{bc:.3g}'} |")
    lines += ["", "Template arguments:"]
    lines += [f"* `{k}`: {v}." for k, v in LEGEND.items()]
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    res = summarise(sys.argv[1])
    with open(os.path.join(sys.argv[2], "counters_line_kernels.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    text = report(res)
    with open(os.path.join(sys.argv[2], "line_kernels_bench_forms.md"), "w") as fh:
        fh.write(text)
    print(text)
