"""Summaries of rocprofv3 runs of ``bench.py`` on the 256^3 workload.

Reads the CSV output of three rocprofv3 runs from one directory:
  kt_kernel_stats.csv           --kernel-trace --stats   (per-kernel durations)
  fetch_counter_collection.csv  --pmc FETCH_SIZE         (KiB read per dispatch)
  write_counter_collection.csv  --pmc WRITE_SIZE         (KiB written per dispatch)
and optionally
  valu_counter_collection.csv   --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES
and writes ``traffic_gpe3d_256[_semi_implicit].json`` (read by bench.py) plus a markdown
summary, for the RK4IP step or (with bench.py --semi-implicit) the semi-implicit step.

The counters are scaled to bytes with the same counters read for one elementwise copy of
known size (bench.py --calibrate-copy: 256 MiB in, 256 MiB out).

    python -m paper_1204_4255_amd.rocprof_summary <csv dir> <out dir> [rk4ip | semi_implicit]
"""
from __future__ import annotations

import csv
import json
import os
import re
import sys
from collections import defaultdict

from .build import source_hash

POINTS = 256 ** 3
KINDS = {0: "D1", 1: "D2", 2: "FIRST", 4: "LAST2", 5: "U", 6: "AW", 7: "AS", 8: "AF", 9: "LF", 10: "XF", 11: "SI"}
# algorithmic HBM bytes per lattice point of each pass kind (complex64 = 8 B); the
# semi-implicit step's passes (D1, applied once or twice, and SI) read and write psi once
PASS_BYTES = {"FIRST": 24, "D2": 32, "LF": 32, "XF": 32, "LAST2": 24, "D1": 16, "SI": 16}
# the step forms profiled: file-name suffix and the extra benchmark switch
FORMS = {"rk4ip": ("", ""), "semi_implicit": ("_semi_implicit", " --semi-implicit")}
COPY_BYTES = 256 << 20
AXIS_RE = re.compile(r"k_axis<(\d+), (\d+), (true|false), (\d+), (true|false), (\d), (\d+)(?:, (true|false), (\d+))?>")


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def pass_of(name: str):
    """('LF:strided', template text) for a k_axis kernel name, else None."""
    m = AXIS_RE.search(name)
    if not m:
        return None
    kind = KINDS.get(int(m.group(2)), "?")
    layout = "contig" if m.group(3) == "true" else "strided"
    return f"{kind}:{layout}", m.group(0)


def _counters(path: str):
    """{kernel name: {counter: [values per dispatch]}}"""
    out = defaultdict(lambda: defaultdict(list))
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for r in csv.DictReader(fh):
            out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def _copy_kernel(cnt, counter: str):
    """The calibration copy: the elementwise kernel with the largest reading."""
    best = None
    for name, c in cnt.items():
        if "elementwise" in name and counter in c:
            v = max(c[counter])
            if best is None or v > best:
                best = v
    return best


def summarise(src: str, dst: str, commands: str, form: str = "rk4ip") -> dict:
    fetch = _counters(os.path.join(src, "fetch_counter_collection.csv"))
    write = _counters(os.path.join(src, "write_counter_collection.csv"))
    valu = _counters(os.path.join(src, "valu_counter_collection.csv"))
    stats = {}
    with open(os.path.join(src, "kt_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            stats[r["Name"]] = r
    cf = _copy_kernel(fetch, "FETCH_SIZE")
    cw = _copy_kernel(write, "WRITE_SIZE")
    fetch_factor = COPY_BYTES / 1024 / cf
    write_factor = COPY_BYTES / 1024 / cw
    kernels = {}
    rows = []
    for name in sorted(set(fetch) | set(stats)):
        p = pass_of(name)
        if not p or p[0].split(":")[0] not in PASS_BYTES:
            continue
        key, templ = p
        f = fetch.get(name, {}).get("FETCH_SIZE")
        w = write.get(name, {}).get("WRITE_SIZE")
        st = stats.get(name)
        alg = PASS_BYTES[key.split(":")[0]] * POINTS
        rec = {"kernel": templ, "algorithmic_bytes": alg}
        if f and w:
            fb = sum(f) / len(f) * 1024 * fetch_factor
            wb = sum(w) / len(w) * 1024 * write_factor
            rec.update({"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb, "ratio": (fb + wb) / alg,
                        "dispatches": len(f)})
        if st:
            rec.update({"calls": int(st["Calls"]), "average_ns": float(st["AverageNs"]),
                        "min_ns": float(st["MinNs"]), "max_ns": float(st["MaxNs"]),
                        "percent": float(st["Percentage"])})
            rec["achieved_GBps"] = alg / float(st["AverageNs"])
        v = valu.get(name)
        if v and "SQ_INSTS_VALU" in v:
            mean = lambda c: sum(v[c]) / len(v[c]) if c in v else None
            rec["valu_insts"] = mean("SQ_INSTS_VALU")
            rec["lds_insts"] = mean("SQ_INSTS_LDS")
            rec["lds_bank_conflict_cycles"] = mean("SQ_LDS_BANK_CONFLICT")
            rec["waves"] = mean("SQ_WAVES")
            rec["valu_lane_insts_per_point"] = rec["valu_insts"] * 64 / POINTS
            if st:
                # one wave64 VALU instruction per CU per clock: 256 CUs at 2.4 GHz
                rec["valu_issue_frac"] = rec["valu_insts"] / (256 * 2.4e9 * float(st["AverageNs"]) * 1e-9)
        # several template instances can map to one pass kind: keep the one with most calls
        if key in kernels and kernels[key].get("calls", 0) >= rec.get("calls", 0):
            continue
        kernels[key] = rec
    out = {"source_hash": source_hash(), "workload": "gpe3d_256^3", "form": form,
           "calibration": {"kernel": "torch elementwise x*1.0, 256 MiB in + 256 MiB out", "FETCH_SIZE_KiB": cf,
                           "WRITE_SIZE_KiB": cw, "fetch_factor": fetch_factor, "write_factor": write_factor},
           "commands": commands, "kernels": kernels}
    os.makedirs(dst, exist_ok=True)
    with open(os.path.join(dst, f"traffic_gpe3d_256{FORMS[form][0]}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def markdown(out: dict) -> str:
    lines = ["| pass | kernel | calls | average us | min us | max us | % GPU time | algorithmic GB/s | "
             "measured / algorithmic bytes | VALU lane-instr per point | VALU issue | LDS bank-conflict cycles |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for key, r in sorted(out["kernels"].items(), key=lambda kv: -kv[1].get("percent", 0)):
        f = lambda k, fmt: (fmt % r[k]) if r.get(k) is not None else "-"
        lines.append(f"| {key} | `{r['kernel']}` | {f('calls', '%d')} | {r.get('average_ns', 0) / 1e3:.1f} | "
                     f"{r.get('min_ns', 0) / 1e3:.1f} | {r.get('max_ns', 0) / 1e3:.1f} | {f('percent', '%.2f')} | "
                     f"{f('achieved_GBps', '%.0f')} | {f('ratio', '%.4f')} | {f('valu_lane_insts_per_point', '%.0f')} | "
                     f"{f('valu_issue_frac', '%.2f')} | {f('lds_bank_conflict_cycles', '%.3g')} |")
    return "\n".join(lines)


COMMANDS = """    cd /tmp && export TMPDIR=/tmp
    R=<repository root>; OUT=<a writable output directory>
    export RK4IP_TUNE_CACHE=$OUT/tune_gpe3d_256{sfx}.json
    python3 $R/bench.py --no-cpu-baseline --no-forms{sw} --steps 20 --warmup 5
    rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof{sfx} -o kt -- python3 $R/bench.py --no-cpu-baseline --no-forms{sw} --steps 50 --warmup 5 --calibrate-copy
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/prof{sfx} -o fetch -- python3 $R/bench.py --no-cpu-baseline --no-forms{sw} --steps 3 --warmup 1 --profile-steps 2 --calibrate-copy
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/prof{sfx} -o write -- python3 $R/bench.py --no-cpu-baseline --no-forms{sw} --steps 3 --warmup 1 --profile-steps 2 --calibrate-copy
    rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES --output-format csv -d $OUT/prof{sfx} -o valu -- python3 $R/bench.py --no-cpu-baseline --no-forms{sw} --steps 3 --warmup 1 --profile-steps 2
    cd $R && python3 -m paper_1204_4255_amd.rocprof_summary $OUT/prof{sfx} profiles {form}"""

COPY_GBPS = 5900.0  # a plain elementwise copy of 256 MiB in and out on this GPU


def report(out: dict, tune: str = "") -> str:
    cal = out["calibration"]
    form = out.get("form", "rk4ip")
    sfx, sw = FORMS[form]
    title = "the RK4IP step" if form == "rk4ip" else "the semi-implicit step"
    lines = [
        f"# Step kernels of the 256^3 3D GPE workload, {title}: rocprofv3 kernel trace and counters",
        "",
        "Commands (one MI355X, repository root). `RK4IP_TUNE_CACHE` keeps the schedules the",
        "autotuner picks in the first run, so every later run launches the same kernels:",
        "",
        COMMANDS.format(sfx=sfx, sw=sw, form=form),
        "",
        f"The last command writes this file and `traffic_gpe3d_256{sfx}.json`, which `bench.py{sw}` reads",
        f"for `roofline.traffic` while the kernel sources still hash to `{out['source_hash']}`.",
        "",
    ]
    if tune:
        lines += ["Schedules picked (tune cache: lines or columns, field order, values per thread,",
                  "minimum waves per SIMD):", "", "```", tune.strip(), "```", ""]
    lines += [
        "Calibration: `--calibrate-copy` runs one torch elementwise kernel that reads 256 MiB and",
        f"writes 256 MiB. It reads FETCH_SIZE = {cal['FETCH_SIZE_KiB']:.1f} KiB and WRITE_SIZE =",
        f"{cal['WRITE_SIZE_KiB']:.1f} KiB, so the counters are scaled by {cal['fetch_factor']:.4f} (fetch) and",
        f"{cal['write_factor']:.4f} (write) to bytes of HBM traffic.",
        "",
        "Columns:",
        "* Calls, durations and % of GPU time come from `kt_kernel_stats.csv`. That run also holds the",
        "  profiling plan's eager steps and the autotuner's launches, so call counts are not whole steps.",
        "* Algorithmic GB/s = the pass's algorithmic bytes (16, 24 or 32 B per point x 256^3) / average",
        "  duration.",
        "* Measured / algorithmic = (scaled FETCH + WRITE) / algorithmic bytes.",
        "* VALU lane-instructions per point = SQ_INSTS_VALU x 64 / 256^3.",
        "* VALU issue = SQ_INSTS_VALU / (256 CUs x 2.4 GHz x duration): the fraction of the chip's wave64",
        "  VALU issue slots (one per CU per clock without packed FP32).",
        "",
        markdown(out),
        "",
        "Template arguments of `k_axis`: (length, pass kind, contiguous axis, lines or columns per",
        "workgroup, noise drawn, field order 0 joint / 1 one after the other / 2 the same with the",
        "second load deferred / 3 one thread per field, values per thread, FP64 transforms, minimum",
        "waves per SIMD). Pass",
        "kinds: 0 = D1 (once, or twice where two semi-implicit steps meet), 1 = D2, 2 = FIRST,",
        "4 = LAST2, 9 = LF, 10 = XF, 11 = SI.",
        "",
        "Reading (thresholds: within 10% of the copy rate = HBM-bound; VALU issue above 0.6 and",
        "under half the copy rate = VALU-bound):",
    ]
    for key, r in sorted(out["kernels"].items(), key=lambda kv: -kv[1].get("percent", 0)):
        gbs = r.get("achieved_GBps")
        issue = r.get("valu_issue_frac")
        ratio = r.get("ratio")
        if gbs is None:
            continue
        kind = "HBM-bound" if gbs > 0.9 * COPY_GBPS else ("VALU-bound" if issue and issue > 0.6 else "mixed")
        lines.append(f"* {key}: {gbs:.0f} GB/s ({gbs / 8000:.0%} of 8 TB/s, {gbs / COPY_GBPS:.0%} of a copy), "
                     f"VALU issue {issue:.2f}, traffic {ratio:.3f}x algorithmic: {kind}."
                     if issue is not None and ratio is not None else f"* {key}: {gbs:.0f} GB/s: {kind}.")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    # python -m paper_1204_4255_amd.rocprof_summary <csv dir> <out dir> [rk4ip | semi_implicit]
    form = sys.argv[3] if len(sys.argv) > 3 else "rk4ip"
    res = summarise(sys.argv[1], sys.argv[2], COMMANDS.format(sfx=FORMS[form][0], sw=FORMS[form][1], form=form), form)
    tune = ""
    path = os.environ.get("RK4IP_TUNE_CACHE")
    if path and os.path.exists(path):
        tune = open(path).read()
    text = report(res, tune)
    with open(os.path.join(sys.argv[2], f"step_kernels_gpe3d_256{FORMS[form][0]}.md"), "w") as fh:
        fh.write(text)
    print(text)
