"""Text summaries of rocprofv3 runs of bench.py, for the profiles/ folder.

Inputs are the rocpd databases rocprofv3 writes: one kernel-trace run with
--stats, and one --pmc run per HBM counter (FETCH_SIZE, then WRITE_SIZE), each
of a bench.py run that ends with the calibration kernel (--calib-copy-mib):
an elementwise negation that reads and writes a float32 buffer of known size
once.  The counters of that kernel against its true bytes give the scale of
each counter on the device; the kernels of the GLD step are then reported in
calibrated HBM bytes per launch.

Writes
  profiles/<name>.md            the kernel table and the traffic table, with
                                the commands that produced them
  profiles/<name>_traffic.json  per kernel class: calibrated bytes read and
                                written per launch, and the hash of the kernel
                                sources they were measured on (bench.py
                                reports the traffic only while it matches)

usage: python -m paper_1808_00270_amd.profile_summary --name NAME --kt DIR
       [--fetch DIR --write DIR --calib-bytes B] --cmd-kt "..." [--cmd-fetch
       "..." --cmd-write "..."] [--note "..."]
"""
from __future__ import annotations

import argparse
import collections
import glob
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# the kernels and their launchers (the traffic of a launch depends on these only)
SOURCES = ["gld_kernels.hip", "gld_pairs.hip", "gld_internal.h", "gld_device.h"]
SOURCES_KIND = {
    "single": SOURCES,
    "batch": ["gld_batch.hip", "gld_batch_dev.h", "gld_batch.cpp", "gld_device.h", "gld_internal.h"],
    "general": ["gld_general.hip", "gld_device.h"],
}

# kernel classes of the step (the names bench.py uses) -> kernel symbol, for
# the work type T of the precision (F: suffix of the FP64 filter-bank kernel)
CLASSES = {
    "noise_spmv": r"k_mvw?<{T}",  # k_mvw: the first pair term with P Y
    "history_step": r"k_history_step<{T}",
    "history_block": r"k_fir_mfma{F}<1[,>]",  # FP64: k_fir_mfma64<ROLE, row tiles>
    "noise_fir": r"k_fir_mfma{F}<0[,>]",
    "noise_white": r"k_white_ring<{T}",
    "neighbor_refresh": r"k_refresh<{T}",
    "neighbor_build": r"k_build<{T}",
    "update": r"k_update_[rv]\b",  # FP64 in both paths
}
# the batched engine's and the general engine's kernel classes
CLASSES_BATCH = {
    "noise_spmv": r"kb_spmv<{T}",
    "history": r"kb_history<{T}",
    "noise_fir": r"kb_fir",
    "noise_premix": r"kb_premix<{T}",
    "noise_white": r"kb_white<{T}",
    "neighbor_build": r"kb_build<{T}",
    "update": r"kb_update_[rv]<{T}",
}
CLASSES_GENERAL = {
    "lanczos": r"gen::.*k_lanczos\(",
    "dissipative": r"gen::.*k_dissipative\(",
    "dft": r"gen::.*k_dft_(slide|full)\(",
    "pairs": r"gen::.*k_pairs\(",
    "combine": r"gen::.*k_combine\(",
    "update": r"gen::.*k_(update_[rv]|white_step)\(",
}
CALIB = r"neg"


def source_hash(kind: str = "single") -> str:
    h = hashlib.sha256()
    for s in SOURCES_KIND[kind]:
        with open(os.path.join(HERE, "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^>(]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name if len(name) <= 60 else name[:57] + "..."


def db(path: str) -> sqlite3.Connection:
    files = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
    if not files:
        raise SystemExit(f"no rocpd database under {path}")
    return sqlite3.connect(files[0])


def kernel_table(path: str):
    c = db(path)
    return c.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()


def kernel_durations(path: str):
    """Per-dispatch durations (us), by kernel name."""
    c = db(path)
    acc = collections.defaultdict(list)
    for name, start, end in c.execute("select name, start, end from kernels"):
        acc[name].append((end - start) / 1e3)
    return acc


def counter_values(path: str, counter: str):
    """Counter value (KiB) of every dispatch, by kernel name."""
    c = db(path)
    rows = c.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    acc = collections.defaultdict(list)
    for _, name, v in rows:
        acc[name].append(v)
    return acc


def working(values):
    """The dispatches that did the class's work, and the number of the
    others: a launch below a quarter of the class median did next to nothing
    (the Chebyshev chain's first term, which has no pair term, and the terms
    beyond the K of the step's plan, which return at once).  The rebuild
    kernels and the filter bank work one launch in several; their median
    launch is the empty one, so they keep every launch."""
    v = sorted(values)
    med = v[len(v) // 2]
    keep = [x for x in values if x >= 0.25 * med]
    return keep, len(values) - len(keep)


def pick(table: dict, pattern: str):
    """(mean over the working dispatches, their count, launches that returned at once)."""
    vals = [x for k, v in table.items() if re.search(pattern, k) for x in v]
    if not vals:
        return None
    keep, skipped = working(vals)
    return (sum(keep) / len(keep), len(keep), skipped)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-bytes", type=float, default=0.0)
    ap.add_argument("--cmd-kt", required=True)
    ap.add_argument("--cmd-fetch", default="")
    ap.add_argument("--cmd-write", default="")
    ap.add_argument("--note", default="")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="kernel classes of this path (work type float or double)")
    ap.add_argument("--kind", choices=("single", "batch", "general"), default="single",
                    help="which engine's kernel classes to report")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args()
    table = {"single": CLASSES, "batch": CLASSES_BATCH, "general": CLASSES_GENERAL}[a.kind]
    classes = {k: v.format(T="float" if a.precision == "fp32" else "double", F="" if a.precision == "fp32" else "64")
               for k, v in table.items()}

    lines = [f"# {a.name}", ""]
    if a.note:
        lines += [a.note, ""]
    lines += ["Kernel trace:", "", "    " + a.cmd_kt, "",
              "| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    kt = kernel_table(a.kt)
    for name, calls, total, avg, pctg in kt[:16]:
        lines.append(f"| `{short(name)}` | {calls} | {avg:.1f} | {total / 1e3:.2f} | {pctg:.1f} |")
    lines += ["", "Average duration per launch by kernel class (" + a.precision + " path; launches below a "
              "quarter of the class median did next to nothing and are counted apart"
              + (": the chain's first term and the terms beyond the K of the step's noise plan" if a.kind == "single"
                 else "") + "):", ""]
    avg_by_class = {}
    durs = kernel_durations(a.kt)
    for cls, pat in classes.items():
        d = pick(durs, pat)
        if d:
            avg_by_class[cls] = d[0]
            extra = f" (+ {d[2]} that did next to nothing)" if d[2] else ""
            lines.append(f"- {cls} (`{pat}`): {d[0]:.1f} us over {d[1]} launches{extra}")
    out = {"name": a.name, "precision": a.precision, "kind": a.kind, "source_sha256": source_hash(a.kind),
           "avg_us": avg_by_class, "kernels": {}}

    if a.fetch and a.write and a.calib_bytes > 0:
        fe = counter_values(a.fetch, "FETCH_SIZE")
        wr = counter_values(a.write, "WRITE_SIZE")
        cf, cw = pick(fe, CALIB), pick(wr, CALIB)
        if cf is None or cw is None:
            raise SystemExit("calibration kernel not found in the counter runs")
        sf = cf[0] * 1024.0 / a.calib_bytes  # counter bytes per true byte
        sw = cw[0] * 1024.0 / a.calib_bytes
        out["calibration"] = {"bytes": a.calib_bytes, "fetch_kib": cf[0], "write_kib": cw[0],
                              "fetch_scale": sf, "write_scale": sw}
        lines += ["", "HBM traffic per launch (FETCH_SIZE and WRITE_SIZE, one counter per run):", "",
                  "    " + a.cmd_fetch, "    " + a.cmd_write, "",
                  f"Calibration: negation of {a.calib_bytes / 2**20:.0f} MiB float32 (reads and writes "
                  f"{a.calib_bytes:.0f} B): FETCH_SIZE {cf[0]:.0f} KiB (scale {sf:.4f}), "
                  f"WRITE_SIZE {cw[0]:.0f} KiB (scale {sw:.4f}).", "",
                  "| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | read (MB) | written (MB) |",
                  "|---|---:|---:|---:|---:|---:|"]
        for cls, pat in classes.items():
            f, w = pick(fe, pat), pick(wr, pat)
            if f is None or w is None:
                continue
            rb, wb = f[0] * 1024.0 / sf, w[0] * 1024.0 / sw
            out["kernels"][cls] = {"read_bytes": rb, "write_bytes": wb, "traffic_bytes": rb + wb,
                                   "dispatches": f[1]}
            lines.append(f"| {cls} (`{pat}`) | {f[1]} | {f[0]:.0f} | {w[0]:.0f} | {rb / 1e6:.1f} | "
                         f"{wb / 1e6:.1f} |")
    lines += ["", f"Kernel sources (sha256 over csrc): `{out['source_sha256'][:16]}`", ""]
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, a.name + ".md"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(a.out, a.name + "_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
