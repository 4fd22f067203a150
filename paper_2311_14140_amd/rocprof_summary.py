"""Summaries of rocprofv3 output for the kernels of a DSMC step.

    python -m paper_2311_14140_amd.rocprof_summary stats DIR [--last N]
    python -m paper_2311_14140_amd.rocprof_summary traffic --stats DIR --fetch DIR \\
        --write DIR --tag NAME --workload TEXT [--copy-mib 256] [--json FILE]
    python -m paper_2311_14140_amd.rocprof_summary issue DIR [DIR ...]

``stats`` prints the kernel statistics of a ``--kernel-trace --stats -f csv``
run as a table; with ``--last N`` it averages only each step kernel's last N
dispatches from the kernel trace (bench.py's per-kernel profile launches
its steps last, one lane after another, where the timed graph replays run
the lanes concurrently).  ``traffic`` reads two counter runs (``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE``, each in its own run) and converts each kernel's average
KiB per dispatch to bytes, scaled by what the same counter reads for a plain
device copy of known size in the same run (the bench's calibration copy):
the largest copy dispatch is taken as that copy.  It prints a table per step
kernel and records the bytes per launch with the hash of the sources in the
JSON file that bench.py reads for its ``traffic`` field.  ``issue`` reads SQ
counter runs (``--pmc SQ_...``, any split of the counters over runs) and
prints, per step kernel averaged over its dispatches, the fraction of its
wavefronts' cycles spent issuing each kind of instruction or waiting, and
its instructions per wavefront.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# kernel name prefix -> step slot (the slots of dsmc_profile_step; a resident
# lane's whole-step kernel is kept apart, as that call reports its share)
PHASE_OF = (("k_count", "count"), ("k_colsum", "colsum"), ("k_scan_small", "scan"),
            ("k_scan_seg", "scan"),
            ("k_scan", "scan"), ("k_colprefix", "colprefix"), ("k_move_scatter", "move_scatter"),
            ("k_move_scatter_wide", "move_scatter"),
            ("k_collide_bucket", "collide"), ("k_collide_fast", "collide"),
            ("k_collide_det", "collide"), ("k_resident", "resident"),
            ("k_finalize", "finalize"))
SOURCES = ("kernels.hip", "runtime.hip", "rng.hpp", "common.hpp", "kernels.hpp")


def _code_only(text: str) -> str:
    """The source without its comments and with whitespace runs collapsed, so
    that a change of comments alone keeps the hash (string and character
    literals are kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if ch in "\"'":
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    """Hash of the kernel and runtime sources' code (comments excluded)."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, "paper_2311_14140_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """A kernel's name without return type, namespaces and parameters."""
    base = name.replace("void ", "", 1).strip()
    for ns in ("dsmc::(anonymous namespace)::", "dsmc::"):
        if base.startswith(ns):
            base = base[len(ns):]
    depth = 0
    for i, ch in enumerate(base):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return base[:i]
    return base


def phase(name: str):
    base = short_name(name)
    for prefix, ph in PHASE_OF:
        if base.startswith(prefix + "<") or base == prefix:
            return ph
    return None


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def kernel_stats(directory: str):
    """[(name, calls, total_ns, average_ns, percent)] of a kernel-trace run."""
    out = []
    for r in _rows(directory, "kernel_stats.csv"):
        out.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                    float(r["AverageNs"]), float(r["Percentage"])))
    out.sort(key=lambda x: -x[2])
    return out


def counter_per_dispatch(directory: str, counter: str):
    """{kernel name: [value per dispatch]} of one counter run."""
    per = defaultdict(float)
    names = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r.get("Dispatch_Id") or r.get("Correlation_Id"), r["Kernel_Name"])
        per[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    out = defaultdict(list)
    for key, v in per.items():
        out[names[key]].append(v)
    return out


def copy_scale(values: dict, copy_mib: int) -> float:
    copies = [v for name, vs in values.items() if "copy" in name.lower() for v in vs]
    if not copies:
        raise SystemExit("no copy dispatch found for the calibration")
    return copy_mib * 1024.0 / max(copies)


def cmd_issue(a):
    per_kernel = defaultdict(lambda: defaultdict(list))
    for directory in a.dirs:
        per = defaultdict(float)
        for r in _rows(directory, "counter_collection.csv"):
            key = (r.get("Dispatch_Id") or r.get("Correlation_Id"), r["Kernel_Name"], r["Counter_Name"])
            per[key] += float(r["Counter_Value"])
        for (_, name, counter), v in per.items():
            per_kernel[short_name(name)][counter].append(v)
    for name in sorted(per_kernel):
        if not phase(name) or phase(name) in ("finalize",):
            continue
        m = {c: sum(v) / len(v) for c, v in per_kernel[name].items()}
        if "SQ_WAVE_CYCLES" in m:
            wc = m["SQ_WAVE_CYCLES"]
            parts = [(k, "SQ_ACTIVE_INST_" + k) for k in ("VALU", "LDS", "VMEM", "SCA", "ANY")]
            parts += [("WAIT_ANY", "SQ_WAIT_ANY"), ("WAIT_INST_ANY", "SQ_WAIT_INST_ANY")]
            print(f"== {name}")
            print("  per wave-cycle: " + " ".join(f"{k} {m[c] / wc:.3f}" for k, c in parts if c in m))
        if "SQ_WAVES" in m:
            w = m["SQ_WAVES"]
            parts = [(k, "SQ_INSTS_" + k) for k in ("VALU", "LDS", "SALU", "VMEM_RD", "VMEM_WR", "BRANCH")]
            line = " ".join(f"{k} {m[c] / w:.0f}" for k, c in parts if c in m)
            if "SQ_LDS_BANK_CONFLICT" in m and m.get("SQ_INSTS_LDS"):
                line += f"; bank conflicts per LDS instruction {m['SQ_LDS_BANK_CONFLICT'] / m['SQ_INSTS_LDS']:.3f}"
            if "SQ_WAVE_CYCLES" not in m:
                print(f"== {name}")
            print("  instructions per wavefront: " + line)


def last_dispatches(directory: str, last: int):
    """[(name, dispatches averaged, average ns)] over each step kernel's last
    `last` dispatches of a kernel trace (not the estimators' kernel, and not
    a resident lane's, whose launches carry different numbers of steps)."""
    per = defaultdict(list)
    for r in _rows(directory, "kernel_trace.csv"):
        if phase(r["Kernel_Name"]) not in (None, "finalize", "resident"):
            per[r["Kernel_Name"]].append((int(r["Dispatch_Id"]),
                                          int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = []
    for name, ds in per.items():
        ds.sort()
        tail = [t for _, t in ds[-last:]]
        out.append((name, len(tail), sum(tail) / len(tail)))
    out.sort(key=lambda x: -x[2] * x[1])
    return out


def cmd_stats(a):
    if a.last:
        print(f"| kernel | last dispatches | average us |")
        print("|---|---|---|")
        for name, n, avg in last_dispatches(a.dir, a.last):
            print(f"| {short_name(name)} | {n} | {avg / 1e3:.3f} |")
        return
    print("| kernel | calls | total us | average us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in kernel_stats(a.dir):
        print(f"| {short_name(name)} | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.3f} | {pct:.1f} |")


def cmd_traffic(a):
    stats = kernel_stats(a.stats)
    fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(a.write, "WRITE_SIZE")
    fs, ws = copy_scale(fetch, a.copy_mib), copy_scale(write, a.copy_mib)
    avg_us = defaultdict(list)
    for name, calls, tot, avg, _ in stats:
        ph = phase(name)
        if ph:
            avg_us[ph].append((calls, tot))
    by_phase = defaultdict(lambda: [[], []])
    for name, vs in fetch.items():
        if phase(name):
            by_phase[phase(name)][0] += vs
    for name, vs in write.items():
        if phase(name):
            by_phase[phase(name)][1] += vs
    rec = {"workload": a.workload, "fetch_scale": fs, "write_scale": ws,
           "kernel_source_hash": source_hash(), "avg_us": {}, "bytes_per_launch": {},
           "fetch_KiB": {}, "write_KiB": {}}
    for ph, cts in avg_us.items():
        calls = sum(c for c, _ in cts)
        rec["avg_us"][ph] = sum(t for _, t in cts) / calls / 1e3
    print(f"Calibration: a plain {a.copy_mib} MiB device copy scales FETCH_SIZE by {fs:.3f} "
          f"and WRITE_SIZE by {ws:.3f}.\n")
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated MB per launch |")
    print("|---|---|---|---|")
    for ph in sorted(by_phase):
        f, w = by_phase[ph]
        if not f or not w:
            continue
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        b = (fk * fs + wk * ws) * 1024.0
        rec["fetch_KiB"][ph], rec["write_KiB"][ph] = fk, wk
        rec["bytes_per_launch"][ph] = b
        print(f"| {ph} | {fk:.1f} | {wk:.1f} | {b / 1e6:.3f} |")
    print(f"\nKernel source hash (code without comments): {rec['kernel_source_hash']}")
    if a.json:
        data = {}
        if os.path.exists(a.json):
            with open(a.json) as fh:
                data = json.load(fh)
        data[a.tag] = rec
        with open(a.json, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--last", type=int, default=0)
    t = sub.add_parser("traffic")
    t.add_argument("--stats", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--tag", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--copy-mib", type=int, default=256)
    t.add_argument("--json", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"))
    i = sub.add_parser("issue")
    i.add_argument("dirs", nargs="+")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "issue": cmd_issue}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
