"""Summaries of rocprofv3 runs of bench.py, as short text under profiles/.

Reads the CSV output of one `rocprofv3 --kernel-trace --stats` run and of two
`rocprofv3 --pmc` runs (FETCH_SIZE, then WRITE_SIZE) of the same bench
command with `--copy-ref-mib`, and writes

    profiles/<tag>_kernel_trace.md   calls, total and average time per kernel
    profiles/<tag>_hbm_traffic.md    HBM bytes per dispatch, scaled by a copy
    profiles/<tag>_traffic.json      the same numbers for bench.py

The copy reference is the plain device copy that bench.py runs with
`--copy-ref-mib M` (M MiB read and written): the ratio of its known bytes to
what each counter reports for it scales the counter for every kernel.

    python -m paper_2606_09799_amd.profiling --tag c2_fp64 \\
        --trace out/trace_fp64 --fetch out/fetch_fp64 \\
        --write out/write_fp64 --copy-mib 1024 \\
        --trace-cmd "<bench.py args>" --pmc-cmd "<bench.py args>"
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def csrc_sha() -> str:
    """Hash of the kernel sources (the same one bench.py checks)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_09799_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(raw: str) -> str:
    """'void ibm::k_fftz<HIP_vector_type<double, 2u>, false>(ibm::PoisK<...>)'
    -> 'k_fftz<double2, false>'."""
    k = raw.replace("void ", "")
    depth, cut = 0, len(k)
    for i, ch in enumerate(k):  # drop the argument list (outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    k = k[:cut].replace("ibm::", "")
    k = re.sub(r"HIP_vector_type<(\w+), 2u>", r"\g<1>2", k)
    return k.strip()


def _one(path_dir: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(path_dir, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {path_dir}")
    return hits[0]


def pmc_per_kernel(path_dir: str):
    """Counter values per kernel, and the values of the copy reference: the
    last three dispatches of the runtime's copy kernel (bench.py runs the
    reference copy three times after everything else; other copies of the
    run, such as state clones, may be larger)."""
    out = collections.defaultdict(list)
    copies = []
    with open(_one(path_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = kernel_name(r["Kernel_Name"])
            out[k].append(float(r["Counter_Value"]))
            if "copyBuffer" in k:
                copies.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    ref = sorted(v for _, v in sorted(copies)[-3:])
    return out, (ref[len(ref) // 2] if ref else None)


def summarise(tag, trace, fetch, write, copy_mib, trace_cmd, pmc_cmd, workload):
    sha = csrc_sha()
    with open(_one(trace, "kernel_stats.csv")) as f:
        stats = list(csv.DictReader(f))
    lines = [f"# Kernel trace, {workload}, rocprofv3 --stats", "",
             "Command (from the repository root on one MI355X):", "",
             "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats "
             f"--output-format csv -d $REPO/{trace} -o run -- python3 $REPO/bench.py {trace_cmd}",
             "", f"Kernel sources hash (paper_2606_09799_amd/csrc): `{sha}`", "",
             "| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
    for r in stats[:32]:
        lines.append(f"| {kernel_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{tag}_kernel_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    if not fetch or not write:  # a trace-only summary
        return sha, None, None

    (fe, cf), (wr, cw) = pmc_per_kernel(fetch), pmc_per_kernel(write)
    ref_kib = copy_mib * 1024.0
    fs, ws = ref_kib / cf, ref_kib / cw
    lines = [f"# HBM traffic per dispatch, {workload}, rocprofv3 --pmc", "",
             "Two passes, one counter each (from the repository root on one MI355X):", "",
             "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
             f"-d $REPO/{fetch} -o run -- python3 $REPO/bench.py {pmc_cmd} --copy-ref-mib {copy_mib}",
             "    cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
             f"-d $REPO/{write} -o run -- python3 $REPO/bench.py {pmc_cmd} --copy-ref-mib {copy_mib}",
             "", "Summary: `python -m paper_2606_09799_amd.profiling` (this module).", "",
             f"Scale factors from the plain {copy_mib} MiB device copy of the same runs "
             f"({ref_kib:.0f} KiB read and written): FETCH_SIZE reads {cf:.0f} KiB -> x{fs:.3f}; "
             f"WRITE_SIZE reads {cw:.0f} KiB -> x{ws:.3f}.", "",
             f"Kernel sources hash: `{sha}`", "",
             "| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | HBM read MB (scaled) "
             "| HBM write MB (scaled) |", "|---|---|---|---|---|---|"]
    traffic = {}
    for k, v in fe.items():
        if not k.startswith("k_"):
            continue
        w = wr.get(k, [0.0])
        f_ = sum(v) / len(v)
        w_ = sum(w) / len(w)
        rd, wt = f_ * fs * 1024, w_ * ws * 1024
        lines.append(f"| {k} | {len(v)} | {f_:.0f} | {w_:.0f} | {rd / 1e6:.1f} | {wt / 1e6:.1f} |")
        traffic[k] = {"read_bytes": rd, "write_bytes": wt, "dispatches": len(v)}
    with open(os.path.join(ROOT, "profiles", f"{tag}_hbm_traffic.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", f"{tag}_traffic.json"), "w") as f:
        json.dump({"csrc_sha": sha, "fetch_scale": fs, "write_scale": ws, "kernels": traffic},
                  f, indent=1)
    return sha, fs, ws


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--tag", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", default="", help="FETCH_SIZE run (omit for a trace-only summary)")
    ap.add_argument("--write", default="", help="WRITE_SIZE run (omit for a trace-only summary)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--trace-cmd", default="", help="bench.py arguments of the traced run")
    ap.add_argument("--pmc-cmd", default="", help="bench.py arguments of the counter runs")
    ap.add_argument("--workload", default="256x192x256 plate workload")
    a = ap.parse_args()
    print(summarise(a.tag, a.trace, a.fetch, a.write, a.copy_mib, a.trace_cmd, a.pmc_cmd,
                    a.workload))


if __name__ == "__main__":
    main()
