"""Build libibm.so (the HIP kernels for gfx950 and the C-ABI host code) in
place, next to this file.  Usage: python -m paper_2606_09799_amd.build"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libibm.so")

ARCH = os.environ.get("IBM_OFFLOAD_ARCH", "gfx950")
# packed FP32 instructions stay off (the compiler may not form them itself)
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-result"]
# geometry whose integer outcome must be reproducible bit for bit: no FMA
NO_CONTRACT = {"tag.hip", "force.hip", "body.hip"}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    procs, objs = [], []
    for f in sources():
        obj = os.path.join(BUILD, f + ".o")
        flags = list(COMMON)
        if f in NO_CONTRACT:
            flags.append("-ffp-contract=off")
        if f.endswith(".cpp"):
            flags = ["-x", "hip"] + flags
        cmd = [hipcc] + flags + ["-c", os.path.join(CSRC, f), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((f, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for f, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the GPU target feature: harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(f)
            sys.stderr.write(f"--- {f}\n" + "\n".join(lines) + "\n")
        elif verbose and any(ln.strip() for ln in lines):
            sys.stderr.write(f"--- {f}\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode(errors="replace"))
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
