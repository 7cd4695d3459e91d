"""Throughput of the hot path on one MI355X.

One "step" is one full time step of the scheme (tagging of the moving body
at t^n, then two RK2 sub-stages of IB forcing, predictor, consistent mass
correction, Poisson solve and projection) on the 256x192x256 stretched
channel with the heaving/pitching zero-thickness plate, inputs resident in
HBM.  The body vertices are recomputed on the device every step from
host-evaluated coefficients (included in the timing).

Prints one JSON line: cell-steps/s per fractional step (cells x sub-stages /
s) of the first precision form (FP64 by default), the roofline of its
dominant kernel (algorithmic bytes per launch over its average duration,
from HIP events recorded around that kernel inside the timed region), the
CPU oracle timed on a bounded sample, and under "forms" the same
measurement for every form timed (the mixed form with its FP64-residual
refinement counts).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s per fractional step, 1 MI355X: FP64 vs mixed vs batched; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(name, nx, ny, nz, form="fp64"):
    """Bytes a launch of kernel `name` must move at minimum: the fields it
    reads and writes once, per the pass model of the step.  The velocity and
    phi are FP64 in every form; p, H, R and the line-solve data are FP32 in
    the mixed forms; the spectrum is FP32 in mixed_refined (whose refinement
    passes are not counted here)."""
    N = nx * ny * nz
    Nv = nx * (ny + 1) * nz
    U = N + Nv + N                       # u, v, w values
    r = 8 if form == "fp64" else 4       # p, H, R, line-solve data
    spec = ny * nz * (nx // 2 + 1) * (8 if form == "mixed_refined" else 16)
    table = {
        "rhs": 8 * U + r * N + r * U * 2,          # u,v,w (f64), p + H + R
        "adi_x": 2 * r * N, "adi_z": 2 * r * N,    # per component
        "adi_y": r * N + 16 * N,                   # w2, u (f64) -> u_hat
        "pois_fftx_fwd": 8 * U + spec + (8 * N if form == "mixed_refined" else 0),
        "pois_fftz_fwd": 2 * spec, "pois_fftz_inv": 2 * spec,
        "pois_tri_y": 2 * spec,
        "pois_fftx_inv": spec + 8 * N,
        "project": 8 * U * 2 + 8 * N + r * N * 2,  # u_hat, phi, p -> u, p
    }
    return table.get(name)


# kernel name in the library's event profile -> prefixes of its kernel symbols
# in the rocprofv3 summaries (every variant the launcher may pick: flags of
# the RHS march, the line-solve and transform kernels by line length)
def counter_names(kernel, form):
    T = "double" if form == "fp64" else "float"
    C = "float2" if form == "mixed_refined" else "double2"
    return {"rhs": [f"k_rhs<{T},"],
            "adi_x": [f"k_line_xw<{T}>", f"k_line<{T}, 0,"],
            "adi_z": [f"k_line_col<{T}, 1>", f"k_line<{T}, 1,"],
            "adi_y": [f"k_line_col<{T}, 2>", f"k_line<{T}, 2,"],
            "pois_fftx_fwd": [f"k_fftx256_fwd<{C}", f"k_fftx_fwd<{C}"],
            "pois_fftz_fwd": [f"k_fftz256<{C}, false>", f"k_fftz<{C}, false>"],
            "pois_fftz_inv": [f"k_fftz256<{C}, true>", f"k_fftz<{C}, true>"],
            "pois_tri_y": [f"k_tri_y<{C}", f"k_tri_y_blk<{C}"],
            "pois_fftx_inv": [f"k_fftx256_inv<{C}", f"k_fftx_inv<{C}"],
            "project": [f"k_project<{T}>"]}.get(kernel, [])


def csrc_sha():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_09799_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, form="fp64"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy; averaged over
    the kernel's symbol variants by dispatch count), or None when no summary
    exists for this workload and form or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{form}_traffic.json")
    names = counter_names(kernel, form)
    if not names or not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("csrc_sha") != csrc_sha():
        return None
    tot, n = 0.0, 0
    for sym, k in t["kernels"].items():
        if any(sym.startswith(nm) for nm in names):
            tot += (k["read_bytes"] + k["write_bytes"]) * k["dispatches"]
            n += k["dispatches"]
    return int(tot / n) if n else None


def cpu_baseline(wl):
    """The oracle as it stands, on one full time step (tagging and both RK2
    sub-stages: IB forcing, predictor, mass correction, Poisson, projection)
    of the same workload from t = 0."""
    import numpy as np
    from oracle import kinematics, step as ostep
    from oracle.grid import Grid
    g = Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces)
    f = wl.fields()
    X, U = kinematics.body_at(wl.bodies[0], 0.0)
    T = wl.bodies[0].tris
    t0 = time.perf_counter()
    ostep.step(g, f, np.zeros(g.shape), (X, U, T), wl.dt, wl.re, (-wl.dpdx, 0.0, 0.0))
    el = time.perf_counter() - t0
    return {"value": g.cells * 2 / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one full time step (tagging + 2 RK2 sub-stages) of the "
                      f"{wl.nx}x{wl.ny}x{wl.nz} workload from t=0 ({el:.1f} s, numpy, "
                      f"one thread)"}


def progress(msg):
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def run_form(args, wl, form, dev):
    """Times args.steps full steps of workload wl in one precision form.
    Returns (elapsed s, warm-up per-kernel profile, dominant kernel, its
    timed-region event profile, refinement statistics or None)."""
    import numpy as np
    import torch
    from paper_2606_09799_amd import ibm

    ctx = ibm.Context(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces, wl.re, wl.dpdx,
                      precision="fp64" if form == "fp64" else "mixed",
                      mixed_poisson="refined" if form == "mixed_refined" else "fp64")
    progress(f"{form}: context created, generating the initial field")
    u0, v0, w0 = wl.fields()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    u, v, w = T(u0), T(v0), T(w0)
    del u0, v0, w0
    p = torch.zeros(ctx.cells, dtype=ctx.pdtype, device=dev)
    dbodies = []
    for b in wl.bodies:
        ref = T(b.ref)
        xyz = torch.empty(b.ref.shape[0], 3, dtype=torch.float64, device=dev)
        vel = torch.empty_like(xyz)
        dbodies.append((b, ref, xyz, vel, T(b.tris.astype(np.int32))))
    bodies = [ibm.Body(x, vv, tr) for (_, _, x, vv, tr) in dbodies]
    progress(f"{form}: state on the device, warming up")

    def one_step(s):
        tt = s * wl.dt
        for (b, ref, xyz, vel, _) in dbodies:
            if b.kind == "rigid":
                ibm.ibm_body_rigid(ctx, ref, b.coef(tt), xyz, vel)
            else:
                ibm.ibm_body_deform(ctx, ref, b.coef(tt), xyz, vel)
        ibm.ibm_step(ctx, u, v, w, p, bodies, wl.dt)

    # warm-up, profiling every kernel to find the dominant one (the first
    # step, which pays for code loading and cold caches, is not profiled)
    for s in range(args.warmup):
        if s == min(1, args.warmup - 1):
            ibm.ibm_profile(ctx, True, None)
        one_step(s)
    prof = ibm.ibm_profile_read(ctx)
    dominant = max((k for k in prof if algorithmic_bytes(k, wl.nx, wl.ny, wl.nz, form)),
                   key=lambda k: prof[k][1], default=None)
    stats = ibm.ibm_refine_stats(ctx, reset=True) if form == "mixed_refined" else None
    progress(f"{form}: warm-up done, timing {args.steps} steps")
    # timed region: events only around the dominant kernel
    ibm.ibm_profile(ctx, True, dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        one_step(s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"{form}: {el / args.steps * 1e3:.3f} ms per step")
    dom = ibm.ibm_profile_read(ctx)
    ibm.ibm_profile(ctx, False, None)
    if form == "mixed_refined":
        stats = ibm.ibm_refine_stats(ctx, after_first=True)
    flags = ibm.ibm_check(ctx)
    if flags:
        print(f"bench.py: device flags {flags} after the {form} run", file=sys.stderr)
        sys.exit(1)
    # no-slip error (Sec. 4.4) of the final fields against the body at the
    # final time (untimed: body transform and tagging at t, then the error)
    tend = (args.warmup + args.steps) * wl.dt
    for (b, ref, xyz, vel, _) in dbodies:
        if b.kind == "rigid":
            ibm.ibm_body_rigid(ctx, ref, b.coef(tend), xyz, vel)
        else:
            ibm.ibm_body_deform(ctx, ref, b.coef(tend), xyz, vel)
    ibm.ibm_tag(ctx, bodies)
    eps, eps_c = ibm.ibm_noslip_error(ctx, u, v, w)
    noslip = {"mean": eps, "u": eps_c[0], "v": eps_c[1], "w": eps_c[2], "time": tend}
    if not all(torch.isfinite(x).all().item() for x in (u, v, w, p)):
        print(f"bench.py: non-finite state after the {form} run", file=sys.stderr)
        sys.exit(1)
    ctx.close()
    return el, prof, dominant, dom, stats, noslip


def run_batched(args, dev, nsim):
    """Times the batched workload (nsim simulations of different sizes, one
    body each) in each execution mode, then autotunes the plan (stream
    groups, RHS tile, graph or streams) and times the tuned plan; returns
    {mode: (cell-steps/s, ms per step)}, the total cell count and the tuner's
    report."""
    import numpy as np
    import torch
    import workloads
    from paper_2606_09799_amd import ibm

    wls = workloads.batch(nsim)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sims = []
    for wl in wls:
        u, v, w = (T(a) for a in wl.fields())
        b = wl.bodies[0]
        nv = b.ref.shape[0]
        sims.append({"nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "lx": wl.lx, "lz": wl.lz,
                     "y_faces": wl.y_faces, "re": wl.re, "dpdx": wl.dpdx, "u": u, "v": v, "w": w,
                     "p": torch.zeros(wl.cells, dtype=torch.float64, device=dev),
                     "motion": b.kind, "ref": T(b.ref),
                     "xyz": torch.empty(nv, 3, dtype=torch.float64, device=dev),
                     "vel": torch.empty(nv, 3, dtype=torch.float64, device=dev),
                     "tri": T(b.tris.astype(np.int32))})
    batch = ibm.Batch(sims)
    dt = wls[0].dt
    cells = sum(wl.cells for wl in wls)
    out = {}
    k = 0
    for name, mode in (("serial", ibm.BATCH_SERIAL), ("streams", ibm.BATCH_STREAMS),
                       ("graph", ibm.BATCH_GRAPH)):
        for _ in range(args.warmup):
            batch.step([wl.bodies[0].coef(k * dt) for wl in wls], dt, mode)
            k += 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.step([wl.bodies[0].coef(k * dt) for wl in wls], dt, mode)
            k += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = (cells * 2 * args.steps / el, el / args.steps * 1e3)
        progress(f"batched {name}: {el / args.steps * 1e3:.3f} ms per step")
    progress("batched: autotuning the plan")
    t0 = time.perf_counter()
    best, tried = batch.tune([wl.bodies[0].coef(k * dt) for wl in wls], dt, steps=3)
    tune_s = time.perf_counter() - t0
    progress(f"batched: tuned plan {best} in {tune_s:.1f} s")
    for _ in range(args.warmup):
        batch.step([wl.bodies[0].coef(k * dt) for wl in wls], dt, ibm.BATCH_PLAN)
        k += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.step([wl.bodies[0].coef(k * dt) for wl in wls], dt, ibm.BATCH_PLAN)
        k += 1
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["tuned"] = (cells * 2 * args.steps / el, el / args.steps * 1e3)
    progress(f"batched tuned: {el / args.steps * 1e3:.3f} ms per step")
    tune = {"plan": best, "tune_seconds": round(tune_s, 2),
            "tried": [{k2: (round(v, 3) if isinstance(v, float) else v) for k2, v in p.items()}
                      for p in tried]}
    flags = batch.check()
    if flags:
        print(f"bench.py: device flags {flags} after the batched run", file=sys.stderr)
        sys.exit(1)
    for d in sims:
        if not all(torch.isfinite(d[q]).all().item() for q in ("u", "v", "w", "p")):
            print("bench.py: non-finite state after the batched run", file=sys.stderr)
            sys.exit(1)
    batch.close()
    return out, cells, tune


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--forms", default="fp64,mixed,mixed_refined",
                    help="precision forms to time (fp64; mixed: FP32 predictor and FP64 "
                         "Poisson; mixed_refined: also FP32 Poisson transforms refined with "
                         "FP64 residuals); the first one is the headline value")
    ap.add_argument("--batch-sims", type=int, default=64,
                    help="simulations of the batched workload (0 = skip it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run a plain device copy of this size (PMC scale reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU design is documented, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads

    torch.cuda.set_device(0)
    dev = "cuda:0"
    wl = workloads.config(args.workload)
    forms = [f for f in args.forms.split(",") if f]
    substeps = 2
    results = {}
    for form in forms:
        el, prof, dominant, dom, stats, noslip = run_form(args, wl, form, dev)
        r = {"value": wl.cells * substeps * args.steps / el, "ms_per_step": el / args.steps * 1e3,
             "kernel_ms_per_step": {k: round(vv[1] / max(1, args.warmup - 1), 4)
                                    for k, vv in prof.items()}}
        if dominant and dominant in dom:
            launches, total_ms = dom[dominant]
            avg_s = total_ms / launches / 1e3
            ab = algorithmic_bytes(dominant, wl.nx, wl.ny, wl.nz, form)
            ach = ab / avg_s / 1e9
            r["roofline"] = {"bound": "hbm", "kernel": dominant, "achieved": round(ach, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(ach / HBM_PEAK_GBS, 4),
                             "traffic": measured_traffic(dominant, wl.name, form),
                             "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes": ab}
        # whole step: algorithmic bytes of every dense kernel per step over the
        # step time
        nprof = max(1, args.warmup - 1)
        path_bytes = sum((algorithmic_bytes(k, wl.nx, wl.ny, wl.nz, form) or 0) * vv[0] / nprof
                         for k, vv in prof.items())
        path_gbs = path_bytes / (el / args.steps) / 1e9
        r["path_roofline"] = {"bound": "hbm", "achieved": round(path_gbs, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                              "algorithmic_bytes_per_step": int(path_bytes)}
        if stats is not None:
            solves, corr, worst, first = stats
            r["refinement"] = {"poisson_solves": solves, "corrections": corr,
                               "corrections_per_solve": round(corr / max(1, solves), 3),
                               "max_final_divergence": worst,
                               "max_divergence_after_first_correction": first}
        r["noslip_error"] = noslip
        results[form] = r
    batched = None
    if args.batch_sims > 0:
        try:
            modes, bcells, tune = run_batched(args, dev, args.batch_sims)
        except Exception as e:  # the single-grid results above stand on their own
            print(f"bench.py: the batched workload failed: {type(e).__name__}: {e}",
                  file=sys.stderr, flush=True)
            modes = None
            batched = {"error": f"{type(e).__name__}: {e}"}
    if args.batch_sims > 0 and modes is not None:
        best = max(modes, key=lambda m: modes[m][0])
        batched = {"workload": f"c4: {args.batch_sims} simulations, {bcells} cells in total "
                               "(uniform spacing 1/32, 32..128 x 32..96 x 32..128, one sphere, "
                               "plate or deforming body each), Re 100, dt 1e-3, FP64",
                   "value": modes[best][0], "ms_per_step": modes[best][1], "mode": best,
                   "modes": {m: {"value": v, "ms_per_step": ms} for m, (v, ms) in modes.items()},
                   "speedup_vs_serial": modes[best][0] / modes["serial"][0],
                   "autotune": tune}
    head = results[forms[0]]
    copy_ref = None
    if args.copy_ref_mib:
        nb = args.copy_ref_mib * 1024 * 1024 // 8
        a = torch.ones(nb, dtype=torch.float64, device=dev)
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        copy_ref = {"bytes_read": nb * 8, "bytes_written": nb * 8, "launches": 3}
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle on one step")
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)
    out = {
        "metric": METRIC, "value": head["value"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.nx}x{wl.ny}x{wl.nz} channel, tanh-stretched y, "
                               f"Re {wl.re:g}, dt {wl.dt:g}, RK2+CN, "
                               f"{sum(b.tris.shape[0] for b in wl.bodies)} triangles",
                   "cells": wl.cells, "substeps_per_step": substeps,
                   "form": forms[0], "parallelism": "single GPU"},
        "roofline": head.get("roofline"),
        "cpu_baseline": cpu,
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "forms": {f: dict(r) for f, r in results.items()},
    }
    if batched:
        out["forms"]["batched"] = batched
    if copy_ref:
        out["copy_ref"] = copy_ref
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
