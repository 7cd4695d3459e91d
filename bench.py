"""Throughput of the hot path on one MI355X.

One "step" is one full time step of the scheme: tagging of the moving bodies
at t^n, then two RK2 sub-stages of IB forcing, predictor, consistent mass
correction, Poisson solve and projection, on a synthetic workload shaped like
the paper's tests, with every input resident in HBM (the body vertices are
recomputed on the device every step from host-evaluated coefficients, inside
the timed region).

The headline is the largest single-GPU workload, the 1024x768x1024 stretched
channel with 67 moving bodies, in the mixed form: p, H, R and the line-solve
data in FP32, the velocity, the Poisson solve, the projection and every
global reduction in FP64.  The same line carries, under "forms", the FP64
form and the refined mixed form (FP32 forward Poisson transforms, FP64
wall-normal solves and inverse transforms, FP64-residual refinement to the
post-projection divergence bound) on that workload, each mixed form with its
velocity error against the FP64 run and every form with its post-projection
divergence; the three forms on the 256x192x256 plate workload; and the
batched workload (64 independent simulations) in FP64 and the mixed form.

Prints one JSON line: cell-steps/s per fractional step (cells x sub-stages /
s); the roofline of the headline's dominant kernel (algorithmic bytes per
launch over its average duration, from HIP events recorded around that
kernel on the library's stream inside the timed region); the whole step
against the pass model of the path (bytes per cell and sub-stage of each
form) and against the implementation's own pass bytes; the CPU oracle timed
on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s per fractional step, 1 MI355X: FP64 vs mixed vs batched; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FORMS = ("fp64", "mixed", "mixed_refined")

# Pass model of one sub-stage, bytes per cell (the minimum global passes the
# data dependencies force; FP64 8 B, FP32 4 B; the velocity is FP64 in every
# form):
#   fp64           RHS + x sweep 80, z sweep 48, y sweep 72, Poisson 96
#                  (x forward 32, z/y/z 48, x inverse 16), projection 72: 368
#   mixed_refined  RHS + x sweep 52, z 24, y 24, Poisson 76 (FP32 spectrum),
#                  projection 76: 252, plus 64 per FP64-residual refinement
#   mixed          the mixed predictor and projection with the FP64 Poisson
#                  passes: 100 + 96 + 76 = 272
MODEL_BYTES = {"fp64": 368.0, "mixed": 272.0, "mixed_refined": 252.0}
# the post-projection divergence bound max |D u - q| that the refined form's
# FP64-residual refinement enforces (max |rhs - L_c phi| alpha dt)
DIV_BOUND = 1e-10
MODEL_REFINEMENT_BYTES = 64.0


def algorithmic_bytes(name, nx, ny, nz, form="fp64"):
    """Bytes a launch of kernel `name` must move at minimum: the fields it
    reads and writes once, as this implementation's passes are cut.  The
    velocity and phi are FP64 in every form; p, H, R and the line-solve data
    are FP32 in the mixed forms; the refined form keeps an FP64 copy of the
    Poisson right-hand side (written by the first pass, read by each
    residual pass with phi), transforms forward on an FP32 spectrum and back
    on an FP64 one."""
    N = nx * ny * nz
    Nv = nx * (ny + 1) * nz
    U = N + Nv + N                       # u, v, w values
    r = 8 if form == "fp64" else 4       # p, H, R, line-solve data
    S = ny * nz * (nx // 2 + 1)          # spectrum values
    ref = form == "mixed_refined"
    s_fwd = S * (8 if ref else 16)
    s_inv = S * 16
    table = {
        "rhs": 8 * U + r * N + r * U * 2,          # u,v,w (f64), p + H + R
        "adi_x": 2 * r * N, "adi_z": 2 * r * N,    # per component
        "adi_y": r * N + 16 * N,                   # w2, u (f64) -> u_hat
        "pois_fftx_fwd": 8 * U + s_fwd + (8 * N if ref else 0),
        "pois_fftz_fwd": 2 * s_fwd,
        "pois_tri_y": s_fwd + s_inv,
        "pois_fftz_inv": 2 * s_inv,
        "pois_fftx_inv": s_inv + 8 * N,
        "pois_resid_fftx": 16 * N + s_fwd,
        "project": 8 * U * 2 + 8 * N + r * N * 2,
    }
    return table.get(name)


# kernel name in the library's event profile -> prefixes of its kernel symbols
# in the rocprofv3 summaries (every variant the launcher may pick)
def counter_names(kernel, form):
    T = "double" if form == "fp64" else "float"
    C = "float2" if form == "mixed_refined" else "double2"
    return {"rhs": [f"k_rhs<{T},"],
            "adi_x": [f"k_line_xw<{T},", f"k_line<{T}, 0,"],
            "adi_z": [f"k_line_col<{T}, 1,", f"k_line<{T}, 1,"],
            "adi_y": [f"k_line_col<{T}, 2,", f"k_line_col_reg<{T}, 2,", f"k_line<{T}, 2,"],
            "pois_fftx_fwd": [f"k_fftx256_fwd<{C}", f"k_fftx_fwd<{C}"],
            "pois_fftz_fwd": [f"k_fftz256<{C}, false,", f"k_fftz<{C}, false,",
                              f"k_fftz4s<{C}, false,"],
            "pois_fftz_inv": ["k_fftz256<double2, true,", "k_fftz<double2, true,",
                              "k_fftz4s<double2, true,"],
            "pois_tri_y": [f"k_tri_y<{C},", f"k_tri_y_blk<{C},"],
            "pois_fftx_inv": ["k_fftx256_inv<double2", "k_fftx_inv<double2",
                              "k_fftx4s_inv<double2,"],
            "project": [f"k_project<{T},"]}.get(kernel, [])


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl):
    """The oracle as it stands, on one full time step (tagging and both RK2
    sub-stages: IB forcing, predictor, mass correction, Poisson, projection)
    of workload wl from t = 0."""
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
            "cpu": cpu_model(),
            "sample": f"one full time step (tagging + 2 RK2 sub-stages) of the "
                      f"{wl.nx}x{wl.ny}x{wl.nz} plate workload from t=0 ({el:.1f} s; numpy, "
                      f"one thread)"}


def progress(msg):
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def describe(wl):
    if wl.vforce == "vortex":
        kind = "immersed-plane channel y in [-1/4, 2], vortex forcing below the plane"
    elif wl.vforce == "relax":
        kind = "immersed-plane channel y in [-1/4, 2], Re_tau 200, relaxation forcing below"
    else:
        kind = "channel, tanh-stretched y"
    return (f"{wl.name}: {wl.nx}x{wl.ny}x{wl.nz} {kind}, Re {wl.re:g}, "
            f"dt {wl.dt:g}, {'AB2' if wl.scheme == 'ab2' else 'RK2'}+CN, {len(wl.bodies)} bodies, "
            f"{sum(b.tris.shape[0] for b in wl.bodies)} triangles")


def run_form(args, wl, form, dev, fields0):
    """Times args.steps full steps of workload wl in one precision form from
    the initial field fields0 (device tensors, copied).  Returns a dict of
    results and the final velocity (device tensors)."""
    import numpy as np
    import torch
    from paper_2606_09799_amd import ibm

    ctx = ibm.Context(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces, wl.re, wl.dpdx,
                      scheme=wl.scheme,
                      precision="fp64" if form == "fp64" else "mixed",
                      mixed_poisson="refined" if form == "mixed_refined" else "fp64",
                      refine_tol=DIV_BOUND if form == "mixed_refined" else 0.0)
    u, v, w = (x.clone() for x in fields0)
    p = torch.zeros(ctx.cells, dtype=ctx.pdtype, device=dev)
    T = lambda a: torch.from_numpy(a).to(dev)
    import workloads
    vf = []
    for c in range(3):  # the volume forces of the immersed-plane channels
        f0, kap = workloads.volume_force(wl, c)
        if f0 is not None:
            vf.append((T(np.ascontiguousarray(f0)),
                       T(np.ascontiguousarray(kap)) if kap is not None else None))
            ibm.ibm_set_volume_force(ctx, c, *vf[-1])
    # AB2 + CN: H^{n-1} in and H^n out through the state (zero before the
    # first step)
    hbuf = ([torch.zeros(ctx.comp_numel(c), dtype=ctx.pdtype, device=dev) for c in range(3)]
            if wl.scheme == "ab2" else None)
    dbodies = []
    for b in wl.bodies:
        ref = T(np.ascontiguousarray(b.ref))
        xyz = torch.empty(b.ref.shape[0], 3, dtype=torch.float64, device=dev)
        vel = torch.empty_like(xyz)
        dbodies.append((b, ref, xyz, vel, T(np.ascontiguousarray(b.tris.astype(np.int32)))))
    bodies = [ibm.Body(x, vv, tr) for (_, _, x, vv, tr) in dbodies]
    progress(f"{wl.name} {form}: state on the device, warming up")

    def move(tt):
        for (b, ref, xyz, vel, _) in dbodies:
            if b.kind == "rigid":
                ibm.ibm_body_rigid(ctx, ref, b.coef(tt), xyz, vel)
            else:
                ibm.ibm_body_deform(ctx, ref, b.coef(tt), xyz, vel)

    def one_step(s):
        move(s * wl.dt)
        ibm.ibm_step(ctx, u, v, w, p, bodies, wl.dt, h=hbuf)

    # warm-up, profiling every kernel to find the dominant one (the first
    # step, which pays for code loading and cold caches, is not profiled)
    for s in range(args.warmup):
        if s == min(1, args.warmup - 1):
            ibm.ibm_profile(ctx, True, None)
        one_step(s)
    prof = ibm.ibm_profile_read(ctx)
    nprof = max(1, args.warmup - 1)
    dominant = max((k for k in prof if algorithmic_bytes(k, wl.nx, wl.ny, wl.nz, form)),
                   key=lambda k: prof[k][1], default=None)
    if form == "mixed_refined":
        ibm.ibm_refine_stats(ctx, reset=True)
    progress(f"{wl.name} {form}: warm-up done, timing {args.steps} steps")
    # timed region: events only around the dominant kernel
    ibm.ibm_profile(ctx, True, dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        one_step(s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"{wl.name} {form}: {el / args.steps * 1e3:.3f} ms per step")
    dom = ibm.ibm_profile_read(ctx)
    ibm.ibm_profile(ctx, False, None)
    flags = ibm.ibm_check(ctx)
    if flags:
        print(f"bench.py: device flags {flags} after the {wl.name} {form} run", file=sys.stderr)
        sys.exit(1)
    cells = wl.cells
    r = {"value": cells * 2 * args.steps / el, "ms_per_step": el / args.steps * 1e3,
         "kernel_ms_per_step_warmup_events":
             {k: round(vv[1] / nprof, 4) for k, vv in prof.items()}}
    if form == "mixed_refined":
        solves, corr, worst, first, init_max, init_mean = ibm.ibm_refine_stats(
            ctx, after_first=True, initial=True)
        r["refinement"] = {"poisson_solves": solves, "corrections": corr,
                           "corrections_per_solve": round(corr / max(1, solves), 3),
                           "max_final_divergence": worst,
                           "max_divergence_after_first_correction": first,
                           "max_divergence_of_uncorrected_solve": init_max,
                           "mean_divergence_of_uncorrected_solve": init_mean}
    # post-projection divergence of the final field (last tags, last q_F)
    div, qf = ibm.ibm_divergence(ctx, u, v, w)
    r["post_projection_divergence"] = {"max_abs_Du_minus_qF": div, "qF": qf}
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
    # the whole step against the pass model of the form
    b_model = MODEL_BYTES[form]
    if form == "mixed_refined":
        b_model += MODEL_REFINEMENT_BYTES * r["refinement"]["corrections_per_solve"]
    model_gbs = r["value"] * b_model / 1e9
    r["path_roofline"] = {"bound": "hbm", "model_bytes_per_cell_substep": b_model,
                          "achieved": round(model_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(model_gbs / HBM_PEAK_GBS, 4)}
    impl = sum((algorithmic_bytes(k, wl.nx, wl.ny, wl.nz, form) or 0) * vv[0] / nprof
               for k, vv in prof.items())
    r["impl_pass_bytes"] = {"bytes_per_step": int(impl),
                            "per_cell_substep": round(impl / (2 * cells), 1),
                            "achieved_gbs": round(impl / (el / args.steps) / 1e9, 1)}
    # no-slip error (Sec. 4.4) of the final fields against the bodies at the
    # final time (untimed: body transform and tagging at t, then the error)
    tend = (args.warmup + args.steps) * wl.dt
    move(tend)
    ibm.ibm_tag(ctx, bodies)
    eps, eps_c = ibm.ibm_noslip_error(ctx, u, v, w)
    r["noslip_error"] = {"mean": eps, "u": eps_c[0], "v": eps_c[1], "w": eps_c[2], "time": tend}
    if not all(torch.isfinite(x).all().item() for x in (u, v, w, p)):
        print(f"bench.py: non-finite state after the {wl.name} {form} run", file=sys.stderr)
        sys.exit(1)
    ctx.close()
    return r, (u, v, w)


def run_workload(args, wl, forms, dev):
    """Every form of one workload from the same initial field; the mixed
    forms report their velocity error against the FP64 run (same steps)."""
    import torch
    progress(f"{wl.name}: generating the initial field on the device")
    fields0 = wl.fields_torch(dev)
    order = (["fp64"] if "fp64" in forms else []) + [f for f in forms if f != "fp64"]
    out, ref = {}, None
    for form in order:
        r, final = run_form(args, wl, form, dev, fields0)
        if form == "fp64":
            ref = final
        elif ref is not None:
            # max |difference| per component over the velocity scale of the
            # FP64 run (its largest |u|, |v| or |w|): a component that stays
            # near zero (w of the spanwise-uniform plane workload) would make
            # a per-component ratio meaningless
            scale = max(float(b.abs().max()) for b in ref)
            errs = [float((a - b).abs().max()) / scale for a, b in zip(final, ref)]
            r["velocity_error_vs_fp64"] = {"max_rel": max(errs), "u": errs[0], "v": errs[1],
                                           "w": errs[2], "scale": scale,
                                           "steps": args.warmup + args.steps}
        del final
        out[form] = r
        torch.cuda.empty_cache()
    del fields0, ref
    torch.cuda.empty_cache()
    return {f: out[f] for f in forms}


def run_batched(args, dev, nsim, form):
    """Times the batched workload (nsim simulations of different sizes, one
    body each) in each execution mode (serial, streams, graph, grouped
    launches); the best mode is the form's value."""
    import numpy as np
    import torch
    import workloads
    from paper_2606_09799_amd import ibm

    # the bodies' wall clearance covers every step the modes below run
    nmodes = len([m for m in args.batch_modes.split(",") if m])
    wls = workloads.batch(nsim, steps=nmodes * (args.warmup + args.steps))
    pdt = torch.float64 if form == "fp64" else torch.float32
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sims = []
    for wl in wls:
        u, v, w = wl.fields_torch(dev)
        b = wl.bodies[0]
        nv = b.ref.shape[0]
        sims.append({"nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "lx": wl.lx, "lz": wl.lz,
                     "y_faces": wl.y_faces, "re": wl.re, "dpdx": wl.dpdx, "u": u, "v": v, "w": w,
                     "p": torch.zeros(wl.cells, dtype=pdt, device=dev),
                     "motion": b.kind, "ref": T(b.ref),
                     "xyz": torch.empty(nv, 3, dtype=torch.float64, device=dev),
                     "vel": torch.empty(nv, 3, dtype=torch.float64, device=dev),
                     "tri": T(b.tris.astype(np.int32))})
    batch = ibm.Batch(sims, precision="fp64" if form == "fp64" else "mixed",
                      mixed_poisson="refined" if form == "mixed_refined" else "fp64",
                      refine_tol=DIV_BOUND if form == "mixed_refined" else 0.0)
    dt = wls[0].dt
    cells = sum(wl.cells for wl in wls)
    out = {}
    k = 0

    def coefs():
        return [wl.bodies[0].coef(k * dt) for wl in wls]

    modes = {"serial": ibm.BATCH_SERIAL, "streams": ibm.BATCH_STREAMS,
             "graph": ibm.BATCH_GRAPH, "grouped": ibm.BATCH_GROUPED}
    for name in [m for m in args.batch_modes.split(",") if m]:
        mode = modes[name]
        for _ in range(args.warmup):
            batch.step(coefs(), dt, mode)
            k += 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.step(coefs(), dt, mode)
            k += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = (cells * 2 * args.steps / el, el / args.steps * 1e3)
        progress(f"batched {form} {name}: {el / args.steps * 1e3:.3f} ms per step")
    tune = None  # the library's autotuner is switched off
    flags = batch.check()
    if flags:
        print(f"bench.py: device flags {flags} after the batched {form} run", file=sys.stderr)
        sys.exit(1)
    for d in sims:
        if not all(torch.isfinite(d[q]).all().item() for q in ("u", "v", "w", "p")):
            print(f"bench.py: non-finite state after the batched {form} run", file=sys.stderr)
            sys.exit(1)
    batch.close()
    del sims
    torch.cuda.empty_cache()
    best_mode = max(out, key=lambda m: out[m][0])
    return {"workload": f"c4: {nsim} simulations, {cells} cells in total (uniform spacing 1/32, "
                        "32..128 x 32..96 x 32..128, one sphere, plate or deforming body each), "
                        f"Re 100, dt 1e-3, form {form}",
            "value": out[best_mode][0], "ms_per_step": out[best_mode][1], "mode": best_mode,
            "modes": {m: {"value": v, "ms_per_step": ms} for m, (v, ms) in out.items()},
            "speedup_vs_serial": (out[best_mode][0] / out["serial"][0]) if "serial" in out else None,
            "autotune": tune}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5",
                    help="headline workload (c5: 1024x768x1024 with 67 bodies)")
    ap.add_argument("--forms", default="mixed,fp64,mixed_refined",
                    help="forms of the headline workload; the first one is the headline value")
    ap.add_argument("--also", default="c2,plane,turb",
                    help="further workloads timed in every form (comma list, empty: none)")
    ap.add_argument("--batch-sims", type=int, default=64,
                    help="simulations of the batched workload (0 = skip it)")
    ap.add_argument("--batch-forms", default="fp64,mixed")
    ap.add_argument("--batch-modes", default="serial,streams,graph,grouped",
                    help="batched execution modes to time")

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
    forms = [f for f in args.forms.split(",") if f]
    for f in forms:
        if f not in FORMS:
            raise SystemExit(f"unknown form {f}")
    wl = workloads.config(args.workload)
    head_results = run_workload(args, wl, forms, dev)
    extra = {}
    for name in [x for x in args.also.split(",") if x and x != args.workload]:
        w2 = workloads.config(name)
        extra[name] = {"workload": describe(w2), "cells": w2.cells,
                       "forms": run_workload(args, w2, list(FORMS), dev)}
    batched = {}
    if args.batch_sims > 0:
        for bf in [x for x in args.batch_forms.split(",") if x]:
            try:
                batched[bf] = run_batched(args, dev, args.batch_sims, bf)
            except Exception as e:  # the single-grid results above stand on their own
                print(f"bench.py: the batched workload ({bf}) failed: {type(e).__name__}: {e}",
                      file=sys.stderr, flush=True)
                batched[bf] = {"error": f"{type(e).__name__}: {e}"}
    copy_ref = None
    if args.copy_ref_mib:
        nb = args.copy_ref_mib * 1024 * 1024 // 8
        a = torch.ones(nb, dtype=torch.float64, device=dev)
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        copy_ref = {"bytes_read": nb * 8, "bytes_written": nb * 8, "launches": 3}
    cpu = None
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle on one step of the 256x192x256 plate workload")
        cpu = cpu_baseline(workloads.config("c2"))
    head = head_results[forms[0]]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "cells": wl.cells, "substeps_per_step": 2,
                   "form": forms[0], "parallelism": "single GPU"},
        "roofline": head.get("roofline"),
        "cpu_baseline": cpu,
        "path_roofline": head.get("path_roofline"),
        "forms": {f"{wl.name}_{f}": r for f, r in head_results.items()},
    }
    for name, e in extra.items():
        for f, r in e["forms"].items():
            out["forms"][f"{name}_{f}"] = dict(r, workload=e["workload"])
    for bf, b in batched.items():
        out["forms"][f"batched_{bf}"] = b
    if copy_ref:
        out["copy_ref"] = copy_ref
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
