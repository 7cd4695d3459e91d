"""Edge cases and degenerate inputs of the HIP path (through the C-ABI):
no body at all, forcing lists that overflow their capacity, a probe that
would leave the channel, the AB+CN scheme against the oracle, run-to-run
determinism, and the largest single-grid workload (512x384x512 with a
20480-triangle deforming body) in both precision forms."""
import numpy as np
import pytest
import torch

import workloads
from gpu_harness import Case, DEV, n, rel, t
from oracle import kinematics, operators as op, projection, step as ostep

pytestmark = pytest.mark.gpu


def test_empty_body_list():
    """Without bodies the step is the plain channel step: no forcing node,
    no boundary cell, q_F = 0, and the oracle's result within 1e-10."""
    case = Case("tiny")
    g, wl = case.g, case.wl
    f = wl.fields()
    d = [t(a) for a in f]
    pd = torch.zeros(g.cells, dtype=torch.float64, device=DEV)
    p = np.zeros(g.shape)
    empty = (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    for _ in range(2):
        case.ibm.ibm_step(case.ctx, *d, pd, [], wl.dt)
        f, p, _, tags = ostep.step(g, f, p, empty, wl.dt, wl.re, case.fext)
    assert case.ibm.ibm_tags_count_host(case.ctx) == [0, 0, 0, 0]
    assert case.ibm.ibm_check(case.ctx) == 0
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c


def test_capacity_overflow_is_flagged():
    """A forcing-list capacity far below the node count: the lists hold
    their first entries, nothing is written past them, and the sticky flag
    reports the overflow; a second context with room agrees on those
    entries."""
    small = Case("tiny", force_cap=16)
    bodies, (X, U, T) = small.bodies_at(0.0)
    small.ibm.ibm_tag(small.ctx, bodies)
    counts = small.ibm.ibm_tags_count_host(small.ctx)
    assert min(counts[:3]) > 16
    assert small.ibm.ibm_check(small.ctx) & small.ibm.FLAG_CAPACITY
    tags = ostep.compute_tags(small.g, X, T)
    for c in range(3):
        idx = torch.empty(16, dtype=torch.int64, device=DEV)
        tri = torch.empty(16, dtype=torch.int32, device=DEV)
        small.ibm._ok(small.ibm._tags_copy(small.ctx.handle, c, small.ibm.c_void_p(idx.data_ptr()),
                                           small.ibm.c_void_p(tri.data_ptr()), 16), "copy")
        assert np.array_equal(n(idx), tags.idx[c][:16])
        assert np.array_equal(n(tri), tags.tri[c][:16])
    # a step on the truncated lists completes; the flag is raised again
    d = [t(a) for a in small.fields()]
    pd = torch.zeros(small.g.cells, dtype=torch.float64, device=DEV)
    small.ibm.ibm_step(small.ctx, *d, pd, bodies, small.wl.dt)
    assert small.ibm.ibm_check(small.ctx) & small.ibm.FLAG_CAPACITY
    assert all(torch.isfinite(x).all().item() for x in d)


def test_probe_leaving_the_channel_is_flagged():
    """A sphere so close to the lower wall that outward probes (length
    h = 2 x cell diagonal) cross it: the forcing flags the geometry limit
    and falls back to the wall velocity for those nodes."""
    wl = workloads.config("tiny")
    b = wl.bodies[0]
    r = float(np.linalg.norm(b.ref[0]))
    c0 = np.array([3.0, -1.0 + r + 0.08, 1.6])
    wl.bodies = [workloads.Body("rigid", b.ref, b.tris,
                                lambda tt: workloads.sphere_translation(tt, c0, (0.0, 0.0, 0.0)))]
    case = Case(wl)
    bodies, _ = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    d = [t(a) for a in wl.fields()]
    case.ibm.ibm_force(case.ctx, *d)
    assert case.ibm.ibm_check(case.ctx) & case.ibm.FLAG_GEOM


def test_ab2_parity():
    """AB+CN: the first step is taken by the oracle (explicit Euler on H, as
    the scheme starts); from then on both sides run AB+CN from the same
    state and H, and H^n comes back through the state."""
    case = Case("tiny_plate", scheme="ab2")
    g, wl = case.g, case.wl
    f = wl.fields()
    p = np.zeros(g.shape)
    _, surf = case.bodies_at(0.0)
    f, p, H, _ = ostep.step(g, f, p, surf, wl.dt, wl.re, case.fext, scheme="ab2")
    d = [t(a) for a in f]
    pd = t(p)
    hd = [t(a) for a in H]
    for s in (1, 2):
        bodies, surf = case.bodies_at(s * wl.dt)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt, h=hd)
        f, p, H, tags = ostep.step(g, f, p, surf, wl.dt, wl.re, case.fext, scheme="ab2",
                                   hprev=H)
    assert case.ibm.ibm_check(case.ctx) == 0
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c
        assert rel(n(hd[c], f[c].shape), H[c]) < 1e-10, c


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steps_are_deterministic(precision):
    """The same steps from the same state give the same bits (no
    floating-point atomics on the path; fixed-order reductions)."""
    outs = []
    for _ in range(2):
        case = Case("c1", precision=precision)
        d = [t(a) for a in case.fields()]
        pd = torch.zeros(case.g.cells, dtype=case.ctx.pdtype, device=DEV)
        for s in range(2):
            bodies, _ = case.bodies_at(s * case.wl.dt)
            case.ibm.ibm_step(case.ctx, *d, pd, bodies, case.wl.dt)
        assert case.ibm.ibm_check(case.ctx) == 0
        outs.append([x.clone() for x in d + [pd]])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_c3_full_size_mixed_against_fp64():
    """The largest single-grid workload, 512x384x512 with a 20480-triangle
    deforming body: two steps in each form from the same state; the mixed
    velocity within 1e-6 of the FP64 one and D u = q_F on C_F to 1e-10 in
    both."""
    wl = workloads.config("c3")
    f0 = wl.fields()
    res = {}
    for precision in ("fp64", "mixed"):
        case = Case(wl, precision=precision)
        d = [t(a) for a in f0]
        pd = torch.zeros(case.g.cells, dtype=case.ctx.pdtype, device=DEV)
        for s in range(2):
            bodies, _ = case.bodies_at(s * wl.dt)
            case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt)
        assert case.ibm.ibm_check(case.ctx) == 0
        res[precision] = [n(x, f0[c].shape) for c, x in enumerate(d)]
        lists, cb = case.ibm.tag_lists(case.ctx)
        g = case.g
        D = op.divergence(g, *res[precision])
        mB = projection.cell_mask(g, n(cb))
        qF = np.median(D[~mB])
        assert np.max(np.abs(D[~mB] - qF)) < 1e-10, precision
        del case, d, pd
        torch.cuda.empty_cache()
    for c in range(3):
        assert rel(res["mixed"][c], res["fp64"][c]) < 1e-6, c


def test_incompatible_poisson_rhs_is_flagged():
    """poisson_solve checks the compatibility condition of the Neumann
    problem (App. A: sum rhs dV = 0): a right-hand side with its volume mean
    removed passes; adding a constant (the mean of |rhs| times 1e-6) makes
    |sum rhs dV| exceed 1e-12 sum |rhs| dV and raises IBM_FLAG_COMPAT, also
    on the mixed form's refined solve."""
    for opts in ({}, {"precision": "mixed", "mixed_poisson": "refined"}):
        case = Case("tiny", **opts)
        g = case.g
        rng = np.random.default_rng(5)
        r = rng.standard_normal(g.shape)
        dV = g.cell_volume()
        r -= np.sum(r * dV) / np.sum(dV)
        phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
        case.ibm.poisson_solve(case.ctx, t(r), phi)
        assert case.ibm.ibm_check(case.ctx) & case.ibm.FLAG_COMPAT == 0
        bad = r + 1e-6 * np.mean(np.abs(r))
        case.ibm.poisson_solve(case.ctx, t(bad), phi)
        fl = case.ibm.ibm_check(case.ctx)
        assert fl & case.ibm.FLAG_COMPAT, fl
        assert torch.isfinite(phi).all().item()


def test_body_displacement_over_half_a_cell_is_flagged():
    """ibm_step flags (IBM_FLAG_CFL) a body whose vertices move more than
    half the local spacing in one step (the one-layer fresh-cell treatment of
    Sec. 3.1 needs less): the sphere of the ragged case moved at 0.4 of the
    x spacing per step passes, at 0.6 of it the flag is raised; the step
    itself still runs."""
    for frac, expect in ((0.4, False), (0.6, True)):
        wl = workloads.config("tiny")
        b = wl.bodies[0]
        dx = wl.lx / wl.nx
        U = np.array([frac * dx / wl.dt, 0.0, 0.0])
        c0 = np.array([3.0, 0.0, 1.6])
        wl.bodies = [workloads.Body("rigid", b.ref, b.tris,
                                    lambda tt, U=U: workloads.sphere_translation(tt, c0, U))]
        case = Case(wl)
        bodies, _ = case.bodies_at(0.0)
        d = [t(a) for a in wl.fields()]
        pd = torch.zeros(case.g.cells, dtype=torch.float64, device=DEV)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt)
        fl = case.ibm.ibm_check(case.ctx)
        assert bool(fl & case.ibm.FLAG_CFL) == expect, (frac, fl)
        assert fl & ~case.ibm.FLAG_CFL == 0, fl


def test_first_step_at_a_new_dt_needs_no_host_wait():
    """A new dt rebuilds the line-solve tables on the host and copies them in
    stream order: steps at dt, 2 dt and back at dt, enqueued with no
    synchronisation in between, equal the same steps taken one at a time with
    a synchronisation after each."""
    case = Case("tiny")
    wl = case.wl
    bodies, _ = case.bodies_at(0.0)
    dts = (wl.dt, 2 * wl.dt, wl.dt, 0.5 * wl.dt)
    a = [t(x) for x in wl.fields()]
    pa = torch.zeros(case.g.cells, dtype=torch.float64, device=DEV)
    for dt in dts:
        case.ibm.ibm_step(case.ctx, *a, pa, bodies, dt)
    case2 = Case("tiny")
    bodies2, _ = case2.bodies_at(0.0)
    b = [t(x) for x in wl.fields()]
    pb = torch.zeros(case2.g.cells, dtype=torch.float64, device=DEV)
    for dt in dts:
        case2.ibm.ibm_step(case2.ctx, *b, pb, bodies2, dt)
        torch.cuda.synchronize()
    assert case.ibm.ibm_check(case.ctx) == 0 and case2.ibm.ibm_check(case2.ctx) == 0
    for x, y in zip(a + [pa], b + [pb]):
        assert torch.equal(x, y)
