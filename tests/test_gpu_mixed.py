"""The mixed-precision form against the FP64 oracle (through the C-ABI).

The mixed form keeps u, v, w in FP64 and stores p, H, the predictor
right-hand side and the line-solve intermediates in FP32.  Its Poisson solve
is FP64 (the default), or FP32 transforms refined with FP64 residuals until
max|rhs - L_c phi| * alpha_dt <= 1e-11, which after the projection is
max|D u - q| (paper Eq. mod_div).  Bars: tags bit-exact (the geometry is FP64
in both forms); velocity after whole steps within 1e-6 relative of the FP64
oracle; post-projection divergence on C_F within 1e-10 absolute at every
sub-stage (device statistics) and after every step (host check); single
stages within the FP32 rounding they store."""
import numpy as np
import pytest
import torch

from gpu_harness import Case, DEV, n, rel, t
from oracle import operators as op
from oracle import poisson, predictor, projection, step as ostep

pytestmark = pytest.mark.gpu

SMALL = ["tiny", "tiny_plate", "c1"]


def _tags_equal(case, tags):
    lists, cb = case.ibm.tag_lists(case.ctx)
    for c in range(3):
        assert np.array_equal(n(lists[c][0]), tags.idx[c])
        assert np.array_equal(n(lists[c][1]), tags.tri[c])
    assert np.array_equal(n(cb), tags.cb)


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("stage", [0, 1])
def test_mixed_viscous(name, stage):
    case = Case(name, precision="mixed")
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    masks = ostep.masks_of(g, tags)
    f = case.random_fields(2)
    rng = np.random.default_rng(3)
    p = rng.standard_normal(g.shape).astype(np.float32)
    hprev = [rng.standard_normal(g.comp_shape(c)).astype(np.float32) for c in range(3)]
    hprev[1][0] = hprev[1][-1] = 0.0
    gamma, rho = ostep.SCHEMES["rk2"][stage]
    dt = case.wl.dt
    # the oracle sees the same FP32-representable p and H_prev, in FP64
    ref, Href = predictor.predictor(g, f, p.astype(np.float64),
                                    [h.astype(np.float64) for h in hprev] if rho else None,
                                    masks, gamma, rho, gamma + rho, dt, case.wl.re, case.fext)
    d = [t(a) for a in f]
    hp = [t(a) for a in hprev]
    ho = [torch.zeros(x.numel(), dtype=torch.float32, device=DEV) for x in d]
    case.ibm.ibm_viscous(case.ctx, t(p), hp if rho else None, ho, gamma, rho, dt, *d)
    for c in range(3):
        # du from FP32 line solves of an FP32-stored right-hand side
        assert rel(n(d[c], f[c].shape) - f[c], ref[c] - f[c]) < 2e-6, c
        # forcing nodes are not predicted: du = 0 there exactly
        m = masks[c].reshape(-1)
        assert np.array_equal(n(d[c]).reshape(-1)[m], f[c].reshape(-1)[m])
        assert rel(n(ho[c], f[c].shape).astype(np.float64), Href[c]) < 1e-7, c


@pytest.mark.parametrize("name", SMALL + ["c2"])
def test_mixed_poisson_refined(name):
    """FP32 transforms + FP64-residual refinement reach the requested
    residual; the result agrees with the FP64 oracle solve."""
    case = Case(name, precision="mixed", mixed_poisson="refined", refine_tol=1e-9)
    g = case.g
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.ibm_refine_stats(case.ctx, reset=True)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    solves, corr, final = case.ibm.ibm_refine_stats(case.ctx)
    assert case.ibm.ibm_check(case.ctx) == 0
    assert solves == 1 and 0 <= corr <= 3 and final <= 1e-9
    got = n(phi, g.shape)
    res = op.lap_c(g, got) - rhs
    assert np.max(np.abs(res)) <= 1.5e-9
    assert abs(np.sum(got * dV)) < 1e-12 * np.sum(np.abs(got) * dV)
    if g.cells <= 300_000:
        assert rel(got, poisson.solve(g, rhs)) < 1e-8


def test_mixed_poisson_aliased_rhs():
    case = Case("tiny", precision="mixed", mixed_poisson="refined", refine_tol=1e-9)
    g = case.g
    rng = np.random.default_rng(8)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    x = t(rhs)
    case.ibm.poisson_solve(case.ctx, x, x)
    assert case.ibm.ibm_check(case.ctx) == 0
    assert rel(n(x, g.shape), poisson.solve(g, rhs)) < 1e-8


def test_mixed_refinement_flag():
    """An unreachable tolerance with one refinement allowed: exactly one
    correction runs and the sticky flag reports it (forced from the host)."""
    case = Case("tiny", precision="mixed", mixed_poisson="refined", refine_max=1,
                refine_tol=1e-300)
    g = case.g
    rng = np.random.default_rng(9)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    solves, corr, _ = case.ibm.ibm_refine_stats(case.ctx)
    assert (solves, corr) == (1, 1)
    assert case.ibm.ibm_check(case.ctx) == case.ibm.FLAG_REFINE
    assert case.ibm.ibm_check(case.ctx) == 0  # cleared


@pytest.mark.parametrize("name", SMALL)
def test_mixed_project(name):
    case = Case(name, precision="mixed")
    g = case.g
    f = case.random_fields(6)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(g.shape)
    p = rng.standard_normal(g.shape).astype(np.float32)
    ref, pref = projection.project(g, f, p.astype(np.float64), phi, 0.5, case.wl.dt, case.wl.re)
    d = [t(a) for a in f]
    pd = t(p)
    case.ibm.ibm_project(case.ctx, t(phi), 0.5 * case.wl.dt, *d, pd)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), ref[c]) < 1e-12
    # FP64 update rounded once to FP32
    assert rel(n(pd, g.shape).astype(np.float64), pref) < 1e-7


def _run_mixed(name, steps, mixed_poisson):
    case = Case(name, precision="mixed", mixed_poisson=mixed_poisson)
    g, wl = case.g, case.wl
    f = wl.fields()
    d = [t(a) for a in f]
    pd = torch.zeros(g.cells, dtype=torch.float32, device=DEV)
    p = np.zeros(g.shape)
    worst_div = 0.0
    case.ibm.ibm_refine_stats(case.ctx, reset=True)
    for s in range(steps):
        time = s * wl.dt
        bodies, surf = case.bodies_at(time)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt)
        f, p, _, tags = ostep.step(g, f, p, surf, wl.dt, wl.re, case.fext)
        u = [n(x, f[c].shape) for c, x in enumerate(d)]
        D = op.divergence(g, *u)
        mB = projection.cell_mask(g, tags.cb)
        qF = np.median(D[~mB])
        worst_div = max(worst_div, float(np.max(np.abs(D[~mB] - qF))))
    assert case.ibm.ibm_check(case.ctx) == 0
    return case, g, d, pd, f, p, tags, worst_div


@pytest.mark.parametrize("mixed_poisson", ["fp64", "refined"])
@pytest.mark.parametrize("name,steps", [("tiny", 3), ("tiny_plate", 3), ("c1", 10)])
def test_mixed_step_against_fp64_oracle(name, steps, mixed_poisson):
    case, g, d, pd, f, p, tags, worst_div = _run_mixed(name, steps, mixed_poisson)
    _tags_equal(case, tags)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-6, c
    assert worst_div < 1e-10
    if mixed_poisson == "refined":
        solves, corr, final = case.ibm.ibm_refine_stats(case.ctx)
        assert solves == 2 * steps
        assert final <= 1e-11
        assert corr <= 3 * solves
    mB = projection.cell_mask(g, tags.cb)
    dV = g.cell_volume()
    got = n(pd, g.shape).astype(np.float64)

    def centred(a):
        return a[~mB] - np.sum(a[~mB] * dV[~mB]) / np.sum(dV[~mB])
    assert rel(centred(got), centred(p)) < 1e-5


def test_mixed_refined_step_x256():
    """The refined mixed step on x lines of 256 cells, where the length-256 x
    transforms run on the FP32 spectrum: the velocity source, kept in FP64
    for the refinement, and the residual passes are formed by their
    branch-free row stagings.  A sphere in the channel, two steps: velocity
    within 1e-6 of the FP64 oracle, post-projection divergence below 1e-10,
    the refinement reaching its tolerance."""
    import workloads
    d = 2.0 / 12
    wl = workloads.Workload("x256", 256, 12, 16, 256 * d, 16 * d, workloads.uniform_faces(12),
                            100.0, 1e-3, 2, 1.0, 0.01, 17, -0.02,
                            [workloads._sphere_body(2, 0.3, (128 * d, 0.0, 8 * d),
                                                    (0.2, 0.05, -0.1))])
    case, g, dv, pd, f, p, tags, worst_div = _run_mixed(wl, 2, "refined")
    _tags_equal(case, tags)
    for c in range(3):
        assert rel(n(dv[c], f[c].shape), f[c]) < 1e-6, c
    assert worst_div < 1e-10
    solves, corr, final = case.ibm.ibm_refine_stats(case.ctx)
    assert solves == 4 and final <= 1e-11
