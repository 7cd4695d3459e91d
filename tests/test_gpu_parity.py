"""Parity of the HIP path (called through the C-ABI) with the CPU oracle on
identical seeded inputs.

Bar: bit-exact for the integer outputs (body vertices, forcing lists,
forcing triangles, C_B); FP64 single-stage outputs within 1e-12 of the
oracle relative to the field's max-norm (Poisson 1e-11: the low wall-normal
modes amplify rounding); whole steps within 1e-10 relative (velocity; the
pressure on C_F after removing its volume-weighted mean)."""
import numpy as np
import pytest
import torch

from gpu_harness import Case, DEV, n, rel, t
from oracle import diagnostics, forcing, poisson, predictor, projection, step as ostep
from oracle import operators as op

pytestmark = pytest.mark.gpu

SMALL = ["tiny", "tiny_plate", "c1"]


def _tags_equal(case, tags):
    lists, cb = case.ibm.tag_lists(case.ctx)
    for c in range(3):
        assert np.array_equal(n(lists[c][0]), tags.idx[c]), f"forcing nodes, component {c}"
        assert np.array_equal(n(lists[c][1]), tags.tri[c]), f"forcing triangles, component {c}"
    assert np.array_equal(n(cb), tags.cb), "boundary cells"


@pytest.mark.parametrize("name", SMALL)
def test_body_transform_bit_exact(name):
    case = Case(name)
    for time in (0.0, 0.0137, 0.5):
        bodies, (X, U, _) = case.bodies_at(time)
        assert np.array_equal(n(bodies[0].xyz), X)
        assert np.array_equal(n(bodies[0].vel), U)


@pytest.mark.parametrize("name,time", [("tiny", 0.0), ("tiny", 0.011), ("tiny_plate", 0.0),
                                       ("tiny_plate", 0.137), ("c1", 0.0), ("c1", 0.009)])
def test_tags_bit_exact(name, time):
    case = Case(name)
    bodies, surf = case.bodies_at(time)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(case.g, surf[0], surf[2])
    assert sum(tags.counts) > 0
    _tags_equal(case, tags)
    assert case.ibm.ibm_check(case.ctx) == 0


@pytest.mark.parametrize("name", SMALL)
def test_force_parity(name):
    case = Case(name)
    bodies, (X, U, T) = case.bodies_at(0.003)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(case.g, X, T)
    f = case.random_fields(1)
    ref = forcing.apply_ib(case.g, f, list(zip(tags.idx, tags.tri)), X, U, T)
    d = [t(a) for a in f]
    case.ibm.ibm_force(case.ctx, *d)
    for c in range(3):
        got = n(d[c], f[c].shape)
        assert rel(got, ref[c]) < 1e-12, c
        # untouched elsewhere
        m = np.ones(f[c].size, bool)
        m[tags.idx[c]] = False
        assert np.array_equal(got.reshape(-1)[m], f[c].reshape(-1)[m])
    assert case.ibm.ibm_check(case.ctx) == 0


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("stage", [0, 1])
def test_viscous_parity(name, stage):
    case = Case(name)
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    masks = ostep.masks_of(g, tags)
    f = case.random_fields(2)
    rng = np.random.default_rng(3)
    p = rng.standard_normal(g.shape)
    hprev = [rng.standard_normal(g.comp_shape(c)) for c in range(3)]
    hprev[1][0] = hprev[1][-1] = 0.0
    gamma, rho = ostep.SCHEMES["rk2"][stage]
    dt = case.wl.dt
    ref, Href = predictor.predictor(g, f, p, hprev if rho else None, masks, gamma, rho,
                                    gamma + rho, dt, case.wl.re, case.fext)
    d = [t(a) for a in f]
    hp = [t(a) for a in hprev]
    ho = [torch.zeros_like(x) for x in d]
    case.ibm.ibm_viscous(case.ctx, t(p), hp if rho else None, ho, gamma, rho, dt, *d)
    for c in range(3):
        assert rel(n(d[c], f[c].shape) - f[c], ref[c] - f[c]) < 1e-12, c
        assert rel(n(ho[c], f[c].shape), Href[c]) < 1e-12, c


def _long_line_workload(axis, nx=16, nz_y=16):
    """Lines of 64 segments (blocks of 1024 threads in the column sweeps), with
    a sphere so that segments hold forcing nodes: y lines of 768 rows
    (12-row segments) or z lines of 1024 rows (16-row segments); with nx = 32
    the FP32 line data of the mixed form take 24-row (y) and 32-row (z)
    segments instead, 32 lines per block."""
    import workloads
    if axis == "y":
        return workloads.Workload("long_y", nx, 768, nz_y, 0.01 * nx, 0.01 * nz_y,
                                  workloads.uniform_faces(768), 100.0, 1e-3, 2, 1.0, 0.01, 13,
                                  -0.02, [workloads._sphere_body(2, 0.04, (0.08, 0.0, 0.08),
                                                                 (0.2, 0.05, -0.1))])
    return workloads.Workload("long_z", nx, 24, 1024, nx * 2.0 / 24, 1024 * 2.0 / 24,
                              workloads.uniform_faces(24), 100.0, 1e-3, 2, 1.0, 0.01, 13, -0.02,
                              [workloads._sphere_body(2, 0.3, (0.66, 0.0, 40.0), (0.2, 0.05, -0.1))])


@pytest.mark.parametrize("axis", ["y", "z"])
@pytest.mark.parametrize("stage", [0, 1])
def test_viscous_parity_long_lines(axis, stage):
    case = Case(_long_line_workload(axis))
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    assert min(len(i) for i in tags.idx) > 0
    masks = ostep.masks_of(g, tags)
    f = case.random_fields(4)
    rng = np.random.default_rng(6)
    p = rng.standard_normal(g.shape)
    hprev = [rng.standard_normal(g.comp_shape(c)) for c in range(3)]
    hprev[1][0] = hprev[1][-1] = 0.0
    gamma, rho = ostep.SCHEMES["rk2"][stage]
    dt = case.wl.dt
    ref, Href = predictor.predictor(g, f, p, hprev if rho else None, masks, gamma, rho,
                                    gamma + rho, dt, case.wl.re, case.fext)
    d = [t(a) for a in f]
    hp = [t(a) for a in hprev]
    ho = [torch.zeros_like(x) for x in d]
    case.ibm.ibm_viscous(case.ctx, t(p), hp if rho else None, ho, gamma, rho, dt, *d)
    for c in range(3):
        assert rel(n(d[c], f[c].shape) - f[c], ref[c] - f[c]) < 1e-12, c
        assert rel(n(ho[c], f[c].shape), Href[c]) < 1e-12, c


@pytest.mark.parametrize("axis,nz_y", [("y", 16), ("y", 14), ("z", 16)])
@pytest.mark.parametrize("stage", [0, 1])
def test_mixed_viscous_long_segments(axis, nz_y, stage):
    """The mixed form's FP32 column sweeps in 24-row (y, 768 rows) and
    32-row (z, 1024 rows) segments, 32 lines per block, with forcing nodes
    inside segments (the y sweep's whole z rows per XCD also with 14 z
    rows: a last round of 6): du within the FP32 rounding of its stored
    right-hand side of the FP64 oracle, du = 0 exactly on forcing nodes."""
    case = Case(_long_line_workload(axis, nx=32, nz_y=nz_y), precision="mixed")
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    assert min(len(i) for i in tags.idx) > 0
    masks = ostep.masks_of(g, tags)
    f = case.random_fields(5)
    rng = np.random.default_rng(7)
    p = rng.standard_normal(g.shape).astype(np.float32)
    hprev = [rng.standard_normal(g.comp_shape(c)).astype(np.float32) for c in range(3)]
    hprev[1][0] = hprev[1][-1] = 0.0
    gamma, rho = ostep.SCHEMES["rk2"][stage]
    dt = case.wl.dt
    ref, Href = predictor.predictor(g, f, p.astype(np.float64),
                                    [h.astype(np.float64) for h in hprev] if rho else None,
                                    masks, gamma, rho, gamma + rho, dt, case.wl.re, case.fext)
    d = [t(a) for a in f]
    hp = [t(a) for a in hprev]
    ho = [torch.zeros(x.numel(), dtype=torch.float32, device=DEV) for x in d]
    case.ibm.ibm_viscous(case.ctx, t(p), hp if rho else None, ho, gamma, rho, dt, *d)
    for c in range(3):
        assert rel(n(d[c], f[c].shape) - f[c], ref[c] - f[c]) < 2e-6, c
        m = masks[c].reshape(-1)
        assert np.array_equal(n(d[c]).reshape(-1)[m], f[c].reshape(-1)[m])
        assert rel(n(ho[c], f[c].shape).astype(np.float64), Href[c]) < 1e-7, c
    case.ctx.close()


@pytest.mark.parametrize("name,time", [("tiny", 0.011), ("tiny_plate", 0.137), ("c1", 0.0)])
def test_noslip_error_parity(name, time):
    """No-slip error of Sec. 4.4 at the forcing nodes of the current tags,
    per component and averaged, against the oracle's diagnostics on the same
    fields (random, so that every node contributes)."""
    case = Case(name)
    bodies, (X, U, T) = case.bodies_at(time)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(case.g, X, T)
    f = case.random_fields(7)
    eps, per = case.ibm.ibm_noslip_error(case.ctx, *[t(a) for a in f])
    eps_ref, per_ref = diagnostics.noslip_error(case.g, f, tags, X, U, T)
    assert eps_ref > 0
    assert abs(eps - eps_ref) <= 1e-12 * eps_ref
    for a, b in zip(per, per_ref):
        assert abs(a - b) <= 1e-12 * max(b, 1e-300)
    assert case.ibm.ibm_check(case.ctx) == 0


@pytest.mark.parametrize("name,time,precision", [("c1", 0.0, "fp64"), ("c1", 0.009, "fp64"),
                                                  ("tiny", 0.011, "fp64"), ("c1", 0.0, "mixed")])
def test_pressure_cb_parity(name, time, precision):
    """Pressure rebuilt on the boundary cells (Sec. 2, after Eq. q_F; the
    reading of the oracle) against the oracle on the same random p; the
    mixed form reads an FP32 p.  An output shorter than the boundary-cell
    count raises the capacity flag."""
    case = Case(name, precision=precision)
    bodies, (X, U, T) = case.bodies_at(time)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(case.g, X, T)
    assert len(tags.cb) > 0
    p = np.random.default_rng(9).standard_normal(case.g.shape)
    pd = t(p).to(torch.float32 if precision == "mixed" else torch.float64)
    ref = diagnostics.pressure_cb(case.g, n(pd.double(), case.g.shape), tags, X, T)
    out = torch.full((len(tags.cb),), float("nan"), dtype=torch.float64, device=DEV)
    case.ibm.ibm_pressure_cb(case.ctx, pd, out)
    assert np.max(np.abs(n(out) - ref)) <= 1e-12 * np.max(np.abs(p))
    assert case.ibm.ibm_check(case.ctx) == 0
    short = torch.zeros(len(tags.cb) - 1, dtype=torch.float64, device=DEV)
    case.ibm.ibm_pressure_cb(case.ctx, pd, short)
    assert case.ibm.ibm_check(case.ctx) & case.ibm.FLAG_CAPACITY


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("use_q", [True, False])
def test_mass_rhs_parity(name, use_q):
    case = Case(name, use_q=use_q)
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    f = case.random_fields(4)
    adt = 0.5 * case.wl.dt
    rhs_ref, qf_ref, _ = projection.mass_correction(g, f, tags.cb, 0.5, case.wl.dt, use_q)
    rhs = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    qf = torch.zeros(1, dtype=torch.float64, device=DEV)
    case.ibm.ibm_mass_rhs(case.ctx, *[t(a) for a in f], adt, rhs, qf)
    assert abs(n(qf)[0] - qf_ref) <= 1e-12 * max(abs(qf_ref), 1e-300) + 1e-300
    assert rel(n(rhs, g.shape), rhs_ref) < 1e-12


@pytest.mark.parametrize("name", SMALL + ["c2"])
def test_poisson_parity(name):
    case = Case(name)
    g = case.g
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    got = n(phi, g.shape)
    if g.cells <= 300_000:
        assert rel(got, poisson.solve(g, rhs)) < 1e-11
    # at any size: the discrete residual and the gauge
    res = op.lap_c(g, got) - rhs
    assert np.max(np.abs(res)) < 1e-9 * np.max(np.abs(rhs))
    assert abs(np.sum(got * dV)) < 1e-12 * np.sum(np.abs(got) * dV)


@pytest.mark.parametrize("shape", [(256, 12, 16), (16, 12, 256), (16, 800, 8), (16, 528, 16),
                                   (16, 500, 16), (16, 8, 512), (24, 6, 1024), (16, 192, 16),
                                   (24, 100, 16), (1024, 5, 9), (512, 7, 9)])
def test_poisson_parity_kernel_paths(shape):
    """Shapes that select the other kernel paths, compared with the oracle
    value by value: length-256 x transforms (four-step), length-256 z
    transforms (four-step), a wall-normal solve with more than 64
    separators per mode even in 12-row segments (ny = 800: block-wide
    reduction), the wavefront solve in 44 equal 12-row segments (ny = 528)
    and in 42 unequal ones of at most 12 rows (ny = 500), length-512 and
    -1024 z transforms (16 x 16 x R; 24 x-points: a partial last tile of
    modes), the wall-normal solve of 32 equal 6-row segments (ny = 192,
    straight-line rows) and of 17 unequal ones (ny = 100), the inverse x
    transforms of lengths 1024 and 512 (16 x 16 x R, one row pair per 64 or
    32 lanes; an odd row count leaves a last pair of one row); stretched y."""
    import workloads
    nx, ny, nz = shape
    wl = workloads.Workload("paths", nx, ny, nz, 2 * np.pi, np.pi, workloads.tanh_faces(ny),
                            1.0, 1.0, 1, 0.0, 0.0, 1, 0.0, [])
    case = Case(wl)
    g = case.g
    rng = np.random.default_rng(11)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    assert rel(n(phi, g.shape), poisson.solve(g, rhs)) < 1e-11


@pytest.mark.parametrize("shape", [(16, 8, 512), (24, 6, 1024), (16, 192, 16)])
def test_poisson_refined_long_z(shape):
    """The FP32 length-512 and -1024 z transforms, and the wall-normal solve
    of an FP32 spectrum in 32 equal segments, inside the refined mixed solve:
    the refined result agrees with the FP64 oracle solve."""
    import workloads
    nx, ny, nz = shape
    wl = workloads.Workload("paths", nx, ny, nz, 2 * np.pi, np.pi, workloads.tanh_faces(ny),
                            1.0, 1.0, 1, 0.0, 0.0, 1, 0.0, [])
    case = Case(wl, precision="mixed", mixed_poisson="refined", refine_tol=1e-9)
    g = case.g
    rng = np.random.default_rng(12)
    rhs = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    assert case.ibm.ibm_check(case.ctx) == 0
    assert rel(n(phi, g.shape), poisson.solve(g, rhs)) < 1e-8


def test_poisson_closed_form_eigenmode():
    import workloads
    wl = workloads.Workload("eig", 16, 12, 10, 2 * np.pi, np.pi, workloads.uniform_faces(12),
                            1.0, 1.0, 1, 0.0, 0.0, 1, 0.0, [])
    case = Case(wl)
    g = case.g
    p, m, q = 3, 2, 4
    xc = (np.arange(g.nx) + 0.5) * g.dx
    zc = (np.arange(g.nz) + 0.5) * g.dz
    ph = (np.cos(np.pi * q * (g.yc + 1) / 2)[:, None, None]
          * np.cos(2 * np.pi * m * zc / g.lz)[None, :, None]
          * np.cos(2 * np.pi * p * xc / g.lx)[None, None, :])
    lam = (-(4 / g.dx ** 2) * np.sin(np.pi * p / g.nx) ** 2
           - (4 / g.dz ** 2) * np.sin(np.pi * m / g.nz) ** 2
           - (4 / g.dy[0] ** 2) * np.sin(np.pi * q / (2 * g.ny)) ** 2)
    out = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(lam * ph), out)
    assert np.max(np.abs(n(out, g.shape) - ph)) < 1e-13


@pytest.mark.parametrize("name", SMALL)
def test_project_parity(name):
    case = Case(name)
    g = case.g
    f = case.random_fields(6)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(g.shape)
    p = rng.standard_normal(g.shape)
    adt = 0.5 * case.wl.dt
    ref, pref = projection.project(g, f, p, phi, 0.5, case.wl.dt, case.wl.re)
    d = [t(a) for a in f]
    pd = t(p)
    case.ibm.ibm_project(case.ctx, t(phi), adt, *d, pd)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), ref[c]) < 1e-12
    assert rel(n(pd, g.shape), pref) < 1e-12


def _run_both(name, steps, use_q=True):
    case = Case(name, use_q=use_q)
    g, wl = case.g, case.wl
    f = wl.fields()
    d = [t(a) for a in f]
    pd = torch.zeros(g.cells, dtype=torch.float64, device=DEV)
    p = np.zeros(g.shape)
    for s in range(steps):
        time = s * wl.dt
        bodies, surf = case.bodies_at(time)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt)
        f, p, _, tags = ostep.step(g, f, p, surf, wl.dt, wl.re, case.fext, use_q=use_q)
    assert case.ibm.ibm_check(case.ctx) == 0
    return case, g, d, pd, f, p, tags


@pytest.mark.parametrize("name,steps", [("tiny", 3), ("tiny_plate", 3), ("c1", 10)])
def test_step_parity(name, steps):
    case, g, d, pd, f, p, tags = _run_both(name, steps)
    _tags_equal(case, tags)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c
    mB = projection.cell_mask(g, tags.cb)
    dV = g.cell_volume()
    got = n(pd, g.shape)

    def centred(a):
        return a[~mB] - np.sum(a[~mB] * dV[~mB]) / np.sum(dV[~mB])
    assert rel(centred(got), centred(p)) < 1e-10


@pytest.mark.parametrize("nx,use_q", [(512, True), (1024, True), (1024, False)])
def test_step_parity_long_x(nx, use_q):
    """Whole steps on x lines of 512 and 1024 cells (the x sweep on 32 and 64
    segments per line, the generic x transforms with the velocity source
    formed branch-free, with and without the C_B mask), a sphere in the
    channel: velocity within 1e-10 of the oracle after two steps."""
    import workloads
    d = 2.0 / 24
    wl = workloads.Workload("long_x", nx, 24, 16, nx * d, 16 * d, workloads.uniform_faces(24),
                            100.0, 1e-3, 2, 1.0, 0.01, 13, -0.02,
                            [workloads._sphere_body(2, 0.3, (nx * d / 2, 0.0, 8 * d),
                                                    (0.2, 0.05, -0.1))])
    case, g, d, pd, f, p, tags = _run_both(wl, 2, use_q=use_q)
    _tags_equal(case, tags)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c


def test_step_parity_without_mass_correction():
    case, g, d, pd, f, p, tags = _run_both("tiny", 2, use_q=False)
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c


def test_c2_full_size_tags_and_step_properties():
    """256x192x256 stretched channel with the heaving/pitching plate: tags
    bit-exact at t = 0 (plate on the v-node plane: the |N| = 0 case) and at
    t = 0.37; after one GPU step D u = q holds on C_F to 1e-10 and the total
    divergence vanishes."""
    case = Case("c2")
    g = case.g
    for time in (0.0, 0.37):
        bodies, (X, U, T) = case.bodies_at(time)
        case.ibm.ibm_tag(case.ctx, bodies)
        tags = ostep.compute_tags(g, X, T)
        _tags_equal(case, tags)
    bodies, (X, U, T) = case.bodies_at(0.0)
    tags = ostep.compute_tags(g, X, T)
    f = case.wl.fields()
    d = [t(a) for a in f]
    # forcing values at full size against the oracle on the same field
    ref = forcing.apply_ib(g, f, list(zip(tags.idx, tags.tri)), X, U, T)
    case.ibm.ibm_tag(case.ctx, bodies)
    case.ibm.ibm_force(case.ctx, *d)
    for c in range(3):
        got = n(d[c]).reshape(-1)[tags.idx[c]]
        assert rel(got, ref[c].reshape(-1)[tags.idx[c]]) < 1e-12
    d = [t(a) for a in f]
    pd = torch.zeros(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.ibm_step(case.ctx, *d, pd, bodies, case.wl.dt)
    assert case.ibm.ibm_check(case.ctx) == 0
    u = [n(x, f[c].shape) for c, x in enumerate(d)]
    D = op.divergence(g, *u)
    mB = projection.cell_mask(g, tags.cb)
    qF = np.median(D[~mB])
    assert np.max(np.abs(D[~mB] - qF)) < 1e-10
    assert abs(np.sum(D * g.cell_volume())) < 1e-10


@pytest.mark.parametrize("shape,stretch", [((32, 96, 16), 2.5), ((16, 390, 16), 2.5),
                                           ((16, 768, 8), 2.0), ((16, 800, 8), 2.0)])
def test_poisson_residual_at_the_rounding_floor(shape, stretch):
    """The discrete residual max|rhs - L_c phi| of the direct solve on
    strongly stretched grids is that of the oracle's own solve (paper
    Eq. elliptic_mod; its size is the post-projection divergence over alpha
    dt): wall-normal solves of 16 separators per mode (6-row segments), 33
    and 64 (12-row segments) and 67 (12-row segments, block-wide).  A
    separator system formed and reduced from the diagonal b = lambda - a - c
    loses digits for the low modes where a + c is large (near the walls);
    such a solve left about 50 times the oracle's residual here."""
    import workloads
    nx, ny, nz = shape
    wl = workloads.Workload("resid", nx, ny, nz, 2 * np.pi, np.pi,
                            workloads.tanh_faces(ny, stretch), 1.0, 1.0, 1, 0.0, 0.0, 1, 0.0, [])
    case = Case(wl)
    g = case.g
    rhs = np.random.default_rng(3).standard_normal(g.shape) * 1e3
    dV = g.cell_volume()
    rhs -= np.sum(rhs * dV) / np.sum(dV)
    phi = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    case.ibm.poisson_solve(case.ctx, t(rhs), phi)
    got = n(phi, g.shape)
    ref = poisson.solve(g, rhs)
    floor = np.max(np.abs(rhs - op.lap_c(g, ref)))
    assert np.max(np.abs(rhs - op.lap_c(g, got))) < 3.0 * floor
    assert rel(got, ref) < 1e-11
    case.ctx.close()
