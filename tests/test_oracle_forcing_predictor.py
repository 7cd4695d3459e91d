"""Pins of the oracle's IB forcing (Eqs. probe, new_IB), predictor (Eq.
NS_prov with approximate factorisation) and mass correction / projection
(Eqs. mod_div .. q_F, projection), against closed forms, brute force and
exact invariants.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import forcing, geometry, operators as op, poisson, predictor, projection
from oracle.grid import Grid
from oracle.linsolve import thomas
from oracle.step import compute_tags, masks_of, step


def _grid(nx=24, ny=20, nz=16, stretched=True):
    yf = workloads.tanh_faces(ny, 1.2) if stretched else workloads.uniform_faces(ny)
    return Grid(nx, ny, nz, 2 * np.pi, np.pi, yf)


def _plane(g, y0, nq=6):
    P, T = workloads.plate_mesh(g.lx, g.lz, nq, nq)
    return P + np.array([g.lx / 2, y0, g.lz / 2]), T


# ------------------------------------------------------------- forcing
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_forcing_exact_for_linear_shear(comp):
    """u = a (y - y0) with a wall plane at y0 moving at U = 0: the linear
    reconstruction along the normal probe and trilinear interpolation are
    exact for linear fields, so u^f = a (y^f - y0) to round-off."""
    g = _grid()
    y0 = 0.113
    V, F = _plane(g, y0)
    vel = np.zeros_like(V)
    idx, tri = geometry.tag(g, comp, V, F)
    ext = g.y_nodes_ext(comp)
    if comp == 1:
        yn = g.yf
    else:
        yn = g.yc
    a = 1.7
    field = np.broadcast_to((a * (yn - y0))[:, None, None], g.comp_shape(comp)).copy()
    if comp == 1:
        field[0] = field[-1] = 0.0   # unused: the probes stay away from walls
    uf = forcing.forced_values(g, comp, idx, tri, V, vel, F, field)
    jj = idx // (g.nx * g.nz)
    assert np.allclose(uf, a * (yn[jj] - y0), rtol=0, atol=1e-13)
    del ext


def test_forcing_on_surface_node_takes_wall_velocity():
    """Reading |N| = 0: the node takes U bit-for-bit."""
    g = _grid()
    jf = 10
    V, F = _plane(g, g.yf[jf])
    vel = np.zeros_like(V)
    vel[:, 1] = 0.37
    idx, tri = geometry.tag(g, 1, V, F)
    rng = np.random.default_rng(3)
    field = rng.standard_normal(g.comp_shape(1))
    uf = forcing.forced_values(g, 1, idx, tri, V, vel, F, field)
    # weight a = |N|/h = 0 (or ~1e-16 where the closest point carries
    # rounding in its in-plane coordinates): the result is the barycentric
    # wall velocity and does not depend on the flow field
    assert np.allclose(uf, 0.37, rtol=1e-13, atol=0)
    uf2 = forcing.forced_values(g, 1, idx, tri, V, vel, F, 1e3 * field)
    assert np.max(np.abs(uf - uf2)) < 1e-15 * np.max(np.abs(1e3 * field))


def test_jacobi_equals_sequential_on_flat_plate():
    """On a full-span flat plate no probe stencil contains a forcing node, so
    computing all u^f first (Jacobi) equals writing each one as soon as it is
    computed (the paper's on-line forcing), bit for bit."""
    g = _grid()
    V, F = _plane(g, -0.21)
    vel = np.zeros_like(V)
    vel[:, 0] = 0.4
    rng = np.random.default_rng(5)
    for comp in range(3):
        idx, tri = geometry.tag(g, comp, V, F)
        field = rng.standard_normal(g.comp_shape(comp))
        jac = forcing.forced_values(g, comp, idx, tri, V, vel, F, field)
        seq = field.copy().reshape(-1)
        for n in range(len(idx)):
            val = forcing.forced_values(g, comp, idx[n:n + 1], tri[n:n + 1], V, vel, F,
                                        seq.reshape(field.shape))
            seq[idx[n]] = val[0]
        assert np.array_equal(seq[idx], jac)


def test_probe_length_uniform_grid():
    """h = 2 sqrt(3) Delta on a uniform grid (Sec. 3.1)."""
    n = 16
    g = Grid(n, n, n, 2.0, 2.0, workloads.uniform_faces(n))
    h = forcing.probe_length(g, 0, 5)
    assert np.isclose(h, 2 * np.sqrt(3) * (2.0 / n), rtol=1e-15)


# ----------------------------------------------------------- predictor
def test_af_closed_form_stokes_mode():
    """No body, p = 0, H off: u = sin(2 pi x/Lx) sin(2 pi z/Lz) sin(pi q (j+1/2)/ny)
    is an eigenvector of every 1-D factor; then
    du = dt (alpha/Re) lambda u / [(1-b lx)(1-b lz)(1-b ly)]."""
    g = _grid(stretched=False)
    x = np.arange(g.nx) * g.dx
    z = (np.arange(g.nz) + 0.5) * g.dz
    q = 3
    u = (np.sin(np.pi * q * (np.arange(g.ny) + 0.5) / g.ny)[:, None, None]
         * np.sin(2 * np.pi * z / g.lz)[None, :, None] * np.sin(2 * np.pi * x / g.lx)[None, None, :])
    lx = -(4 / g.dx ** 2) * np.sin(np.pi / g.nx) ** 2
    lz = -(4 / g.dz ** 2) * np.sin(np.pi / g.nz) ** 2
    ly = -(4 / g.dy[0] ** 2) * np.sin(np.pi * q / (2 * g.ny)) ** 2
    dt, re, alpha = 0.05, 10.0, 0.5
    beta = alpha * dt / (2 * re)
    R = dt * (alpha / re) * op.lap_cc(g, u)
    masks = [np.zeros(g.comp_shape(c), bool) for c in range(3)]
    zeros = np.zeros(g.comp_shape(1))
    du = predictor.factored_solve(g, [R, zeros, R], masks, alpha, dt, re)
    expect = dt * (alpha / re) * (lx + ly + lz) * u / ((1 - beta * lx) * (1 - beta * lz) * (1 - beta * ly))
    assert np.allclose(du[0], expect, rtol=0, atol=1e-13 * np.abs(expect).max())


def test_af_sweeps_invert_factored_operator_with_identity_rows(rng):
    """Applying the factored operator (stencil form) to the swept solution
    returns R; the forcing nodes stay exactly 0."""
    g = _grid()
    V, F = workloads.icosphere(1)
    V = V * 0.6 + np.array([3.0, 0.1, 1.5])
    tags = compute_tags(g, V, F)
    masks = masks_of(g, tags)
    R = [rng.standard_normal(g.comp_shape(c)) for c in range(3)]
    R[1][0] = R[1][-1] = 0.0
    for c in range(3):
        R[c][masks[c]] = 0.0
    dt, re, alpha = 0.3, 5.0, 0.5
    du = predictor.factored_solve(g, R, masks, alpha, dt, re)
    back = predictor.apply_factored(g, du, masks, alpha, dt, re)
    for c in range(3):
        assert np.allclose(back[c], R[c], atol=1e-12)
        assert np.all(du[c][masks[c]] == 0.0)


def test_steady_discrete_poiseuille_is_a_fixed_point():
    """No body: the discrete steady profile of nu L_y u = dP/dx (u = 0 at the
    walls, H = 0 for a parallel flow, D u = 0) is left unchanged by a full
    RK2 step; this pins the sign and the time weight of the driving force."""
    g = _grid(nx=8, ny=24, nz=6)
    re, dpdx = 100.0, -2.0 / 100.0
    ny = g.ny
    lo = 1.0 / (g.dyc[:-1] * g.dy)
    hi = 1.0 / (g.dyc[1:] * g.dy)
    a = np.zeros(ny); a[1:] = lo[1:]
    c = np.zeros(ny); c[:-1] = hi[:-1]
    b = -(lo + hi)
    prof = thomas(a, b, c, np.full(ny, re * dpdx))
    u = np.broadcast_to(prof[:, None, None], g.shape).copy()
    v = np.zeros(g.comp_shape(1))
    w = np.zeros(g.shape)
    p = np.zeros(g.shape)
    empty = (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int64))
    (u2, v2, w2), p2, _, _ = step(g, (u, v, w), p, empty, 0.01, re, (-dpdx, 0, 0))
    assert np.max(np.abs(u2 - u)) < 1e-13
    assert np.max(np.abs(v2)) < 1e-13 and np.max(np.abs(w2)) < 1e-13


# ------------------------------------------------------ mass correction
def _body_case(rng):
    g = _grid()
    V, F = workloads.icosphere(2)
    V = V * 0.7 + np.array([3.0, 0.05, 1.5])
    tags = compute_tags(g, V, F)
    f = [rng.standard_normal(g.comp_shape(c)) for c in range(3)]
    f[1][0] = f[1][-1] = 0.0
    return g, tags, f


def test_mass_correction_invariants(rng):
    """Eq. constraint_q: sum (D u_hat - q) dV = 0; the RHS vanishes on C_B
    (Eq. q_boundary); q_F is the minimal-L2 solution of the constraint
    (App. B), checked against the least-squares minimum-norm solution."""
    g, tags, f = _body_case(rng)
    alpha, dt = 0.5, 1e-3
    rhs, qF, D = projection.mass_correction(g, f, tags.cb, alpha, dt)
    dV = g.cell_volume()
    mB = projection.cell_mask(g, tags.cb)
    assert len(tags.cb) > 0
    assert np.all(rhs[mB] == 0.0)
    tot = np.sum(rhs * alpha * dt * dV)
    assert abs(tot) <= 1e-12 * np.sum(np.abs(D) * dV)
    # minimal weighted-L2 q_F: min sum q^2 dV s.t. sum_F q dV = -sum_B D dV
    s = np.sqrt(dV[~mB])
    A = np.sum(D[mB] * dV[mB])
    y = np.linalg.lstsq(s[None, :], np.array([-A]), rcond=None)[0]
    qmin = y / s
    assert np.allclose(qmin, qF, rtol=1e-10)


def test_projection_meets_modified_divergence(rng):
    """After the projection D u^{s+1} = q to round-off (Eq. mod_div) and the
    total divergence vanishes (App. A)."""
    g, tags, f = _body_case(rng)
    alpha, dt, re = 0.5, 1e-3, 100.0
    rhs, qF, _ = projection.mass_correction(g, f, tags.cb, alpha, dt)
    phi = poisson.solve(g, rhs)
    (u, v, w), _ = projection.project(g, f, np.zeros(g.shape), phi, alpha, dt, re)
    D = op.divergence(g, u, v, w)
    mB = projection.cell_mask(g, tags.cb)
    Dq = np.where(mB, D - op.divergence(g, *f), D - qF)
    assert np.max(np.abs(Dq)) < 1e-10
    assert abs(np.sum(D * g.cell_volume())) < 1e-12


def test_uncorrected_projection_is_standard(rng):
    """Without q (standard scheme, Eq. elliptic) D u^{s+1} = 0 everywhere."""
    g, tags, f = _body_case(rng)
    rhs, qF, _ = projection.mass_correction(g, f, tags.cb, 0.5, 1e-3, use_q=False)
    phi = poisson.solve(g, rhs)
    (u, v, w), _ = projection.project(g, f, np.zeros(g.shape), phi, 0.5, 1e-3, 100.0)
    assert qF == 0.0
    assert np.max(np.abs(op.divergence(g, u, v, w))) < 1e-10
