"""Pins of the mass- and energy-conserving shape of q_F (App. B, Eq.
unif_shape) in the oracle, against facts that do not come from its formula:
the two constraints it must satisfy, the minimum-norm solution of those
constraints from a least-squares solve, the degenerate case where the two
constraints coincide, and the discrete energy identity of the cell-centred
kinetic energy."""
import numpy as np

from oracle import operators as op, poisson, projection
from oracle.grid import Grid
from oracle.step import compute_tags
import workloads

from test_oracle_forcing_predictor import _body_case


def test_kinetic_energy_identity(rng):
    """On a uniform grid sum over cells of e dV = 1/2 sum over faces of
    u^2 dV (every face shared by two cells, the v wall faces hold 0), and a
    uniform velocity gives e = |U|^2/2 away from the walls."""
    g = Grid(12, 10, 8, 2.0, 1.5, workloads.uniform_faces(10))
    u = rng.standard_normal(g.shape)
    v = rng.standard_normal(g.comp_shape(1))
    v[0] = v[-1] = 0.0
    w = rng.standard_normal(g.shape)
    e = op.kinetic_energy(g, u, v, w)
    dV = g.cell_volume()
    assert np.isclose(np.sum(e * dV), 0.5 * dV[0, 0, 0] * (np.sum(u * u) + np.sum(v * v) + np.sum(w * w)),
                      rtol=1e-13)
    U = (0.3, -1.2, 0.7)
    e = op.kinetic_energy(g, np.full(g.shape, U[0]), np.full(g.comp_shape(1), U[1]),
                          np.full(g.shape, U[2]))
    assert np.allclose(e, 0.5 * sum(x * x for x in U), rtol=1e-15)


def _energy_case(rng):
    g, tags, f = _body_case(rng)
    p = rng.standard_normal(g.shape)
    return g, tags, f, p


def test_energy_shape_meets_both_constraints(rng):
    """sum_F q dV + sum_B D u dV = 0 (mass) and sum_F r q dV + sum_B r D u dV
    = 0 (energy in the inviscid limit), r = p - e, to round-off."""
    g, tags, f, p = _energy_case(rng)
    rhs, q, D, (c0, c1) = projection.mass_correction_energy(g, f, p, tags.cb, 0.5, 1e-3)
    dV = g.cell_volume()
    mB = projection.cell_mask(g, tags.cb)
    r = p - op.kinetic_energy(g, *f)
    assert len(tags.cb) > 0 and c1 != 0.0
    mass = np.sum(q[~mB] * dV[~mB]) + np.sum(D[mB] * dV[mB])
    energy = np.sum(r[~mB] * q[~mB] * dV[~mB]) + np.sum(r[mB] * D[mB] * dV[mB])
    scale = np.sum(np.abs(D[mB]) * dV[mB])
    assert abs(mass) <= 1e-12 * scale
    assert abs(energy) <= 1e-12 * scale * np.max(np.abs(r))
    assert np.all(rhs[mB] == 0.0)


def test_energy_shape_is_the_minimum_norm_solution(rng):
    """q_F minimises sum_F q^2 dV under the two constraints: the same as the
    least-squares minimum-norm solution of the weighted 2-row system."""
    g, tags, f, p = _energy_case(rng)
    _, q, D, _ = projection.mass_correction_energy(g, f, p, tags.cb, 0.5, 1e-3)
    dV = g.cell_volume()
    mB = projection.cell_mask(g, tags.cb)
    r = p - op.kinetic_energy(g, *f)
    s = np.sqrt(dV[~mB])
    M = np.stack([s, r[~mB] * s])               # constraints on y = s q
    b = -np.array([np.sum(D[mB] * dV[mB]), np.sum(r[mB] * D[mB] * dV[mB])])
    y = np.linalg.lstsq(M, b, rcond=None)[0]
    assert np.allclose(y / s, q[~mB], rtol=1e-9, atol=1e-12 * np.max(np.abs(q[~mB])))


def test_energy_shape_reduces_to_uniform_when_r_is_constant(rng):
    """With p - e constant on the fluid cells the two constraints coincide
    (C = 0) and the uniform q_F of Eq. q_F is the answer."""
    g, tags, f, _ = _energy_case(rng)
    p = op.kinetic_energy(g, *f) + 0.37
    _, q, _, (c0, c1) = projection.mass_correction_energy(g, f, p, tags.cb, 0.5, 1e-3)
    _, qF, _ = projection.mass_correction(g, f, tags.cb, 0.5, 1e-3)
    mB = projection.cell_mask(g, tags.cb)
    assert c1 == 0.0
    assert np.allclose(q[~mB], qF, rtol=1e-12)


def test_projection_with_energy_shape(rng):
    """After the projection D u^{s+1} = q cell by cell (the fluid cells carry
    the shaped q_F), so both constraints hold for the projected field."""
    g, tags, f, p = _energy_case(rng)
    alpha, dt = 0.5, 1e-3
    rhs, q, _, _ = projection.mass_correction_energy(g, f, p, tags.cb, alpha, dt)
    phi = poisson.solve(g, rhs)
    (u, v, w), _ = projection.project(g, f, p, phi, alpha, dt, 100.0)
    D = op.divergence(g, u, v, w)
    mB = projection.cell_mask(g, tags.cb)
    Dhat = op.divergence(g, *f)
    assert np.max(np.abs(np.where(mB, D - Dhat, D - q))) < 1e-10
    assert abs(np.sum(D * g.cell_volume())) < 1e-12
