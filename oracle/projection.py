"""Consistent mass correction, projection and pressure update.

Mass correction (paper Sec. 3.2): the divergence constraint is modified to
D u^{s+1} = q (Eq. mod_div) with q_B = D u_hat on the boundary cells C_B
(Eq. q_boundary) and a uniform q_F on the fluid cells C_F,

    q_F = -(1/|C_F|) sum_{C_B} D u_hat dV      (Eq. q_F),

the minimal-L2 solution of the global constraint (Eq. constraint_q, App. B);
the pseudo-pressure then solves L_c phi = (D u_hat - q)/(alpha dt)
(Eq. elliptic_mod), whose right-hand side vanishes on C_B.

Projection (Eq. projection) and pressure update (Eq. update_pressure):
    u^{s+1} = u_hat - alpha dt G phi,
    p^{s+1} = p^s + phi - alpha dt/(2 Re) L_c phi.
"""
from __future__ import annotations

import numpy as np

from . import operators as op


def cell_mask(g, cb):
    m = np.zeros(g.cells, bool)
    m[cb] = True
    return m.reshape(g.shape)


def mass_correction(g, fields, cb, alpha, dt, use_q=True, p=None):
    """Returns (rhs of Eq. elliptic_mod, q_F, D u_hat).  With use_q=False the
    standard right-hand side D u_hat/(alpha dt) of Eq. elliptic is returned
    (the uncorrected scheme, used by the accuracy tests); with
    use_q="energy" the shape of mass_correction_energy (p required), and the
    second value is its pair (c0, c1)."""
    if use_q == "energy":
        rhs, _, D, coef = mass_correction_energy(g, fields, p, cb, alpha, dt)
        return rhs, coef, D
    D = op.divergence(g, *fields)
    if not use_q or len(cb) == 0:
        return D / (alpha * dt), 0.0, D
    dV = g.cell_volume()
    mB = cell_mask(g, cb)
    A = float(np.sum(D[mB] * dV[mB]))
    vol_f = float(np.sum(dV[~mB]))
    qF = -A / vol_f
    rhs = np.where(mB, 0.0, (D - qF) / (alpha * dt))
    return rhs, qF, D


def mass_correction_energy(g, fields, p, cb, alpha, dt):
    """The mass- and energy-conserving shape of q_F (App. B, Eq. unif_shape;
    the formulas are followed, the equation labels of the appendix are
    swapped).  With r = p - e (p the pressure of the sub-stage, e the
    cell-centred kinetic energy of u_hat):

        q_F^k = (-A S2 + B S1)/C + (A S1 - B S0)/C r^k   on C_F,
        S_i = sum_{C_F} r^i dV,  A = sum_{C_B} D u_hat dV,
        B = sum_{C_B} r D u_hat dV,  C = S0 S2 - S1^2,

    the minimal-L2 q_F that satisfies both the mass constraint
    (Eq. constraint_q) and sum_{C_F} r q dV + sum_{C_B} r D u_hat dV = 0.
    C >= 0 (Cauchy-Schwarz) and vanishes only when r is constant on C_F,
    where the two constraints coincide: then the uniform shape (Eq. q_F) is
    used.  Returns (rhs of Eq. elliptic_mod, q on every cell (q_B on C_B),
    D u_hat, (c0, c1)) with q_F = c0 + c1 r."""
    D = op.divergence(g, *fields)
    if len(cb) == 0:
        return D / (alpha * dt), np.zeros(g.shape), D, (0.0, 0.0)
    dV = g.cell_volume()
    mB = cell_mask(g, cb)
    r = p - op.kinetic_energy(g, *fields)
    S0 = float(np.sum(dV[~mB]))
    S1 = float(np.sum(r[~mB] * dV[~mB]))
    S2 = float(np.sum(r[~mB] * r[~mB] * dV[~mB]))
    A = float(np.sum(D[mB] * dV[mB]))
    B = float(np.sum(r[mB] * D[mB] * dV[mB]))
    C = S0 * S2 - S1 * S1
    if C <= 1e-14 * S0 * S2:
        c0, c1 = -A / S0, 0.0
    else:
        c0, c1 = (-A * S2 + B * S1) / C, (A * S1 - B * S0) / C
    q = np.where(mB, D, c0 + c1 * r)
    rhs = np.where(mB, 0.0, (D - q) / (alpha * dt))
    return rhs, q, D, (c0, c1)


def project(g, fields, p, phi, alpha, dt, re):
    """Eqs. projection and update_pressure; the v wall planes stay 0."""
    gu, gv, gw = op.gradient(g, phi)
    u = fields[0] - (alpha * dt) * gu
    v = fields[1] - (alpha * dt) * gv
    w = fields[2] - (alpha * dt) * gw
    v[0] = 0.0
    v[g.ny] = 0.0
    pn = p + phi - (alpha * dt / (2.0 * re)) * op.lap_c(g, phi)
    return (u, v, w), pn
