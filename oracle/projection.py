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


def mass_correction(g, fields, cb, alpha, dt, use_q=True):
    """Returns (rhs of Eq. elliptic_mod, q_F, D u_hat).  With use_q=False the
    standard right-hand side D u_hat/(alpha dt) of Eq. elliptic is returned
    (the uncorrected scheme, used by the accuracy tests)."""
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
