"""Predictor on the fluid nodes (paper Eq. NS_prov, Sec. 2).

    (u_hat - u^s)/dt = gamma H^s + rho H^{s-1} - alpha G p^s
                       + alpha/(2 Re) L (u_hat + u^s)          on fluid nodes

written in delta form, du = u_hat - u^s:

    (I - beta L) du = R,  beta = alpha dt / (2 Re),
    R = dt [gamma H^s + rho H^{s-1} - alpha (G p^s - f) + (alpha/Re) L u^s],

with f the constant driving pressure gradient (a volume force of Eq. ns1,
integrated like the pressure gradient).  L is approximately factorised into
three one-dimensional operators (Sec. 2, "approximate factorization of L,
yielding three tridiagonal systems"):

    (I - beta L_x)(I - beta L_z)(I - beta L_y) du = R,

solved as the three sweeps x, z, y (reading: delta form, that sweep order).
Every forcing node is an identity row in all three sweeps, so du = 0 there and
u_hat keeps the IB value (Sec. 3.1 and Fig. 3: the stencil never crosses the
interface).  x and z are periodic (cyclic systems); y has Dirichlet walls.
"""
from __future__ import annotations

import numpy as np

from . import operators as op
from .linsolve import cyclic, thomas


def explicit_rhs(g, fields, p, hprev, masks, gamma, rho, alpha, dt, re, fext, kappa=None):
    """R of the delta form at every node; 0 on the forcing nodes and on the
    v wall planes.  Returns (R, H) with H = H(u^s) for reuse by a later
    sub-stage.  The volume force of component c is fext[c] (a constant or an
    array on the component's lattice) plus kappa[c] * u_c^s when kappa[c] is
    given (a force linear in the component itself, evaluated explicitly like
    the constant part: Sec. 4.2 and 4.3 add such forces to Eq. NS_prov)."""
    u, v, w = fields
    H = op.conv(g, u, v, w)
    G = op.gradient(g, p)
    Lu = (op.lap_cc(g, u), op.lap_v(g, v), op.lap_cc(g, w))
    R = []
    for c in range(3):
        f = fext[c]
        if kappa is not None and kappa[c] is not None:
            f = f + kappa[c] * fields[c]
        r = gamma * H[c] - alpha * (G[c] - f) + (alpha / re) * Lu[c]
        if rho != 0.0:
            r = r + rho * hprev[c]
        r = dt * r
        if c == 1:
            r[0] = 0.0
            r[g.ny] = 0.0
        r[masks[c]] = 0.0
        R.append(r)
    return R, H


def _sweep_periodic(d, mask, r, axis):
    """(I - beta L_1d) x = d along a periodic axis with r = beta/h^2;
    identity rows where mask."""
    dm = np.moveaxis(d, axis, 0)
    mm = np.moveaxis(mask, axis, 0)
    a = np.where(mm, 0.0, -r)
    c = np.where(mm, 0.0, -r)
    b = np.where(mm, 1.0, 1.0 + 2.0 * r)
    x = cyclic(a, b, c, np.where(mm, 0.0, dm))
    return np.moveaxis(x, 0, axis)


def _sweep_y(g, comp, d, mask, beta):
    """(I - beta L_y) x = d with the wall values fixed (x = 0 at the walls);
    identity rows where mask.  For v only the interior planes are unknowns."""
    if comp == 1:
        lo = 1.0 / (g.dy[:-1] * g.dyc[1:g.ny])      # rows j = 1..ny-1
        hi = 1.0 / (g.dy[1:] * g.dyc[1:g.ny])
        dd, mm = d[1:g.ny], mask[1:g.ny]
    else:
        lo = 1.0 / (g.dyc[:-1] * g.dy)               # rows j = 0..ny-1
        hi = 1.0 / (g.dyc[1:] * g.dy)
        dd, mm = d, mask
    lo, hi = lo[:, None, None], hi[:, None, None]
    a = np.where(mm, 0.0, -beta * lo)
    c = np.where(mm, 0.0, -beta * hi)
    b = np.where(mm, 1.0, 1.0 + beta * (lo + hi))
    x = thomas(a, b, c, np.where(mm, 0.0, dd))
    if comp == 1:
        out = np.zeros_like(d)
        out[1:g.ny] = x
        return out
    return x


def factored_solve(g, R, masks, alpha, dt, re):
    """Three sweeps of the approximate factorisation; returns du per
    component."""
    beta = alpha * dt / (2.0 * re)
    rx = beta / (g.dx * g.dx)
    rz = beta / (g.dz * g.dz)
    out = []
    for c in range(3):
        w1 = _sweep_periodic(R[c], masks[c], rx, axis=2)
        w2 = _sweep_periodic(w1, masks[c], rz, axis=1)
        out.append(_sweep_y(g, c, w2, masks[c], beta))
    return out


def predictor(g, fields, p, hprev, masks, gamma, rho, alpha, dt, re, fext, kappa=None):
    """u_hat = u^s + du on every node (du = 0 on the forcing nodes and
    walls).  Returns ((u_hat, v_hat, w_hat), H(u^s))."""
    R, H = explicit_rhs(g, fields, p, hprev, masks, gamma, rho, alpha, dt, re, fext, kappa)
    du = factored_solve(g, R, masks, alpha, dt, re)
    return tuple(fields[c] + du[c] for c in range(3)), H


def apply_factored(g, du, masks, alpha, dt, re):
    """The factored operator (I - bL_x)(I - bL_z)(I - bL_y) applied to du with
    identity rows on the forcing nodes (used by tests as a residual check)."""
    beta = alpha * dt / (2.0 * re)
    out = []
    for c in range(3):
        x = du[c]
        # y
        if c == 1:
            z = np.zeros((1,) + x.shape[1:])
            fl = (x[1:] - x[:-1]) / g.dy[:, None, None]
            ly = np.zeros_like(x)
            ly[1:g.ny] = (fl[1:] - fl[:-1]) / g.dyc[1:g.ny, None, None]
        else:
            z = np.zeros((1,) + x.shape[1:])
            xe = np.concatenate((z, x, z))
            fl = (xe[1:] - xe[:-1]) / g.dyc[:, None, None]
            ly = (fl[1:] - fl[:-1]) / g.dy[:, None, None]
        y1 = np.where(masks[c], x, x - beta * ly)
        lz = ((op.zp(y1) - y1) - (y1 - op.zm(y1))) / (g.dz * g.dz)
        y2 = np.where(masks[c], y1, y1 - beta * lz)
        lx = ((op.xp(y2) - y2) - (y2 - op.xm(y2))) / (g.dx * g.dx)
        y3 = np.where(masks[c], y2, y2 - beta * lx)
        if c == 1:
            y3[0] = 0.0
            y3[g.ny] = 0.0
        out.append(y3)
    return out
