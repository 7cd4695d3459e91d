"""Order of accuracy of the whole oracle step (paper Sec. 4.2: the error of
the bulk flow and of the no-slip condition at an immersed plane decays as
O(N^-2)).

Adapted setup: a channel with walls at y = +-1 split by a full-span immersed
plane at the off-node height y0 = -1/2 + 0.37 Delta; a pressure gradient
drives plane Poiseuille flow on both sides (the closed form of Sec. 4.2 on
the upper side, u_e = (y - y0)(1 - y) for -dP/dx = 2/Re, and its mirror
below).  The flow is invariant in x and z, so a few cells of size Delta
(12 x 12, so that each triangle's inflated box fits the periodic box)
suffice horizontally.  Re = 1 and a convective CFL of 1/2 reach the steady
state of the discrete scheme in a few hundred steps (the profile and its
error do not depend on Re once -dP/dx = 2/Re).  The mass correction q plays no role here
(D u_hat = 0 for a parallel flow), so this pins the forcing, the viscous
operator and the time integration, not the splitting-error reduction: at
the steady state phi = 0, the projection leaves the forcing nodes untouched
and the no-slip error is round-off (checked), while the bulk error must fall
at second order.
"""
import numpy as np
import pytest

import workloads
from oracle import diagnostics
from oracle.grid import Grid
from oracle.step import step


def _steady_error(N, re=1.0, t_end=7.0):
    d = 2.0 / N
    dt = 0.5 * d
    max_steps = int(t_end / dt)
    g = Grid(12, N, 12, 12 * d, 12 * d, workloads.uniform_faces(N))
    y0 = -0.5 + 0.37 * d
    P, T = workloads.plate_mesh(g.lx, g.lz, 6, 6)
    P = P + np.array([g.lx / 2, y0, g.lz / 2])
    vel = np.zeros_like(P)

    def exact(y):
        return np.where(y > y0, (y - y0) * (1 - y), (y + 1) * (y0 - y))

    u = np.broadcast_to(exact(g.yc)[:, None, None], g.shape).copy()
    v = np.zeros(g.comp_shape(1))
    w = np.zeros(g.shape)
    p = np.zeros(g.shape)
    fext = (2.0 / re, 0.0, 0.0)
    for _ in range(max_steps):
        (u2, v, w), p, _, tags = step(g, (u, v, w), p, (P, vel, T), dt, re, fext)
        change = np.max(np.abs(u2 - u))
        u = u2
        if change < 1e-14:
            break
    upper = (g.yc > y0 + 2 * d)
    bulk = np.mean(np.abs(u[upper] - exact(g.yc)[upper, None, None]))
    eps, _ = diagnostics.noslip_error(g, (u, v, w), tags, P, vel, T)
    return bulk, eps, change


@pytest.mark.slow
def test_second_order_bulk_error_and_exact_noslip():
    Ns = (24, 48, 96)
    res = [_steady_error(N) for N in Ns]
    for r in res:
        assert r[2] < 1e-13            # reached the discrete steady state
        assert r[1] < 1e-14            # no splitting error at phi = 0
    bulk = np.array([r[0] for r in res])
    sb = np.polyfit(np.log(Ns), np.log(bulk), 1)[0]
    assert sb <= -1.8, (bulk, sb)
