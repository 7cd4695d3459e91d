"""No-slip error of the oracle with and without the consistent mass correction
(paper Sec. 3.2, Eqs. mod_div, q_F, elliptic_mod; Sec. 4.2 for the setup;
Sec. 4.4 for the error measure).

Adapted from the Poiseuille flow over an immersed plane of Sec. 4.2: a
channel with walls at y = -1/2 and y = 2, split by a full-span zero-thickness
plane at the off-node height y0 = 0.37 Delta.  Above the plane a pressure
gradient drives plane Poiseuille flow, u_e = (Re G / 2)(y - y0)(2 - y); below
it a wall-normal volume force F_y = A sin(pi (y + 1/2)/(1/2)) cos(pi x)
(zero outside -1/2 < y < 0) drives a row of steady vortices, so that the flow
below the plane crosses the forcing layer and the cut cells C_B carry a
nonzero divergence.  Re = 1 (the scheme's diffusion reaches the discrete
steady state in a few hundred steps), uniform spacing Delta = 2/N in x and y,
12 cells of Delta in z (the flow is invariant in z).

At the steady state:
  * with q the projection leaves the forcing nodes as the IB step set them:
    the no-slip error of Sec. 4.4 (the flow extrapolated to the wall with the
    forcing interpolator, minus the wall velocity) is round-off, and the bulk
    error above the plane falls at second order;
  * with the standard projection (q = 0, Eq. elliptic) the correction of the
    divergence of the cut cells moves the forcing nodes every step: the
    no-slip error stays at the 1e-4 level and does not fall with N over this
    range (the splitting error that Sec. 4.2 attributes to the unmodified
    elliptic equation).
"""
import numpy as np
import pytest

import workloads
from oracle import diagnostics
from oracle.grid import Grid
from oracle.step import step


def _steady(N, use_q, re=1.0, amp=20.0, lo=-0.5, nz=12, tol=1e-12, tmax=40.0):
    d = 2.0 / N
    ny = int(round((2.0 - lo) / d))
    g = Grid(N, ny, nz, 2.0, nz * d, workloads.uniform_faces(ny, lo, 2.0))
    y0 = 0.37 * d
    P, T = workloads.plate_mesh(g.lx, g.lz, N // 4, nz // 2)
    P = P + np.array([g.lx / 2, y0, g.lz / 2])
    vel = np.zeros_like(P)
    G = 2.0 / re                              # -dP/dx

    def exact(y):
        return np.where(y > y0, 0.5 * re * G * (y - y0) * (2.0 - y), 0.0)

    u = np.broadcast_to(exact(g.yc)[:, None, None], g.shape).copy()
    v = np.zeros(g.comp_shape(1))
    w = np.zeros(g.shape)
    p = np.zeros(g.shape)
    xv = (np.arange(N) + 0.5) * d            # x of the v nodes
    fy = np.zeros(g.comp_shape(1))
    below = (g.yf > lo) & (g.yf < 0.0)
    fy[below] = ((amp * np.sin(np.pi * (g.yf[below] - lo) / (-lo)))[:, None, None]
                 * np.cos(np.pi * xv)[None, None, :])
    dt = 0.5 * d
    change = np.inf
    for _ in range(int(tmax / dt)):
        (u2, v, w), p, _, tags = step(g, (u, v, w), p, (P, vel, T), dt, re, (G, fy, 0.0),
                                      use_q=use_q)
        change = np.max(np.abs(u2 - u))
        u = u2
        if change < tol:
            break
    above = g.yc > y0 + 1.5 * d
    bulk = np.mean(np.abs(u[above] - exact(g.yc)[above, None, None]))
    eps, _ = diagnostics.noslip_error(g, (u, v, w), tags, P, vel, T)
    return bulk, eps, change, np.max(np.abs(v))


@pytest.mark.slow
def test_mass_correction_removes_the_noslip_splitting_error():
    Ns = (16, 24, 32)
    with_q = [_steady(N, True) for N in Ns]
    for bulk, eps, change, vmax in with_q:
        assert change < 1e-12                 # the discrete steady state
        assert vmax > 1e-2                    # the vortices cross the plane's layer
        assert eps < 1e-13                    # no splitting error with q
    bulk = np.array([r[0] for r in with_q])
    slope = np.polyfit(np.log(Ns), np.log(bulk), 1)[0]
    assert slope <= -1.8, (bulk, slope)
    without_q = [_steady(N, False) for N in (16, 32)]
    for bulk_n, eps_n, change, _ in without_q:
        assert change < 1e-12
        assert eps_n > 1e-5                   # the standard projection moves the forcing nodes
    # and that error does not fall with the grid (first order at best)
    assert without_q[1][1] > 0.5 * without_q[0][1], [r[1] for r in without_q]
