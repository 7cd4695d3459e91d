"""Order of accuracy of the HIP time step against a closed form (paper
Sec. 4.2: the error of the bulk flow at an immersed plane decays as O(N^-2)
and the no-slip condition holds there).

The same adapted setup as the oracle's convergence test: walls at y = +-1, a
full-span immersed plane at the off-node height y0 = -1/2 + 0.37 Delta, plane
Poiseuille flow on both sides driven by -dP/dx = 2/Re (upper side
u_e = (y - y0)(1 - y), its mirror below), 12 x N x 12 cells of size
Delta = 2/N, Re = 1, convective CFL 1/2.  Here every step runs through
`ibm_step` on the GPU (tagging, forcing, predictor, mass correction, Poisson
solve, projection) until the discrete steady state; the no-slip error comes
from `ibm_noslip_error`.  The comparison is with the exact solution, not with
the oracle.
"""
import numpy as np
import pytest
import torch

import workloads
from gpu_harness import Case, DEV, n, t

pytestmark = pytest.mark.gpu


def _plane_workload(N, re=1.0):
    d = 2.0 / N
    lx = lz = 12 * d
    y0 = -0.5 + 0.37 * d
    P, T = workloads.plate_mesh(lx, lz, 6, 6)
    centre = (lx / 2, y0, lz / 2)
    body = workloads.Body("rigid", P, T,
                          lambda tt: workloads.sphere_translation(tt, centre, (0.0, 0.0, 0.0)))
    return workloads.Workload("plane", 12, N, 12, lx, lz, workloads.uniform_faces(N), re,
                              0.5 * d, 1, 1.0, 0.0, 0, -2.0 / re, [body]), y0


def _steady_error(N, t_end=7.0):
    wl, y0 = _plane_workload(N)
    case = Case(wl)
    g = case.g
    d = 2.0 / N

    def exact(y):
        return np.where(y > y0, (y - y0) * (1 - y), (y + 1) * (y0 - y))

    u = np.broadcast_to(exact(g.yc)[:, None, None], g.shape).copy()
    dev = [t(u), t(np.zeros(g.comp_shape(1))), t(np.zeros(g.shape))]
    pd = torch.zeros(g.cells, dtype=case.ctx.pdtype, device=DEV)
    change = np.inf
    steps = int(t_end / wl.dt)
    for s in range(steps):
        prev = dev[0].clone() if s % 10 == 9 else None
        bodies, _ = case.bodies_at(s * wl.dt)
        case.ibm.ibm_step(case.ctx, *dev, pd, bodies, wl.dt)
        if prev is not None:
            change = torch.max(torch.abs(dev[0] - prev)).item()
            if change < 1e-14:
                break
    assert case.ibm.ibm_check(case.ctx) == 0
    eps, _ = case.ibm.ibm_noslip_error(case.ctx, *dev)
    uh = n(dev[0], g.shape)
    upper = g.yc > y0 + 2 * d
    bulk = np.mean(np.abs(uh[upper] - exact(g.yc)[upper, None, None]))
    return bulk, eps, change


def test_second_order_bulk_error_and_exact_noslip():
    Ns = (24, 48, 96)
    res = [_steady_error(N) for N in Ns]
    for r in res:
        assert r[2] < 1e-13            # reached the discrete steady state
        assert r[1] < 1e-14            # no splitting error at phi = 0
    bulk = np.array([r[0] for r in res])
    slope = np.polyfit(np.log(Ns), np.log(bulk), 1)[0]
    assert slope <= -1.8, (bulk, slope)
