"""Volume forces (the forces that paper Sec. 4.2 and 4.3 add to Eq.
NS_prov) through the C-ABI against the oracle, on the immersed-plane
channel of those sections: walls at y = -1/4 and 2, a full-span
zero-thickness plane at y0 = 0.37 Delta, and

* Sec. 4.2: a wall-normal vortex forcing F_y = A sin(pi (y + 1/4)/(1/4))
  cos(pi x) below the plane and a driving gradient above it, RK2 + CN;
* Sec. 4.3: the relaxation F_y = -5 (v - 1) below the plane (f0 = 5,
  kappa = -5) and a driving force 1 along x above it, AB2 + CN.

Bar: whole steps within 1e-10 of the oracle in FP64, 1e-6 in the mixed
form."""
import numpy as np
import pytest
import torch

import workloads
from gpu_harness import Case, DEV, n, rel, t
from oracle import step as ostep

pytestmark = pytest.mark.gpu


def _plane_channel(N=32, nz=12, re=100.0, scheme="rk2"):
    """Walls at y = -1/4 and 2, uniform spacing 2/N (the probe of the
    forcing, two cell diagonals, stays inside the lower region), a full-span
    plane at y0 = 0.37 Delta, a 0.05 perturbation on every unknown."""
    d = 2.0 / N
    lo = -0.25
    ny = int(round((2.0 - lo) / d))
    yf = workloads.uniform_faces(ny, lo, 2.0)
    lx, lz = N * d, nz * d
    y0 = 0.37 * d
    P, T = workloads.plate_mesh(lx, lz, N // 4, nz // 2)
    centre = (lx / 2, y0, lz / 2)
    body = workloads.Body("rigid", P, T,
                          lambda tt: workloads.sphere_translation(tt, centre, (0.0, 0.0, 0.0)))
    wl = workloads.Workload("plane_vf", N, ny, nz, lx, lz, yf, re, 0.25 * d, 3, 1.0, 0.05, 13, 0.0,
                            [body])
    wl.scheme = scheme
    return wl


def _lattice(g, c):
    ox, oz = {0: (0.0, 0.5), 1: (0.5, 0.5), 2: (0.5, 0.0)}[c]
    ys = g.yf if c == 1 else g.yc
    x = (np.arange(g.nx) + ox) * g.dx
    z = (np.arange(g.nz) + oz) * g.dz
    return np.meshgrid(ys, z, x, indexing="ij")


def _forces(g, case_name):
    """(f0, kappa) per component as the two sections set them."""
    f0 = [np.zeros(g.comp_shape(c)) for c in range(3)]
    kap = [None, None, None]
    Yu, _, _ = _lattice(g, 0)
    Yv, _, Xv = _lattice(g, 1)
    below = (Yv > -0.25) & (Yv < 0.0)
    f0[0][Yu > 0.0] = 1.0                      # driving force above the plane
    if case_name == "vortex":
        f0[1][below] = 20.0 * (np.sin(np.pi * (Yv - (-0.25)) / 0.25) * np.cos(np.pi * Xv))[below]
    else:
        f0[1][below] = 5.0
        kap[1] = np.where(below, -5.0, 0.0)
    return f0, kap


@pytest.mark.parametrize("case_name,scheme", [("vortex", "rk2"), ("relax", "ab2")])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_volume_force_steps_against_oracle(case_name, scheme, precision):
    wl = _plane_channel(scheme=scheme)
    case = Case(wl, precision=precision, scheme=scheme)
    g = case.g
    f0, kap = _forces(g, case_name)
    for c in range(3):
        case.ibm.ibm_set_volume_force(case.ctx, c, t(f0[c]),
                                      t(kap[c]) if kap[c] is not None else None)
    pdt = case.ctx.pdtype
    f = list(wl.fields())
    p = np.zeros(g.shape)
    H, hdev, start = None, None, 0
    if scheme == "ab2":
        # AB+CN starts with an explicit Euler step on H: taken by the oracle,
        # then both sides continue from its state and H
        _, surf = case.bodies_at(0.0)
        f, p, H, _ = ostep.step(g, f, p, surf, wl.dt, wl.re, tuple(f0), scheme, kappa=kap)
        hdev = [t(a, pdt) for a in H]
        start = 1
    d = [t(a) for a in f]
    pd = t(p, pdt)
    for s in range(start, start + 3):
        bodies, surf = case.bodies_at(s * wl.dt)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt, h=hdev)
        f, p, H, tags = ostep.step(g, f, p, surf, wl.dt, wl.re, tuple(f0), scheme, H,
                                   kappa=kap)
    assert case.ibm.ibm_check(case.ctx) == 0
    bar = 1e-10 if precision == "fp64" else 1e-6
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < bar, c
    # the fluid below the plane moves (the vortex forcing drives it; the
    # relaxation acts on the perturbation)
    assert np.max(np.abs(f[1][g.yf < 0.0])) > 1e-3
    case.ctx.close()
