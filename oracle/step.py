"""One sub-stage and one time step of the scheme (paper Sec. 2 and Sec. 3).

Per sub-stage s (Sec. 2, Eqs. IB_step .. update_pressure; Sec. 3.2):
  1. IB step on the forcing nodes (Eq. IB_step / new_IB), from u^s and U^n;
  2. predictor on the fluid nodes (Eq. NS_prov, approximate factorisation);
  3. consistent mass correction and L_c phi = (D u_hat - q)/(alpha dt)
     (Eqs. mod_div .. q_F, elliptic_mod);
  4. projection and pressure update (Eqs. projection, update_pressure).

Time schemes (Sec. 2): RK2+CN with (gamma, rho) = (1/2, 0), (1, -1/2);
AB+CN with (3/2, -1/2); alpha = gamma + rho.

Reading "body fixed within the step": the body stays at X(t^n) with velocity
U^n for every sub-stage of step n (Sec. 2 uses the wall velocity of the
previous time step; Fig. 5 moves the structure after the step), so the tags
are computed once per step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry, forcing, predictor, poisson, projection
from .grid import Grid

SCHEMES = {
    "rk2": ((0.5, 0.0), (1.0, -0.5)),
    "ab2": ((1.5, -0.5),),
}


@dataclass
class Tags:
    idx: list     # per component, int64 ascending
    tri: list     # per component, int32
    cb: np.ndarray

    @property
    def counts(self):
        return [len(i) for i in self.idx]


def compute_tags(g, verts, tris):
    t = geometry.tag_all(g, verts, tris)
    idx = [a for a, _ in t]
    tri = [b for _, b in t]
    return Tags(idx, tri, geometry.boundary_cells(g, *idx))


def masks_of(g, tags):
    return [geometry.forcing_mask(g, c, tags.idx[c]) for c in range(3)]


def substage(g, fields, p, hprev, tags, verts, vel, tris, gamma, rho, dt, re, fext,
             use_q=True, diag=None, kappa=None):
    """One sub-stage.  Returns (fields^{s+1}, p^{s+1}, H^s)."""
    alpha = gamma + rho
    masks = masks_of(g, tags)
    fib = forcing.apply_ib(g, fields, list(zip(tags.idx, tags.tri)), verts, vel, tris)
    uhat, H = predictor.predictor(g, fib, p, hprev, masks, gamma, rho, alpha, dt, re, fext,
                                  kappa)
    rhs, qF, _ = projection.mass_correction(g, uhat, tags.cb, alpha, dt, use_q, p)
    phi = poisson.solve(g, rhs)
    new, pn = projection.project(g, uhat, p, phi, alpha, dt, re)
    if diag is not None:
        diag.append({"qF": qF, "n_cb": len(tags.cb), "counts": tags.counts})
    return new, pn, H


def step(g, fields, p, surface, dt, re, fext, scheme="rk2", hprev=None, use_q=True,
         diag=None, kappa=None):
    """One time step from t^n.  surface = (verts, vel, tris) at t^n.
    Returns (fields^{n+1}, p^{n+1}, H for a following AB step, tags)."""
    verts, vel, tris = surface
    tags = compute_tags(g, verts, tris)
    coefs = SCHEMES[scheme]
    if scheme == "ab2" and hprev is None:
        coefs = ((1.0, 0.0),)          # first AB step: explicit Euler on H
    H = hprev
    for gamma, rho in coefs:
        fields, p, Hs = substage(g, fields, p, H, tags, verts, vel, tris, gamma, rho,
                                 dt, re, fext, use_q, diag, kappa)
        H = Hs
    return fields, p, H, tags


def run(workload, steps=None, use_q=True, diag=None, callback=None):
    """March a workloads.Workload from t = 0 for `steps` steps."""
    from .kinematics import body_at, concat_bodies
    wl = workload
    g = Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces)
    fields = wl.fields()
    p = np.zeros(g.shape)
    fext = (-wl.dpdx, 0.0, 0.0)
    H = None
    n = wl.steps if steps is None else steps
    for s in range(n):
        t = s * wl.dt
        parts = [body_at(b, t) + (b.tris,) for b in wl.bodies]
        surface = concat_bodies(parts)
        fields, p, H, tags = step(g, fields, p, surface, wl.dt, wl.re, fext, wl.scheme, H,
                                  use_q, diag)
        if callback is not None:
            callback(s, fields, p, tags)
    return g, fields, p
