"""Shared setup for the GPU parity tests: builds the oracle grid and the HIP
context from the same seeded inputs, moves arrays between numpy and torch,
and measures relative errors.  Not a test module."""
import numpy as np
import torch

import workloads
from oracle import kinematics
from oracle.grid import Grid

DEV = "cuda:0"


def t(a, dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        x = x.to(dtype)
    return x.to(DEV)


def n(x, shape=None):
    a = x.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def rel(a, ref):
    den = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(a - ref))) / (den if den > 0 else 1.0)


class Case:
    """A workload on both sides: oracle grid + HIP context + bodies."""

    def __init__(self, name, use_q=True, force_cap=0, **ctx_opts):
        from paper_2606_09799_amd import ibm
        self.ibm = ibm
        self.wl = wl = workloads.config(name) if isinstance(name, str) else name
        self.g = Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces)
        self.ctx = ibm.Context(wl.nx, wl.ny, wl.nz, wl.lx, wl.lz, wl.y_faces, wl.re, wl.dpdx,
                               use_q=use_q, force_cap=force_cap, **ctx_opts)
        self.fext = (-wl.dpdx, 0.0, 0.0)
        self.dev_bodies = []
        for b in wl.bodies:
            ref = t(b.ref)
            nv = b.ref.shape[0]
            xyz = torch.empty(nv, 3, dtype=torch.float64, device=DEV)
            vel = torch.empty(nv, 3, dtype=torch.float64, device=DEV)
            self.dev_bodies.append((b, ref, xyz, vel, t(b.tris.astype(np.int32))))

    def bodies_at(self, time):
        """Body transforms on the device; returns (device Body list, oracle
        surface (verts, vel, tris) computed by the oracle's own transform)."""
        out, parts = [], []
        for b, ref, xyz, vel, tri in self.dev_bodies:
            coef = b.coef(time)
            if b.kind == "rigid":
                self.ibm.ibm_body_rigid(self.ctx, ref, coef, xyz, vel)
            else:
                self.ibm.ibm_body_deform(self.ctx, ref, coef, xyz, vel)
            out.append(self.ibm.Body(xyz, vel, tri))
            parts.append(kinematics.body_at(b, time) + (b.tris,))
        return out, kinematics.concat_bodies(parts)

    def fields(self):
        return self.wl.fields()

    def random_fields(self, seed):
        rng = np.random.default_rng(seed)
        g = self.g
        u = rng.standard_normal(g.shape)
        v = rng.standard_normal(g.comp_shape(1))
        v[0] = 0.0
        v[-1] = 0.0
        w = rng.standard_normal(g.shape)
        return u, v, w
