"""The mass- and energy-conserving shape of q_F (paper App. B, Eq.
unif_shape; IBM_Q_ENERGY) on the GPU against the oracle: the right-hand
side and the two coefficients of a single mass correction, whole steps in
FP64 within 1e-10, and the mixed form within 1e-6 of the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_harness import Case, DEV, n, rel, t
from oracle import projection, step as ostep

pytestmark = pytest.mark.gpu

SMALL = ["tiny", "tiny_plate", "c1"]


@pytest.mark.parametrize("name", SMALL)
def test_mass_rhs_energy_parity(name):
    case = Case(name, use_q="energy")
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    tags = ostep.compute_tags(g, X, T)
    f = case.random_fields(4)
    p = np.random.default_rng(14).standard_normal(g.shape)
    adt = 0.5 * case.wl.dt
    rhs_ref, _, _, (c0, c1) = projection.mass_correction_energy(g, f, p, tags.cb, 0.5,
                                                                case.wl.dt)
    rhs = torch.empty(g.cells, dtype=torch.float64, device=DEV)
    qf = torch.zeros(2, dtype=torch.float64, device=DEV)
    case.ibm.ibm_mass_rhs(case.ctx, *[t(a) for a in f], adt, rhs, qf, p=t(p))
    got = n(qf)
    assert abs(got[0] - c0) <= 1e-10 * abs(c0) and abs(got[1] - c1) <= 1e-10 * abs(c1)
    assert rel(n(rhs, g.shape), rhs_ref) < 1e-11
    assert case.ibm.ibm_check(case.ctx) == 0


def _run(name, steps, precision):
    case = Case(name, use_q="energy", precision=precision)
    g, wl = case.g, case.wl
    f = wl.fields()
    d = [t(a) for a in f]
    pd = torch.zeros(g.cells, dtype=case.ctx.pdtype, device=DEV)
    p = np.zeros(g.shape)
    for s in range(steps):
        bodies, surf = case.bodies_at(s * wl.dt)
        case.ibm.ibm_step(case.ctx, *d, pd, bodies, wl.dt)
        f, p, _, tags = ostep.step(g, f, p, surf, wl.dt, wl.re, case.fext, use_q="energy")
    assert case.ibm.ibm_check(case.ctx) == 0
    return case, g, d, pd, f, p, tags


@pytest.mark.parametrize("name,steps", [("tiny", 3), ("tiny_plate", 3), ("c1", 5)])
def test_step_parity_energy(name, steps):
    case, g, d, pd, f, p, tags = _run(name, steps, "fp64")
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-10, c
    mB = projection.cell_mask(g, tags.cb)
    dV = g.cell_volume()
    got = n(pd, g.shape)

    def centred(a):
        return a[~mB] - np.sum(a[~mB] * dV[~mB]) / np.sum(dV[~mB])
    assert rel(centred(got), centred(p)) < 1e-10


def test_mixed_step_energy_against_fp64_oracle():
    case, g, d, pd, f, p, tags = _run("c1", 5, "mixed")
    for c in range(3):
        assert rel(n(d[c], f[c].shape), f[c]) < 1e-6, c
