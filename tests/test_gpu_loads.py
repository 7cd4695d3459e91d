"""Hydrodynamic loads (paper Sec. 3.3) through the C-ABI against the
oracle: per-marker tractions and per-body force and torque of a closed
icosphere and a two-sided plate that crosses the periodic boundary, on a
stretched grid with random fields, in FP64 and with an FP32 pressure (the
mixed form); and the loads of the 67 bodies of the 1024x768x1024 workload
at its initial field, against the oracle on a sample of markers.

Bar: 1e-10 relative (FP64 arithmetic on both sides; the MLS normal
equations have a condition number of about 10)."""
import numpy as np
import pytest
import torch

import workloads
from gpu_harness import Case, DEV, n, rel, t
from oracle import loads as oloads
from oracle import step as ostep

pytestmark = pytest.mark.gpu


def _two_bodies():
    V, T1 = workloads.icosphere(2)
    S = V * 0.3 + np.array([0.95, 0.1, 1.1])
    P, T2 = workloads.plate_mesh(0.8, 0.6, 5, 4)
    Pl = P + np.array([1.9, -0.35, 0.4])       # crosses x = lx
    return [(S, T1, 1), (Pl, T2, 2)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loads_against_oracle(precision):
    wl = workloads.Workload("loads", 24, 32, 24, 2.0, 2.0, workloads.tanh_faces(32, 1.8), 50.0,
                            1e-3, 1, 1.0, 0.0, 0, 0.0, [])
    case = Case(wl, precision=precision)
    g = case.g
    bodies = _two_bodies()
    dbod = [case.ibm.Body(t(X), t(np.zeros_like(X)), t(T.astype(np.int32))) for X, T, _ in bodies]
    case.ibm.ibm_tag(case.ctx, dbod)
    rng = np.random.default_rng(4)
    f = [rng.standard_normal(g.shape), rng.standard_normal(g.comp_shape(1)),
         rng.standard_normal(g.shape)]
    f[1][0] = f[1][-1] = 0.0
    p = rng.standard_normal(g.shape)
    if precision == "mixed":
        p = p.astype(np.float32).astype(np.float64)  # the oracle sees the stored FP32 values
    Xc = np.concatenate([b[0] for b in bodies])
    Tc = np.concatenate([bodies[0][1], bodies[1][1] + bodies[0][0].shape[0]])
    tags = ostep.compute_tags(g, Xc, Tc)
    cbm = np.zeros(g.cells, bool)
    cbm[np.asarray(tags.cb)] = True
    assert cbm.any()
    sides = np.array([b[2] for b in bodies], np.int32)
    pole = np.array([[0.9, 0.1, 1.0], [1.9, -0.3, 0.5]])
    ntri = len(Tc)
    tr = torch.zeros(ntri, 3, dtype=torch.float64, device=DEV)
    ld = torch.zeros(2, 6, dtype=torch.float64, device=DEV)
    case.ibm.ibm_loads(case.ctx, *(t(a) for a in f), t(p, case.ctx.pdtype), t(sides), t(pole),
                       tr, ld)
    tg, lg = n(tr), n(ld)
    off = 0
    for q, (X, T, sd) in enumerate(bodies):
        tq, F, M = oloads.loads(g, f, p, X, T, wl.re, pole[q], two_sided=(sd == 2), cb_mask=cbm)
        assert rel(tg[off:off + len(T)], tq) < 1e-10, q
        off += len(T)
        assert rel(lg[q, :3], F) < 1e-10, q
        assert rel(lg[q, 3:], M) < 1e-10, q
    case.ctx.close()


def test_loads_of_the_large_multibody_workload_sampled():
    """All 67 bodies of the 1024x768x1024 channel (111920 markers) at t = 0
    with its initial field and a smooth pressure: the tractions of 16
    sampled markers of every eighth sphere and of each leaflet against the
    oracle's (same marker, same tags), and every body's force and torque
    against FP64 sums of the GPU tractions (the per-body summation is
    checked, not only the markers)."""
    case = Case("c5", precision="mixed")
    g = case.g
    bodies, (X, U, T) = case.bodies_at(0.0)
    case.ibm.ibm_tag(case.ctx, bodies)
    u, v, w = case.wl.fields_torch(DEV)
    yc = torch.tensor(g.yc, device=DEV)
    pg = (0.3 * yc[:, None, None] + 0.1 * yc[:, None, None] ** 2).expand(g.ny, g.nz, g.nx)
    pg = pg.to(torch.float32).contiguous().view(-1)
    nb = len(bodies)
    # the three leaflets are zero-thickness surfaces (two-sided), the
    # spheres closed
    sides = torch.tensor([2 if b.tris.shape[0] > 5000 else 1 for b in case.wl.bodies],
                         dtype=torch.int32, device=DEV)
    kinds = n(sides)
    pole = torch.zeros(nb, 3, dtype=torch.float64, device=DEV)
    ntri = sum(b.tris.shape[0] for b in case.wl.bodies)
    tr = torch.zeros(ntri, 3, dtype=torch.float64, device=DEV)
    ld = torch.zeros(nb, 6, dtype=torch.float64, device=DEV)
    case.ibm.ibm_loads(case.ctx, u, v, w, pg, sides, pole, tr, ld)
    tg, lg = n(tr), n(ld)
    assert np.isfinite(tg).all() and np.isfinite(lg).all()
    lists, cb = case.ibm.tag_lists(case.ctx)
    cbm = np.zeros(g.cells, bool)
    cbm[n(cb)] = True
    fields = None
    rng = np.random.default_rng(9)
    off = 0
    for q, b in enumerate(case.wl.bodies):
        verts = n(bodies[q].xyz)
        tris = b.tris
        Xm, nm, A = oloads.markers(verts, tris)
        F = np.sum(tg[off:off + len(tris)] * A[:, None], axis=0)
        M = np.sum(np.cross(Xm, tg[off:off + len(tris)]) * A[:, None], axis=0)
        assert np.max(np.abs(lg[q, :3] - F)) < 1e-10 * (1 + np.max(np.abs(F))), q
        assert np.max(np.abs(lg[q, 3:] - M)) < 1e-10 * (1 + np.max(np.abs(M))), q
        if q % 8 == 0 or kinds[q] == 2:
            if fields is None:
                fields = [n(x, s) for x, s in ((u, g.shape), (v, g.comp_shape(1)), (w, g.shape))]
                pn = n(pg, g.shape).astype(np.float64)
            for m in rng.choice(len(tris), size=16, replace=False):
                tm = sum(oloads.marker_traction(g, fields, pn, Xm[m], nm[m], s, case.wl.re,
                                                cbm.reshape(g.shape))
                         for s in ((1.0, -1.0) if kinds[q] == 2 else (1.0,)))
                ref = np.max(np.abs(tm)) + 1.0
                assert np.max(np.abs(tg[off + m] - tm)) < 1e-10 * ref, (q, m)
        off += len(tris)
    case.ctx.close()
