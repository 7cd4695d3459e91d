"""Pins of the oracle's hydrodynamic loads (paper Sec. 3.3) against what the
mathematics fixes, each chosen so that a plausible slip fails one of them:

* the MLS fit reproduces quadratic fields exactly (value, gradient,
  Hessian), on every staggered lattice (a wrong basis term, scale or
  lattice offset fails);
* Archimedes: a linear pressure on a closed icosphere gives F = -grad(p) V
  with V the polyhedron's volume (midpoint quadrature is exact for a linear
  p on flat triangles; a wrong sign, area or normal fails);
* a pressure quadratic in the wall-normal distance above a plate gives the
  wall value at every marker (the h and h^2 Taylor terms of Sec. 3.3; a
  dropped or mis-signed term fails);
* a zero-thickness plate in the shear layer u = g |y - y_p| (opposite
  shear on its two faces) feels F_x = 2 g A / Re (the symmetric gradient and
  1/Re; G in place of G + G^T, or one side only fails), and its torque
  about a pole is (X_c - pole) x F;
* nodes behind the marker's tangent plane are left out of the fit (a
  field that is quadratic in front and arbitrary behind is reproduced).
"""
import numpy as np
import pytest

import workloads
from oracle import loads
from oracle.grid import Grid


def _grid(n=24, ny=24, stretch=None):
    yf = workloads.tanh_faces(ny, stretch) if stretch else workloads.uniform_faces(ny)
    return Grid(n, ny, n, 2.0, 2.0, yf)


def _quad(rng):
    c0, g = rng.standard_normal(), rng.standard_normal(3)
    H = rng.standard_normal((3, 3))
    H = H + H.T
    return c0, g, H


@pytest.mark.parametrize("q", ["p", 0, 1, 2])
@pytest.mark.parametrize("stretch", [None, 1.5])
def test_mls_reproduces_quadratics(q, stretch):
    g = _grid(stretch=stretch)
    rng = np.random.default_rng(3)
    c0, gr, H = _quad(rng)
    xe = np.array([1.013, 0.071, 0.977])          # mid-channel, away from x, z = 0
    from oracle.grid import COMP_OFFSETS
    ox, oz = (0.5, 0.5) if q == "p" else COMP_OFFSETS[q]
    ys = g.yc if q in ("p", 0, 2) else g.yf
    shape = g.shape if q != 1 else g.comp_shape(1)
    x = (np.arange(g.nx) + ox) * g.dx
    z = (np.arange(g.nz) + oz) * g.dz
    Y, Z, X = np.meshgrid(ys, z, x, indexing="ij")
    d = np.stack([X - xe[0], Y - xe[1], Z - xe[2]], axis=-1)
    f = c0 + d @ gr + 0.5 * np.einsum("...i,ij,...j->...", d, H, d)
    assert f.shape == shape
    Xm = xe - np.array([0.0, 0.3, 0.0])           # marker below: every node passes
    val, grad, Hf = loads.mls_fit(g, q, f, xe, Xm, np.array([0.0, 1.0, 0.0]),
                                  max(g.dx, g.dz, g.dy[loads.cell_j(g, Xm[1])]))
    assert abs(val - c0) < 1e-11 * (1 + abs(c0))
    assert np.max(np.abs(grad - gr)) < 1e-9 * (1 + np.max(np.abs(gr)))
    assert np.max(np.abs(Hf - H)) < 1e-7 * (1 + np.max(np.abs(H)))


def test_archimedes_on_a_closed_icosphere():
    g = _grid(32, 32)
    V, T = workloads.icosphere(2)
    r, c = 0.35, np.array([1.02, 0.03, 0.97])
    verts = V * r + c
    a = np.array([0.7, -1.9, 0.4])                # grad p
    xc = (np.arange(g.nx) + 0.5) * g.dx
    zc = (np.arange(g.nz) + 0.5) * g.dz
    Y, Z, X = np.meshgrid(g.yc, zc, xc, indexing="ij")
    p = 0.3 + a[0] * X + a[1] * Y + a[2] * Z
    zero = [np.zeros(g.shape), np.zeros(g.comp_shape(1)), np.zeros(g.shape)]
    t, F, M = loads.loads(g, zero, p, verts, T, 100.0, c)
    Xm, n, A = loads.markers(verts, T)
    vol = np.sum(np.einsum("ij,ij->i", Xm - c, n) * A) / 3.0
    assert vol > 0.9 * 4.0 / 3.0 * np.pi * r ** 3   # outward normals
    assert np.max(np.abs(F + a * vol)) < 1e-10 * np.linalg.norm(a) * vol


def _plate(g, yp, nq=6):
    P, T = workloads.plate_mesh(0.9, 0.7, nq, nq)
    return P + np.array([1.03, yp, 0.98]), T


def test_pressure_taylor_terms_above_a_plate():
    g = _grid(32, 32)
    yp = 0.013
    verts, T = _plate(g, yp)
    xc = (np.arange(g.nx) + 0.5) * g.dx
    zc = (np.arange(g.nz) + 0.5) * g.dz
    Y, _, _ = np.meshgrid(g.yc, zc, xc, indexing="ij")
    c, b, a = 0.83, -1.7, 2.9
    p = c + b * (Y - yp) + a * (Y - yp) ** 2
    zero = [np.zeros(g.shape), np.zeros(g.comp_shape(1)), np.zeros(g.shape)]
    t, F, M = loads.loads(g, zero, p, verts, T, 100.0, np.zeros(3))
    _, n, A = loads.markers(verts, T)
    side = np.sign(n[0, 1])                       # the winding's side of the plate
    assert np.all(n[:, 1] == side)
    # at y_p the pressure is c on the normal's side: t = -c n
    assert np.max(np.abs(t[:, 1] + c * side)) < 1e-10
    assert np.max(np.abs(t[:, [0, 2]])) < 1e-10
    assert abs(F[1] + c * side * np.sum(A)) < 1e-10


def test_two_sided_plate_in_a_shear_layer():
    g = _grid(32, 32)
    yp = 0.013
    verts, T = _plate(g, yp)
    gam, re = 1.3, 50.0
    u = np.broadcast_to((gam * np.abs(g.yc - yp))[:, None, None], g.shape).copy()
    zero_v, zero_w = np.zeros(g.comp_shape(1)), np.zeros(g.shape)
    pole = np.array([0.2, -0.4, 0.3])
    t, F, M = loads.loads(g, [u, zero_v, zero_w], np.zeros(g.shape), verts, T, re, pole,
                          two_sided=True)
    Xm, _, A = loads.markers(verts, T)
    assert np.max(np.abs(t - np.array([2 * gam / re, 0.0, 0.0]))) < 1e-10
    assert abs(F[0] - 2 * gam * np.sum(A) / re) < 1e-10
    Xc = np.sum(Xm * A[:, None], axis=0) / np.sum(A)
    assert np.max(np.abs(M - np.cross(Xc - pole, F))) < 1e-10
    # one side only: half of it
    t1, F1, _ = loads.loads(g, [u, zero_v, zero_w], np.zeros(g.shape), verts, T, re, pole)
    assert abs(F1[0] - gam * np.sum(A) / re) < 1e-10


def test_mls_uses_only_nodes_in_front_of_the_marker():
    """With the marker close to the probe point, the nodes behind the
    marker's tangent plane (here holding unrelated values) are left out:
    the fit still reproduces the quadratic of the front side exactly."""
    g = _grid()
    rng = np.random.default_rng(8)
    c0, gr, H = _quad(rng)
    xe = np.array([1.013, 0.071, 0.977])
    n = np.array([0.3, 0.9, -0.2])
    n /= np.linalg.norm(n)
    Xm = xe - 0.4 * g.dx * n
    x = (np.arange(g.nx) + 0.5) * g.dx
    z = (np.arange(g.nz) + 0.5) * g.dz
    Y, Z, X = np.meshgrid(g.yc, z, x, indexing="ij")
    d = np.stack([X - xe[0], Y - xe[1], Z - xe[2]], axis=-1)
    f = c0 + d @ gr + 0.5 * np.einsum("...i,ij,...j->...", d, H, d)
    behind = (np.stack([X, Y, Z], axis=-1) - Xm) @ n <= 0.0
    f[behind] = 1e3 * rng.standard_normal(np.count_nonzero(behind))
    val, grad, Hf = loads.mls_fit(g, "p", f, xe, Xm, n, g.dx)
    assert abs(val - c0) < 1e-9 * (1 + abs(c0))
    assert np.max(np.abs(grad - gr)) < 1e-7 * (1 + np.max(np.abs(gr)))
