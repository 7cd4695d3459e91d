"""Pins of the oracle's pressure reconstruction on the boundary cells (paper
Sec. 2, after Eq. q_F; the reading: the probe of the velocity forcing from
the closest wall point, twice the cell diagonal along N, and a zero normal
gradient, p(x_cb) = p(x^e)).  A full-span plate makes C_B exactly one cell
layer with N along y: a field linear in x and z (constant along the normal)
is reproduced exactly; a field linear in y gives b (y_w +- h), fixing the
side and the length of the probe; on a sphere every value is a convex
combination of the field.  CPU only."""
from types import SimpleNamespace

import numpy as np

import workloads
from oracle import diagnostics, geometry
from oracle.grid import Grid


def _plate_tags(g, y0, nq=8):
    P, T = workloads.plate_mesh(g.lx, g.lz, nq, nq)
    P = P + np.array([g.lx / 2, y0, g.lz / 2])
    lists = [geometry.tag(g, c, P, T) for c in range(3)]
    idx = [a[0] for a in lists]
    tri = [a[1] for a in lists]
    cb = geometry.boundary_cells(g, *idx)
    return SimpleNamespace(idx=idx, tri=tri, cb=cb), P, T


def _grid():
    ny = 14
    return Grid(48, ny, 24, 2 * np.pi, np.pi, workloads.uniform_faces(ny))


def _centres(g, cb):
    i, k, j = cb % g.nx, (cb // g.nx) % g.nz, cb // (g.nx * g.nz)
    return (i + 0.5) * g.dx, g.yc[j], (k + 0.5) * g.dz, j


def test_field_constant_along_the_normal_is_reproduced():
    g = _grid()
    jl = 7
    tags, P, T = _plate_tags(g, g.yf[jl] + 0.35 * g.dy[jl])
    assert len(tags.cb) == g.nx * g.nz
    X, Y, Z = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx))
    xc, zc = (Z + 0.5) * g.dx, (X + 0.5) * g.dz
    p = 0.3 * np.sin(xc) + 0.7 * np.cos(2 * zc) + 1.25   # periodic, no y dependence
    got = diagnostics.pressure_cb(g, p, tags, P, T)
    x, y, z, _ = _centres(g, tags.cb)
    assert np.max(np.abs(got - (0.3 * np.sin(x) + 0.7 * np.cos(2 * z) + 1.25))) < 1e-12


def test_probe_side_and_length_from_a_field_linear_in_y():
    g = _grid()
    jl = 7
    b = 2.5
    for frac, side in ((0.35, 1.0), (0.65, -1.0)):
        yw = g.yf[jl] + frac * g.dy[jl]
        tags, P, T = _plate_tags(g, yw)
        assert len(tags.cb) == g.nx * g.nz
        p = b * np.broadcast_to(g.yc[:, None, None], g.shape).copy()
        got = diagnostics.pressure_cb(g, p, tags, P, T)
        h = 2.0 * np.sqrt(g.dx ** 2 + g.dy[jl] ** 2 + g.dz ** 2)
        assert g.yc[0] <= yw - h and yw + h <= g.yc[-1]
        assert np.max(np.abs(got - b * (yw + side * h))) < 1e-12


def test_sphere_values_are_convex_combinations(rng):
    ny = 24
    g = Grid(32, ny, 24, 2 * np.pi, np.pi, workloads.uniform_faces(ny))
    S, T = workloads.icosphere(2)
    S = S * 0.9 + np.array([3.0, 0.0, 1.5])
    lists = [geometry.tag(g, c, S, T) for c in range(3)]
    tags = SimpleNamespace(idx=[a[0] for a in lists], tri=[a[1] for a in lists],
                           cb=geometry.boundary_cells(g, *[a[0] for a in lists]))
    assert len(tags.cb) > 0
    p = rng.standard_normal(g.shape)
    got = diagnostics.pressure_cb(g, p, tags, S, T)
    assert np.all(got >= p.min() - 1e-12) and np.all(got <= p.max() + 1e-12)
    assert np.all(diagnostics.pressure_cb(g, np.full(g.shape, 3.5), tags, S, T) - 3.5 < 1e-12)
