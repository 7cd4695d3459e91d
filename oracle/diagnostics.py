"""No-slip (transpiration) error (paper Sec. 4.4): the mismatch between the
wall velocity and the flow velocity interpolated on the surface with the IB
interpolator of Eq. new_IB, i.e. the linear extrapolation to the wall
through the forcing node and its probe point:

    eps = (u(x^f) - a u(x^e)) / (1 - a) - U(X^f),   a = |N|/h,

averaged in absolute value over the forcing nodes of each component and then
over the three components (reading: the "L1 norm" is a mean).
"""
from __future__ import annotations

import numpy as np

from .forcing import node_images, probe_length, trilinear
from .geometry import closest_point, dot3
from .grid import COMP_OFFSETS


def noslip_error(g, fields, tags, verts, vel, tris):
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    per = []
    for c in range(3):
        idx, tri = tags.idx[c], tags.tri[c]
        if len(idx) == 0:
            per.append(0.0)
            continue
        ox, oz = COMP_OFFSETS[c]
        iu, j, ku = node_images(g, c, idx, tri, verts, tris)
        ext = g.y_nodes_ext(c)
        e = j if c == 1 else j + 1
        x = ((iu + ox) * g.dx, ext[e], (ku + oz) * g.dz)
        T = tris[tri]
        A = tuple(verts[T[:, 0], d] for d in range(3))
        B = tuple(verts[T[:, 1], d] for d in range(3))
        C = tuple(verts[T[:, 2], d] for d in range(3))
        X, (wa, wb, wc), _ = closest_point(x, A, B, C)
        N = (x[0] - X[0], x[1] - X[1], x[2] - X[2])
        nn = np.sqrt(dot3(*N, *N))
        U = (wa * vel[T[:, 0], c] + wb * vel[T[:, 1], c]) + wc * vel[T[:, 2], c]
        uf = fields[c].reshape(-1)[idx]
        h = probe_length(g, c, j)
        on = nn == 0.0
        safe = np.where(on, 1.0, nn)
        xe = tuple(X[d] + h * (N[d] / safe) for d in range(3))
        a = nn / h
        ue = trilinear(g, c, fields[c], xe)
        wall = np.where(on, uf, (uf - a * ue) / (1.0 - a))
        per.append(float(np.mean(np.abs(wall - U))))
    return float(np.mean(per)), per


# --------------------------------------------------------------------------
# Pressure on the boundary cells (paper Sec. 2, after Eq. q_F): p is not
# defined on C_B by the solve and is rebuilt from the surrounding field with
# the strategy of the velocity forcing, as post-processing.  Reading (the
# paper gives no formula): for a C_B cell, the wall point X is the closest
# point of the cell centre on the forcing triangles of the cell's six faces
# (least |N|^2, ties to the lowest triangle id; the centre's periodic image
# nearest the triangle's centroid); the probe x^e = X + h N/|N| with h twice
# the cell's diagonal, as in Eq. probe; the wall carries no pressure value,
# so the linear profile of Eq. new_IB reduces to a zero normal gradient and
# the cell takes p(x^e), trilinear on the cell-centre lattice (constant
# beyond the first and last centres: homogeneous Neumann at the walls).  A
# centre on the surface (|N| = 0) takes the mean of the probes on both sides
# along the triangle's normal.
# --------------------------------------------------------------------------

def pressure_trilinear(g, p, xe):
    """Trilinear interpolation of a cell-centred field at points xe (tuple of
    3 arrays), periodic in x and z, clamped to the first/last centre in y."""
    sx = xe[0] / g.dx - 0.5
    ix = np.floor(sx)
    tx = sx - ix
    ix = ix.astype(np.int64)
    sz = xe[2] / g.dz - 0.5
    iz = np.floor(sz)
    tz = sz - iz
    iz = iz.astype(np.int64)
    ey = np.clip(np.searchsorted(g.yc, xe[1], side="right") - 1, 0, g.ny - 2)
    ty = np.clip((xe[1] - g.yc[ey]) / (g.yc[ey + 1] - g.yc[ey]), 0.0, 1.0)
    out = np.zeros_like(np.asarray(xe[0], np.float64))
    for a in (0, 1):
        wx = tx if a else 1.0 - tx
        ii = np.mod(ix + a, g.nx)
        for b in (0, 1):
            wy = ty if b else 1.0 - ty
            for d in (0, 1):
                wz = tz if d else 1.0 - tz
                kk = np.mod(iz + d, g.nz)
                out += (wx * wy * wz) * p[ey + b, kk, ii]
    return out


def pressure_cb(g, p, tags, verts, tris):
    """Reconstructed pressure at every cell of tags.cb (ascending), as an
    array in that order.  tags: .idx[c], .tri[c] (sorted forcing nodes and
    their triangles), .cb."""
    cb = np.asarray(tags.cb, np.int64)
    if len(cb) == 0:
        return np.zeros(0)
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    p = np.asarray(p, np.float64).reshape(g.shape)
    plane = g.nx * g.nz
    i, k, j = cb % g.nx, (cb // g.nx) % g.nz, cb // plane
    faces = [(0, cb), (0, j * plane + k * g.nx + (i + 1) % g.nx), (1, cb), (1, cb + plane),
             (2, cb), (2, j * plane + ((k + 1) % g.nz) * g.nx + i)]
    centre = ((i + 0.5) * g.dx, g.yc[j], (k + 0.5) * g.dz)
    best_n2 = np.full(len(cb), np.inf)
    best_t = np.full(len(cb), np.iinfo(np.int64).max)
    best_X = [np.zeros(len(cb)) for _ in range(3)]
    best_p = [np.zeros(len(cb)) for _ in range(3)]
    for c, node in faces:
        pos = np.searchsorted(tags.idx[c], node)
        assert np.all(np.asarray(tags.idx[c])[pos] == node), "a C_B face is not a forcing node"
        t = np.asarray(tags.tri[c], np.int64)[pos]
        T = tris[t]
        A = tuple(verts[T[:, 0], d] for d in range(3))
        B = tuple(verts[T[:, 1], d] for d in range(3))
        C = tuple(verts[T[:, 2], d] for d in range(3))
        cx = (A[0] + B[0] + C[0]) / 3.0
        cz = (A[2] + B[2] + C[2]) / 3.0
        pc = (centre[0] + g.lx * np.round((cx - centre[0]) / g.lx), centre[1],
              centre[2] + g.lz * np.round((cz - centre[2]) / g.lz))
        X, _, _ = closest_point(pc, A, B, C)
        N = (pc[0] - X[0], pc[1] - X[1], pc[2] - X[2])
        n2 = dot3(*N, *N)
        better = (n2 < best_n2) | ((n2 == best_n2) & (t < best_t))
        best_n2 = np.where(better, n2, best_n2)
        best_t = np.where(better, t, best_t)
        for d in range(3):
            best_X[d] = np.where(better, X[d], best_X[d])
            best_p[d] = np.where(better, pc[d], best_p[d])
    h = 2.0 * np.sqrt(g.dx * g.dx + g.dz * g.dz + g.dy[j] * g.dy[j])
    nn = np.sqrt(best_n2)
    on = nn == 0.0
    safe = np.where(on, 1.0, nn)
    n = [(best_p[d] - best_X[d]) / safe for d in range(3)]
    out = pressure_trilinear(g, p, tuple(best_X[d] + h * n[d] for d in range(3)))
    if np.any(on):
        T = tris[best_t[on]]
        e1 = verts[T[:, 1]] - verts[T[:, 0]]
        e2 = verts[T[:, 2]] - verts[T[:, 0]]
        nr = np.cross(e1, e2)
        nr /= np.linalg.norm(nr, axis=1)[:, None]
        Xo = [best_X[d][on] for d in range(3)]
        ho = h[on]
        plus = pressure_trilinear(g, p, tuple(Xo[d] + ho * nr[:, d] for d in range(3)))
        minus = pressure_trilinear(g, p, tuple(Xo[d] - ho * nr[:, d] for d in range(3)))
        out[on] = 0.5 * (plus + minus)
    return out
