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
