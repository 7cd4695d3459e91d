"""Two-sided Eulerian IB forcing (paper Sec. 3.1, Eqs. probe and new_IB).

For a forcing node x^f with wall point X^f (closest point on its forcing
triangle) and N^f = x^f - X^f, a probe of length h is cast along
n^f = N^f/|N^f| to the external point x^e = X^f + h n^f (Eq. probe); the
forced value is u^f = (1 - a) U + a u^e with a = |N^f|/h (Eq. new_IB), where U
is the wall velocity at X^f and u^e the trilinear interpolation of the same
velocity component at x^e.  h is twice the diagonal of the local cell
(Sec. 3.1; 2 sqrt(3) Delta on a uniform grid).

Readings: the local cell of a u/w node has height dy[j], that of
a v node dyc[j]; U inside a triangle is the barycentric interpolation of the
vertex velocities; a node on the surface (|N| = 0) takes u^f = U; all u^f are
computed from the unmodified field and written afterwards (Jacobi), and the
wall values act as interpolation nodes between a wall and its first node.
"""
from __future__ import annotations

import numpy as np

from .geometry import _ranges, closest_point, dot3
from .grid import COMP_OFFSETS


class GeometryError(ValueError):
    """A probe leaves the domain or its stencil contains its own node."""


def _wrapped_ijk(g, c, idx):
    nx, nz = g.nx, g.nz
    i = idx % nx
    k = (idx // nx) % nz
    j = idx // (nx * nz)
    return i, j, k


def node_images(g, c, idx, tri_ids, verts, tris):
    """Unwrapped lattice indices of each forcing node: the periodic image that
    lies inside its forcing triangle's candidate box (the image used by the
    tagging)."""
    i, j, k = _wrapped_ijk(g, c, idx)
    P = verts[tris[tri_ids]]
    i0, i1, _, _, k0, k1 = _ranges(g, c, P.min(1), P.max(1), g.delta_max())
    iu = i + g.nx * np.ceil((i0 - i) / g.nx).astype(np.int64)
    ku = k + g.nz * np.ceil((k0 - k) / g.nz).astype(np.int64)
    return iu, j, ku


def trilinear(g, c, field, xe, node=None):
    """Trilinear interpolation of component c (its own staggered lattice) at
    points xe (tuple of 3 arrays), periodic in x and z; in y the bracket is
    the largest lattice height <= y, with the wall points as nodes.
    If node=(i, j, k) is given, raises GeometryError when the 8-node stencil
    contains that node."""
    ox, oz = COMP_OFFSETS[c]
    ext = g.y_nodes_ext(c)
    if c == 1:
        fe = field
    else:
        z = np.zeros((1,) + field.shape[1:])
        fe = np.concatenate((z, field, z), axis=0)
    if np.any(xe[1] < ext[0]) or np.any(xe[1] > ext[-1]):
        raise GeometryError("probe point outside the channel")
    sx = xe[0] / g.dx - ox
    ix = np.floor(sx)
    tx = sx - ix
    ix = ix.astype(np.int64)
    sz = xe[2] / g.dz - oz
    iz = np.floor(sz)
    tz = sz - iz
    iz = iz.astype(np.int64)
    ey = np.clip(np.searchsorted(ext, xe[1], side="right") - 1, 0, len(ext) - 2)
    ty = (xe[1] - ext[ey]) / (ext[ey + 1] - ext[ey])
    out = np.zeros_like(xe[0])
    for a in (0, 1):
        wx = tx if a else 1.0 - tx
        ii = np.mod(ix + a, g.nx)
        for b in (0, 1):
            wy = ty if b else 1.0 - ty
            ee = ey + b
            for d in (0, 1):
                wz = tz if d else 1.0 - tz
                kk = np.mod(iz + d, g.nz)
                out += (wx * wy * wz) * fe[ee, kk, ii]
                if node is not None:
                    jj = ee if c == 1 else ee - 1
                    if np.any((ii == node[0]) & (jj == node[1]) & (kk == node[2])):
                        raise GeometryError("probe stencil contains its forcing node")
    return out


def probe_length(g, c, j):
    """h = 2 x (diagonal of the local cell) (Sec. 3.1)."""
    dyl = g.dyc[j] if c == 1 else g.dy[j]
    return 2.0 * np.sqrt(g.dx * g.dx + g.dz * g.dz + dyl * dyl)


def forced_values(g, c, idx, tri_ids, verts, vel, tris, field):
    """u^f of Eq. new_IB at every forcing node of component c, evaluated from
    the given (unmodified) field."""
    verts = np.asarray(verts, np.float64)
    vel = np.asarray(vel, np.float64)
    tris = np.asarray(tris, np.int64)
    if len(idx) == 0:
        return np.zeros(0)
    ox, oz = COMP_OFFSETS[c]
    iu, j, ku = node_images(g, c, idx, tri_ids, verts, tris)
    ext = g.y_nodes_ext(c)
    e = j if c == 1 else j + 1
    x = ((iu.astype(np.float64) + ox) * g.dx, ext[e], (ku.astype(np.float64) + oz) * g.dz)
    T = tris[tri_ids]
    A = tuple(verts[T[:, 0], d] for d in range(3))
    B = tuple(verts[T[:, 1], d] for d in range(3))
    C = tuple(verts[T[:, 2], d] for d in range(3))
    X, (wa, wb, wc), _ = closest_point(x, A, B, C)
    N = (x[0] - X[0], x[1] - X[1], x[2] - X[2])
    n2 = dot3(*N, *N)
    U = (wa * vel[T[:, 0], c] + wb * vel[T[:, 1], c]) + wc * vel[T[:, 2], c]
    on = n2 == 0.0
    nn = np.sqrt(np.where(on, 1.0, n2))
    h = probe_length(g, c, j)
    xe = tuple(X[d] + h * (N[d] / nn) for d in range(3))
    w = nn / h
    i_w, j_w, k_w = _wrapped_ijk(g, c, idx)
    off = ~on
    ue = np.zeros_like(w)
    if np.any(off):
        ue[off] = trilinear(g, c, field, tuple(a[off] for a in xe),
                            node=(i_w[off], j_w[off], k_w[off]))
    return np.where(on, U, (1.0 - w) * U + w * ue)


def apply_ib(g, fields, tags, verts, vel, tris):
    """Eq. IB_step: replace the velocity at every forcing node by u^f, all
    values computed from the input fields before any is written (Jacobi).
    fields = (u, v, w); tags = [(idx, tri) per component].  Returns copies."""
    out = []
    for c in range(3):
        f = fields[c].copy()
        idx, tri = tags[c]
        if len(idx):
            vals = forced_values(g, c, idx, tri, verts, vel, tris, fields[c])
            f.reshape(-1)[idx] = vals
        out.append(f)
    return tuple(out)
