"""Hydrodynamic loads on the bodies (paper Sec. 3.3): tractions at the
triangle centres from second-order moving-least-squares (MLS) fits of p and
of the velocity components, Taylor-expanded from a probe point back to the
surface, summed into force and torque.

Test infrastructure only: plain FP64 numpy, one marker at a time, no
blocking or reordering beyond what the definitions state.  Readings of the
paper (it gives the method, not the MLS weight and support, which come from
a cited companion paper):

* markers X^l are the triangle centroids, n^l the unit normal of the
  triangle's winding, A^l its area;
* the probe length h is twice the diagonal of the grid cell containing X^l,
  sqrt(dx^2 + dz^2 + dy_j^2), as for the forcing probe; the probe point is
  x^e = X^l + s h n^l for side s = +1, and also s = -1 for a two-sided
  (zero-thickness) body, whose marker traction is the sum of both sides;
* each quantity is fitted on its own lattice (p at cell centres; u, v, w on
  their faces, with the wall points as nodes): the 4 x 4 x 4 nodes around
  x^e (periodic images in x and z; in y four consecutive lattice heights
  bracketing x^e, shifted inside at the walls), keeping only nodes strictly
  on the probe side of the marker's tangent plane, (x_i - X^l).(s n^l) > 0,
  and, for p, only fluid cells (not C_B, where the solve does not define p);
* weights w_i = exp(-|x_i - x^e|^2 / D^2) with D = max(dx, dz, dy_j); basis
  1, X, Y, Z, X^2, Y^2, Z^2, XY, YZ, XZ in the scaled coordinates
  (x - x^e)/D; the fit is the weighted least-squares solution;
* with a quadratic basis the third derivatives vanish, so the h^2 term of
  the velocity-gradient expansion is zero;
* a probe point exactly on a lattice line (the paper is silent): the window
  follows from floor(x^e/dx - o) as evaluated, and the tangent-plane test is
  the three products summed left to right, both in plain binary64.
"""
from __future__ import annotations

import numpy as np

from .grid import COMP_OFFSETS

NB = 10  # basis size


def markers(verts, tris):
    """Centroids (M, 3), unit normals (M, 3) and areas (M,) of the triangles."""
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    A, B, C = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    X = (A + B + C) / 3.0
    cr = np.cross(B - A, C - A)
    nrm = np.linalg.norm(cr, axis=1)
    return X, cr / nrm[:, None], 0.5 * nrm


def cell_j(g, y):
    """Index of the cell whose [yf_j, yf_{j+1}) holds y (clamped)."""
    return int(np.clip(np.searchsorted(g.yf, y, side="right") - 1, 0, g.ny - 1))


def _y_lattice(g, q):
    """Heights of the y-lattice of quantity q ('p' or component 0-2) and a
    map from a lattice index to the array row (None: a wall point, value 0
    for u, w)."""
    if q == "p":
        return g.yc, lambda e: e
    if q == 1:
        return g.yf, lambda e: e
    ext = np.concatenate(([g.yf[0]], g.yc, [g.yf[-1]]))
    return ext, lambda e: (None if e == 0 or e == g.ny + 1 else e - 1)


def stencil(g, q, xe):
    """The 4 x 4 x 4 nodes of quantity q around xe: list of (position,
    (j_row or None, k, i))."""
    ox, oz = (0.5, 0.5) if q == "p" else COMP_OFFSETS[q]
    ys, row = _y_lattice(g, q)
    e0 = int(np.searchsorted(ys, xe[1], side="right")) - 2
    e0 = min(max(e0, 0), len(ys) - 4)
    i0 = int(np.floor(xe[0] / g.dx - ox)) - 1
    k0 = int(np.floor(xe[2] / g.dz - oz)) - 1
    out = []
    for e in range(e0, e0 + 4):
        for kk in range(k0, k0 + 4):
            for ii in range(i0, i0 + 4):
                pos = np.array([(ii + ox) * g.dx, ys[e], (kk + oz) * g.dz])
                out.append((pos, (row(e), kk % g.nz, ii % g.nx)))
    return out


def basis(d):
    """Quadratic basis at scaled offsets d = (X, Y, Z)."""
    X, Y, Z = d
    return np.array([1.0, X, Y, Z, X * X, Y * Y, Z * Z, X * Y, Y * Z, X * Z])


def mls_fit(g, q, field, xe, X, ns, D, cb_mask=None):
    """Weighted least-squares quadratic fit of quantity q around xe: returns
    (value, gradient (3,), Hessian (3, 3)) at xe."""
    rows, rhs, wts = [], [], []
    for pos, (j, k, i) in stencil(g, q, xe):
        r = pos - X
        if r[0] * ns[0] + r[1] * ns[1] + r[2] * ns[2] <= 0.0:
            continue                        # behind the marker's tangent plane
        if q == "p" and cb_mask is not None and cb_mask[j, k, i]:
            continue                        # C_B cell: p is not defined there
        val = 0.0 if j is None else field[j, k, i]
        d = (pos - xe) / D
        rows.append(basis(d))
        rhs.append(val)
        wts.append(np.exp(-np.dot(d, d)))
    P = np.array(rows)
    sw = np.sqrt(np.array(wts))
    c = np.linalg.lstsq(P * sw[:, None], np.array(rhs) * sw, rcond=None)[0]
    grad = c[1:4] / D
    H = np.array([[2 * c[4], c[7], c[9]],
                  [c[7], 2 * c[5], c[8]],
                  [c[9], c[8], 2 * c[6]]]) / (D * D)
    return c[0], grad, H


def marker_traction(g, fields, p, X, n, side, re, cb_mask=None):
    """Traction at marker X with normal side*n (Sec. 3.3): the probe, the
    MLS fits, the Taylor expansions back to X and t = -p n + (1/Re)(G + G^T) n."""
    j = cell_j(g, X[1])
    h = 2.0 * np.sqrt(g.dx * g.dx + g.dz * g.dz + g.dy[j] * g.dy[j])
    D = max(g.dx, g.dz, g.dy[j])
    ns = side * n
    xe = X + h * ns
    pe, gp, Hp = mls_fit(g, "p", p, xe, X, ns, D, cb_mask)
    pl = pe - h * np.dot(ns, gp) + 0.5 * h * h * (ns @ Hp @ ns)
    G = np.zeros((3, 3))                    # G[i, j] = d u_i / d x_j at X
    for c in range(3):
        _, gu, Hu = mls_fit(g, c, fields[c], xe, X, ns, D)
        G[c] = gu - h * (Hu @ ns)
    return -pl * ns + (G + G.T) @ ns / re


def loads(g, fields, p, verts, tris, re, pole, two_sided=False, cb_mask=None):
    """Per-marker tractions (M, 3), force (3,) and torque about `pole` (3,)
    of one body (Sec. 3.3)."""
    X, n, A = markers(verts, tris)
    p = np.asarray(p, np.float64).reshape(g.shape)
    if cb_mask is not None:
        cb_mask = np.asarray(cb_mask, bool).reshape(g.shape)
    sides = (1.0, -1.0) if two_sided else (1.0,)
    t = np.zeros_like(X)
    for m in range(len(X)):
        for s in sides:
            t[m] += marker_traction(g, fields, p, X[m], n[m], s, re, cb_mask)
    F = np.sum(t * A[:, None], axis=0)
    M = np.sum(np.cross(X - np.asarray(pole, np.float64), t) * A[:, None], axis=0)
    return t, F, M
