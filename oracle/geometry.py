"""Closest point on a triangle, the tagging algorithm and the cell classes.

Tagging follows Alg. 1 of the paper (Sec. 3.1): for every surface triangle,
the Eulerian nodes of one staggered lattice inside the triangle's inflated
Cartesian bounding box are visited; the closest point X on the triangle to a
node x is found (the paper cites Ericson's point-triangle algorithm, Real-Time
Collision Detection, 2004, Sec. 5.1.5, restated below), N = x - X, and x is a
forcing node if the scalar product of N with x_n - X is negative for at least
one of the six same-lattice neighbours x_n.

Readings of points the paper leaves open:
  * a node lying on the surface (|N| = 0) is a forcing node (weight 0);
  * the bounding box is inflated by the largest neighbour spacing of the
    grid (plus one node), so culling never changes the set: the
    "|N| <= cell diagonal" test of Alg. 1 is implied by the sign test on the
    grids used here, and the set is defined by the sign test alone;
  * when several triangles classify a node, the forcing triangle is the one
    with the smallest |N|^2 (ties to the lowest triangle id);
  * the wall-normal neighbour of the first/last node of a lattice is the
    wall point itself;
  * boundary cells C_B are the cells all six of whose faces carry forcing
    nodes (Sec. 3.2, "all of its faces contain forcing nodes").

Arithmetic contract: the decision uses only IEEE binary64 +, -, *, / in the
order written here (no fused multiply-add: numpy evaluates each operation
separately), and no square root.
"""
from __future__ import annotations

import numpy as np

from .grid import COMP_OFFSETS


def dot3(a0, a1, a2, b0, b1, b2):
    """Dot product in the pinned order (a0*b0 + a1*b1) + a2*b2."""
    return (a0 * b0 + a1 * b1) + a2 * b2


def closest_point(p, A, B, C):
    """Closest point on triangle ABC to each point p (Ericson 2004, Sec.
    5.1.5: Voronoi regions of the vertices, the edges and the face, tested in
    that order).  All arguments are tuples of three arrays (broadcastable).
    Returns (X, bary, region): X the closest point, bary its barycentric
    weights on (A, B, C), region 0..6 = A, B, AB, C, AC, BC, face."""
    ab = (B[0] - A[0], B[1] - A[1], B[2] - A[2])
    ac = (C[0] - A[0], C[1] - A[1], C[2] - A[2])
    ap = (p[0] - A[0], p[1] - A[1], p[2] - A[2])
    d1 = dot3(*ab, *ap)
    d2 = dot3(*ac, *ap)
    bp = (p[0] - B[0], p[1] - B[1], p[2] - B[2])
    d3 = dot3(*ab, *bp)
    d4 = dot3(*ac, *bp)
    cp = (p[0] - C[0], p[1] - C[1], p[2] - C[2])
    d5 = dot3(*ab, *cp)
    d6 = dot3(*ac, *cp)
    vc = d1 * d4 - d3 * d2
    vb = d5 * d2 - d1 * d6
    va = d3 * d6 - d5 * d4

    in_a = (d1 <= 0) & (d2 <= 0)
    in_b = (d3 >= 0) & (d4 <= d3)
    in_ab = (vc <= 0) & (d1 >= 0) & (d3 <= 0)
    in_c = (d6 >= 0) & (d5 <= d6)
    in_ac = (vb <= 0) & (d2 >= 0) & (d6 <= 0)
    in_bc = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)

    region = np.full(np.broadcast(d1, d2).shape, 6, dtype=np.int8)
    # first matching region wins: assign in reverse priority
    for code, m in ((5, in_bc), (4, in_ac), (3, in_c), (2, in_ab), (1, in_b), (0, in_a)):
        region[m] = code

    with np.errstate(divide="ignore", invalid="ignore"):
        t_ab = d1 / (d1 - d3)
        t_ac = d2 / (d2 - d6)
        t_bc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        den = 1.0 / ((va + vb) + vc)
        s_f = vb * den
        t_f = vc * den

    X = []
    for c in range(3):
        cb = C[c] - B[c]
        shape = d1.shape
        cand = [np.broadcast_to(A[c], shape), np.broadcast_to(B[c], shape),
                A[c] + ab[c] * t_ab, np.broadcast_to(C[c], shape),
                A[c] + ac[c] * t_ac, B[c] + cb * t_bc, (A[c] + ab[c] * s_f) + ac[c] * t_f]
        X.append(np.choose(region, cand))
    one = np.ones_like(d1)
    zero = np.zeros_like(d1)
    wa = np.choose(region, [one, zero, 1.0 - t_ab, zero, 1.0 - t_ac, zero, 1.0 - s_f - t_f])
    wb = np.choose(region, [zero, one, t_ab, zero, zero, 1.0 - t_bc, s_f])
    wc = np.choose(region, [zero, zero, zero, one, t_ac, t_bc, t_f])
    return tuple(X), (wa, wb, wc), region


# ------------------------------------------------------------ tagging
def _ranges(g, c, lo, hi, dm):
    """Candidate unwrapped index ranges of lattice c for boxes [lo, hi]
    inflated by dm, with one extra node of margin on each side."""
    ox, oz = COMP_OFFSETS[c]
    ext = g.y_nodes_ext(c)
    e_first = 1
    e_last = g.ny - 1 if c == 1 else g.ny
    i0 = np.floor((lo[:, 0] - dm) / g.dx - ox).astype(np.int64) - 1
    i1 = np.floor((hi[:, 0] + dm) / g.dx - ox).astype(np.int64) + 1
    k0 = np.floor((lo[:, 2] - dm) / g.dz - oz).astype(np.int64) - 1
    k1 = np.floor((hi[:, 2] + dm) / g.dz - oz).astype(np.int64) + 1
    e0 = np.searchsorted(ext, lo[:, 1] - dm, side="left") - 1
    e1 = np.searchsorted(ext, hi[:, 1] + dm, side="right")
    e0 = np.clip(e0, e_first, e_last)
    e1 = np.clip(e1, e_first, e_last)
    return i0, i1, e0, e1, k0, k1


def check_extent(g, verts, tris):
    """Every inflated bounding box must span fewer nodes than the periodic
    length, so that each node has a single image near a triangle."""
    dm = g.delta_max()
    P = verts[tris]
    ex = (P[:, :, 0].max(1) - P[:, :, 0].min(1) + 2 * dm) / g.dx + 4
    ez = (P[:, :, 2].max(1) - P[:, :, 2].min(1) + 2 * dm) / g.dz + 4
    if np.any(ex >= g.nx) or np.any(ez >= g.nz):
        raise ValueError("triangle bounding box too large for the periodic box")


def classify_pairs(g, c, verts, tris, tri_ids, ii, ee, kk):
    """Alg. 1 inner loop for explicit (triangle, node-image) candidate pairs.
    ii, kk are unwrapped lattice indices, ee indices into the lattice's y
    array with walls.  Returns (forcing mask, |N|^2)."""
    ox, oz = COMP_OFFSETS[c]
    ext = g.y_nodes_ext(c)
    T = tris[tri_ids]
    A = tuple(verts[T[:, 0], d] for d in range(3))
    B = tuple(verts[T[:, 1], d] for d in range(3))
    Cv = tuple(verts[T[:, 2], d] for d in range(3))
    px = (ii.astype(np.float64) + ox) * g.dx
    py = ext[ee]
    pz = (kk.astype(np.float64) + oz) * g.dz
    X, _, _ = closest_point((px, py, pz), A, B, Cv)
    N = (px - X[0], py - X[1], pz - X[2])
    n2 = dot3(*N, *N)
    forcing = n2 == 0.0
    neigh = (
        ((ii - 1).astype(np.float64) + ox) * g.dx, py, pz,
        ((ii + 1).astype(np.float64) + ox) * g.dx, py, pz,
        px, ext[ee - 1], pz,
        px, ext[ee + 1], pz,
        px, py, ((kk - 1).astype(np.float64) + oz) * g.dz,
        px, py, ((kk + 1).astype(np.float64) + oz) * g.dz,
    )
    for n in range(6):
        xn = neigh[3 * n:3 * n + 3]
        vn = (xn[0] - X[0], xn[1] - X[1], xn[2] - X[2])
        forcing |= dot3(*vn, *N) < 0.0
    return forcing, n2


def node_index(g, c, ii, ee, kk):
    """Linear index [y][z][x] of the wrapped node."""
    j = ee if c == 1 else ee - 1
    return (j * g.nz + np.mod(kk, g.nz)) * g.nx + np.mod(ii, g.nx)


def tag_pairs(g, c, verts, tris, chunk=4096):
    """All classifying (node, |N|^2, triangle) pairs of lattice c, visiting
    for every triangle the nodes of its inflated bounding box (Alg. 1)."""
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    check_extent(g, verts, tris)
    dm = g.delta_max()
    nodes, dists, owners = [], [], []
    for t0 in range(0, len(tris), chunk):
        tid = np.arange(t0, min(len(tris), t0 + chunk))
        P = verts[tris[tid]]
        i0, i1, e0, e1, k0, k1 = _ranges(g, c, P.min(1), P.max(1), dm)
        ni, ne, nk = i1 - i0 + 1, np.maximum(e1 - e0 + 1, 0), k1 - k0 + 1
        cnt = ni * ne * nk
        if cnt.sum() == 0:
            continue
        tt = np.repeat(tid, cnt)
        local = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        nir, ner = np.repeat(ni, cnt), np.repeat(ne, cnt)
        ii = np.repeat(i0, cnt) + local % nir
        ee = np.repeat(e0, cnt) + (local // nir) % ner
        kk = np.repeat(k0, cnt) + local // (nir * ner)
        f, n2 = classify_pairs(g, c, verts, tris, tt, ii, ee, kk)
        nodes.append(node_index(g, c, ii[f], ee[f], kk[f]))
        dists.append(n2[f])
        owners.append(tt[f])
    if not nodes:
        return np.zeros(0, np.int64), np.zeros(0), np.zeros(0, np.int64)
    return np.concatenate(nodes), np.concatenate(dists), np.concatenate(owners)


def select(nodes, dists, owners):
    """Forcing set and forcing triangle: for each node the classifying
    triangle with the smallest |N|^2, ties to the lowest triangle id.
    Returns (idx int64 ascending, tri int32)."""
    if len(nodes) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int32)
    order = np.lexsort((owners, dists, nodes))
    n = nodes[order]
    first = np.ones(len(n), bool)
    first[1:] = n[1:] != n[:-1]
    return n[first].astype(np.int64), owners[order][first].astype(np.int32)


def tag(g, c, verts, tris):
    """Forcing nodes of lattice c: (sorted idx, forcing triangle)."""
    return select(*tag_pairs(g, c, verts, tris))


def tag_all(g, verts, tris):
    return [tag(g, c, verts, tris) for c in range(3)]


def forcing_mask(g, c, idx):
    m = np.zeros(int(np.prod(g.comp_shape(c))), bool)
    m[idx] = True
    return m.reshape(g.comp_shape(c))


def boundary_cells(g, idx_u, idx_v, idx_w):
    """C_B: cells all six of whose faces carry forcing nodes of their own
    lattice (u at i and i+1, v at j and j+1, w at k and k+1).  Sorted."""
    mu = forcing_mask(g, 0, idx_u)
    mv = forcing_mask(g, 1, idx_v)
    mw = forcing_mask(g, 2, idx_w)
    cb = (mu & np.roll(mu, -1, axis=2) & mv[:-1] & mv[1:]
          & mw & np.roll(mw, -1, axis=1))
    return np.flatnonzero(cb.ravel()).astype(np.int64)


# --------------------------------------------- brute force (for the pins)
def tag_bruteforce(g, c, verts, tris):
    """Every node of lattice c against every triangle at every periodic image
    shift in {-1, 0, 1}^2, with no culling.  Returns the sorted set of forcing
    nodes.  Used only to pin the culled enumeration."""
    ox, oz = COMP_OFFSETS[c]
    jlo, jhi = g.node_j_range(c)
    ext = g.y_nodes_ext(c)
    J, K, I = np.meshgrid(np.arange(jlo, jhi + 1), np.arange(g.nz), np.arange(g.nx),
                          indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    E = J if c == 1 else J + 1
    hit = np.zeros(len(I), bool)
    for t in range(len(tris)):
        tt = np.full(len(I), t)
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                f, _ = classify_pairs(g, c, verts, tris, tt, I + a * g.nx, E, K + b * g.nz)
                hit |= f
    idx = (J * g.nz + K) * g.nx + I
    return np.sort(idx[hit]).astype(np.int64)
