"""Second-order centred finite-difference operators on the staggered grid
(paper Sec. 2: "second-order accurate centered finite-difference schemes";
Eq. discrete_div for D; L_c = DG in Eq. elliptic; H in conservative form in
Eq. NS_prov; App. A for the discrete divergence theorem).

The paper names these operators but does not print their stencils on a
stretched staggered grid; the stencils below are this implementation's
reading of them (flux-form H with linear face interpolation in y, finite-
volume Laplacian with the wall value at half a cell, D as Eq. discrete_div).  Periodic shifts use np.roll; walls are at the two
y boundaries, where v = 0 and u = w = 0 (no-slip, stationary walls).
"""
from __future__ import annotations

import numpy as np


def xm(a):  # value at i-1
    return np.roll(a, 1, axis=2)


def xp(a):  # value at i+1
    return np.roll(a, -1, axis=2)


def zm(a):  # value at k-1
    return np.roll(a, 1, axis=1)


def zp(a):  # value at k+1
    return np.roll(a, -1, axis=1)


def _col(a):
    return np.asarray(a)[:, None, None]


# ---------------------------------------------------------------- D and G
def divergence(g, u, v, w):
    """Eq. discrete_div on a stretched grid: sum over directions of the face
    difference divided by the cell width, at every cell centre."""
    return ((xp(u) - u) / g.dx
            + (v[1:] - v[:-1]) / _col(g.dy)
            + (zp(w) - w) / g.dz)


def gradient(g, p):
    """G: face-normal differences of a cell-centred field.  The wall-normal
    component is zero on the two wall planes (homogeneous Neumann for the
    pressure, Eq. elliptic)."""
    gu = (p - xm(p)) / g.dx
    gv = np.zeros(g.comp_shape(1))
    gv[1:g.ny] = (p[1:] - p[:-1]) / _col(g.dyc[1:g.ny])
    gw = (p - zm(p)) / g.dz
    return gu, gv, gw


def lap_c(g, phi):
    """L_c = D G (Eq. elliptic), written literally as the composition."""
    return divergence(g, *gradient(g, phi))


# ---------------------------------------------------------- viscous L
def lap_cc(g, a):
    """Viscous Laplacian at u or w nodes (cell-centred in y).  In y the flux
    through face f is (a[f] - a[f-1]) / dyc[f]; at the walls the missing
    neighbour is the wall value 0 at distance dyc[0] (dyc[ny])."""
    lx = ((xp(a) - a) - (a - xm(a))) / (g.dx * g.dx)
    lz = ((zp(a) - a) - (a - zm(a))) / (g.dz * g.dz)
    z = np.zeros((1,) + a.shape[1:])
    ae = np.concatenate((z, a, z), axis=0)                 # ny+2 planes
    flux = (ae[1:] - ae[:-1]) / _col(g.dyc)                  # faces 0..ny
    ly = (flux[1:] - flux[:-1]) / _col(g.dy)
    return lx + ly + lz


def lap_v(g, v):
    """Viscous Laplacian at interior v nodes (faces j = 1..ny-1); the wall
    planes of the result are zero.  In y the flux through the cell centre j is
    (v[j+1] - v[j]) / dy[j]."""
    out = np.zeros_like(v)
    lx = ((xp(v) - v) - (v - xm(v))) / (g.dx * g.dx)
    lz = ((zp(v) - v) - (v - zm(v))) / (g.dz * g.dz)
    flux = (v[1:] - v[:-1]) / _col(g.dy)                     # centres 0..ny-1
    ly = (flux[1:] - flux[:-1]) / _col(g.dyc[1:g.ny])        # faces 1..ny-1
    out[1:g.ny] = lx[1:g.ny] + ly + lz[1:g.ny]
    return out


# ------------------------------------------------------ convective H
def _to_faces(g, a):
    """Linear interpolation of a u/w (cell-centred in y) field to the faces
    f = 0..ny; the wall faces take the wall value 0."""
    out = np.zeros((g.ny + 1,) + a.shape[1:])
    d0, d1 = _col(g.dy[:-1]), _col(g.dy[1:])
    out[1:g.ny] = (a[:-1] * d1 + a[1:] * d0) / (d0 + d1)
    return out


def conv_u(g, u, v, w):
    """H for the x-momentum at u nodes: H_u = -div(u u) in flux form."""
    ub = 0.5 * (u + xp(u))                       # u at cell centres (i+1/2)
    tx = (ub * ub - xm(ub) * xm(ub)) / g.dx
    fy = _to_faces(g, u) * (0.5 * (xm(v) + v))   # (u v) at faces, x = i dx
    ty = (fy[1:] - fy[:-1]) / _col(g.dy)
    fz = (0.5 * (u + zp(u))) * zp(0.5 * (xm(w) + w))   # (u w) at z=(k+1)dz
    tz = (fz - zm(fz)) / g.dz
    return -(tx + ty + tz)


def conv_w(g, u, v, w):
    """H for the z-momentum at w nodes (x and z roles of conv_u swapped)."""
    wb = 0.5 * (w + zp(w))                       # w at cell centres (k+1/2)
    tz = (wb * wb - zm(wb) * zm(wb)) / g.dz
    fy = _to_faces(g, w) * (0.5 * (zm(v) + v))   # (w v) at faces, z = k dz
    ty = (fy[1:] - fy[:-1]) / _col(g.dy)
    fx = (0.5 * (w + xp(w))) * xp(0.5 * (zm(u) + u))   # (w u) at x=(i+1)dx
    tx = (fx - xm(fx)) / g.dx
    return -(tx + ty + tz)


def conv_v(g, u, v, w):
    """H for the y-momentum at interior v nodes; wall planes are zero."""
    ny = g.ny
    out = np.zeros_like(v)
    uy = _to_faces(g, u)[1:ny]                         # u at faces 1..ny-1
    wy = _to_faces(g, w)[1:ny]                         # w at faces 1..ny-1
    vi = v[1:ny]
    fx = xp(uy) * (0.5 * (vi + xp(vi)))                # (u v) at x=(i+1)dx
    tx = (fx - xm(fx)) / g.dx
    vc = 0.5 * (v[:-1] + v[1:])                        # v at centres 0..ny-1
    ty = (vc[1:] * vc[1:] - vc[:-1] * vc[:-1]) / _col(g.dyc[1:ny])
    fz = zp(wy) * (0.5 * (vi + zp(vi)))                # (w v) at z=(k+1)dz
    tz = (fz - zm(fz)) / g.dz
    out[1:ny] = -(tx + ty + tz)
    return out


def conv(g, u, v, w):
    return conv_u(g, u, v, w), conv_v(g, u, v, w), conv_w(g, u, v, w)


def kinetic_energy(g, u, v, w):
    """Cell-centred kinetic energy e = u.u/2 of a staggered field (the e of
    App. B): each component's square averaged over the two faces of the cell
    normal to it (x and z periodic; the v wall faces hold 0)."""
    eu = 0.5 * (u * u + xp(u) * xp(u))
    ev = 0.5 * (v[:-1] * v[:-1] + v[1:] * v[1:])
    ew = 0.5 * (w * w + zp(w) * zp(w))
    return 0.5 * (eu + ev + ew)
