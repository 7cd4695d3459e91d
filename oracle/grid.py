"""Staggered channel grid (paper Sec. 2 and Fig. 1).

The paper's box is periodic and uniform in x1, x2 and stretched in x3 between
two walls.  Here the periodic directions are x (streamwise) and z (spanwise)
and the wall-normal direction is y, with walls at y_f[0] and y_f[ny].
Pressure sits at cell centres and each velocity component on the faces normal
to it.  Arrays are laid out [y][z][x] (numpy shape (ny, nz, nx)); v carries
the two wall planes, shape (ny+1, nz, nx).
"""
from __future__ import annotations

import numpy as np

# lattice of each velocity component: (x offset, z offset) in cell units
COMP_OFFSETS = {0: (0.0, 0.5), 1: (0.5, 0.5), 2: (0.5, 0.0)}


class Grid:
    """Grid metrics (Sec. 2: uniform dx1, dx2; variable dx3^k).

    dx, dz     periodic spacings  L/n
    yf[0..ny]  face heights (caller-supplied, strictly increasing)
    yc[j]      cell-centre heights (yf[j] + yf[j+1]) / 2
    dy[j]      cell heights yf[j+1] - yf[j]
    dyc[j]     distance between the u/w nodes around face j; at the walls the
               distance from the first/last centre to the wall
    """

    def __init__(self, nx, ny, nz, lx, lz, y_faces):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.lz = float(lx), float(lz)
        yf = np.array(y_faces, dtype=np.float64)
        if yf.shape != (ny + 1,) or not np.all(np.diff(yf) > 0):
            raise ValueError("y_faces must hold ny+1 strictly increasing values")
        self.yf = yf
        self.dx = self.lx / self.nx
        self.dz = self.lz / self.nz
        self.yc = (yf[:-1] + yf[1:]) * 0.5
        self.dy = yf[1:] - yf[:-1]
        dyc = np.empty(ny + 1)
        dyc[0] = self.yc[0] - yf[0]
        dyc[1:ny] = self.yc[1:] - self.yc[:-1]
        dyc[ny] = yf[ny] - self.yc[ny - 1]
        self.dyc = dyc

    # shapes -------------------------------------------------------------
    @property
    def shape(self):
        return (self.ny, self.nz, self.nx)

    def comp_shape(self, c):
        return (self.ny + 1, self.nz, self.nx) if c == 1 else self.shape

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    def cell_volume(self):
        """Delta V per cell, broadcastable to (ny, nz, nx)."""
        return (self.dx * self.dz) * self.dy[:, None, None] * np.ones((1, self.nz, self.nx))

    # node coordinates (Fig. 1b) ----------------------------------------
    def y_nodes_ext(self, c):
        """Heights of the y-lattice of component c including the two wall
        points, so that a node's y-neighbours are ext[e-1], ext[e+1]:
        u, w: [yf[0], yc[0..ny-1], yf[ny]], node j <-> ext index j+1;
        v:    yf[0..ny],                     node j <-> ext index j."""
        if c == 1:
            return self.yf.copy()
        return np.concatenate(([self.yf[0]], self.yc, [self.yf[-1]]))

    def node_j_range(self, c):
        """Valid (unknown) j indices of component c: v excludes the walls."""
        return (1, self.ny - 1) if c == 1 else (0, self.ny - 1)

    def ext_index(self, c, j):
        return j if c == 1 else j + 1

    def delta_max(self):
        """Largest distance between a node and any of its six same-lattice
        neighbours, over all three lattices."""
        return max(self.dx, self.dz, float(self.dyc.max()), float(self.dy.max()))

    def local_dy(self, c, j):
        """Wall-normal size of the local cell around a node of component c
        (u, w: the cell height dy[j]; v: the distance dyc[j] between the
        centres around face j)."""
        return self.dyc[j] if c == 1 else self.dy[j]
