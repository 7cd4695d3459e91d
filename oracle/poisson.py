"""Direct solve of the pressure-correction equation L_c phi = rhs (paper
Eqs. elliptic / elliptic_mod; Sec. 2: "FFTs along the periodic directions, and
the Thomas algorithm ... in the non-periodic direction").

L_c = D G is diagonalised by the discrete Fourier transform in x and z: a
mode (p, m) turns the periodic three-point second differences into the
eigenvalues lambda_x(p) = -(4/dx^2) sin^2(pi p/nx) and
lambda_z(m) = -(4/dz^2) sin^2(pi m/nz), leaving for each mode a tridiagonal
system in y with homogeneous Neumann rows at the walls.

The (0, 0) mode is singular (Neumann at both walls, A24 of the readings);
its first row is replaced by phi_0 = 0 and the solution is then shifted to a
zero volume-weighted mean (reading "gauge").
"""
from __future__ import annotations

import numpy as np

from .linsolve import thomas


def mode_eigenvalues(g):
    p = np.arange(g.nx // 2 + 1)
    m = np.arange(g.nz)
    lx = -(4.0 / (g.dx * g.dx)) * np.sin(np.pi * p / g.nx) ** 2
    lz = -(4.0 / (g.dz * g.dz)) * np.sin(np.pi * m / g.nz) ** 2
    return lx, lz


def solve(g, rhs):
    """phi with L_c phi = rhs (rhs compatible: sum rhs dV = 0), zero
    volume-weighted mean."""
    F = np.fft.rfft(rhs, axis=2)
    F = np.fft.fft(F, axis=1)                     # (ny, nz, nx/2+1)
    lx, lz = mode_eigenvalues(g)
    lam = lz[:, None] + lx[None, :]               # (nz, nx/2+1)
    ny = g.ny
    lo = np.zeros(ny)
    hi = np.zeros(ny)
    lo[1:] = 1.0 / (g.dyc[1:ny] * g.dy[1:])       # couples phi[j-1]
    hi[:-1] = 1.0 / (g.dyc[1:ny] * g.dy[:-1])     # couples phi[j+1]
    a = np.broadcast_to(lo[:, None, None], F.shape).copy()
    c = np.broadcast_to(hi[:, None, None], F.shape).copy()
    b = (-(lo + hi))[:, None, None] + lam[None, :, :]
    b = np.broadcast_to(b, F.shape).copy()
    # gauge of the singular (0, 0) mode: first row -> phi_0 = 0
    a[0, 0, 0] = 0.0
    b[0, 0, 0] = 1.0
    c[0, 0, 0] = 0.0
    F[0, 0, 0] = 0.0
    X = thomas(a, b, c, F)
    phi = np.fft.irfft(np.fft.ifft(X, axis=1), n=g.nx, axis=2)
    dV = g.cell_volume()
    return phi - (phi * dV).sum() / dV.sum()
