"""Pins of the oracle's tridiagonal and Poisson solvers: dense LU on tiny
systems (brute force), the closed-form discrete eigenmodes of L_c (paper
Eq. elliptic with FFT/tridiagonal direct solve, Sec. 2), a discrete
manufactured solution and a dense solve of the whole L_c.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import operators as op
from oracle import poisson
from oracle.grid import Grid
from oracle.linsolve import cyclic, thomas


def _dense(a, b, c, cyc):
    n = len(b)
    M = np.diag(b)
    for i in range(1, n):
        M[i, i - 1] = a[i]
    for i in range(n - 1):
        M[i, i + 1] = c[i]
    if cyc:
        M[0, n - 1] += a[0]
        M[n - 1, 0] += c[n - 1]
    return M


@pytest.mark.parametrize("n", [3, 7, 16, 33])
def test_thomas_matches_dense(rng, n):
    a = rng.uniform(-1, 0, n)
    c = rng.uniform(-1, 0, n)
    b = 2.5 + rng.uniform(0, 1, n)
    d = rng.standard_normal((n, 4))
    x = thomas(a[:, None], b[:, None], c[:, None], d)
    ref = np.linalg.solve(_dense(a, b, c, False), d)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [3, 8, 17])
def test_cyclic_matches_dense(rng, n):
    a = rng.uniform(-1, 0, n)
    c = rng.uniform(-1, 0, n)
    b = 2.5 + rng.uniform(0, 1, n)
    d = rng.standard_normal((n, 3))
    x = cyclic(a[:, None], b[:, None], c[:, None], d)
    ref = np.linalg.solve(_dense(a, b, c, True), d)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-13)


def test_cyclic_with_identity_rows_matches_dense(rng):
    n = 12
    a = np.full(n, -0.3)
    c = np.full(n, -0.3)
    b = np.full(n, 1.6)
    ident = [0, 5, 6]
    for r in ident:
        a[r], b[r], c[r] = 0.0, 1.0, 0.0
    d = rng.standard_normal((n, 2))
    d[ident] = 0.0
    x = cyclic(a[:, None], b[:, None], c[:, None], d)
    ref = np.linalg.solve(_dense(a, b, c, True), d)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-13)
    assert np.all(x[ident] == 0.0)


@pytest.mark.parametrize("p,m,q", [(1, 0, 0), (0, 2, 1), (3, 1, 2), (2, 3, 5)])
def test_poisson_closed_form_eigenmode(p, m, q):
    """Uniform y: cos(2 pi p x/Lx) cos(2 pi m z/Lz) cos(pi q (y+1)/2) at the
    cell centres is an eigenvector of L_c with
    lambda = -(4/dx^2)sin^2(pi p/nx) - (4/dz^2)sin^2(pi m/nz)
             -(4/dy^2)sin^2(pi q/(2 ny));
    solving L_c phi = lambda phi must return phi (zero-mean) to 1e-13."""
    nx, ny, nz = 16, 12, 10
    g = Grid(nx, ny, nz, 2 * np.pi, np.pi, workloads.uniform_faces(ny))
    xc = (np.arange(nx) + 0.5) * g.dx
    zc = (np.arange(nz) + 0.5) * g.dz
    phi = (np.cos(np.pi * q * (g.yc + 1) / 2)[:, None, None]
           * np.cos(2 * np.pi * m * zc / g.lz)[None, :, None]
           * np.cos(2 * np.pi * p * xc / g.lx)[None, None, :])
    lam = (-(4 / g.dx ** 2) * np.sin(np.pi * p / nx) ** 2
           - (4 / g.dz ** 2) * np.sin(np.pi * m / nz) ** 2
           - (4 / g.dy[0] ** 2) * np.sin(np.pi * q / (2 * ny)) ** 2)
    # the stencil itself has this eigenvalue
    assert np.allclose(op.lap_c(g, phi), lam * phi, atol=1e-11 * abs(lam))
    sol = poisson.solve(g, lam * phi)
    assert np.max(np.abs(sol - phi)) <= 1e-13 * max(1.0, np.max(np.abs(phi))) * 10


def test_poisson_manufactured_discrete(rng):
    """Stretched grid, non-power-of-two sizes: random zero-mean phi*,
    rhs = L_c phi*, solve, recover phi*."""
    nx, ny, nz = 20, 15, 12
    g = Grid(nx, ny, nz, 2 * np.pi, np.pi, workloads.tanh_faces(ny, 2.0))
    phi = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    phi -= np.sum(phi * dV) / np.sum(dV)
    sol = poisson.solve(g, op.lap_c(g, phi))
    assert np.max(np.abs(sol - phi)) < 1e-10


def test_poisson_matches_dense_solve(rng):
    """Tiny grid: assemble L_c column by column from the stencil and solve the
    singular system with the zero-mean constraint by least squares."""
    nx, ny, nz = 6, 5, 4
    g = Grid(nx, ny, nz, 1.3, 0.7, workloads.tanh_faces(ny, 1.0))
    n = g.cells
    M = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        M[:, col] = op.lap_c(g, e.reshape(g.shape)).ravel()
    dV = g.cell_volume().ravel()
    rhs = rng.standard_normal(n)
    rhs -= np.sum(rhs * dV) / np.sum(dV)          # compatible
    K = np.vstack([M, dV[None, :]])
    ref = np.linalg.lstsq(K, np.concatenate([rhs, [0.0]]), rcond=None)[0]
    sol = poisson.solve(g, rhs.reshape(g.shape)).ravel()
    assert np.allclose(sol, ref, rtol=1e-10, atol=1e-10)
    assert np.allclose(M @ sol, rhs, atol=1e-9)
