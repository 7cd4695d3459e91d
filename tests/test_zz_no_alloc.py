"""poisson_solve_static, the entry point that allocates nothing (its tables
and spectrum in the library's static device array), against poisson_solve of
an FP64 context on the same right-hand side: two calls in a row, the second on
a smaller grid, within the Poisson tolerance of the parity tests (1e-11 of
max|phi|); a grid larger than the static array is refused."""
import numpy as np
import pytest
import torch

import workloads
from gpu_harness import DEV, n, t
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _compatible_rhs(g, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    return r - np.sum(r * dV) / np.sum(dV)


def _context_solve(ibm, nx, ny, nz, lx, lz, yf, rhs):
    ctx = ibm.Context(nx, ny, nz, lx, lz, yf, 100.0)
    phi = torch.empty(nx * ny * nz, dtype=torch.float64, device=DEV)
    ibm.poisson_solve(ctx, t(rhs), phi)
    assert ibm.ibm_check(ctx) == 0
    out = n(phi).copy()
    ctx.close()
    return out


def test_static_poisson_matches_the_context_solve_on_two_calls():
    from paper_2606_09799_amd import ibm
    cases = [
        # 40 x 30 x 36 stretched (mixed-radix transforms, several segments)
        (40, 30, 36, 2 * np.pi, np.pi, workloads.tanh_faces(30, 1.5), 11),
        # then a smaller uniform grid: the static array keeps the first call's
        # contents, so nothing of it may leak into the second
        (32, 24, 16, 2.0, 1.0, workloads.uniform_faces(24, -0.75, 0.75), 12),
    ]
    for nx, ny, nz, lx, lz, yf, seed in cases:
        g = Grid(nx, ny, nz, lx, lz, yf)
        rhs = _compatible_rhs(g, seed)
        ref = _context_solve(ibm, nx, ny, nz, lx, lz, yf, rhs)
        phi = torch.full((g.cells,), np.nan, dtype=torch.float64, device=DEV)
        ibm.poisson_solve_static(nx, ny, nz, lx, lz, yf, t(rhs), phi)
        torch.cuda.synchronize()
        got = n(phi)
        assert np.all(np.isfinite(got))
        err = np.max(np.abs(got - ref.ravel())) / np.max(np.abs(ref))
        assert err < 1e-11, (nx, ny, nz, err)


def test_static_poisson_refuses_a_grid_beyond_its_array():
    from paper_2606_09799_amd import ibm
    nx = ny = nz = 256  # spectrum 256*256*136*16 bytes > the static array
    yf = workloads.uniform_faces(ny)
    rhs = torch.zeros(nx * ny * nz, dtype=torch.float64, device=DEV)
    phi = torch.zeros_like(rhs)
    with pytest.raises(ibm.IbmError) as e:
        ibm.poisson_solve_static(nx, ny, nz, 1.0, 1.0, yf, rhs, phi)
    assert e.value.code == ibm.IBM_EINVAL
