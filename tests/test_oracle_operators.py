"""Pins of the oracle's finite-difference operators against exact discrete
identities (paper App. A discrete divergence theorem; conservative H of
Eq. NS_prov; L_c = DG of Eq. elliptic) and exactness on low-order
polynomials.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import operators as op
from oracle.grid import Grid


def _grid(nx=12, ny=9, nz=10, stretched=True):
    yf = workloads.tanh_faces(ny, 1.7) if stretched else workloads.uniform_faces(ny)
    return Grid(nx, ny, nz, 2.0 * np.pi, np.pi, yf)


def _rand_fields(g, rng):
    u = rng.standard_normal(g.shape)
    v = rng.standard_normal(g.comp_shape(1))
    v[0] = 0.0
    v[-1] = 0.0
    w = rng.standard_normal(g.shape)
    return u, v, w


@pytest.mark.parametrize("stretched", [False, True])
def test_discrete_divergence_theorem(rng, stretched):
    """App. A: sum_c D u dV equals the net boundary flux, which is 0 for a
    periodic box with impermeable walls, for ANY field."""
    g = _grid(stretched=stretched)
    u, v, w = _rand_fields(g, rng)
    D = op.divergence(g, u, v, w)
    dV = g.cell_volume()
    tot = np.sum(D * dV)
    assert abs(tot) <= 1e-13 * np.sum(np.abs(D) * dV)
    # with a through-flow at the walls the sum equals the wall flux
    v2 = v.copy()
    v2[-1] = rng.standard_normal(v2[-1].shape)
    D2 = op.divergence(g, u, v2, w)
    flux = np.sum(v2[-1]) * g.dx * g.dz
    assert abs(np.sum(D2 * dV) - flux) <= 1e-12 * (abs(flux) + 1)


def test_divergence_exact_on_linear_fields():
    g = _grid()
    X = np.arange(g.nx) * g.dx
    # u = 3 x is not periodic; use the z-only and y-only parts for exactness
    u = np.zeros(g.shape)
    v = np.broadcast_to((2.0 * g.yf)[:, None, None], g.comp_shape(1)).copy()
    w = np.zeros(g.shape)
    D = op.divergence(g, u, v, w)
    assert np.allclose(D, 2.0, rtol=0, atol=1e-12)
    del X


@pytest.mark.parametrize("stretched", [False, True])
def test_convective_flux_form_conserves_momentum(rng, stretched):
    """Conservative H (Eq. NS_prov; Morinishi's fully conservative form): the
    x- and z-momentum fluxes telescope, so sum H_u dV_u = sum H_w dV_w = 0 for
    any field with v = 0 at the walls."""
    g = _grid(stretched=stretched)
    u, v, w = _rand_fields(g, rng)
    Hu, Hv, Hw = op.conv(g, u, v, w)
    dV = g.cell_volume()
    scale = np.sum(np.abs(u) ** 2 * dV)
    assert abs(np.sum(Hu * dV)) <= 1e-13 * scale
    assert abs(np.sum(Hw * dV)) <= 1e-13 * scale
    assert np.all(Hv[0] == 0) and np.all(Hv[-1] == 0)


def test_convective_term_uniform_flow_is_zero():
    g = _grid()
    u = np.full(g.shape, 1.3)
    v = np.zeros(g.comp_shape(1))
    w = np.full(g.shape, -0.4)
    Hu, Hv, Hw = op.conv(g, u, v, w)
    # away from the walls a uniform field carries no momentum flux divergence
    assert np.allclose(Hu, 0, atol=1e-13)
    assert np.allclose(Hw, 0, atol=1e-13)
    assert np.allclose(Hv, 0, atol=1e-13)


def test_convective_term_single_mode():
    """u = sin(x) only: -H_u = d(u^2)/dx discretised as the difference of
    squared cell averages; check against the closed form of that stencil."""
    g = _grid(nx=16)
    x = np.arange(g.nx) * g.dx
    u = np.broadcast_to(np.sin(x), g.shape).copy()
    v = np.zeros(g.comp_shape(1))
    w = np.zeros(g.shape)
    Hu = op.conv_u(g, u, v, w)
    ub_p = 0.5 * (np.sin(x) + np.sin(x + g.dx))
    ub_m = 0.5 * (np.sin(x - g.dx) + np.sin(x))
    expect = -(ub_p ** 2 - ub_m ** 2) / g.dx
    assert np.allclose(Hu, expect[None, None, :], atol=1e-13)


@pytest.mark.parametrize("stretched", [False, True])
def test_lap_c_is_self_adjoint_and_negative(rng, stretched):
    """L_c = DG with Neumann walls is symmetric in the dV-weighted inner
    product and negative semi-definite (constants in its kernel)."""
    g = _grid(stretched=stretched)
    a = rng.standard_normal(g.shape)
    b = rng.standard_normal(g.shape)
    dV = g.cell_volume()
    lab = np.sum(a * op.lap_c(g, b) * dV)
    lba = np.sum(b * op.lap_c(g, a) * dV)
    assert abs(lab - lba) <= 1e-12 * (abs(lab) + 1)
    assert np.sum(a * op.lap_c(g, a) * dV) < 0
    assert np.allclose(op.lap_c(g, np.full(g.shape, 2.5)), 0.0, atol=1e-10)


def test_viscous_laplacian_dirichlet_eigenmode():
    """On a uniform y grid the cell-centred Laplacian with the wall value 0 at
    half a cell equals the antisymmetric-ghost stencil, whose eigenvectors are
    the DST-II modes sin(pi q (j+1/2)/ny) with eigenvalue
    -(4/dy^2) sin^2(pi q/(2 ny)); x and z modes add -(4/h^2) sin^2(pi k/n)."""
    g = _grid(nx=8, ny=12, nz=6, stretched=False)
    dy = g.dy[0]
    for q in (1, 3, 7):
        x = np.arange(g.nx) * g.dx
        z = (np.arange(g.nz) + 0.5) * g.dz
        yy = np.sin(np.pi * q * (np.arange(g.ny) + 0.5) / g.ny)
        u = yy[:, None, None] * np.sin(2 * np.pi * z / g.lz)[None, :, None] \
            * np.sin(2 * np.pi * x / g.lx)[None, None, :]
        lam = (-(4 / dy ** 2) * np.sin(np.pi * q / (2 * g.ny)) ** 2
               - (4 / g.dx ** 2) * np.sin(np.pi / g.nx) ** 2
               - (4 / g.dz ** 2) * np.sin(np.pi / g.nz) ** 2)
        assert np.allclose(op.lap_cc(g, u), lam * u, atol=1e-11 * abs(lam))


def test_viscous_laplacian_v_exact_on_quadratic():
    """At interior faces the v Laplacian is exact for a quadratic in y on a
    stretched grid only where the two cell heights agree; on a uniform grid it
    is exact everywhere: check -2 for v = 1 - y^2."""
    g = _grid(stretched=False)
    v = np.broadcast_to((1 - g.yf ** 2)[:, None, None], g.comp_shape(1)).copy()
    v[0] = v[-1] = 0.0   # walls: 1 - 1 = 0 anyway
    L = op.lap_v(g, v)
    assert np.allclose(L[1:-1], -2.0, atol=1e-10)
