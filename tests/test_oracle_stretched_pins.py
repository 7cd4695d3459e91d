"""Pins of the oracle's wall-normal stencils on a stretched grid (paper Sec. 2:
second-order centred differences on a grid stretched in y; Eq. NS_prov for
the flux-form H and the viscous L), by closed forms written from the grid
geometry and by exact discrete identities.  Each pin fails if a weight of the
stretched stencils is swapped (dy for dyc, or the two neighbouring cell
heights of a face interpolation).  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import operators as op
from oracle.grid import Grid
from oracle.step import step


def _grid(ny=17, nx=12, nz=10, beta=2.0):
    return Grid(nx, ny, nz, 2.0 * np.pi, np.pi, workloads.tanh_faces(ny, beta))


def _col(a):
    return np.asarray(a)[:, None, None]


@pytest.mark.parametrize("ny", [16, 17])
def test_face_interpolation_is_exact_for_fields_linear_in_y(ny):
    """The y interpolation of a cell-centred value to a face is linear in
    distance: a field a = c0 + c1 y sampled at the centres gives c0 + c1 y_f
    at every interior face, on a tanh grid whose neighbouring cells differ in
    height; the wall faces take the wall value 0."""
    g = _grid(ny)
    a = np.broadcast_to(_col(1.7 - 0.9 * g.yc), g.shape).copy()
    f = op._to_faces(g, a)
    expect = 1.7 - 0.9 * g.yf[1:ny]
    assert np.max(np.abs(f[1:ny] - _col(expect))) <= 1e-14
    assert np.all(f[0] == 0.0) and np.all(f[ny] == 0.0)
    # the grid really is stretched: a plain average would miss by O(dy)
    mid = 0.5 * (g.yc[:-1] + g.yc[1:])
    assert np.max(np.abs(mid - g.yf[1:ny])) > 1e-3


def test_conv_v_wall_normal_flux_telescopes(rng):
    """Summing H_v dV_v over the interior v nodes (dV_v = dx dyc[j] dz): the x
    and z flux differences telescope over the periodic directions and the y
    term (vc[j]^2 - vc[j-1]^2)/dyc[j] telescopes in j, leaving
    sum H_v dV_v = -dx dz sum_{i,k} (vc[ny-1]^2 - vc[0]^2), with vc the
    cell-centre average of v.  Holds for any field."""
    g = _grid(13)
    ny = g.ny
    u = rng.standard_normal(g.shape)
    w = rng.standard_normal(g.shape)
    v = rng.standard_normal(g.comp_shape(1))
    v[0] = v[ny] = 0.0
    Hv = op.conv_v(g, u, v, w)
    dVv = g.dx * g.dz * _col(g.dyc[1:ny])
    lhs = np.sum(Hv[1:ny] * dVv)
    vc_top = 0.5 * (v[ny - 1] + v[ny])
    vc_bot = 0.5 * (v[0] + v[1])
    rhs = -g.dx * g.dz * np.sum(vc_top ** 2 - vc_bot ** 2)
    scale = g.dx * g.dz * np.sum(vc_top ** 2 + vc_bot ** 2)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_conv_v_transverse_fluxes_use_the_face_value_of_u_and_w():
    """u = a0 + a1 y and w = b0 + b1 y (uniform in x and z), v = V(x) Z(z) on
    the interior faces: on the faces j = 2..ny-2 the y term of H_v vanishes
    (vc is the same above and below), and
      -H_v = (a0 + a1 y_f) (V_{i+1} - V_{i-1}) Z_k / (2 dx)
           + (b0 + b1 y_f) V_i (Z_{k+1} - Z_{k-1}) / (2 dz),
    the face value y_f of the linear profiles entering exactly."""
    g = _grid(15)
    ny = g.ny
    a0, a1, b0, b1 = 0.4, 1.3, -0.2, 0.7
    u = np.broadcast_to(_col(a0 + a1 * g.yc), g.shape).copy()
    w = np.broadcast_to(_col(b0 + b1 * g.yc), g.shape).copy()
    xv = (np.arange(g.nx) + 0.5) * g.dx
    zv = (np.arange(g.nz) + 0.5) * g.dz
    V = np.sin(2.0 * np.pi * xv / g.lx)
    Z = np.cos(4.0 * np.pi * zv / g.lz)
    v = np.zeros(g.comp_shape(1))
    v[1:ny] = Z[None, :, None] * V[None, None, :]
    Hv = op.conv_v(g, u, v, w)
    dV = (np.roll(V, -1) - np.roll(V, 1)) / (2.0 * g.dx)
    dZ = (np.roll(Z, -1) - np.roll(Z, 1)) / (2.0 * g.dz)
    j = np.arange(2, ny - 1)
    expect = -((a0 + a1 * g.yf[j])[:, None, None] * (Z[None, :, None] * dV[None, None, :])
               + (b0 + b1 * g.yf[j])[:, None, None] * (dZ[None, :, None] * V[None, None, :]))
    assert np.max(np.abs(Hv[j] - expect)) <= 1e-12


def test_cell_centred_viscous_laplacian_closed_forms():
    """Viscous L at u/w nodes on a stretched grid (flux (a_f - a_{f-1})/dyc[f]
    through face f, the wall value 0 at dyc[0] / dyc[ny]):
      a = c0 + c1 y_c       -> 0 on the rows 1..ny-2;
      a = y_c - y_f[0]      -> 0 on row 0 as well (the profile vanishes at the
                               bottom wall), -2/(dyc[ny] dy[ny-1]) on row ny-1;
      a = y_c^2             -> (y_c[j+1] - y_c[j-1]) / dy[j] on rows 1..ny-2."""
    g = _grid(19)
    ny = g.ny
    one = np.ones((1, g.nz, g.nx))
    L = op.lap_cc(g, _col(0.3 + 2.1 * g.yc) * one)
    assert np.max(np.abs(L[1:ny - 1])) <= 1e-9
    L = op.lap_cc(g, _col(g.yc - g.yf[0]) * one)
    assert np.max(np.abs(L[:ny - 1])) <= 1e-9
    top = -(g.yf[ny] - g.yf[0]) / (g.dyc[ny] * g.dy[ny - 1])
    assert np.max(np.abs(L[ny - 1] - top)) <= 1e-9 * abs(top)
    L = op.lap_cc(g, _col(g.yc ** 2) * one)
    j = np.arange(1, ny - 1)
    expect = (g.yc[j + 1] - g.yc[j - 1]) / g.dy[j]
    assert np.max(np.abs(L[j] - _col(expect))) <= 1e-9
    # on this grid the stretched answer is far from the uniform-grid value 2
    assert np.max(np.abs(expect - 2.0)) > 0.03


def test_face_viscous_laplacian_closed_forms():
    """Viscous L at v nodes (faces) on a stretched grid (flux
    (v_{j+1} - v_j)/dy[j] through the centre j, difference over dyc[j]):
      v = c0 + c1 y_f -> 0 on every interior face;
      v = y_f^2       -> (y_f[j+1] - y_f[j-1]) / dyc[j], which is 2 on any
                         grid (dyc[j] is half of y_f[j+1] - y_f[j-1]), while
                         a divisor dy in place of dyc would give
                         (y_f[j+1] - y_f[j-1]) / dy[j] != 2 on this grid."""
    g = _grid(18)
    ny = g.ny
    one = np.ones((1, g.nz, g.nx))
    L = op.lap_v(g, _col(-0.6 + 1.9 * g.yf) * one)
    assert np.max(np.abs(L[1:ny])) <= 1e-9
    assert np.all(L[0] == 0.0) and np.all(L[ny] == 0.0)
    L = op.lap_v(g, _col(g.yf ** 2) * one)
    j = np.arange(1, ny)
    expect = (g.yf[j + 1] - g.yf[j - 1]) / g.dyc[j]
    assert np.max(np.abs(L[j] - _col(expect))) <= 1e-9
    assert np.max(np.abs(expect - 2.0)) <= 1e-12
    wrong = (g.yf[j + 1] - g.yf[j - 1]) / g.dy[j]
    assert np.max(np.abs(wrong - 2.0)) > 0.03


def _steady_channel_profile(g, re, dpdx):
    """The discrete steady profile of a stretched channel, built by summing
    fluxes: in steady parallel flow every cell balances its viscous fluxes
    against the driving gradient, F_{f+1} - F_f = re dpdx dy[f], so
    F_f = F_0 + re dpdx (y_f[f] - y_f[0]); the velocity is the running sum
    u_j = sum_{f <= j} F_f dyc[f] from the bottom wall (distances dyc between
    consecutive values, the first one from the wall), and the top wall value
    0 fixes F_0 = -re dpdx sum_f (y_f[f] - y_f[0]) dyc[f] / sum_f dyc[f]."""
    s = g.yf - g.yf[0]
    F0 = -re * dpdx * np.sum(s * g.dyc) / np.sum(g.dyc)
    F = F0 + re * dpdx * s                      # faces 0..ny
    return np.cumsum(F[:g.ny] * g.dyc[:g.ny])  # centres 0..ny-1


def test_steady_stretched_channel_is_a_fixed_point_of_the_step():
    """No body, a stretched grid: the discrete steady profile (from the flux
    sums above, not from the oracle's solver coefficients) is left unchanged
    by a full RK2 step with v = w = 0 (H = 0 and D u = 0 for a parallel flow);
    this pins the viscous y stencil, the sign and time weight of the driving
    force and the wall treatment together."""
    g = _grid(24, nx=8, nz=6)
    re, dpdx = 100.0, -2.0 / 100.0
    prof = _steady_channel_profile(g, re, dpdx)
    # the flux construction closes at the top wall
    top = prof[-1] + (re * dpdx * (g.yf[g.ny] - g.yf[0])
                      - re * dpdx * np.sum((g.yf - g.yf[0]) * g.dyc) / np.sum(g.dyc)) * g.dyc[g.ny]
    assert abs(top) < 1e-12
    u = np.broadcast_to(_col(prof), g.shape).copy()
    v = np.zeros(g.comp_shape(1))
    w = np.zeros(g.shape)
    p = np.zeros(g.shape)
    empty = (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int64))
    (u2, v2, w2), p2, _, _ = step(g, (u, v, w), p, empty, 0.01, re, (-dpdx, 0, 0))
    assert np.max(np.abs(u2 - u)) < 1e-13
    assert np.max(np.abs(v2)) < 1e-13 and np.max(np.abs(w2)) < 1e-13
    # and it is not the parabola sampled at the centres (wall cells differ)
    assert np.max(np.abs(prof - (1.0 - g.yc ** 2))) > 1e-4
