"""Pins of the oracle's rigid-body dynamics (Sec. 4.5's loose coupling: AB2
for Newton's and Euler's equations and the quaternion) against closed
forms, chosen so that a plausible slip fails one of them:

* free flight: c advances by V dt exactly every step;
* a constant force: V^n = V0 + n dt a exactly, and after the Euler start
  c^n = c0 + n dt V0 + a dt^2 (n^2 - 1)/2 (derived independently: a wrong
  AB2 weight or start fails);
* a constant torque about z on a body with equal moments: Omega_z grows by
  M dt / I per step exactly;
* rotation about a principal axis: the quaternion follows (cos, sin) of half
  the angle, with an error that falls as dt^2 (a wrong factor 1/2 fails);
* a spin about the body axis of a turned body, and a world torque on it
  (the quaternion product order, R^T for the torque);
* the torque-free axisymmetric top (I1 = I2 != I3): Omega_3 stays constant
  and (Omega_1, Omega_2) turns at lambda = (I3 - I1) Omega_3 / I1 (the sign
  of the gyroscopic term), again at second order.
"""
import numpy as np

from oracle import rigid


def _run(state, props, F, M, dt, n):
    coefs = []
    for _ in range(n):
        state, coef = rigid.advance(state, props, F, M, dt)
        coefs.append(coef)
    return state, coefs


def test_free_flight_and_constant_force():
    c0, V0 = np.array([0.3, -0.2, 1.1]), np.array([0.5, 0.1, -0.4])
    a = np.array([0.0, -9.81, 0.0])
    m = 2.5
    props = np.array([m, 1.0, 1.0, 1.0, *(m * a), 0.0])
    dt, n = 0.01, 37
    s0 = rigid.initial_state(c0, [1.0, 0.0, 0.0, 0.0], V0, np.zeros(3))
    s, coefs = _run(s0, props, np.zeros(3), np.zeros(3), dt, n)
    assert np.max(np.abs(s[7:10] - (V0 + n * dt * a))) < 1e-13
    cn = c0 + n * dt * V0 + a * dt * dt * (n * n - 1) / 2.0
    assert np.max(np.abs(s[0:3] - cn)) < 1e-12
    assert np.max(np.abs(coefs[-1][0:3] - s[0:3])) == 0.0
    assert np.max(np.abs(coefs[-1][12:15] - s[7:10])) == 0.0
    # no force: straight line
    props0 = np.array([m, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    s, _ = _run(s0, props0, np.zeros(3), np.zeros(3), dt, n)
    assert np.max(np.abs(s[0:3] - (c0 + n * dt * V0))) < 1e-13


def test_constant_torque_about_z():
    I, Mz, dt, n = 0.7, 0.21, 0.02, 25
    props = np.array([1.0, I, I, I, 0.0, 0.0, 0.0, 0.0])
    s0 = rigid.initial_state(np.zeros(3), [1.0, 0.0, 0.0, 0.0], np.zeros(3), np.zeros(3))
    s, coefs = _run(s0, props, np.zeros(3), np.array([0.0, 0.0, Mz]), dt, n)
    assert abs(s[12] - n * dt * Mz / I) < 1e-13
    assert np.max(np.abs(s[10:12])) < 1e-15
    assert abs(coefs[-1][17] - s[12]) < 1e-15          # omega (world) about z


def _spin_error(dt):
    w, T = 2.3, 1.0
    props = np.array([1.0, 1.0, 2.0, 3.0, 0.0, 0.0, 0.0, 0.0])
    s0 = rigid.initial_state(np.zeros(3), [1.0, 0.0, 0.0, 0.0], np.zeros(3), [0.0, 0.0, w])
    s, coefs = _run(s0, props, np.zeros(3), np.zeros(3), dt, int(round(T / dt)))
    exact = np.array([np.cos(0.5 * w * T), 0.0, 0.0, np.sin(0.5 * w * T)])
    R = coefs[-1][3:12].reshape(3, 3)
    assert abs(np.sum(s[3:7] ** 2) - 1.0) < 1e-14
    assert np.max(np.abs(R @ R.T - np.eye(3))) < 1e-14
    return np.max(np.abs(s[3:7] - exact))


def test_rotation_about_a_principal_axis_is_second_order():
    e1, e2 = _spin_error(0.02), _spin_error(0.01)
    assert e1 < 1e-3
    assert 3.5 < e1 / e2 < 4.5


def _top_error(dt):
    I1, I3, w3, T = 1.0, 1.7, 1.9, 1.0
    props = np.array([1.0, I1, I1, I3, 0.0, 0.0, 0.0, 0.0])
    om0 = np.array([0.3, 0.0, w3])
    s0 = rigid.initial_state(np.zeros(3), [1.0, 0.0, 0.0, 0.0], np.zeros(3), om0)
    s, _ = _run(s0, props, np.zeros(3), np.zeros(3), dt, int(round(T / dt)))
    lam = (I3 - I1) * w3 / I1
    # dOm1/dt = -lam Om2, dOm2/dt = lam Om1: (Om1 + i Om2) turns by e^{i lam t}
    exact = 0.3 * np.array([np.cos(lam * T), np.sin(lam * T)])
    assert abs(s[12] - w3) < 1e-14
    return np.max(np.abs(s[10:12] - exact))


def test_torque_free_axisymmetric_top_is_second_order():
    e1, e2 = _top_error(0.02), _top_error(0.01)
    assert e1 < 1e-3
    assert 3.5 < e1 / e2 < 4.5


_QX = np.array([np.cos(np.pi / 4), np.sin(np.pi / 4), 0.0, 0.0])   # 90 degrees about x


def _tilted_spin_error(dt):
    """Spin about the body z axis of a body turned 90 degrees about x: the
    motion is q0 (x) (cos, 0, 0, sin) of half the angle (body-frame angular
    velocity; the other product order turns about the world z axis)."""
    w, T = 2.3, 1.0
    props = np.array([1.0, 1.0, 2.0, 3.0, 0.0, 0.0, 0.0, 0.0])
    s0 = rigid.initial_state(np.zeros(3), _QX, np.zeros(3), [0.0, 0.0, w])
    s, _ = _run(s0, props, np.zeros(3), np.zeros(3), dt, int(round(T / dt)))
    exact = rigid.quat_mul(_QX, [np.cos(0.5 * w * T), 0.0, 0.0, np.sin(0.5 * w * T)])
    return np.max(np.abs(s[3:7] - exact))


def test_spin_of_a_turned_body_is_about_its_own_axis():
    e1, e2 = _tilted_spin_error(0.02), _tilted_spin_error(0.01)
    assert e1 < 1e-3
    assert 3.5 < e1 / e2 < 4.5


def test_world_torque_on_a_turned_body():
    """A world torque about z on a turned body with equal moments: the
    world angular velocity grows along z by M dt / I per step (the torque
    is brought into the body frame by R^T)."""
    I, Mz, dt, n = 0.7, 0.21, 0.02, 25
    props = np.array([1.0, I, I, I, 0.0, 0.0, 0.0, 0.0])
    s0 = rigid.initial_state(np.zeros(3), _QX, np.zeros(3), np.zeros(3))
    s, coefs = _run(s0, props, np.zeros(3), np.array([0.0, 0.0, Mz]), dt, n)
    assert np.max(np.abs(coefs[-1][15:18] - np.array([0.0, 0.0, n * dt * Mz / I]))) < 1e-13
