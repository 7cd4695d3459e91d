"""Rigid-body dynamics of the loosely coupled FSI (paper Sec. 4.5, with the
loads of Sec. 3.3): Newton's equations for the translation in the inertial
frame, Euler's equations for the rotation in the body's principal frame, the
orientation as a unit quaternion, all advanced by the AB2 scheme (explicit
Euler on the first step) from the hydrodynamic force and torque of the last
fluid step.

Test infrastructure only: plain FP64 numpy.  Readings: the torque is taken
about the body's centre c; an external force Fext (gravity with buoyancy,
given by the caller) is added to the fluid force; the quaternion is
renormalised after each step.  The paper solves the fluid in a frame moving
with the body; that frame is not built: here the body moves through the
fixed channel.

State of one body (RIGID_STATE doubles):
  [0:3] c, [3:7] q = (w, x, y, z), [7:10] V, [10:13] Om (body frame),
  [13:16] dV/dt, [16:19] dOm/dt, [19:22] dc/dt, [22:26] dq/dt of the last
  step, [26] 1 once a step has been taken, [27] unused.
Properties (RIGID_PROPS doubles): m, I1, I2, I3 (principal moments),
  Fext (3), unused.
"""
from __future__ import annotations

import numpy as np

RIGID_STATE = 28
RIGID_PROPS = 8


def quat_mul(a, b):
    """Hamilton product a b of quaternions (w, x, y, z)."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def quat_matrix(q):
    """Rotation matrix (body -> world) of a unit quaternion."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def initial_state(c, q, V, Om):
    s = np.zeros(RIGID_STATE)
    s[0:3], s[3:7], s[7:10], s[10:13] = c, q, V, Om
    return s


def advance(state, props, F, M, dt):
    """One AB2 step of one body from force F and torque M (world frame, M
    about c).  Returns (new state, the 18 coefficients of the rigid motion at
    the new time: c, R (row-major, body -> world), cdot, omega (world))."""
    s = np.array(state, np.float64)
    c, q, V, Om = s[0:3], s[3:7], s[7:10], s[10:13]
    m, I = props[0], np.asarray(props[1:4], np.float64)
    Fext = np.asarray(props[4:7], np.float64)
    R = quat_matrix(q)
    d_now = [(np.asarray(F, np.float64) + Fext) / m,               # Newton
             (R.T @ np.asarray(M, np.float64) - np.cross(Om, I * Om)) / I,  # Euler
             V.copy(),                                             # dc/dt
             0.5 * quat_mul(q, np.array([0.0, Om[0], Om[1], Om[2]]))]  # dq/dt
    d_prev = [s[13:16], s[16:19], s[19:22], s[22:26]]
    started = s[26] != 0.0
    inc = [dt * ((1.5 * a - 0.5 * b) if started else a) for a, b in zip(d_now, d_prev)]
    out = s.copy()
    out[7:10] = V + inc[0]
    out[10:13] = Om + inc[1]
    out[0:3] = c + inc[2]
    qn = q + inc[3]
    out[3:7] = qn / np.sqrt(np.sum(qn * qn))
    out[13:16], out[16:19], out[19:22], out[22:26] = d_now
    out[26] = 1.0
    Rn = quat_matrix(out[3:7])
    coef = np.concatenate([out[0:3], Rn.reshape(9), out[7:10], Rn @ out[10:13]])
    return out, coef
