"""Vertex positions and velocities at t^n from host-evaluated coefficients
(the wall position X(t) and velocity U(X(t)) of Sec. 2).

Every transcendental is evaluated on the host by the input generators; here
only +, - and * are applied, in the written order, so that any independent
implementation following the same order obtains bit-identical vertices (and
hence bit-identical tags).

rigid:   X = c + R X0,  U = cdot + omega x (X - c)
         coef = [c(3), R(9 row-major), cdot(3), omega(3)]
deform:  X = c + (r0 + f s) d,  U = cdot + (f sdot) d
         per-vertex data [d(3), f], coef = [c(3), r0, s, sdot, cdot(3)]
         (a shape r(theta, t) carried by a centre moving at cdot: the wall
         velocity is the time derivative of X)
"""
from __future__ import annotations

import numpy as np


def rigid(X0, coef):
    X0 = np.asarray(X0, np.float64)
    c, R, cd, om = coef[0:3], coef[3:12], coef[12:15], coef[15:18]
    x0, x1, x2 = X0[:, 0], X0[:, 1], X0[:, 2]
    X = np.empty_like(X0)
    for d in range(3):
        X[:, d] = c[d] + ((R[3 * d] * x0 + R[3 * d + 1] * x1) + R[3 * d + 2] * x2)
    r0, r1, r2 = X[:, 0] - c[0], X[:, 1] - c[1], X[:, 2] - c[2]
    U = np.empty_like(X0)
    U[:, 0] = cd[0] + (om[1] * r2 - om[2] * r1)
    U[:, 1] = cd[1] + (om[2] * r0 - om[0] * r2)
    U[:, 2] = cd[2] + (om[0] * r1 - om[1] * r0)
    return X, U


def deform(data, coef):
    data = np.asarray(data, np.float64)
    c, r0, s, sd, cd = coef[0:3], coef[3], coef[4], coef[5], coef[6:9]
    f = data[:, 3]
    rad = r0 + f * s
    rd = f * sd
    X = np.empty((len(data), 3))
    U = np.empty((len(data), 3))
    for d in range(3):
        X[:, d] = c[d] + rad * data[:, d]
        U[:, d] = cd[d] + rd * data[:, d]
    return X, U


def body_at(body, t):
    """(verts, vel) of a workloads.Body at time t."""
    coef = body.coef(t)
    if body.kind == "rigid":
        return rigid(body.ref, coef)
    return deform(body.ref, coef)


def concat_bodies(parts):
    """Concatenate several bodies [(verts, vel, tris)] into one surface with
    global triangle ids (body offset + local id)."""
    vs, us, ts = [], [], []
    off = 0
    for X, U, T in parts:
        vs.append(X)
        us.append(U)
        ts.append(np.asarray(T, np.int64) + off)
        off += len(X)
    return np.concatenate(vs), np.concatenate(us), np.concatenate(ts)
