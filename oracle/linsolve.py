"""Tridiagonal solves used by the approximate factorisation and the Poisson
solver (paper Sec. 2: "tridiagonal systems ... solved using the Thomas
algorithm").  The periodic directions give cyclic systems, solved here with
the Sherman-Morrison correction of a Thomas solve (the paper names only
Thomas; the periodic lines are read as cyclic systems).

Lines run along axis 0; any trailing axes are a batch.  a[i], b[i], c[i] are
the sub-, main and super-diagonal of row i; for the cyclic solver a[0]
multiplies x[n-1] and c[n-1] multiplies x[0].
"""
from __future__ import annotations

import numpy as np


def thomas(a, b, c, d):
    """Solve a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i]  (a[0], c[n-1]
    unused).  Coefficients broadcast against d."""
    n = d.shape[0]
    a = np.broadcast_to(a, d.shape)
    b = np.broadcast_to(b, d.shape)
    c = np.broadcast_to(c, d.shape)
    rdt = np.result_type(d, b)
    cp = np.empty(d.shape, dtype=np.result_type(b))
    dp = np.empty(d.shape, dtype=rdt)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.empty(d.shape, dtype=rdt)
    x[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def cyclic(a, b, c, d):
    """Cyclic tridiagonal solve (Sherman-Morrison on top of Thomas)."""
    n = d.shape[0]
    a = np.broadcast_to(a, d.shape).astype(np.float64)
    b = np.broadcast_to(b, d.shape).astype(np.float64)
    c = np.broadcast_to(c, d.shape).astype(np.float64)
    beta = a[0]           # A[0, n-1]
    alpha = c[n - 1]      # A[n-1, 0]
    gamma = -b[0]
    bb = b.copy()
    bb[0] = b[0] - gamma
    bb[n - 1] = b[n - 1] - alpha * beta / gamma
    x = thomas(a, bb, c, d)
    u = np.zeros(d.shape)
    u[0] = gamma
    u[n - 1] = alpha
    z = thomas(a, bb, c, u)
    fact = (x[0] + beta * x[n - 1] / gamma) / (1.0 + z[0] + beta * z[n - 1] / gamma)
    return x - fact * z
