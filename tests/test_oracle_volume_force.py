"""Pin of the oracle's volume force (the forces that Sec. 4.2 and 4.3 add
to Eq. NS_prov, here F_c = f0 + kappa u_c, explicit like the driving
gradient): a uniform streamwise flow with no body, no viscosity (Re -> inf:
the CN factors are the identity) and v = w = 0 has H = 0, a divergence-free
predictor (phi = 0) and wall terms that vanish with 1/Re, so every RK2
sub-stage is one explicit Euler step of u' = f0 + kappa u over alpha dt.
The closed form after two steps fails for a force taken at the wrong time
level, weighted by gamma instead of alpha, or applied twice."""
import numpy as np

import workloads
from oracle.grid import Grid
from oracle.step import SCHEMES, step


def test_linear_volume_force_is_explicit_euler_per_substage():
    g = Grid(8, 8, 8, 1.0, 1.0, workloads.uniform_faces(8))
    u0 = 0.37
    fields = [np.full(g.shape, u0), np.zeros(g.comp_shape(1)), np.zeros(g.shape)]
    p = np.zeros(g.shape)
    f0, kap, dt = 0.7, -3.0, 0.05
    kappa = [np.full(g.shape, kap), None, None]
    fext = (np.full(g.shape, f0), 0.0, 0.0)
    surface = (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int64))
    u = u0
    for _ in range(2):
        fields, p, _, _ = step(g, fields, p, surface, dt, 1e300, fext, kappa=kappa)
        for gamma, rho in SCHEMES["rk2"]:
            u = u + (gamma + rho) * dt * (f0 + kap * u)
    assert np.max(np.abs(fields[0] - u)) < 1e-14
    assert np.max(np.abs(fields[1])) < 1e-14 and np.max(np.abs(fields[2])) < 1e-14
