"""Pin of the oracle's deforming-body law (the wall position X(t) and the
wall velocity U(X(t)) of Sec. 2): U must be the time derivative of X.  The
coefficients come from the workload generator (the shape
r0 (1 + a Y20 sin(4 pi t)) carried by a centre moving at a constant
velocity); a central difference of X over +-h agrees with U to O(h^2), so a
dropped centre velocity or shape-rate term fails it.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import kinematics


@pytest.mark.parametrize("U", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.7)])
def test_deforming_wall_velocity_is_the_time_derivative(U):
    V, _ = workloads.icosphere(2)
    data = workloads.deform_vertex_data(V, 0.3)
    c0 = (1.0, 0.1, 0.5)
    h = 1e-5
    for t in (0.0, 0.07, 0.31):
        X, Ut = kinematics.deform(data, workloads.deform_coef(t, c0, 0.3, U=U))
        Xp, _ = kinematics.deform(data, workloads.deform_coef(t + h, c0, 0.3, U=U))
        Xm, _ = kinematics.deform(data, workloads.deform_coef(t - h, c0, 0.3, U=U))
        fd = (Xp - Xm) / (2.0 * h)
        # truncation (2 pi f)^3 a r0 h^2 / 6 ~ 1e-8 plus rounding 1e-16/h
        assert np.max(np.abs(fd - Ut)) < 1e-7, t
        # the centre moves with U: the mean vertex velocity of the symmetric
        # icosphere is U plus the mean of the shape rate (f sdot d)
        f = data[:, 3]
        shape_rate = (f[:, None] * data[:, :3]) * workloads.deform_coef(t, c0, 0.3)[5]
        assert np.allclose(Ut - shape_rate, np.asarray(U)[None, :], atol=1e-14, rtol=0)
