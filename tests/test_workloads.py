"""The seeded input generators: the torch generator of the initial field
(used on the device for the large workloads) gives the numpy generator's
values bit for bit.  CPU only (torch on the CPU)."""
import numpy as np
import pytest

import workloads
from oracle import kinematics


@pytest.mark.parametrize("name", ["tiny", "tiny_plate", "c1"])
def test_torch_initial_field_is_bit_identical(name):
    wl = workloads.config(name)
    a = wl.fields()
    b = wl.fields_torch("cpu")
    for x, y in zip(a, b):
        assert np.array_equal(x.ravel(), y.numpy())


def test_torch_generator_chunks_and_offsets():
    """Counter-based: any range [start, start + n) equals the same slice of
    one long draw."""
    import torch
    full = workloads.splitmix64_uniform(7, 2, 5000)
    part = workloads.splitmix64_uniform_torch(7, 2, 1234, "cpu", start=3000)
    assert np.array_equal(full[3000:4234], part.numpy())
    assert part.dtype == torch.float64


@pytest.mark.parametrize("steps", [20, 92])
def test_batched_bodies_stay_clear_of_the_walls(steps):
    """Every batched simulation's body keeps the wall clearance of its
    generator (radius, probe length and two cells) over the given number of
    steps at its drawn speed; the deforming bodies translate too."""
    import math
    d0 = 1.0 / 32.0
    h = 2.0 * math.sqrt(3.0) * d0
    moving_deform = 0
    for s in range(64):
        wl = workloads.batch_sim(s, steps)
        b = wl.bodies[0]
        X0, _ = kinematics.body_at(b, 0.0)
        X1, U1 = kinematics.body_at(b, steps * wl.dt)
        half = 0.5 * wl.ny * d0
        for X in (X0, X1):
            assert np.max(np.abs(X[:, 1])) + h + 2.0 * d0 <= half + 1e-12, (s, steps)
        if b.kind == "deform" and np.linalg.norm(b.coef(0.0)[6:9]) > 0:
            moving_deform += 1
    assert moving_deform > 0
