"""The seeded input generators: the torch generator of the initial field
(used on the device for the large workloads) gives the numpy generator's
values bit for bit.  CPU only (torch on the CPU)."""
import numpy as np
import pytest

import workloads


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
