"""The seeded input recipes (no GPU): the chunked generators reproduce the
plain recipe value for value, so that the full-size workloads are the same
PCG64 streams the small ones are."""
import numpy as np
import pytest

from paper_2606_23698_amd import inputs


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("chunk", [1, 37, 1 << 10])
def test_uniform_chunked_equals_uniform(dtype, chunk):
    a = inputs.uniform((5, 7, 9), 2, dtype)
    b = inputs.uniform_chunked((5, 7, 9), 2, dtype, chunk=chunk)
    assert a.dtype == b.dtype and np.array_equal(a, b)


def test_uniform_draws_real_parts_first():
    x = inputs.uniform((2, 3, 4), 7)
    r = np.random.default_rng(7).uniform(-1.0, 1.0, 48)
    assert np.array_equal(x.real.reshape(-1), r[:24]) and np.array_equal(x.imag.reshape(-1), r[24:])


def test_batch_stream_continues_after_shapes():
    shapes, xs = inputs.batch_inputs(3, 4)
    s2, rng = inputs.batch_shapes(3, 4)
    assert shapes == s2
    for s, x in zip(shapes, xs):
        n = int(np.prod(s))
        assert np.array_equal(x.real.reshape(-1), rng.uniform(-1.0, 1.0, n))
        assert np.array_equal(x.imag.reshape(-1), rng.uniform(-1.0, 1.0, n))
