"""Seeded synthetic inputs shared by the tests, the bench and the oracle runs.

Holds no arithmetic of the method.  Recipes (numpy PCG64 streams, C order,
all real parts drawn before all imaginary parts):

* uniform(shape, seed):   Re, Im i.i.d. U[-1, 1)  (32^3 seed 0, 1024^3 seed 2,
  512^3 seed 4, batch members seed 3) -- stands in for the paper's
  well-conditioned 1024^3 field;
* wide_range(shape, seed): sign * 2^u * exp(i phi), u ~ U[-20, 20],
  sign = +-1, phi ~ U[0, 2 pi)  (256^3 seed 1);
* batch_shapes(seed=3): 64 shapes, each extent drawn from
  {64, 96, 128, 192, 256}, then the member inputs from the same stream.

``uniform_chunked`` and ``uniform_to_device`` produce exactly ``uniform``'s
values (the same PCG64 stream, consumed in order) in bounded-size pieces, for
the 1024^3 and 512^3 workloads: the first builds the host array, the second
fills a device tensor without holding the whole array on the host.
``device_uniform`` draws the same distribution with torch's seeded device
generator (not the host stream) for auxiliary inputs that no oracle reads.
"""
import numpy as np

BATCH_EXTENTS = (64, 96, 128, 192, 256)


def uniform(shape, seed, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, shape)
    im = rng.uniform(-1.0, 1.0, shape)
    out = np.empty(shape, dtype=np.complex128)
    out.real = re
    out.imag = im
    return out.astype(dtype)


_CHUNK = 1 << 24


def _stream_parts(shape, seed, chunk, rng=None):
    """Yields (part, start, values): part 0 = real parts, 1 = imaginary parts,
    C order, in the order uniform() draws them (from `rng` if given, else a
    fresh stream of `seed`)."""
    n = int(np.prod(shape))
    rng = np.random.default_rng(seed) if rng is None else rng
    for part in (0, 1):
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            yield part, a, rng.uniform(-1.0, 1.0, b - a)


def uniform_chunked(shape, seed, dtype=np.complex128, chunk=_CHUNK):
    """uniform(shape, seed) built chunk by chunk (identical values)."""
    out = np.empty(int(np.prod(shape)), dtype=dtype)
    for part, a, v in _stream_parts(shape, seed, chunk):
        if part == 0:
            out.real[a:a + len(v)] = v
        else:
            out.imag[a:a + len(v)] = v
    return out.reshape(shape)


def uniform_to_device(shape, seed, device="cuda", dtype=None, chunk=_CHUNK, rng=None):
    """A device tensor holding uniform(shape, seed) (identical values), filled
    chunk by chunk from the host stream."""
    import torch
    dtype = dtype or torch.complex128
    x = torch.empty(tuple(shape), dtype=dtype, device=device)
    xr = torch.view_as_real(x).view(-1, 2)
    real_dtype = torch.float64 if dtype == torch.complex128 else torch.float32
    for part, a, v in _stream_parts(shape, seed, chunk, rng):
        xr[a:a + len(v), part].copy_(torch.from_numpy(v).to(real_dtype))
    return x


def batch_to_device(seed=3, count=64, device="cuda"):
    """batch_inputs(seed, count) as device tensors (identical values)."""
    shapes, rng = batch_shapes(seed, count)
    return shapes, [uniform_to_device(s, None, device, rng=rng) for s in shapes]


def wide_range(shape, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-20.0, 20.0, shape)
    sign = rng.choice(np.array([-1.0, 1.0]), size=shape)
    phi = rng.uniform(0.0, 2.0 * np.pi, shape)
    mag = sign * np.exp2(u)
    out = np.empty(shape, dtype=np.complex128)
    out.real = mag * np.cos(phi)
    out.imag = mag * np.sin(phi)
    return out


def batch_shapes(seed=3, count=64):
    rng = np.random.default_rng(seed)
    ext = rng.choice(np.array(BATCH_EXTENTS), size=(count, 3))
    return [tuple(int(v) for v in row) for row in ext], rng


def batch_inputs(seed=3, count=64):
    shapes, rng = batch_shapes(seed, count)
    xs = []
    for s in shapes:
        re = rng.uniform(-1.0, 1.0, s)
        im = rng.uniform(-1.0, 1.0, s)
        x = np.empty(s, dtype=np.complex128)
        x.real = re
        x.imag = im
        xs.append(x)
    return shapes, xs


def device_uniform(shape, seed, device="cuda", dtype=None):
    import torch
    dtype = dtype or torch.complex128
    real_dtype = torch.float64 if dtype == torch.complex128 else torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.empty(tuple(shape) + (2,), dtype=real_dtype, device=device)
    x[..., 0].uniform_(-1.0, 1.0, generator=g)
    x[..., 1].uniform_(-1.0, 1.0, generator=g)
    return torch.view_as_complex(x)
