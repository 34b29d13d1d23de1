"""Pins of the double-double sampled-line mode of the accuracy oracle (no GPU).

The sampled-line mode evaluates one final-axis output line of a 3-D DFT from
its cost cone (one output of every first-axis line, then of every
second-axis line, then the whole third-axis line), without rounding to
binary64 between the axes.  It is checked against the textbook DFT in mpmath
and against the full double-double transform (itself pinned to mpmath).
"""
import mpmath
import numpy as np

from oracle import exact as ox


def _mp_line(x, k2, k3, sign=-1):
    """X[:, k2, k3] of the separable DFT, evaluated in mpmath from the definition."""
    mpmath.mp.dps = 40
    n1, n2, n3 = x.shape

    def w(n, t):
        return mpmath.expj(sign * 2 * mpmath.pi * t / n)
    s = [sum(mpmath.mpc(complex(x[i, j, k])) * w(n2, j * k2) * w(n3, k * k3)
             for j in range(n2) for k in range(n3)) for i in range(n1)]
    return [sum(s[i] * w(n1, i * k1) for i in range(n1)) for k1 in range(n1)]


def test_cone_against_mpmath_definition():
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, (6, 5, 7)) + 1j * rng.uniform(-1, 1, (6, 5, 7))
    samples = [(0, 0), (4, 6), (2, 3)]
    got = ox.dd_cone_lines(x, samples)
    for k2, k3 in samples:
        ref = _mp_line(x, k2, k3)
        hi, lo = got[(k2, k3)]
        for k1 in range(6):
            err = abs(mpmath.mpc(complex(hi[k1])) + mpmath.mpc(complex(lo[k1])) - ref[k1])
            assert err < 1e-28, (k2, k3, k1, err)


def test_cone_inverse_against_mpmath_definition():
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, (4, 3, 8)) + 1j * rng.uniform(-1, 1, (4, 3, 8))
    hi, lo = ox.dd_cone_lines(x, [(1, 5)], inverse=True)[(1, 5)]
    ref = _mp_line(x, 1, 5, sign=+1)
    for k1 in range(4):
        assert abs(mpmath.mpc(complex(hi[k1])) + mpmath.mpc(complex(lo[k1])) - ref[k1]) < 1e-28


def test_cone_equals_full_double_double_transform():
    rng = np.random.default_rng(13)
    x = rng.uniform(-1, 1, (16, 12, 32)) + 1j * rng.uniform(-1, 1, (16, 12, 32))
    fhi, flo = ox.fft3_dd(x)
    samples = [(0, 0), (11, 31), (5, 16), (7, 16)]
    for (k2, k3), (hi, lo) in ox.dd_cone_lines(x, samples).items():
        # same value to double-double precision (the summation orders differ)
        d = (hi - fhi[:, k2, k3]) + (lo - flo[:, k2, k3])
        assert np.max(np.abs(d)) < 1e-27 * np.max(np.abs(fhi))


def test_cone_single_tone_closed_form():
    # x = exp(+2 pi i (j1 a + j2 b + j3 c)/n): the DFT is n1 n2 n3 at (a, b, c), 0 elsewhere
    n1, n2, n3 = 8, 4, 16
    a, b, c = 3, 1, 5
    j1, j2, j3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    x = np.exp(2j * np.pi * (j1 * a / n1 + j2 * b / n2 + j3 * c / n3))
    got = ox.dd_cone_lines(x, [(b, c), (0, c)])
    hi, _ = got[(b, c)]
    assert abs(hi[a] - n1 * n2 * n3) < 1e-11
    assert np.max(np.abs(np.delete(hi, a))) < 1e-11
    assert np.max(np.abs(got[(0, c)][0])) < 1e-11
