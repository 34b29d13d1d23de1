"""Quantised roots of unity and double-double twiddles (oracle, test infrastructure only).

The emulated transform multiplies integer data by integer twiddles.  A
twiddle is one quantised root of unity: for the length-N transform and an
exponent t,

    Q(omega_N^t) = ( RNE(2^B cos(2 pi t / N)),  RNE(-2^B sin(2 pi t / N)) )

with B = 52 for the FP64 target (k = 53 signed significand bits, Sec. 2,
Eq. capacity) and B = 23 for the FP32 target (k = 24, Sec. 7).  The fused
second-stage coefficient omega_p^{j1 k1} omega_N^{j1 k2} is quantised as ONE
root omega_N^{j1 (k2 + q k1)} (Sec. 4.1, Eq. twiddle-fusion).  The forward
transform uses omega_N = exp(-2 pi i / N); the conjugate transform negates the
sine column, which is exact because round-to-nearest-even is odd-symmetric.

Values are computed with mpmath at 90 significant digits and rounded from the
exact real number; a tie can only happen where 2^B cos is already an integer.
"""
from functools import lru_cache

import mpmath
import numpy as np

_DPS = 90


def _rne_mp(x):
    """Round an mpmath real to the nearest integer, ties to even."""
    fl = int(mpmath.floor(x))
    d = x - fl
    half = mpmath.mpf(1) / 2
    if d > half:
        return fl + 1
    if d < half:
        return fl
    return fl if fl % 2 == 0 else fl + 1


@lru_cache(maxsize=None)
def quantised_roots(N, bits=52, inverse=False):
    """int64 array [N, 2] of Q(omega_N^t), t = 0..N-1 (forward unless inverse)."""
    out = np.zeros((N, 2), dtype=np.int64)
    with mpmath.workdps(_DPS):
        scale = mpmath.mpf(2) ** bits
        for t in range(N):
            ang = 2 * mpmath.pi * t / N
            c = _rne_mp(scale * mpmath.cos(ang))
            s = _rne_mp(-scale * mpmath.sin(ang))
            out[t, 0] = c
            out[t, 1] = -s if inverse else s
    out.setflags(write=False)
    return out


@lru_cache(maxsize=None)
def dd_twiddles(N, inverse=False):
    """float64 array [N, 4] of exp(-+2 pi i t / N) as (re_hi, re_lo, im_hi, im_lo)."""
    out = np.zeros((N, 4), dtype=np.float64)
    sign = 1 if inverse else -1
    with mpmath.workdps(_DPS):
        for t in range(N):
            ang = 2 * mpmath.pi * t / N
            c = mpmath.cos(ang)
            s = sign * mpmath.sin(ang)
            ch = float(c)
            sh = float(s)
            out[t] = (ch, float(c - ch), sh, float(s - sh))
    out.setflags(write=False)
    return out
