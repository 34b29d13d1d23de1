"""ctypes front end of the C oracle (test infrastructure only).

``fft3_exact``  -- ORACLE-X: the exact-pipeline transform (exact.c)
``fft3_dd``     -- ORACLE-DD: the double-double separable DFT (dd.c)
``dd_cone_lines`` -- ORACLE-DD on sampled final-axis lines of a large
                   transform (the cost cone of each line, in double-double)
``line_stage``  -- one stage of one line with the exact Re/Im integers, the
                   column exponents and the packed outputs (checkpoints)
``pack``        -- the single correctly rounded conversion, exposed for pins
"""
import ctypes
import os

import numpy as np

from . import build as _build
from . import roots as _roots

_lib = None
_I64P = ctypes.POINTER(ctypes.c_int64)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        # OBFFT_ORACLE_LIB: another build of the same sources (the host
        # sanitizer test loads an instrumented one)
        path = os.environ.get("OBFFT_ORACLE_LIB") or _build.ensure_built()
        L = ctypes.CDLL(path)
        L.oracle_fft3.restype = ctypes.c_int
        L.oracle_fft3.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _I64P, _I64P, _I64P, _IP,
                                  ctypes.POINTER(_I64P), ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_line_stage.restype = ctypes.c_int
        L.oracle_line_stage.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, _I64P, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, _I64P, _U64P, _I64P, _U64P, _IP]
        L.oracle_dd_fft3.restype = ctypes.c_int
        L.oracle_dd_fft3.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _I64P,
                                     ctypes.POINTER(_DP), ctypes.c_int]
        L.oracle_lines.restype = ctypes.c_int
        L.oracle_lines.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int64, _I64P, ctypes.c_int, ctypes.c_int]
        L.oracle_lines_at.restype = ctypes.c_int
        L.oracle_lines_at.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, _I64P, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int]
        L.oracle_dd_lines_at.restype = ctypes.c_int
        L.oracle_dd_lines_at.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, _DP, ctypes.c_int]
        L.oracle_dd_lines.restype = ctypes.c_int
        L.oracle_dd_lines.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, _DP]
        L.oracle_pack_hilo.restype = ctypes.c_double
        L.oracle_pack_hilo.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a, t):
    return a.ctypes.data_as(t)


def fft3_exact(x, pq, order=(2, 1, 0), precision=0, inverse=False, final_shift=0,
               nthreads=None):
    """Exact-pipeline transform of complex array x (shape (n1, n2, n3)).

    pq: ((p1, q1), (p2, q2), (p3, q3)) per axis; order: axes in execution order
    (0 = n1); precision 0 = FP64 target, 1 = FP32 target; inverse selects the
    conjugate roots; final_shift is added to the exponent of the last pack.
    Returns complex128 (FP64 target) or complex64 (FP32 target).
    """
    x = np.asarray(x)
    shape = x.shape
    assert len(shape) == 3
    work = np.ascontiguousarray(x.astype(np.complex128))
    out = np.empty_like(work)
    n = np.array(shape, dtype=np.int64)
    p = np.array([a for a, _ in pq], dtype=np.int64)
    q = np.array([b for _, b in pq], dtype=np.int64)
    ordr = np.array(order, dtype=np.intc)
    bits = 52 if precision == 0 else 23
    tabs = [np.ascontiguousarray(_roots.quantised_roots(int(N), bits, inverse)) for N in shape]
    arr = (_I64P * 3)(*[_ptr(t, _I64P) for t in tabs])
    rc = lib().oracle_fft3(work.ctypes.data, out.ctypes.data, _ptr(n, _I64P), _ptr(p, _I64P),
                           _ptr(q, _I64P), _ptr(ordr, _IP), arr, precision, final_shift,
                           nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_fft3 rejected the factorisation")
    if precision == 1:
        return out.astype(np.complex64)
    return out


def fft3_dd(x, inverse=False, nthreads=None):
    """Double-double DFT; returns (hi, lo) complex128 arrays with value hi + lo."""
    x = np.ascontiguousarray(np.asarray(x).astype(np.complex128))
    shape = x.shape
    out = np.empty(shape + (4,), dtype=np.float64)
    n = np.array(shape, dtype=np.int64)
    tabs = [np.ascontiguousarray(_roots.dd_twiddles(int(N), inverse)) for N in shape]
    arr = (_DP * 3)(*[_ptr(t, _DP) for t in tabs])
    lib().oracle_dd_fft3(x.ctypes.data, out.ctypes.data, _ptr(n, _I64P), arr,
                         nthreads or default_threads())
    hi = out[..., 0] + 1j * out[..., 2]
    lo = out[..., 1] + 1j * out[..., 3]
    return hi, lo


def _to_dd(x):
    """complex128 array -> float64 [..., 4] double-double (re_hi, re_lo, im_hi, im_lo)."""
    x = np.asarray(x, dtype=np.complex128)
    d = np.zeros(x.shape + (4,), dtype=np.float64)
    d[..., 0] = x.real
    d[..., 2] = x.imag
    return d


def dd_lines_at(xd, N, k, inverse=False, nthreads=None):
    """Output position k of the double-double DFT of every contiguous length-N
    line of xd: float64 [..., N, 4] double-double values, or complex [..., N]
    binary64 values.  Returns float64 [..., 4]."""
    if np.iscomplexobj(xd):
        xd = np.ascontiguousarray(xd, dtype=np.complex128)
        assert xd.shape[-1] == N
        in_z, lead = 1, xd.shape[:-1]
    else:
        xd = np.ascontiguousarray(xd, dtype=np.float64)
        assert xd.shape[-2:] == (N, 4)
        in_z, lead = 0, xd.shape[:-2]
    nl = int(np.prod(lead))
    out = np.empty(lead + (4,), dtype=np.float64)
    tw = np.ascontiguousarray(_roots.dd_twiddles(int(N), inverse))
    rc = lib().oracle_dd_lines_at(xd.ctypes.data, in_z, out.ctypes.data, nl, N, k, _ptr(tw, _DP),
                                  nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad position")
    return out


def dd_lines(xd, N, inverse=False):
    """The whole double-double DFT of every contiguous length-N line of xd (float64 [..., N, 4])."""
    xd = np.ascontiguousarray(xd, dtype=np.float64)
    assert xd.shape[-2:] == (N, 4)
    out = np.empty_like(xd)
    tw = np.ascontiguousarray(_roots.dd_twiddles(int(N), inverse))
    lib().oracle_dd_lines(xd.ctypes.data, out.ctypes.data, xd.size // (4 * N), N, _ptr(tw, _DP))
    return out


def dd_cone_lines(x, samples, inverse=False, nthreads=None):
    """ORACLE-DD on sampled lines along axis 0 of the 3-D DFT of x (n1, n2, n3).

    samples: iterable of (k2, k3).  Line (k2, k3) is X[:, k2, k3]; it depends
    on every input: output k3 of all n1 n2 axis-3 lines, then output k2 of
    the n1 axis-2 lines, then the whole axis-1 transform, all in
    double-double.  Returns {(k2, k3): (hi, lo)} with complex128 hi and lo.
    """
    x = np.asarray(x)
    n1, n2, n3 = x.shape
    samples = list(samples)
    out = {}
    for k3 in sorted({k3 for _, k3 in samples}):
        a3 = dd_lines_at(x.reshape(n1 * n2, n3), n3, k3, inverse, nthreads).reshape(n1, n2, 4)
        for k2 in sorted({k2 for k2, kk in samples if kk == k3}):
            a2 = dd_lines_at(a3, n2, k2, inverse, nthreads)            # [n1, 4]
            a1 = dd_lines(a2.reshape(1, n1, 4), n1, inverse)[0]         # [n1, 4]
            out[(k2, k3)] = (a1[:, 0] + 1j * a1[:, 2], a1[:, 1] + 1j * a1[:, 3])
    return out


def _join(hi, lo):
    return [(int(h) << 64) | int(l) for h, l in zip(hi, lo)]


def line_stage(x, N, p, q, stage, precision=0, inverse=False, extra_shift=0):
    """One Bailey stage of one length-N line.

    Returns dict with 'out' (complex, slot order of the stage), 're'/'im'
    (exact Python ints per output slot) and 'exp' (column exponents; None for
    an all-zero column).
    """
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    assert x.shape == (N,)
    out = np.empty(N, dtype=np.complex128)
    rh = np.empty(N, dtype=np.int64)
    rl = np.empty(N, dtype=np.uint64)
    ih = np.empty(N, dtype=np.int64)
    il = np.empty(N, dtype=np.uint64)
    ncol = p if stage == 1 else q
    ex = np.empty(ncol, dtype=np.intc)
    bits = 52 if precision == 0 else 23
    tab = np.ascontiguousarray(_roots.quantised_roots(N, bits, inverse))
    rc = lib().oracle_line_stage(x.ctypes.data, out.ctypes.data, N, p, q, _ptr(tab, _I64P),
                                 precision, stage, extra_shift, _ptr(rh, _I64P), _ptr(rl, _U64P),
                                 _ptr(ih, _I64P), _ptr(il, _U64P), _ptr(ex, _IP))
    if rc != 0:
        raise ValueError("bad factorisation")
    intmin = np.iinfo(np.intc).min
    return {"out": out, "re": _join(rh, rl), "im": _join(ih, il),
            "exp": [None if e == intmin else int(e) for e in ex]}


def lines(x, N, p, q, precision=0, inverse=False, nthreads=None):
    """Both Bailey stages of independent contiguous length-N lines (x: [nlines, N])."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    assert x.shape[-1] == N
    out = np.empty_like(x)
    bits = 52 if precision == 0 else 23
    tab = np.ascontiguousarray(_roots.quantised_roots(N, bits, inverse))
    rc = lib().oracle_lines(x.ctypes.data, out.ctypes.data, x.size // N, N, p, q, _ptr(tab, _I64P),
                            precision, nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad factorisation")
    return out


def lines_at(x, N, p, q, k, precision=0, inverse=False, nthreads=None):
    """Output position k of both Bailey stages of every contiguous line of x ([nlines, N])."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    nl = x.size // N
    out = np.empty(nl, dtype=np.complex128)
    bits = 52 if precision == 0 else 23
    tab = np.ascontiguousarray(_roots.quantised_roots(N, bits, inverse))
    rc = lib().oracle_lines_at(x.ctypes.data, out.ctypes.data, nl, N, p, q, _ptr(tab, _I64P),
                               precision, k, nthreads or default_threads())
    if rc != 0:
        raise ValueError("bad factorisation or position")
    return out


def pack(R, exp, precision=0):
    """The oracle's correctly rounded R * 2^exp (R a Python int, |R| < 2^127)."""
    lo = R & ((1 << 64) - 1)
    hi = R >> 64
    return lib().oracle_pack_hilo(hi, lo, exp, precision)
