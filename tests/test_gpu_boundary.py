"""The C-ABI boundary on the GPU: the debug tap of the fused stage kernel,
the non-finite input flag, the axis-order option and in-place execution.

* Debug tap (Alg. 2 checkpoints of one line): the residues that entered
  Phase A are congruent to the oracle's exact stage integers modulo every m_k
  and centred; P_s, Z_t, E, zhat and R equal the big-integer CRT reference
  (Sec. 4.2, Eqs. fcrt and slicing; Sec. 5.1) evaluated on those residues
  (E modulo 2^128, or 2^96 for the FP32 target: the low words the kernel's
  accumulator holds);
  R equals the oracle's exact integer and the output bits the oracle's.
* A non-finite input raises OBFFT_NONFINITE_INPUT through obfft_last_error
  and the kernels still finish; a finite call afterwards reports success.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import words_to_int
from oracle import constants as K
from oracle import crt_ref
from oracle import exact as ox
from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu

NONFINITE = 4


def _api():
    from paper_2606_23698_amd import api
    return api


def _pq(plan):
    info = plan.info()
    return tuple(zip(info["p"], info["q"]))


def _line_of(x, axis, line):
    """Elements of line `line` (outer * inner + inner index) along `axis`."""
    n = x.shape
    inner = int(np.prod(n[axis + 1:]))
    o, i = divmod(line, inner)
    return x.reshape(-1, n[axis], inner)[o, :, i]


def _check_tap(dump, ref, moduli, precision):
    """dump: [N, 2, 64] records; ref: the oracle's line_stage result."""
    M = K.modulus_product(moduli)
    r = len(moduli)
    S, T = K.n_slices(moduli), K.n_frac_slices(moduli)
    nR = 4
    for t in range(dump.shape[0]):
        for part, exact in ((0, ref["re"][t]), (1, ref["im"][t])):
            rec = dump[t, part].astype(np.int64)
            v = [int(np.int32(rec[40 + k])) for k in range(r)]
            for k, m in enumerate(moduli):
                assert (v[k] - exact) % m == 0, (t, part, k)
                assert abs(v[k]) <= m // 2 + 2, (t, part, k, v[k])
            P, Z = crt_ref.phase_a(v, moduli)
            assert [int(np.int32(rec[s])) for s in range(S)] == P, (t, part)
            assert [int(np.int32(rec[16 + q])) for q in range(T)] == Z, (t, part)
            E = sum(p << (8 * s) for s, p in enumerate(P))
            nw = 4 if precision == 0 else 3   # the accumulator holds E mod 2^(32 nw)
            assert words_to_int([int(w) for w in rec[24:24 + nw]], signed=False) == E % (1 << (32 * nw)), (t, part)
            assert all(int(w) == 0 for w in rec[24 + nw:29]), (t, part)
            zh = crt_ref.zhat_from(Z)
            assert int(np.int32(rec[29])) == zh, (t, part)
            R = words_to_int([int(w) for w in rec[30:30 + nR]], signed=True)
            assert R == E - zh * M == exact, (t, part)
            exp = int(np.int32(rec[34]))
            if precision == 0:
                bits = int(rec[35]) | (int(rec[36]) << 32)
                y = np.array([bits], dtype=np.uint64).view(np.float64)[0]
                assert y == crt_ref.pack_f64(R, exp)
            else:
                y = np.array([int(rec[35])], dtype=np.uint32).view(np.float32)[0]
                assert y == crt_ref.pack_f32(R, exp)
            want = ref["out"][t].real if part == 0 else ref["out"][t].imag
            assert float(y) == float(want) and math.copysign(1, y) == math.copysign(1, want), (t, part)


@pytest.mark.parametrize("shape,substrate,precision", [
    ((32, 32, 32), "fp16", "fp64"),
    ((32, 32, 32), "fp8", "fp64"),
    ((32, 32, 32), "int8", "fp64"),
    ((8, 12, 16), "fp16", "fp64"),
    ((2, 2, 1024), "fp8", "fp64"),           # the full-length FP8 tile (K = 32)
    ((16, 8, 32), "fp16", "fp32"),
])
def test_debug_tap_checkpoints_against_crt_reference(gpu, shape, substrate, precision):
    api = _api()
    plan = api.Plan(shape, substrate=substrate, precision=precision)
    prec = 0 if precision == "fp64" else 1
    moduli = plan.info()["moduli"]
    x = inputs.uniform(shape, 0, np.complex128 if prec == 0 else np.complex64)
    xt = torch.from_numpy(x).to(gpu)
    pq = _pq(plan)
    for axis in (2, 1, 0):
        N = shape[axis]
        p, q = pq[axis]
        nlines = int(np.prod(shape)) // N
        for line in sorted({0, nlines // 2 + 1, nlines - 1}):
            y1, dump1 = plan.debug_tap(axis, 1, line, xt)
            ref1 = ox.line_stage(_line_of(x, axis, line), N, p, q, 1, precision=prec)
            _check_tap(dump1, ref1, moduli, prec)
            # stage 2 on the Y' slots that stage 1 wrote
            y1h = y1.cpu().numpy()
            _, dump2 = plan.debug_tap(axis, 2, line, y1)
            ref2 = ox.line_stage(_line_of(y1h, axis, line), N, p, q, 2, precision=prec)
            _check_tap(dump2, ref2, moduli, prec)


def test_nonfinite_input_sets_the_flag(gpu):
    api = _api()
    shape = (32, 32, 32)
    plan = api.Plan(shape)
    x = inputs.uniform(shape, 0)
    ok = plan.forward(torch.from_numpy(x).to(gpu))
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    for bad in (np.inf, -np.inf, np.nan):
        xb = x.copy()
        xb[3, 17, 5] = complex(bad, 0.5)
        y = plan.forward(torch.from_numpy(xb).to(gpu))
        torch.cuda.synchronize()
        assert plan.last_error() == NONFINITE, bad
        plan.clear_error()
        assert plan.last_error() == 0
        del y
    xb = x.copy()
    xb[0, 0, 0] = complex(0.25, np.nan)   # imaginary part only
    plan.forward(torch.from_numpy(xb).to(gpu))
    torch.cuda.synchronize()
    assert plan.last_error() == NONFINITE
    plan.clear_error()
    # a finite call after the flag was cleared reports success and the usual bits
    y = plan.forward(torch.from_numpy(x).to(gpu))
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(y, ok)


@pytest.mark.parametrize("mode", ["passes", "persistent"])
def test_nonfinite_input_flag_in_a_batch(gpu, mode):
    api = _api()
    shapes = [(8, 16, 32), (16, 16, 16)]
    xs = [torch.from_numpy(inputs.uniform(s, 30 + i)).to(gpu) for i, s in enumerate(shapes)]
    bp = api.BatchPlan(shapes)
    bp.set_mode(mode)
    bp.forward(xs)
    torch.cuda.synchronize()
    assert bp.last_error() == 0
    xs[1][3, 3, 3] = complex(np.inf, 0.0)
    bp.forward(xs)
    torch.cuda.synchronize()
    assert bp.last_error() == NONFINITE


@pytest.mark.parametrize("order", [(0, 1, 2), (1, 0, 2), (2, 0, 1)])
def test_axis_order_bit_exact(gpu, order):
    api = _api()
    shape = (8, 12, 16)
    x = inputs.uniform(shape, 3)
    plan = api.Plan(shape, axis_order=order)
    xt = torch.from_numpy(x).to(gpu)
    y = plan.forward(xt)
    yi = plan.inverse(xt)
    torch.cuda.synchronize()
    pq = _pq(plan)
    assert np.count_nonzero(y.cpu().numpy() != ox.fft3_exact(x, pq, order=order)) == 0
    # n is not a power of two: the inverse multiplies the unnormalised result by fl(1/n)
    f = 1.0 / int(np.prod(shape))
    raw = ox.fft3_exact(x, pq, order=order, inverse=True)
    ref_i = np.empty_like(raw)
    ref_i.real = raw.real * f
    ref_i.imag = raw.imag * f
    assert np.count_nonzero(yi.cpu().numpy() != ref_i) == 0
    # a different order is a different (equally valid) rounding sequence
    y_def = api.Plan(shape).forward(xt)
    assert not torch.equal(y, y_def)


def test_in_place_equals_out_of_place(gpu):
    api = _api()
    for shape, prec in (((32, 32, 32), "fp64"), ((8, 12, 16), "fp64"), ((16, 8, 32), "fp32")):
        plan = api.Plan(shape, precision=prec)
        dt = np.complex128 if prec == "fp64" else np.complex64
        x = torch.from_numpy(inputs.uniform(shape, 5, dt)).to(gpu)
        ref = plan.forward(x)
        ref_inv = plan.inverse(x)
        buf = x.clone()
        plan.forward(buf, out=buf)
        buf2 = x.clone()
        plan.inverse(buf2, out=buf2)
        torch.cuda.synchronize()
        assert torch.equal(buf, ref), shape
        assert torch.equal(buf2, ref_inv), shape
