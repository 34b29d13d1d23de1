"""Bit-exact parity of the GPU CRT epilogue (Phase A + Kulisch + lift + pack).

The GPU entry point takes canonical residues and returns every checkpoint
(P_s, Z_t, E, zhat, R) and the packed value; the oracle (oracle.crt_ref)
computes the same quantities in Python integers following Sec. 4.2 and
Sec. 5.1 (Alg. 2).  Inputs include the boundary values the paper names as
permanent regression tests: C = +-(M/2 - 1), rounding ties of the pack, and
the extremes of the representable range.
"""
import numpy as np
import pytest
import torch

from gpu_util import words_to_int
from oracle import constants as K
from oracle import crt_ref

pytestmark = pytest.mark.gpu


def _cases(moduli, rng, n_random):
    M = K.modulus_product(moduli)
    h = M // 2
    vals = [0, 1, -1, 2, -2, h - 1, -h, -h + 1, h - 2, (1 << 112), -(1 << 112), (1 << 53) + 1,
            -((1 << 53) + 1), (1 << 54) + 2, (3 << 52) + 1, (1 << 100) + (1 << 47)]
    vals += [h - 1 - i for i in range(64)] + [-h + i for i in range(64)]
    vals += [int(v) for v in rng.integers(-(1 << 62), 1 << 62, size=n_random)]
    big = [int.from_bytes(rng.bytes(16), "little") % M - h for _ in range(n_random)]
    vals += big
    # ties of the pack at 53 significant bits: odd multiples of the half-ulp
    for e in (60, 80, 100, 110):
        for odd in (1, 3, 5, 7):
            v = (1 << e) + odd * (1 << (e - 53))
            if v < h:
                vals += [v, -v]
    return [v for v in vals if -h <= v < h]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_crt_reconstruct_bit_exact(gpu, precision):
    from paper_2606_23698_amd import api
    moduli = K.MODULI_FP64 if precision == "fp64" else K.MODULI_FP32
    M = K.modulus_product(moduli)
    rng = np.random.default_rng(5)
    vals = _cases(moduli, rng, 700)
    n = len(vals)
    res = np.array([[v % m for m in moduli] for v in vals], dtype=np.int16)
    exps = rng.integers(-160, -60, size=n).astype(np.int32)
    exps[:8] = [-104, 0, -52, -1, -200, -120, 5, -110]
    out, taps = api.crt_reconstruct(torch.from_numpy(res).to(gpu), torch.from_numpy(exps).to(gpu),
                                    precision, taps=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    taps = taps.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    lay = api.taps_layout()
    S, T = K.n_slices(moduli), K.n_frac_slices(moduli)
    target = "f64" if precision == "fp64" else "f32"
    for i, v in enumerate(vals):
        ref = crt_ref.reconstruct([v % m for m in moduli], moduli, int(exps[i]), target)
        assert ref["R"] == v
        t = taps[i]
        assert list(t[lay["P"]:lay["P"] + S]) == ref["P"], i
        assert list(t[lay["Z"]:lay["Z"] + T]) == ref["Z"], i
        E = words_to_int(t[lay["E"]:lay["E"] + lay["n_E"]])
        assert E == ref["E"], i
        assert int(t[lay["zhat"]]) == ref["zhat"], i
        R = words_to_int(t[lay["R"]:lay["R"] + lay["n_R"]], signed=True)
        assert R == v, (i, v, R)
        got = float(out[i])
        assert got == ref["y"] and np.signbit(got) == np.signbit(ref["y"]), (i, v, got, ref["y"])
    assert M > 0
