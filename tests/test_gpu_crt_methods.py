"""GPU parity of the reconstruction ablations (recursive Garner, plain FP64 sum,
Phase A on INT8 MFMA, 16-bit Kulisch words).

Every kernel is compared with oracle.ablation_ref element by element: Garner,
the INT8 route and the 16-bit words bit for bit (all are exact, so they must also equal the
Kulisch route), the FP64 sum bit for bit as well (the oracle performs the same IEEE binary64 operations
in the same order).  Edge cases: ragged n, n = 1, the boundary values of the
lift, rounding ties, subnormal scaling and a bad method code.
"""
import numpy as np
import pytest
import torch

from oracle import ablation_ref as A
from oracle import constants as K

pytestmark = pytest.mark.gpu


def _values(moduli, rng, n_random):
    M = K.modulus_product(moduli)
    h = M // 2
    vals = [0, 1, -1, 2, h - 1, -h, -h + 1, h - 2, (1 << 53) + 1, -((1 << 53) + 1), (3 << 52) + 1]
    for e in (60, 80, 100, 110):
        for odd in (1, 3, 5):
            v = (1 << e) + odd * (1 << (e - 53))
            if v < h:
                vals += [v, -v]
    for bits in (20, 64, 100, 107, 111, 113):
        for _ in range(n_random // 6):
            c = int.from_bytes(rng.bytes(16), "little") % (1 << bits)
            vals.append(-c if rng.integers(2) else c)
    vals += [int.from_bytes(rng.bytes(16), "little") % M - h for _ in range(n_random // 4)]
    return [v for v in vals if -h <= v < h]


def _run(gpu, moduli, vals, exps, method, precision):
    from paper_2606_23698_amd import api
    res = np.array([[v % m for m in moduli] for v in vals], dtype=np.int16)
    out = api.crt_reconstruct_method(torch.from_numpy(res).to(gpu), torch.from_numpy(exps).to(gpu), method,
                                     precision)
    torch.cuda.synchronize()
    return out.cpu().numpy(), res


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_garner_bit_exact(gpu, precision):
    from paper_2606_23698_amd import api
    moduli = K.MODULI_FP64 if precision == "fp64" else K.MODULI_FP32
    target = "f64" if precision == "fp64" else "f32"
    rng = np.random.default_rng(21)
    vals = _values(moduli, rng, 600)
    exps = rng.integers(-170, -40, size=len(vals)).astype(np.int32)
    exps[:6] = [-104, 0, -52, -1, -1200, -1100]  # the last two scale into the subnormal range
    out, res = _run(gpu, moduli, vals, exps, "garner", precision)
    ref = np.array([A.garner_reconstruct(list(map(int, r)), moduli, int(e), target)["y"]
                    for r, e in zip(res, exps)], dtype=out.dtype)
    assert out.tobytes() == ref.tobytes()
    kul, _ = api.crt_reconstruct(torch.from_numpy(res).to(gpu), torch.from_numpy(exps).to(gpu), precision)
    assert kul.cpu().numpy().tobytes() == out.tobytes()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_int8_phase_a_bit_exact(gpu, precision):
    from paper_2606_23698_amd import api
    moduli = K.MODULI_FP64 if precision == "fp64" else K.MODULI_FP32
    target = "f64" if precision == "fp64" else "f32"
    rng = np.random.default_rng(26)
    vals = _values(moduli, rng, 600)
    exps = rng.integers(-170, -40, size=len(vals)).astype(np.int32)
    exps[:6] = [-104, 0, -52, -1, -1200, -1100]
    out, res = _run(gpu, moduli, vals, exps, "kulisch_int8", precision)
    ref = np.array([A.int8_reconstruct(list(map(int, r)), moduli, int(e), target)["y"]
                    for r, e in zip(res, exps)], dtype=out.dtype)
    assert out.tobytes() == ref.tobytes()
    kul, _ = api.crt_reconstruct(torch.from_numpy(res).to(gpu), torch.from_numpy(exps).to(gpu), precision)
    assert kul.cpu().numpy().tobytes() == out.tobytes()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_int16_words_bit_exact(gpu, precision):
    from paper_2606_23698_amd import api
    moduli = K.MODULI_FP64 if precision == "fp64" else K.MODULI_FP32
    target = "f64" if precision == "fp64" else "f32"
    rng = np.random.default_rng(27)
    vals = _values(moduli, rng, 600)
    exps = rng.integers(-170, -40, size=len(vals)).astype(np.int32)
    exps[:6] = [-104, 0, -52, -1, -1200, -1100]
    out, res = _run(gpu, moduli, vals, exps, "kulisch_int16", precision)
    ref = np.array([A.int16_reconstruct(list(map(int, r)), moduli, int(e), target)["y"]
                    for r, e in zip(res, exps)], dtype=out.dtype)
    assert out.tobytes() == ref.tobytes()
    kul, _ = api.crt_reconstruct(torch.from_numpy(res).to(gpu), torch.from_numpy(exps).to(gpu), precision)
    assert kul.cpu().numpy().tobytes() == out.tobytes()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_fp64_bit_exact(gpu, precision):
    moduli = K.MODULI_FP64 if precision == "fp64" else K.MODULI_FP32
    target = "f64" if precision == "fp64" else "f32"
    rng = np.random.default_rng(22)
    vals = _values(moduli, rng, 600)
    exps = rng.integers(-170, -40, size=len(vals)).astype(np.int32)
    out, res = _run(gpu, moduli, vals, exps, "slice_fp64", precision)
    ref = np.array([A.slice_fp64(list(map(int, r)), moduli, int(e), target)["y"]
                    for r, e in zip(res, exps)], dtype=out.dtype)
    assert out.tobytes() == ref.tobytes()


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_ragged_sizes(gpu, n):
    moduli = K.MODULI_FP64
    rng = np.random.default_rng(23 + n)
    vals = _values(moduli, rng, 600)[:n]
    exps = np.full(len(vals), -104, dtype=np.int32)
    for method, fn in (("garner", A.garner_reconstruct), ("slice_fp64", A.slice_fp64),
                       ("kulisch_int8", A.int8_reconstruct), ("kulisch_int16", A.int16_reconstruct)):
        out, res = _run(gpu, moduli, vals, exps, method, "fp64")
        ref = np.array([fn(list(map(int, r)), moduli, -104)["y"] for r in res])
        assert out.tobytes() == ref.tobytes()


def test_large_n_exact_routes_agree(gpu):
    """At 2^22 outputs of uniformly random residue tuples the four exact
    routes agree everywhere; 512 sampled outputs also match the oracle."""
    from paper_2606_23698_amd import api
    moduli = K.MODULI_FP64
    n = 1 << 22
    g = torch.Generator(device=gpu).manual_seed(24)
    res = torch.stack([torch.randint(0, m, (n,), generator=g, device=gpu, dtype=torch.int16) for m in moduli], 1)
    res = res.contiguous()
    exps = torch.full((n,), -110, dtype=torch.int32, device=gpu)
    gar = api.crt_reconstruct_method(res, exps, "garner")
    kul = api.crt_reconstruct_method(res, exps, "kulisch")
    ki8 = api.crt_reconstruct_method(res, exps, "kulisch_int8")
    k16 = api.crt_reconstruct_method(res, exps, "kulisch_int16")
    torch.cuda.synchronize()
    assert torch.equal(gar.view(torch.int64), kul.view(torch.int64))
    assert torch.equal(ki8.view(torch.int64), kul.view(torch.int64))
    assert torch.equal(k16.view(torch.int64), kul.view(torch.int64))
    idx = np.random.default_rng(25).choice(n, 512, replace=False)
    rs = res[torch.from_numpy(idx).to(gpu)].cpu().numpy()
    ref = np.array([A.garner_reconstruct(list(map(int, r)), moduli, -110)["y"] for r in rs])
    assert gar[torch.from_numpy(idx).to(gpu)].cpu().numpy().tobytes() == ref.tobytes()


def test_errors(gpu):
    from paper_2606_23698_amd import api, _lib
    res = torch.zeros((4, 12), dtype=torch.int16, device=gpu)
    exps = torch.zeros(4, dtype=torch.int32, device=gpu)
    out = torch.empty(4, dtype=torch.float64, device=gpu)
    L = _lib.lib()
    import ctypes
    st = L.obfft_crt_reconstruct_method(0, 7, 4, ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(exps.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), None)
    assert st == 1  # OBFFT_INVALID_VALUE
    assert L.obfft_crt_reconstruct_method(0, 1, 0, None, None, None, None) == 0
    with pytest.raises(ValueError):
        api.crt_reconstruct_method(torch.zeros((4, 6), dtype=torch.int16, device=gpu), exps, "garner", "fp64")
