"""Exactness and layout of the gfx950 instructions the kernels rely on.

The residue GEMMs need FP8 and INT8 MFMA to accumulate small integers
exactly, and Phase A needs FP16 MFMA with FP32 accumulation exact below 2^24
(Sec. 4.2: every column sum stays below 2^24; Sec. 9 item (1d) asks for this
contract to be measured on the silicon).  Each probe runs one instruction on
integer operands laid out in the register layout the kernels assume and
compares with an exact integer matmul.
"""
import numpy as np
import pytest
import torch

from gpu_util import e4m3

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_23698_amd import api
    return api


def test_fp8_mfma_16x16x32_layout_and_exactness(gpu):
    api = _api()
    rng = np.random.default_rng(11)
    for trial in range(4):
        A = rng.integers(-16, 17, size=(16, 32))
        B = rng.integers(-16, 17, size=(32, 16))
        if trial == 0:
            A[:] = 16
            B[:] = 16
        a = np.zeros((64, 8), np.uint8)
        b = np.zeros((64, 8), np.uint8)
        for l in range(64):
            for j in range(8):
                k = 8 * (l // 16) + j
                a[l, j] = e4m3(A[l % 16, k])
                b[l, j] = e4m3(B[k, l % 16])
        d = torch.zeros((64, 4), dtype=torch.float32, device=gpu)
        api.mfma_probe(0, torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu), d)
        torch.cuda.synchronize()
        D = d.cpu().numpy()
        ref = A @ B
        got = np.zeros((16, 16))
        for l in range(64):
            for v in range(4):
                got[4 * (l // 16) + v, l % 16] = D[l, v]
        assert np.array_equal(got, ref)


def _k128_slot(h, j):
    """K index of byte j of lane group h in the scaled 16 x 16 x 128 FP8 MFMA."""
    return 16 * h + j if j < 16 else 64 + 16 * h + (j - 16)


@pytest.mark.parametrize("trial", ["random", "digit_weights"])
def test_fp8_scaled_mfma_16x16x128_layout_and_scales(gpu, trial):
    """The full-length FP8 tile's contract: lane l holds row (column) l % 16
    and bytes of K indices 16 h + j (j < 16) and 64 + 16 h + j - 16 (h = l / 16);
    K block b = k / 32 of row m is scaled by 2^(s - 127), s the scale of lane
    m + 16 b; sums of small scaled integers are exact."""
    api = _api()
    rng = np.random.default_rng(23 if trial == "random" else 29)
    A = rng.integers(-16, 17, size=(16, 128))
    B = rng.integers(-16, 17, size=(128, 16))
    if trial == "random":
        S = rng.choice([127, 132], size=(16, 4))
    else:
        # the tile's use: block scales 32^f, the top digit f = 2 in {-1, 0, 1}
        S = np.tile(np.array([127, 132, 137, 127]), (16, 1))
        A[:, 64:96] = rng.integers(-1, 2, size=(16, 32))
    a = np.zeros(64 * 32 + 64 * 4, np.uint8)
    b = np.zeros((64, 32), np.uint8)
    scales = np.zeros(64, np.int32)
    for l in range(64):
        h, r = l // 16, l % 16
        scales[l] = S[r, h]
        for j in range(32):
            k = _k128_slot(h, j)
            a[l * 32 + j] = e4m3(A[r, k])
            b[l, j] = e4m3(B[k, r])
    a[64 * 32:] = scales.view(np.uint8)
    d = torch.zeros((64, 4), dtype=torch.float32, device=gpu)
    api.mfma_probe(7, torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu), d)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    w = np.exp2(S.astype(np.int64) - 127).astype(np.int64)  # [row, block]
    ref = np.zeros((16, 16), np.int64)
    for blk in range(4):
        ks = slice(32 * blk, 32 * blk + 32)
        ref += (A[:, ks] * w[:, blk:blk + 1]) @ B[ks, :]
    got = np.zeros((16, 16))
    for l in range(64):
        for v in range(4):
            got[4 * (l // 16) + v, l % 16] = D[l, v]
    assert np.array_equal(got, ref)


def test_i8_mfma_16x16x64_layout_and_exactness(gpu):
    api = _api()
    rng = np.random.default_rng(12)
    A = rng.integers(-128, 128, size=(16, 64))
    B = rng.integers(-128, 128, size=(64, 16))
    a = np.zeros((64, 16), np.int8)
    b = np.zeros((64, 16), np.int8)
    for l in range(64):
        for j in range(16):
            k = 16 * (l // 16) + j
            a[l, j] = A[l % 16, k]
            b[l, j] = B[k, l % 16]
    d = torch.zeros((64, 4), dtype=torch.int32, device=gpu)
    api.mfma_probe(1, torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu), d)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    got = np.zeros((16, 16), np.int64)
    for l in range(64):
        for v in range(4):
            got[4 * (l // 16) + v, l % 16] = D[l, v]
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("extreme", [False, True])
def test_i8_mfma_32x32x32_layout_and_exactness(gpu, extreme):
    """INT8 Phase-A contract: signed-byte limbs times balanced slices, 32-term
    sums in INT32, in the lane layout the INT8 reconstruction route assumes."""
    api = _api()
    rng = np.random.default_rng(17)
    A = rng.integers(-128, 128, size=(32, 32))
    B = rng.integers(-128, 128, size=(32, 32))
    if extreme:
        A[:] = -128
        B[:] = -128
    a = np.zeros((64, 16), np.int8)
    b = np.zeros((64, 16), np.int8)
    for l in range(64):
        for j in range(16):
            k = 16 * (l // 32) + j
            a[l, j] = A[l % 32, k]
            b[l, j] = B[k, l % 32]
    d = torch.zeros((64, 16), dtype=torch.int32, device=gpu)
    api.mfma_probe(6, torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu), d)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    got = np.zeros((32, 32), np.int64)
    for l in range(64):
        for v in range(16):
            row = (v % 4) + 8 * (v // 4) + 4 * (l // 32)
            got[row, l % 32] = D[l, v]
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("extreme", [False, True])
def test_f16_mfma_32x32x16_layout_and_exactness(gpu, extreme):
    """Phase-A contract: residues <= 2038 times slices <= 255, 16-term sums, plus 2^23."""
    api = _api()
    rng = np.random.default_rng(13)
    A = rng.integers(0, 256, size=(32, 16))
    B = rng.integers(0, 2039, size=(16, 32))
    if extreme:
        A[:] = 255
        B[:] = 2038
    a = np.zeros((64, 8), np.float16)
    b = np.zeros((64, 8), np.float16)
    for l in range(64):
        for j in range(8):
            k = 8 * (l // 32) + j
            a[l, j] = A[l % 32, k]
            b[l, j] = B[k, l % 32]
    d = torch.zeros((64, 16), dtype=torch.float32, device=gpu)
    api.mfma_probe(2, torch.from_numpy(a.view(np.int16)).to(gpu), torch.from_numpy(b.view(np.int16)).to(gpu), d)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    got = np.zeros((32, 32), np.int64)
    for l in range(64):
        for v in range(16):
            row = (v % 4) + 8 * (v // 4) + 4 * (l // 32)
            got[row, l % 32] = D[l, v]
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("extreme", [False, True])
def test_f16_mfma_16x16x32_layout_and_exactness(gpu, extreme):
    """Residue-GEMM contract of the FP16 substrate: matrix residues |a| <= 1019
    against radix-128 limbs (|d0| <= 64, |d1| <= 8), 32-term sums below 2^23."""
    api = _api()
    rng = np.random.default_rng(14)
    A = rng.integers(-1019, 1020, size=(16, 32))
    B = np.where(np.arange(32)[:, None] % 2 == 0, rng.integers(-64, 65, size=(32, 16)),
                 rng.integers(-8, 9, size=(32, 16)))
    if extreme:
        A[:] = 1019
        B[0::2] = 64
        B[1::2] = 8
    a = np.zeros((64, 8), np.float16)
    b = np.zeros((64, 8), np.float16)
    for l in range(64):
        for j in range(8):
            k = 8 * (l // 16) + j
            a[l, j] = A[l % 16, k]
            b[l, j] = B[k, l % 16]
    d = torch.zeros((64, 4), dtype=torch.float32, device=gpu)
    api.mfma_probe(5, torch.from_numpy(a.view(np.int16)).to(gpu), torch.from_numpy(b.view(np.int16)).to(gpu), d)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    got = np.zeros((16, 16), np.int64)
    for l in range(64):
        for v in range(4):
            got[4 * (l // 16) + v, l % 16] = D[l, v]
    assert np.array_equal(got, A @ B)


def test_permlane32_swap_semantics(gpu):
    api = _api()
    x = torch.arange(64, dtype=torch.int32, device=gpu)
    y = torch.arange(1000, 1064, dtype=torch.int32, device=gpu)
    d = torch.zeros(128, dtype=torch.int32, device=gpu)
    api.mfma_probe(3, x, y, d)
    torch.cuda.synchronize()
    out = d.cpu().numpy()
    nx, ny = out[:64], out[64:]
    # the upper half of x is exchanged with the lower half of y
    assert np.array_equal(nx[:32], np.arange(32))
    assert np.array_equal(nx[32:], np.arange(1000, 1032))
    assert np.array_equal(ny[:32], np.arange(32, 64))
    assert np.array_equal(ny[32:], np.arange(1032, 1064))


def test_e4m3_conversion_of_small_integers(gpu):
    api = _api()
    vals = np.concatenate([np.arange(-16, 17), np.zeros(64 - 33)]).astype(np.float32)
    d = torch.zeros(64, dtype=torch.uint8, device=gpu)
    api.mfma_probe(4, torch.from_numpy(vals).to(gpu), None, d)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    ref = np.array([e4m3(v) for v in vals], dtype=np.uint8)
    assert np.array_equal(got, ref)
