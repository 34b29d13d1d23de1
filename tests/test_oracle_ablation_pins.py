"""Pins of the ablation oracle (Garner, FP64 sum, INT8 Phase A, 16-bit words, H0 folds); no GPU.

Garner is pinned to the mixed-radix representation obtained by repeated
division (a different computation from the paper's recursion), to textbook
examples worked by hand, and to the Kulisch route of oracle.crt_ref (CRT by
idempotents).  The FP64-sum baseline is pinned to a forward error bound of
recursive summation (any dropped slice, wrong weight or wrong sign of the
lift lands far outside it) and to the exact special case of a zero tuple.
The INT8 Phase A is pinned to the defining identities of its columns
(sum_s 256^s P'_s = sum_k v_k u_k with the plain u_k, not the byte slices of
the FP16 route), to their INT32 bound, to hand-worked digit examples and to
the FP16 route's final values.  The 16-bit-word accumulator is pinned to
hand-worked deposits with and without a carry, to the plain value
sum_k v_k u_k and its guard-bit bound, and to the 32-bit route's outputs.
The H0 fold-and-add reduction is pinned to the paper's list of friendly
moduli, to hand-worked folds and to the definition of the centred residue
(congruence and range) over the whole range of the GEMM sums.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ablation_ref as A
from oracle import constants as K
from oracle import crt_ref


def _mixed_radix_by_division(x, moduli):
    """Digits of x in the mixed radix (m_0, m_1, ...) by repeated divmod."""
    d = []
    for m in moduli:
        x, r = divmod(x, m)
        d.append(r)
    assert x == 0
    return d


def test_garner_textbook_examples():
    # 23 = 2 + 3 (2 + 5 * 1): residues (2, 3, 2) mod (3, 5, 7)
    assert A.garner_digits([23 % 3, 23 % 5, 23 % 7], (3, 5, 7)) == [2, 2, 1]
    # 1000 = 6 + 7 (10 + 11 * 12): residues (6, 10, 12) mod (7, 11, 13)
    assert A.garner_digits([6, 10, 12], (7, 11, 13)) == [6, 10, 12]
    assert A.garner_value([6, 10, 12], (7, 11, 13)) == 1000


@pytest.mark.parametrize("moduli", [K.MODULI_FP64, K.MODULI_FP32], ids=["fp64", "fp32"])
def test_garner_digits_are_the_mixed_radix_representation(moduli):
    M = K.modulus_product(moduli)
    rng = np.random.default_rng(11)
    xs = [0, 1, M - 1, M // 2, M // 2 - 1] + [int.from_bytes(rng.bytes(16), "little") % M for _ in range(300)]
    for x in xs:
        d = A.garner_digits([x % m for m in moduli], moduli)
        assert d == _mixed_radix_by_division(x, moduli)
        assert all(0 <= dk < m for dk, m in zip(d, moduli))


@pytest.mark.parametrize("moduli,target", [(K.MODULI_FP64, "f64"), (K.MODULI_FP32, "f32")], ids=["fp64", "fp32"])
def test_garner_equals_idempotent_crt_and_kulisch(moduli, target):
    M = K.modulus_product(moduli)
    h = M // 2
    rng = np.random.default_rng(12)
    vals = [0, 1, -1, h - 1, -h, -h + 1, (1 << 53) + 1, -((1 << 60) + 3)]
    vals += [int.from_bytes(rng.bytes(16), "little") % M - h for _ in range(300)]
    for C in vals:
        v = [C % m for m in moduli]
        exp = int(rng.integers(-200, 10))
        g = A.garner_reconstruct(v, moduli, exp, target)
        ref = crt_ref.reconstruct(v, moduli, exp, target)
        assert g["R"] == C == ref["R"]
        assert np.float64(g["y"]).tobytes() == np.float64(ref["y"]).tobytes()


def test_slice_fp64_zero_tuple_is_exact():
    for moduli in (K.MODULI_FP64, K.MODULI_FP32):
        r = A.slice_fp64([0] * len(moduli), moduli, -104)
        assert r["T"] == 0.0 and r["zhat"] == 0 and r["y"] == 0.0


def test_slice_fp64_within_summation_error_bound():
    moduli = K.MODULI_FP64
    rng = np.random.default_rng(13)
    for bits in (20, 64, 100, 110, 113):
        for _ in range(60):
            C = int.from_bytes(rng.bytes(16), "little") % (1 << bits)
            C = -C if rng.integers(2) else C
            exp = int(rng.integers(-160, 0))
            v = [C % m for m in moduli]
            y = A.slice_fp64(v, moduli, exp)["y"]
            err = abs(Fraction(y) - Fraction(C) * Fraction(2) ** exp)
            assert err <= Fraction(A.slice_fp64_error_bound(v, moduli, exp))


def test_slice_fp64_loses_low_bits_at_the_capacity_scale():
    """The plain FP64 sum spans ~130 bits (T up to 4360 M), so an output near
    the capacity limit 2^113 keeps only about its top 36 bits (Table
    precision reports the same loss mechanism), while Garner is exact."""
    moduli = K.MODULI_FP64
    rng = np.random.default_rng(14)
    rel = []
    for _ in range(200):
        C = (1 << 112) + int.from_bytes(rng.bytes(14), "little")
        v = [C % m for m in moduli]
        y = A.slice_fp64(v, moduli)["y"]
        rel.append(float(abs(Fraction(y) - C) / C))
        assert A.garner_reconstruct(v, moduli)["y"] == crt_ref.pack_f64(C, 0)
    med = float(np.median(rel))
    assert 2.0 ** -45 < med < 2.0 ** -30


# ---- Phase A on signed bytes: two limbs, shifted columns (Sec. 8.3) ----

def test_balanced_bytes_and_limbs_hand_examples():
    assert A.balanced_bytes(200, 2) == [-56, 1]                 # 200 = -56 + 256
    assert A.balanced_bytes(0x7F80, 3) == [-128, -128, 1]       # -128 - 128*256 + 65536
    assert A.int8_limbs(2038) == (-10, 8)                       # 2038 = -10 + 256 * 8
    assert A.int8_limbs(127) == (127, 0)
    assert A.int8_limbs(128) == (-128, 1)
    assert A.int8_limbs(0) == (0, 0)


@pytest.mark.parametrize("moduli", [K.MODULI_FP64, K.MODULI_FP32], ids=["fp64", "fp32"])
def test_int8_columns_sum_to_the_crt_inner_products(moduli):
    """sum_s 256^s P'_s = sum_k v_k u_k and sum_t 256^t Z'_t = sum_k v_k w_k, with
    every column inside r * 128 * (128 + 8) (signed bytes, INT32 accumulation)."""
    rng = np.random.default_rng(15)
    U, W = K.idempotents(moduli), K.lift_weights(moduli)
    bound = len(moduli) * 128 * (128 + 8)
    tuples = [[m - 1 for m in moduli], [0] * len(moduli), [min(127, m - 1) for m in moduli],
              [min(128, m - 1) for m in moduli]]
    tuples += [[int(rng.integers(0, m)) for m in moduli] for _ in range(300)]
    for v in tuples:
        P, Z = A.int8_phase_a(v, moduli)
        assert len(P) == K.n_slices(moduli) + 2 and len(Z) == K.n_frac_slices(moduli) + 2
        assert sum(p << (8 * s) for s, p in enumerate(P)) == sum(a * b for a, b in zip(v, U))
        assert sum(z << (8 * t) for t, z in enumerate(Z)) == sum(a * b for a, b in zip(v, W))
        assert max(abs(x) for x in P + Z) <= bound < 2 ** 31


@pytest.mark.parametrize("moduli,target", [(K.MODULI_FP64, "f64"), (K.MODULI_FP32, "f32")], ids=["fp64", "fp32"])
def test_int8_route_equals_fp16_route(moduli, target):
    M = K.modulus_product(moduli)
    h = M // 2
    rng = np.random.default_rng(16)
    vals = [0, 1, -1, h - 1, -h, -h + 1, (1 << 53) + 1]
    vals += [int.from_bytes(rng.bytes(16), "little") % M - h for _ in range(200)]
    for C in vals:
        v = [C % m for m in moduli]
        exp = int(rng.integers(-200, 10))
        a = A.int8_reconstruct(v, moduli, exp, target)
        b = crt_ref.reconstruct(v, moduli, exp, target)
        assert a["R"] == C == b["R"] and a["zhat"] == b["zhat"]
        assert np.float64(a["y"]).tobytes() == np.float64(b["y"]).tobytes()


# ---- 16-bit Kulisch words, Strategy A (Sec. 6.4) ----

def test_kulisch16_hand_example():
    # P_0 = 0x5BC123 at bit 0 -> words 0x123, 0x5BC; P_1 = 1 at bit 8 -> 0x100 in word 0
    raw, W = A.kulisch16_deposit([0x5BC123, 1])
    assert raw[:3] == [0x123 + 0x100, 0x5BC, 0]
    assert W[:3] == [0x223, 0x5BC, 0]
    # P_1 = 0x10 at bit 8 is 0x1000: nothing in word 0, 1 in word 1
    raw, W = A.kulisch16_deposit([0xFFF, 0x10])
    assert raw[:2] == [0xFFF, 0x1] and W[:2] == [0xFFF, 0x1]
    raw, W = A.kulisch16_deposit([0xFFF, 0x1])
    assert raw[0] == 0xFFF + 0x100 and W[:2] == [0x0FF, 0x1]


@pytest.mark.parametrize("moduli", [K.MODULI_FP64, K.MODULI_FP32], ids=["fp64", "fp32"])
def test_kulisch16_value_and_guard_bits(moduli):
    """The swept words spell sum_s 256^s P_s exactly and no word overflows its
    16 bits before the sweep, for extreme and random tuples."""
    rng = np.random.default_rng(17)
    U = K.idempotents(moduli)
    tuples = [[m - 1 for m in moduli], [0] * len(moduli)]
    tuples += [[int(rng.integers(0, m)) for m in moduli] for _ in range(300)]
    for v in tuples:
        P, _ = crt_ref.phase_a(v, moduli)
        raw, W = A.kulisch16_deposit(P)
        assert sum(x << (12 * i) for i, x in enumerate(W)) == sum(a * b for a, b in zip(v, U))
        assert max(raw) < 1 << 16 and all(0 <= x < 1 << 12 for x in W)


@pytest.mark.parametrize("moduli,target", [(K.MODULI_FP64, "f64"), (K.MODULI_FP32, "f32")], ids=["fp64", "fp32"])
def test_int16_route_equals_int32_route(moduli, target):
    M = K.modulus_product(moduli)
    h = M // 2
    rng = np.random.default_rng(18)
    vals = [0, 1, -1, h - 1, -h, -h + 1, (1 << 53) + 1]
    vals += [int.from_bytes(rng.bytes(16), "little") % M - h for _ in range(200)]
    for C in vals:
        v = [C % m for m in moduli]
        exp = int(rng.integers(-200, 10))
        a = A.int16_reconstruct(v, moduli, exp, target)
        b = crt_ref.reconstruct(v, moduli, exp, target)
        assert a["R"] == C == b["R"]
        assert np.float64(a["y"]).tobytes() == np.float64(b["y"]).tobytes()


# ---- H0 fold-and-add reduction of the friendly moduli (Sec. 2, Sec. 8.3) ----

def test_h0_friendly_set_is_the_papers_seven():
    friendly = [m for m in K.MODULI_FP64 if A.h0_form(m) is not None]
    assert sorted(friendly) == [487, 491, 511, 1024, 2027, 2029, 2039]
    assert A.h0_form(2039) == (11, 9) and A.h0_form(487) == (9, 25) and A.h0_form(1024) == (10, 0)


def test_h0_hand_examples():
    # 2^24 = 8192 * 2^11 -> 9 * 8192 = 73728 = 36 * 2^11 -> 9 * 36 = 324 (2^24 mod 2039 = 324)
    assert A.h0_reduce(1 << 24, 2039) == (324, 2)
    # 5000 mod 1024 = 904 -> centred 904 - 1024 = -120, no fold
    assert A.h0_reduce(5000, 1024) == (-120, 0)
    # 1500 >= 2039 - 1019: one subtraction, no fold
    assert A.h0_reduce(1500, 2039) == (1500 - 2039, 0)


@pytest.mark.parametrize("m", [2039, 2029, 2027, 1024, 511, 491, 487])
def test_h0_reduce_is_the_centred_residue(m):
    """Over the whole range of the GEMM sums (|t| <= 2^24): the fold result is
    congruent to t, lies in [-floor(m/2), m - floor(m/2)), and takes at most
    five folds (the stage kernel's fixed count for the slowest modulus)."""
    rng = np.random.default_rng(19)
    ts = list(range(-5000, 5001)) + [(1 << 24) - k for k in range(300)] + [-(1 << 24) + k for k in range(300)]
    ts += [int(x) for x in rng.integers(-(1 << 24), (1 << 24) + 1, size=20000)]
    worst = 0
    for t in ts:
        r, folds = A.h0_reduce(t, m)
        assert (r - t) % m == 0 and -(m // 2) <= r < m - m // 2
        worst = max(worst, folds)
    assert worst <= 5
