"""Pins of the reconstruction-ablation oracle (recursive Garner, plain FP64 sum); no GPU.

Garner is pinned to the mixed-radix representation obtained by repeated
division (a different computation from the paper's recursion), to textbook
examples worked by hand, and to the Kulisch route of oracle.crt_ref (CRT by
idempotents).  The FP64-sum baseline is pinned to a forward error bound of
recursive summation (any dropped slice, wrong weight or wrong sign of the
lift lands far outside it) and to the exact special case of a zero tuple.
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
