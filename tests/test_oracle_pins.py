"""Pins of the CPU oracle to facts outside itself (no GPU).

Each test checks the oracle against something the paper prints, a closed
form, an invariant, a textbook routine or brute force -- never against a
retyping of the oracle's own formula.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import constants as K
from oracle import crt_ref
from oracle import exact as ox
from oracle import roots


# ---- Sec. 2 (Eq. capacity) and Sec. 4.2 / 5.1 printed constants ----

def test_modulus_set_sizes_printed_in_paper():
    M = K.modulus_product(K.MODULI_FP64)
    assert round(math.log2(M), 2) == 117.88          # Sec. 2
    assert M.bit_length() == 118
    assert K.n_slices(K.MODULI_FP64) == 15            # Sec. 4.2: S = ceil(118/8)
    assert K.pairwise_coprime(K.MODULI_FP64)
    assert round(K.capacity_bits_required(32, 53), 6) == 114.0   # Eq. capacity
    assert round(math.log2(M) - 114, 2) == 3.88       # "3.88 bits of margin"
    assert K.capacity_ok(K.MODULI_FP64, 32, 53)


def test_rev33_set_fails_capacity_by_2_16_bits():
    M33 = K.modulus_product(K.MODULI_REV33)
    assert round(math.log2(M33), 2) == 111.84
    assert round(114 - math.log2(M33), 2) == 2.16
    assert not K.capacity_ok(K.MODULI_REV33, 32, 53)


def test_fp32_set():
    M = K.modulus_product(K.MODULI_FP32)
    assert round(math.log2(M), 1) == 62.6              # Sec. 7
    assert K.n_slices(K.MODULI_FP32) == 8
    assert K.capacity_bits_required(32, 24) == 56.0
    assert K.capacity_ok(K.MODULI_FP32, 32, 24)


def test_idempotents_and_exact_bounds_T9():
    mods = K.MODULI_FP64
    M = K.modulus_product(mods)
    u = K.idempotents(mods)
    for k, m in enumerate(mods):
        for j, mj in enumerate(mods):
            assert u[k] % mj == (1 if j == k else 0)
    # Sec. 8 (T9): sum (m_k - 1) u_k = 4360 M - 1, sum (2 m_k - 1) u_k = 8724 M - 1
    assert sum((m - 1) * uk for m, uk in zip(mods, u)) == 4360 * M - 1
    assert sum((2 * m - 1) * uk for m, uk in zip(mods, u)) == 8724 * M - 1


def test_phase_a_column_sums_below_2_23_T6():
    # Sec. 4.2: every P_s <= 12 * 2038 * 255 = 6,236,280 < 2^23 (FP32 exact)
    mods = K.MODULI_FP64
    U = K.u_slices(mods)
    W = K.w_slices(mods)
    worst = max(sum((m - 1) * U[k][s] for k, m in enumerate(mods)) for s in range(15))
    worst_z = max(sum((m - 1) * W[k][t] for k, m in enumerate(mods)) for t in range(len(W[0])))
    assert worst <= 6_236_280 < 2 ** 23
    assert worst_z <= 6_236_280
    assert 12 * 2038 * 255 == 6_236_280


def test_lift_weights_fit_six_bytes():
    assert K.n_frac_slices(K.MODULI_FP64) == 6           # S_frac = 6 (Sec. 5.1)
    assert all(w < 2 ** 48 for w in K.lift_weights(K.MODULI_FP64))


# ---- the CRT / Kulisch / lift / pack reference (Sec. 4.2, Sec. 5.1, Alg. 2) ----

def _adversarial(M):
    h = M // 2
    return [0, 1, -1, h - 1, -h, -h + 1, -(h - 1), h - 2, 1 << 112, -(1 << 112), (1 << 110) + 12345]


@pytest.mark.parametrize("mods", [K.MODULI_FP64, K.MODULI_FP32])
def test_crt_recovers_every_centred_value(mods):
    M = K.modulus_product(mods)
    rng = np.random.default_rng(1)
    vals = [v for v in _adversarial(M) if -M // 2 <= v < M // 2]
    vals += [int.from_bytes(rng.bytes(16), "little") % M - M // 2 for _ in range(400)]
    h = M // 2
    vals += [h - 1 - i for i in range(200)] + [-h + i for i in range(200)]
    for C in vals:
        v = crt_ref.canonical_residues(C, mods)
        out = crt_ref.reconstruct(v, mods)
        assert out["R"] == C
        assert out["E"] == sum(vk * uk for vk, uk in zip(v, K.idempotents(mods)))
        assert crt_ref.words_value(out["W"]) == out["E"] + K.deposit_bias(len(out["P"]))
        assert 0 <= out["zhat"] <= 4360                 # P11: z <= 4360 for canonical residues
        assert all(0 <= p <= 6_236_280 for p in out["P"])


def test_signed_deposits_T3():
    # a negative slice sum (P_0 = -1) must still give the exact signed E (Alg. 2 bias)
    for P in ([-1] + [0] * 14, [-5, 3, -(2 ** 22), 0, 7] + [0] * 10, [-(2 ** 23 - 1)] * 15):
        raw, W = crt_ref.kulisch_deposit(P)
        E = crt_ref.words_value(W) - K.deposit_bias(15)
        assert E == sum(p << (8 * s) for s, p in enumerate(P))


def test_one_sided_lift_fails_two_sided_exact_T4():
    # Sec. 5.1: near C = +-(M/2 - 1) zhat can be off by one; a one-sided
    # correction then returns a value wrong by exactly M, the two-sided one is exact.
    mods = K.MODULI_FP64
    M = K.modulus_product(mods)
    C = -(M // 2 - 1)
    v = crt_ref.canonical_residues(C, mods)
    out = crt_ref.reconstruct(v, mods)
    assert out["R"] == C
    # canonical residues at C = -(M/2 - 1): zhat is one too small; R = C + M >= M/2
    assert out["zhat"] == (out["E"] - C) // M - 1
    # centred residues at +(M/2 - 1): zhat one too large
    Cp = M // 2 - 1
    vc = [((Cp % m) + m // 2) % m - m // 2 for m in mods]
    P, Z = crt_ref.phase_a(vc, mods)
    E = sum(p << (8 * s) for s, p in enumerate(P))
    zh = crt_ref.zhat_from(Z)
    assert E - zh * M == Cp - M
    assert crt_ref.one_sided_lift(E, zh, M) != Cp
    assert crt_ref.two_sided_lift(E, zh, M) == Cp


def test_rev33_dc_field_wrong_by_exactly_M():
    # Sec. 2: with the Rev-33 set the DC contraction K 2^{2k} reconstructs wrong by exactly M
    C = 32 * (2 ** 53 - 1) ** 2
    for mods, expect_ok in ((K.MODULI_REV33, False), (K.MODULI_FP64, True)):
        M = K.modulus_product(mods)
        R = crt_ref.reconstruct(crt_ref.canonical_residues(C, mods), mods)["R"]
        if expect_ok:
            assert R == C
        else:
            assert R == C - M


def test_pack_is_correctly_rounded_against_python_float():
    rng = np.random.default_rng(2)
    cases = [(1 << 53) + 1, (1 << 53) + 3, (1 << 54) + 2, (1 << 54) + 6, (1 << 112) - 1,
             (1 << 60) + (1 << 7), (1 << 60) + (3 << 7), 12345, 1]
    cases += [int.from_bytes(rng.bytes(15), "little") for _ in range(300)]
    for R in cases:
        for sgn in (1, -1):
            for e in (-104, -52, 0, 7, -200):
                ref = float(Fraction(sgn * R) * Fraction(2) ** e)      # Python: correctly rounded
                assert crt_ref.pack_f64(sgn * R, e) == ref
                assert ox.pack(sgn * R, e, 0) == ref                   # the C oracle's pack
    # a negative value that underflows to zero keeps its sign (IEEE 754 rounding)
    assert math.copysign(1.0, crt_ref.pack_f32(-2, -200)) == -1.0
    assert math.copysign(1.0, ox.pack(-2, -200, 1)) == -1.0
    assert math.copysign(1.0, crt_ref.pack_f64(-1, -1200)) == -1.0
    # binary32 via numpy's correctly rounded float64 -> float32 of exactly representable doubles
    for R in [(1 << 24) + 1, (1 << 24) + 3, (1 << 40) + (1 << 16), 3, (1 << 61) - 1]:
        ref = float(np.float32(Fraction(R) * 1))   # exact Fraction -> RNE float32 via float() first
        f = crt_ref.pack_f32(R, 0)
        # independent check: nearest float32, ties to even, computed with integers
        nb = R.bit_length()
        if nb > 24:
            sh = nb - 24
            q, rem = divmod(R, 1 << sh)
            if rem > (1 << (sh - 1)) or (rem == (1 << (sh - 1)) and q & 1):
                q += 1
            assert f == math.ldexp(q, sh)
        else:
            assert f == float(R)
        assert ox.pack(R, 0, 1) == f
        del ref


# ---- quantised roots ----

@pytest.mark.parametrize("N", [8, 12, 32, 96, 1024])
def test_quantised_roots_closed_forms(N):
    Q = roots.quantised_roots(N, 52)
    B = 1 << 52
    assert tuple(Q[0]) == (B, 0)
    if N % 4 == 0:
        assert tuple(Q[N // 4]) == (0, -B)
        assert tuple(Q[N // 2]) == (-B, 0)
        assert tuple(Q[3 * N // 4]) == (0, B)
    if N % 8 == 0:
        # cos(pi/4) 2^52 = sqrt(2^103): RNE by integer square root
        r = math.isqrt(2 ** 103)
        c = r + 1 if (2 * r + 1) ** 2 < 2 ** 105 else r
        assert tuple(Q[N // 8]) == (c, -c)
    if N % 12 == 0:
        # cos(pi/6) 2^52 = sqrt(3 2^102); sin(pi/6) 2^52 = 2^51 exactly
        r = math.isqrt(3 * 2 ** 102)
        c = r + 1 if (2 * r + 1) ** 2 < 3 * 2 ** 104 else r
        assert tuple(Q[N // 12]) == (c, -(1 << 51))
    for t in range(N):
        c, s = int(Q[t, 0]), int(Q[t, 1])
        # libm on a rounded argument: a few units of 2^-52 (the argument carries ~1e-15)
        assert abs(c - 2 ** 52 * math.cos(2 * math.pi * t / N)) <= 4
        assert abs(s + 2 ** 52 * math.sin(2 * math.pi * t / N)) <= 4
        assert abs(c * c + s * s - 2 ** 104) <= 2 ** 54


def test_conjugate_roots_exact():
    f = roots.quantised_roots(96, 52)
    i = roots.quantised_roots(96, 52, inverse=True)
    assert np.array_equal(f[:, 0], i[:, 0]) and np.array_equal(f[:, 1], -i[:, 1])


# ---- the exact-pipeline transform and the double-double DFT ----

def _mp_dft3(x, sign=-1):
    """Separable direct DFT in mpmath (30 digits): the textbook definition."""
    mpmath.mp.dps = 30
    a = [[[mpmath.mpc(complex(x[i, j, k])) for k in range(x.shape[2])] for j in range(x.shape[1])]
         for i in range(x.shape[0])]
    n1, n2, n3 = x.shape

    def w(n, t):
        return mpmath.expj(sign * 2 * mpmath.pi * t / n)
    b = [[[sum(a[i][j][k] * w(n3, k * kk) for k in range(n3)) for kk in range(n3)] for j in range(n2)]
         for i in range(n1)]
    c = [[[sum(b[i][j][k] * w(n2, j * jj) for j in range(n2)) for k in range(n3)] for jj in range(n2)]
         for i in range(n1)]
    d = [[[sum(c[i][j][k] * w(n1, i * ii) for i in range(n1)) for k in range(n3)] for j in range(n2)]
         for ii in range(n1)]
    return d


def test_dd_oracle_against_mpmath_brute_force():
    x = np.random.default_rng(3).uniform(-1, 1, (4, 6, 8)) + 1j * np.random.default_rng(4).uniform(-1, 1, (4, 6, 8))
    ref = _mp_dft3(x)
    hi, lo = ox.fft3_dd(x)
    for idx in np.ndindex(x.shape):
        r = ref[idx[0]][idx[1]][idx[2]]
        err = abs(mpmath.mpc(complex(hi[idx])) + mpmath.mpc(complex(lo[idx])) - r)
        assert err < 1e-27


def test_exact_oracle_against_mpmath_brute_force_8cubed():
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (8, 8, 8)) + 1j * rng.uniform(-1, 1, (8, 8, 8))
    ref = _mp_dft3(x)
    y = ox.fft3_exact(x, ((2, 4), (4, 2), (2, 4)))
    num = den = 0.0
    for idx in np.ndindex(x.shape):
        r = complex(ref[idx[0]][idx[1]][idx[2]])
        num += abs(y[idx] - r) ** 2
        den += abs(r) ** 2
    # each stage quantises to 53-bit significands and rounds once: a few 2^-53 per stage
    assert math.sqrt(num / den) < 1e-15
    yinv = ox.fft3_exact(x, ((2, 4), (4, 2), (2, 4)), inverse=True)
    refi = _mp_dft3(x, sign=+1)
    assert max(abs(yinv[idx] - complex(refi[idx[0]][idx[1]][idx[2]])) for idx in np.ndindex(x.shape)) < 1e-13


def test_exact_oracle_closed_forms():
    pq = ((4, 8), (8, 4), (4, 8))
    x = np.zeros((32, 32, 32), complex)
    x[0, 0, 0] = 1.0
    assert np.all(ox.fft3_exact(x, pq) == 1.0)           # delta -> exactly all ones
    x = np.full((16, 32, 8), 0.75 - 0.25j)
    y = ox.fft3_exact(x, ((4, 4), (4, 8), (2, 4)))
    ref = np.zeros_like(y)
    ref[0, 0, 0] = 16 * 32 * 8 * (0.75 - 0.25j)
    assert np.array_equal(y, ref)                        # constant -> exact DC, exact zeros
    # single tone exp(2 pi i k0.j / n) -> n1 n2 n3 at k0, near zero elsewhere
    n = (8, 16, 8)
    k0 = (3, 5, 1)
    g = np.meshgrid(*[np.arange(m) for m in n], indexing="ij")
    ph = sum(k * gg / m for k, gg, m in zip(k0, g, n))
    tone = np.exp(2j * np.pi * ph)
    y = ox.fft3_exact(tone, ((2, 4), (4, 4), (2, 4)))
    assert abs(y[k0] - 1024) < 1e-11
    y[k0] = 0
    assert np.max(np.abs(y)) < 1e-11


def test_exact_oracle_scale_invariance_and_parseval():
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (8, 16, 32)) + 1j * rng.uniform(-1, 1, (8, 16, 32))
    pq = ((2, 4), (4, 4), (4, 8))
    y = ox.fft3_exact(x, pq)
    # power-of-two scaling commutes exactly with per-column quantisation
    assert np.array_equal(ox.fft3_exact(x * 2.0 ** -37, pq), y * 2.0 ** -37)
    assert abs(np.sum(np.abs(y) ** 2) / x.size - np.sum(np.abs(x) ** 2)) / np.sum(np.abs(x) ** 2) < 1e-14
    back = ox.fft3_exact(y, pq, inverse=True, final_shift=-12)
    assert np.max(np.abs(back - x)) < 1e-14


def test_stage_conventions_against_definition():
    # stage 1: Y'[j1 + p k2] = sum_j2 x[j1 + p j2] w_q^{j2 k2}; stage 2 uses the fused
    # one-root coefficient w_N^{j1 (k2 + q k1)} (Sec. 2 six-step, Sec. 4.1 Eq. twiddle-fusion)
    N, p, q = 24, 4, 6
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
    s1 = ox.line_stage(x, N, p, q, 1)
    for j1 in range(p):
        for k2 in range(q):
            ref = sum(x[j1 + p * j2] * np.exp(-2j * np.pi * j2 * k2 / q) for j2 in range(q))
            assert abs(s1["out"][j1 + p * k2] - ref) < 1e-14
    s2 = ox.line_stage(s1["out"], N, p, q, 2)
    full = np.fft.fft(x)
    assert np.max(np.abs(s2["out"] - full)) < 1e-13
    # exact integers pack to the outputs
    for t in range(N):
        e = s2["exp"][t % q]
        assert ox.pack(s2["re"][t], e - 104) == s2["out"][t].real


def test_fp32_target_oracle_accuracy():
    rng = np.random.default_rng(8)
    x = (rng.uniform(-1, 1, (8, 16, 8)) + 1j * rng.uniform(-1, 1, (8, 16, 8))).astype(np.complex64)
    y = ox.fft3_exact(x, ((2, 4), (4, 4), (2, 4)), precision=1)
    assert y.dtype == np.complex64
    ref = np.fft.fftn(x.astype(np.complex128))
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-6
