"""Big-integer reference of the exact CRT reconstruction (oracle, test infrastructure only).

Follows Sec. 4.2 (direct CRT with idempotents, Eq. fcrt; byte slicing, Eq.
slicing; Phase A on canonical residues) and Sec. 5.1 (Kulisch Phase B,
two-sided modulo-M lift, correctly rounded pack; Alg. 2), step by step, in
Python integers.  Every intermediate that the GPU epilogue exposes through its
debug entry point is produced here:

    v_k    canonical residues in [0, m_k)
    P_s    Phase-A slice sums  sum_k v_k * byte_s(u_k),  s < S
    Z_t    Phase-A lift sums   sum_k v_k * byte_t(w_k),  t < T
    W      the normalised radix-2^28 Kulisch digits of E + B_tot
    zhat   round-half-up(2^-48 * sum_t 256^t Z_t)
    R      the centred representative in [-M/2, M/2)
    y      RNE(R * 2^exp) in the target format
"""
import math
import struct

from . import constants as K

WORD_BITS = 28
WORD_MASK = (1 << WORD_BITS) - 1


def n_words(S):
    """Carry-save words covering 8S + 24 bits: six for S = 15 (Sec. 5.1, Fig. kulisch)."""
    return -(-(8 * S + 24) // WORD_BITS)


def canonical_residues(C, moduli):
    return [C % m for m in moduli]


def phase_a(v, moduli):
    """P_s and Z_t of Eq. slicing and Sec. 5.1 (the 21 Phase-A columns for r = 12)."""
    U = K.u_slices(moduli)
    W = K.w_slices(moduli)
    S = len(U[0])
    T = len(W[0])
    P = [sum(v[k] * U[k][s] for k in range(len(moduli))) for s in range(S)]
    Z = [sum(v[k] * W[k][t] for k in range(len(moduli))) for t in range(T)]
    return P, Z


def kulisch_deposit(P):
    """Biased carry-save deposits of Alg. 2, then one carry sweep.

    Each (P_s + 2^23) lands at bit 8s, split over word floor(8s/28) and the
    next one.  Returns (raw words before the sweep, normalised words).
    """
    S = len(P)
    nw = n_words(S)
    W = [0] * nw
    for s, ps in enumerate(P):
        val = ps + (1 << K.DEPOSIT_BIAS_BITS)
        assert 0 <= val < (1 << 32)
        pos = 8 * s
        w, off = divmod(pos, WORD_BITS)
        W[w] += (val << off) & WORD_MASK
        hi = val >> (WORD_BITS - off)
        if hi:
            W[w + 1] += hi
    raw = list(W)
    assert all(0 <= x < (1 << 32) for x in raw), "guard bits overflowed"
    for w in range(nw - 1):
        W[w + 1] += W[w] >> WORD_BITS
        W[w] &= WORD_MASK
    return raw, W


def words_value(W):
    return sum(x << (WORD_BITS * i) for i, x in enumerate(W))


def zhat_from(Z, f=K.FRAC_BITS):
    """zhat = round(2^-f sum_t 256^t Z_t), halves rounded up (Sec. 5.1)."""
    zacc = sum(z << (8 * t) for t, z in enumerate(Z))
    return (zacc + (1 << (f - 1))) >> f


def two_sided_lift(E, zhat, M):
    """R = E - zhat M, then the symmetric correction into [-M/2, M/2) (Sec. 5.1)."""
    R = E - zhat * M
    if R >= M // 2:
        R -= M
    if R < -(M // 2):
        R += M
    return R


def one_sided_lift(E, zhat, M):
    """The defective one-sided correction (only R >= M/2 is fixed), kept for T4."""
    R = E - zhat * M
    if R >= M // 2:
        R -= M
    return R


def rne_scaled(R, exp, prec, emin_quantum):
    """Correctly rounded R * 2^exp with a `prec`-bit significand, ties to even.

    `emin_quantum` is the exponent of the smallest subnormal (-1074 for binary64,
    -149 for binary32).  Returns (q, e) with the value q * 2^e exactly.
    """
    if R == 0:
        return 0, 0
    a = abs(R)
    top = a.bit_length() - 1 + exp
    qe = max(top - (prec - 1), emin_quantum)
    shift = qe - exp
    if shift <= 0:
        q = a << (-shift)
    else:
        q, r = divmod(a, 1 << shift)
        half = 1 << (shift - 1)
        if r > half or (r == half and (q & 1)):
            q += 1
    return (q if R > 0 else -q), qe


def pack_f64(R, exp):
    """R = 0 gives +0; a nonzero R that rounds to zero keeps its sign (IEEE 754)."""
    q, e = rne_scaled(R, exp, 53, -1074)
    if q == 0:
        return -0.0 if R < 0 else 0.0
    return math.ldexp(float(q), e)


def pack_f32(R, exp):
    q, e = rne_scaled(R, exp, 24, -149)
    if q == 0:
        return -0.0 if R < 0 else 0.0
    v = math.ldexp(float(q), e)
    return struct.unpack("<f", struct.pack("<f", v))[0]


def reconstruct(v, moduli, exp=0, target="f64"):
    """Full Phase A + Phase B for one scalar output; returns every checkpoint."""
    M = K.modulus_product(moduli)
    P, Z = phase_a(v, moduli)
    raw, W = kulisch_deposit(P)
    E = words_value(W) - K.deposit_bias(len(P))
    zh = zhat_from(Z)
    R = two_sided_lift(E, zh, M)
    y = pack_f64(R, exp) if target == "f64" else pack_f32(R, exp)
    return {"P": P, "Z": Z, "raw": raw, "W": W, "E": E, "zhat": zh, "R": R, "y": y}
