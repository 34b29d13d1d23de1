"""Reference of the reconstruction ablations (oracle, test infrastructure only).

The paper ranks the exact Kulisch Phase B against the reconstructions it
replaces.  Two of them are written out here, in Python integers and Python
floats (IEEE binary64, round to nearest even), from their definitions:

* recursive Garner (Sec. 4.1, paragraph on the recursive Garner count, Eq.
  recursive-garner; App. C, per-formulation costs): the mixed-radix digits
  of the residue tuple, each from the ones before it, then the positional
  value, centred into [-M/2, M/2) and rounded once.  The result is the exact
  CRT integer, so its output equals the Kulisch route's bit for bit.

* slicing direct CRT with a plain FP64 sum (Sec. 4.2, Phase B paragraph on the
  FP vector pipe; App. C, the "fp64 sum" Phase B option and Table precision):
  the Phase-A slice sums P_s of Eq. slicing, summed as FP64 values
  P_s * 256^s with a rounding after every addition, the modulo-M lift taken
  with the same round(2^-48 sum_t 256^t Z_t) as the exact route but applied
  in FP64, and one scaling by 2^exp.  This is the accuracy baseline: the
  unweighted sum spans about 120 bits, so the cancellation against zhat M
  loses the low bits of the result.

A third route keeps the Kulisch Phase B but moves Phase A to the INT8
matrix cores (Sec. 8.2, the B200 cross-check; Sec. 8.3, Eq. h1-group): each
canonical residue is split v = v0 + 256 v1 with v0 in [-128, 128) and v1 in
[0, 8], both signed bytes, and the high limb multiplies the next lower slice
(the shifted-column identity), so the columns are P'_s = sum_k (v0_k u_{k,s}
+ v1_k u_{k,s-1}) and likewise Z'_t over the lift weights.  The matrix cores
here multiply signed bytes only, so the slices of u_k and w_k are taken as
balanced base-256 digits in [-128, 128) (one more digit than the unsigned
bytes); sum_s 256^s P'_s is still sum_k v_k u_k, so the result is the
Kulisch route's bit for bit.

A fourth route keeps Phase A and narrows the Kulisch word (Sec. 6.3, Eq.
kulisch-width; Sec. 6.4, Strategy A and Table substrate): the slice sums
P_s (below 2^23) are deposited at bit 8s into 16-bit words of radix 2^12
(four guard bits each), every slice spread over the three words its bits
touch, and one carry sweep at the end resolves the redundant form.  The
accumulated integer is the same, so is the output.

The fifth ablation sits before the reconstruction, in the residue reduction
of the GEMM sums (Sec. 2, the reduction-friendly moduli; rung H0 of the
co-design ladder, Sec. 8.3): for m = 2^b - c with a small complement c, an
integer t = 2^b h + l (h = floor(t / 2^b), l = t mod 2^b) is congruent to
c h + l, so repeated folds shrink t until one conditional subtraction leaves
the centred residue; m = 2^b needs only its low b bits.  Residues are unique,
so this changes no output; the oracle states the steps so that their count
and range can be checked.

Readings where the paper leaves the order open (recorded in the design notes):
the FP64 sum runs over s = 0, 1, ..., S-1; M enters the FP64 lift as its
nearest binary64 value and zhat * M is rounded before the subtraction; the
FP32 target converts the FP64 result to binary32 at the end.
"""
import math
import struct

from . import constants as K
from . import crt_ref


def garner_digits(v, moduli):
    """Mixed-radix digits d_k in [0, m_k) with sum_k d_k prod_{i<k} m_i = CRT(v).

    Eq. recursive-garner: d_k = (v_k - sum_{j<k} d_j prod_{i<j} m_i)
    * (prod_{i<k} m_i)^-1 mod m_k, taken for k = 0, 1, ... in order.
    """
    d = []
    for k, mk in enumerate(moduli):
        acc = v[k]
        radix = 1  # prod_{i<j} m_i for the current j
        for j in range(k):
            acc -= d[j] * radix
            radix *= moduli[j]
        d.append(acc * pow(radix, -1, mk) % mk)
    return d


def garner_value(d, moduli):
    """The positional value d_0 + m_0 (d_1 + m_1 (d_2 + ...)) in [0, M)."""
    value = 0
    for k in reversed(range(len(moduli))):
        value = value * moduli[k] + d[k]
    return value


def garner_reconstruct(v, moduli, exp=0, target="f64"):
    """Recursive Garner, centring into [-M/2, M/2), one correctly rounded pack."""
    M = K.modulus_product(moduli)
    value = garner_value(garner_digits(v, moduli), moduli)
    R = value - M if value >= M // 2 else value
    y = crt_ref.pack_f64(R, exp) if target == "f64" else crt_ref.pack_f32(R, exp)
    return {"digits": garner_digits(v, moduli), "R": R, "y": y}


def slice_fp64(v, moduli, exp=0, target="f64"):
    """Slicing direct CRT with the plain FP64 Phase B (Sec. 4.2; App. C)."""
    M = K.modulus_product(moduli)
    P, Z = crt_ref.phase_a(v, moduli)
    T = 0.0
    for s, ps in enumerate(P):
        T = T + float(ps) * float(1 << (8 * s))  # the product is exact; the sum rounds
    zhat = crt_ref.zhat_from(Z)
    lift = float(zhat) * float(M)  # float(M) is the nearest binary64 to M
    y = math.ldexp(T - lift, exp)
    if target == "f32":
        y = struct.unpack("<f", struct.pack("<f", y))[0]
    return {"P": P, "T": T, "zhat": zhat, "y": y}


def slice_fp64_error_bound(v, moduli, exp=0):
    """A bound on |y - R 2^exp| for slice_fp64's FP64 target (Higham, Sec. 4.2).

    Recursive summation of S terms rounds S - 1 times, each by at most
    2^-53 times the partial sum; float(M) and zhat * float(M) add at most
    2^-53 |zhat M| each, and the final subtraction 2^-53 |y|.  With
    |partial sums| <= sum_s P_s 256^s = E and u = 2^-53 the bound is
    (S u E + 2 u zhat M + u (|R| + S u E + 2 u zhat M)) 2^exp, to first order
    (a factor 1.01 covers the second-order terms).
    """
    M = K.modulus_product(moduli)
    P, Z = crt_ref.phase_a(v, moduli)
    E = sum(p << (8 * s) for s, p in enumerate(P))
    zhat = crt_ref.zhat_from(Z)
    R = E - zhat * M
    u = 2.0 ** -53
    S = len(P)
    first = S * u * float(E) + 2 * u * float(zhat) * float(M)
    return 1.01 * math.ldexp(first + u * (abs(float(R)) + first), exp)


def balanced_bytes(value, count):
    """Digits d_s in [-128, 128) with sum_s d_s 256^s = value, s < count."""
    d = []
    for _ in range(count):
        r = value & 0xFF
        if r >= 128:
            r -= 256
        d.append(r)
        value = (value - r) >> 8
    assert value == 0, "too few digits"
    return d


def int8_limbs(v):
    """The two-limb split of a canonical residue: v = v0 + 256 v1 (Sec. 8.3)."""
    v0 = (v + 128) % 256 - 128
    return v0, (v - v0) // 256


def int8_phase_a(v, moduli):
    """Shifted-column Phase A on signed bytes: P'_s, s <= S + 1, and Z'_t, t <= T + 1."""
    U = [balanced_bytes(u, K.n_slices(moduli) + 1) for u in K.idempotents(moduli)]
    W = [balanced_bytes(w, K.n_frac_slices(moduli) + 1) for w in K.lift_weights(moduli)]
    limbs = [int8_limbs(x) for x in v]

    def columns(D):
        n = len(D[0]) + 1
        return [sum(l0 * (D[k][s] if s < n - 1 else 0) + l1 * (D[k][s - 1] if s >= 1 else 0)
                    for k, (l0, l1) in enumerate(limbs)) for s in range(n)]
    return columns(U), columns(W)


def int8_reconstruct(v, moduli, exp=0, target="f64"):
    """Phase A on INT8 (two limbs, shifted columns), then the Kulisch Phase B of Sec. 5.1."""
    M = K.modulus_product(moduli)
    P, Z = int8_phase_a(v, moduli)
    E = sum(p << (8 * s) for s, p in enumerate(P))
    zacc = sum(z << (8 * t) for t, z in enumerate(Z))
    zhat = (zacc + (1 << (K.FRAC_BITS - 1))) >> K.FRAC_BITS
    R = crt_ref.two_sided_lift(E, zhat, M)
    y = crt_ref.pack_f64(R, exp) if target == "f64" else crt_ref.pack_f32(R, exp)
    return {"P": P, "Z": Z, "E": E, "zhat": zhat, "R": R, "y": y}


RADIX16 = 12   # usable bits of a 16-bit word (four guard bits), Table substrate
WORDS16 = 11   # 11 x 12 = 132 bits: the accumulator modulo 2^132


def kulisch16_deposit(P):
    """Strategy A: P_s at bit 8s into radix-2^12 words (each < 2^16 before the
    sweep), then the carry sweep; returns (words before, words after), both
    modulo 2^132."""
    mask = (1 << RADIX16) - 1
    w = [0] * (WORDS16 + 2)
    for s, ps in enumerate(P):
        assert 0 <= ps < (1 << 23)
        q, o = divmod(8 * s, RADIX16)
        x = ps << o
        for j in range(3):
            w[q + j] += (x >> (RADIX16 * j)) & mask
    raw = w[:WORDS16]
    assert all(0 <= x < (1 << 16) for x in raw), "guard bits overflowed"
    out = list(raw)
    for i in range(WORDS16 - 1):
        out[i + 1] += out[i] >> RADIX16
        out[i] &= mask
    out[-1] &= mask
    return raw, out


def int16_reconstruct(v, moduli, exp=0, target="f64"):
    """Phase A, the 16-bit-word Kulisch accumulation, the two-sided lift, one pack."""
    M = K.modulus_product(moduli)
    P, Z = crt_ref.phase_a(v, moduli)
    raw, W = kulisch16_deposit(P)
    # sum_s P_s 256^s <= 4360 M < 2^131 (canonical residues), so the 132-bit
    # accumulator holds E exactly
    E = sum(x << (RADIX16 * i) for i, x in enumerate(W))
    zhat = crt_ref.zhat_from(Z)
    R = crt_ref.two_sided_lift(E, zhat, M)
    y = crt_ref.pack_f64(R, exp) if target == "f64" else crt_ref.pack_f32(R, exp)
    return {"raw": raw, "W": W, "E": E, "zhat": zhat, "R": R, "y": y}


# ---- H0: fold-and-add reduction of the friendly moduli (Sec. 2, Sec. 8.3) ----

H0_MAX_COMPLEMENT = 31  # friendly: 2^b - m <= 31 (the FP64 set's seven have <= 25; 961 has 63)


def h0_form(m):
    """(b, c) with m = 2^b - c, 2^(b-1) < m <= 2^b, when m is friendly; else None."""
    b = (m - 1).bit_length()
    c = (1 << b) - m
    return (b, c) if c <= H0_MAX_COMPLEMENT else None


def h0_reduce(t, m):
    """Centred residue of the integer t by folds, and the number of folds.

    Folds t <- c floor(t / 2^b) + (t mod 2^b) until t lies in
    [-c, 2^b - 1 + c], then subtracts m once when t >= m - floor(m/2).  For
    m = 2^b the residue is t mod 2^b taken in [-2^(b-1), 2^(b-1)).
    """
    b, c = h0_form(m)
    B = 1 << b
    if c == 0:
        r = t % B
        return (r - B if r >= B // 2 else r), 0
    folds = 0
    while not (-c <= t <= B - 1 + c):
        t = c * (t // B) + t % B
        folds += 1
    return (t - m if t >= m - m // 2 else t), folds
