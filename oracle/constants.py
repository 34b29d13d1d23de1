"""Number-theoretic constants of the Ozaki-II modulus sets, in Python integers.

Oracle module (test infrastructure only).  Everything here is the plain
definition from the paper:

* the modulus sets and their product M (Sec. 2, paragraph "Ozaki Scheme II");
* the capacity budget  log2 M > 1 + log2 K + 2(k+1)  (Sec. 2, Eq. capacity);
* the CRT idempotents u_k = (M/m_k) * ((M/m_k)^-1 mod m_k) (Sec. 4.2, Eq. fcrt);
* the byte slicing of u_k into S = ceil(bitlen(M)/8) slices (Sec. 4.2, Eq. slicing);
* the fractional-lift weights w_k = round(2^f u_k / M), f = 48 (Sec. 5.1);
* the deposit bias B_tot = sum_s 2^23 256^s (Sec. 5.1, Alg. 2).
"""
from math import ceil, log2, prod

# Sec. 2: the shipping modulus set (five perfect squares, pairwise coprime).
MODULI_FP64 = (2039, 2029, 2027, 1089, 1024, 961, 841, 625, 529, 511, 491, 487)
# Sec. 2: the earlier set, which replaced 2039, 2029, 2027 by 509, 503, 499
# and misses the capacity budget by 2.16 bits (negative test only).
MODULI_REV33 = (509, 503, 499, 1089, 1024, 961, 841, 625, 529, 511, 491, 487)
# Sec. 7 (Ozaki-II for FP32): six moduli of the same class with log2 M = 62.6.
# The paper names only r = 6 and log2 M = 62.6; the unique 6-subset of the
# shipping set with that product is used (reading recorded in the design notes).
MODULI_FP32 = (2039, 2029, 2027, 1024, 961, 841)

FRAC_BITS = 48          # f of the fractional lift (Sec. 5.1)
DEPOSIT_BIAS_BITS = 23  # each P_s is biased by 2^23 before deposit (Alg. 2)


def modulus_product(moduli):
    return prod(moduli)


def pairwise_coprime(moduli):
    from math import gcd
    return all(gcd(a, b) == 1 for i, a in enumerate(moduli) for b in moduli[i + 1:])


def capacity_bits_required(K, k):
    """Right-hand side of Eq. capacity: 1 (sign) + log2 K + 2(k+1)."""
    return 1 + log2(K) + 2 * (k + 1)


def capacity_ok(moduli, K, k):
    return log2(modulus_product(moduli)) > capacity_bits_required(K, k)


def idempotents(moduli):
    """u_k of Eq. fcrt: u_k = 1 (mod m_k), u_k = 0 (mod m_j), j != k."""
    M = modulus_product(moduli)
    return [(M // m) * pow(M // m, -1, m) for m in moduli]


def n_slices(moduli):
    """S = ceil(bitlen(M) / 8) (Sec. 4.2: 15 for the shipping set)."""
    return ceil(modulus_product(moduli).bit_length() / 8)


def byte_slices(value, count):
    return [(value >> (8 * s)) & 0xFF for s in range(count)]


def u_slices(moduli):
    """U[k][s] = byte s of u_k (Eq. slicing)."""
    S = n_slices(moduli)
    return [byte_slices(u, S) for u in idempotents(moduli)]


def lift_weights(moduli, f=FRAC_BITS):
    """w_k = round(2^f u_k / M) (Sec. 5.1), rounding to nearest (no ties occur)."""
    M = modulus_product(moduli)
    out = []
    for u in idempotents(moduli):
        num = (u << f)
        q, rem = divmod(num, M)
        if 2 * rem == M:
            raise ValueError("tie in lift weight")
        out.append(q + (1 if 2 * rem > M else 0))
    return out


def n_frac_slices(moduli, f=FRAC_BITS):
    """Number of byte slices needed for every w_k (6 for f = 48)."""
    return max(ceil(w.bit_length() / 8) for w in lift_weights(moduli, f))


def w_slices(moduli, f=FRAC_BITS):
    T = n_frac_slices(moduli, f)
    return [byte_slices(w, T) for w in lift_weights(moduli, f)]


def deposit_bias(S):
    """B_tot = sum_{s<S} 2^23 * 256^s (Alg. 2)."""
    return sum((1 << DEPOSIT_BIAS_BITS) << (8 * s) for s in range(S))
