"""Bit-level pins of the oracle's data quantisation (no GPU).

Per contraction column the method takes one power-of-two scale shared by the
real and imaginary parts (Alg. 1, scaling invariant): e is the largest binary
exponent (ilogb) over the column's nonzero real AND imaginary parts, and every
part becomes the integer x~ = RNE(x 2^((k-1)-e)) with k = 53 for the FP64
target and k = 24 for the FP32 target (Sec. 2, Eq. ozaki and Eq. capacity:
|x~| < 2^k).  Twiddles are integers scaled by 2^B, B = k - 1.

The pins below read that quantisation off the oracle's exact stage integers
at outputs whose twiddles are all omega^0 = 1, i.e. the integer pair
(2^B, 0): stage 1, output k2 = 0 of column j1 is 2^B (sum_j2 a~, sum_j2 b~),
and stage 2, output k1 = 0 of column k2 = 0 is 2^B (sum_j1 a~, sum_j1 b~).
Every expected integer was worked out by hand from the definition above and
is written out as a literal, so that each of these misreadings fails at
least one test:

* truncation instead of round-to-nearest-even,
* an exponent one too large (a k - 1 bit quantisation),
* an exponent taken from the real parts only,
* an exponent from frexp instead of ilogb (one too large),
* round half away from zero instead of half to even.
"""
import numpy as np
import pytest

from oracle import exact as ox

TWO52 = 2 ** 52
TWO23 = 2 ** 23


def _line(vals, N):
    x = np.zeros(N, dtype=np.complex128)
    for idx, v in vals.items():
        x[idx] = v
    return x


# Stage 1, N = 8 = p q with p = 2, q = 4: column j1 is x[j1], x[j1+2], x[j1+4],
# x[j1+6]; its k2 = 0 output sits in Y' slot j1.
#
# Column 0 (maximum in a real part, e = 0):
#   x[0] = 1 + 2^-52                      a~ = 2^52 + 1
#   x[2] = 3 2^-54 + 2.5 2^-52 i           a~ = RNE(0.75) = 1,   b~ = RNE(2.5) = 2   (tie to even)
#   x[4] = -3.5 2^-52 - 2.5 2^-52 i        a~ = RNE(-3.5) = -4,  b~ = RNE(-2.5) = -2 (ties to even)
#   x[6] = 0.5 - (1 - 2^-53) i             a~ = 2^51,  b~ = RNE(-(2^52 - 1/2)) = -2^52 (tie carries
#                                                         into the next binade)
#   sum a~ = 2^52 + 2^51 - 2,  sum b~ = -2^52
#
# Column 1 (maximum in an imaginary part only, e = 2):
#   x[1] = 0.75 + 4 i                      a~ = 0.75 2^50 = 3 2^48,  b~ = 2^52
#   x[3] = 1.5 2^-49                       a~ = 3
#   x[5] = 5 2^-51 - 7 2^-51 i             a~ = RNE(2.5) = 2,  b~ = RNE(-3.5) = -4
#   x[7] = 0
#   sum a~ = 3 2^48 + 5,  sum b~ = 2^52 - 4
STAGE1_VALS = {
    0: complex(1 + 2.0 ** -52, 0.0),
    2: complex(3 * 2.0 ** -54, 2.5 * 2.0 ** -52),
    4: complex(-3.5 * 2.0 ** -52, -2.5 * 2.0 ** -52),
    6: complex(0.5, -(1 - 2.0 ** -53)),
    1: complex(0.75, 4.0),
    3: complex(1.5 * 2.0 ** -49, 0.0),
    5: complex(5 * 2.0 ** -51, -7 * 2.0 ** -51),
    7: 0j,
}
STAGE1_EXPECT = {  # slot: (exponent, Re integer, Im integer)
    0: (0, TWO52 * (2 ** 52 + 2 ** 51 - 2), TWO52 * (-(2 ** 52))),
    1: (2, TWO52 * (3 * 2 ** 48 + 5), TWO52 * (2 ** 52 - 4)),
}


def test_fp64_stage1_quantisation_hand_worked():
    r = ox.line_stage(_line(STAGE1_VALS, 8), 8, 2, 4, stage=1)
    assert r["exp"] == [0, 2]
    for slot, (_, re, im) in STAGE1_EXPECT.items():
        assert r["re"][slot] == re, slot
        assert r["im"][slot] == im, slot


def test_fp64_stage1_packed_outputs_hand_worked():
    # the single rounding: y = RNE(R 2^(e - 52 - 52)); both sums are exact doubles here
    r = ox.line_stage(_line(STAGE1_VALS, 8), 8, 2, 4, stage=1)
    assert r["out"][0] == complex((2 ** 52 + 2 ** 51 - 2) * 2.0 ** -52, -1.0)
    assert r["out"][1] == complex((3 * 2 ** 48 + 5) * 2.0 ** -50, (2 ** 52 - 4) * 2.0 ** -50)


# Stage 2, N = 8 with p = 4, q = 2: column k2 = 0 is Y' slots 0..3; its k1 = 0
# output sits in slot 0 (k2 + q k1).  Subnormal column: ilogb(3 2^-1074) = -1073.
#   y[0] = 3 2^-1074                       a~ = 3 2^(-1074 + 52 + 1073) = 3 2^51
#   y[1] = 2^-1074 i                       b~ = 2^51
#   y[2] = -(2^-1074) + 2^-1073 i          a~ = -2^51,  b~ = 2^52
#   y[3] = 0
#   sum a~ = 2^52,  sum b~ = 3 2^51
STAGE2_SUBNORMAL = {0: complex(3 * 2.0 ** -1074, 0.0), 1: complex(0.0, 2.0 ** -1074),
                    2: complex(-(2.0 ** -1074), 2.0 ** -1073), 3: 0j,
                    4: complex(1.0, 1.0), 5: 0j, 6: 0j, 7: 0j}


def test_fp64_stage2_subnormal_column_hand_worked():
    r = ox.line_stage(_line(STAGE2_SUBNORMAL, 8), 8, 4, 2, stage=2)
    assert r["exp"][0] == -1073
    assert r["re"][0] == TWO52 * 2 ** 52
    assert r["im"][0] == TWO52 * 3 * 2 ** 51


# Stage 2 with the maximum in an imaginary part and a tie only visible at the
# shared exponent: column k2 = 0 = slots 0..3, e = 1 (from Im of slot 3).
#   y[0] = (2 - 2^-52)      exponent 0: y 2^51 = 2^52 - 1/2 -> tie -> 2^52 (even)
#   y[1] = 2^-51 1.5 + 0.5 2^-51 i: 1.5 -> 2, 0.5 -> 0  (ties to even)
#   y[2] = -(2^-51 2.5)     -2.5 -> -2
#   y[3] = 3 i              b~ = 3 2^51
#   sum a~ = 2^52 + 2 - 2 = 2^52,  sum b~ = 3 2^51
STAGE2_IMAG_MAX = {0: complex(2 - 2.0 ** -52, 0.0), 1: complex(1.5 * 2.0 ** -51, 0.5 * 2.0 ** -51),
                   2: complex(-2.5 * 2.0 ** -51, 0.0), 3: complex(0.0, 3.0),
                   4: 0j, 5: 0j, 6: 0j, 7: 0j}


def test_fp64_stage2_imaginary_maximum_hand_worked():
    r = ox.line_stage(_line(STAGE2_IMAG_MAX, 8), 8, 4, 2, stage=2)
    assert r["exp"][0] == 1
    assert r["re"][0] == TWO52 * 2 ** 52
    assert r["im"][0] == TWO52 * 3 * 2 ** 51
    assert r["exp"][1] is None          # column k2 = 1 (slots 4..7) is all zero
    assert r["re"][1] == 0 and r["im"][1] == 0


# FP32 target (k = 24, B = 23); the values are binary32 numbers.
# Stage 1, N = 8 (p = 2, q = 4), column 0, e = 0:
#   x[0] = 1 + 2^-23          a~ = 2^23 + 1
#   x[2] = 3 2^-25 + 2.5 2^-23 i     a~ = RNE(0.75) = 1, b~ = 2
#   x[4] = -3.5 2^-23 - 2.5 2^-23 i  a~ = -4, b~ = -2
#   x[6] = 0.5 - (1 - 2^-24) i       a~ = 2^22, b~ = -2^23 (tie carries into the next binade)
#   sum a~ = 2^23 + 2^22 - 2, sum b~ = -2^23
# column 1, e = 2 from Im only:
#   x[1] = 0.75 + 4 i         a~ = 0.75 2^21 = 3 2^19, b~ = 2^23
#   x[3] = 1.5 2^-20          a~ = 3
#   x[5] = 5 2^-22 - 7 2^-22 i  a~ = 2, b~ = -4
STAGE1_FP32 = {
    0: complex(1 + 2.0 ** -23, 0.0), 2: complex(3 * 2.0 ** -25, 2.5 * 2.0 ** -23),
    4: complex(-3.5 * 2.0 ** -23, -2.5 * 2.0 ** -23), 6: complex(0.5, -(1 - 2.0 ** -24)),
    1: complex(0.75, 4.0), 3: complex(1.5 * 2.0 ** -20, 0.0), 5: complex(5 * 2.0 ** -22, -7 * 2.0 ** -22),
    7: 0j,
}


def test_fp32_stage1_quantisation_hand_worked():
    x = _line(STAGE1_FP32, 8)
    assert np.all(x.astype(np.complex64).astype(np.complex128) == x)  # binary32 inputs
    r = ox.line_stage(x, 8, 2, 4, stage=1, precision=1)
    assert r["exp"] == [0, 2]
    assert r["re"][0] == TWO23 * (2 ** 23 + 2 ** 22 - 2)
    assert r["im"][0] == TWO23 * (-(2 ** 23))
    assert r["re"][1] == TWO23 * (3 * 2 ** 19 + 5)
    assert r["im"][1] == TWO23 * (2 ** 23 - 4)


def test_quantised_magnitude_below_2_to_k():
    # Eq. capacity: |x~| < 2^k.  The column maximum scales into [2^(k-1), 2^k)
    # exactly; the largest significand 2 - 2^-52 gives 2^53 - 1.
    x = _line({0: complex(-(2 - 2.0 ** -52), 2 - 2.0 ** -52), 2: 0j, 4: 0j, 6: 0j}, 8)
    r = ox.line_stage(x, 8, 2, 4, stage=1)
    assert r["exp"][0] == 0
    assert r["re"][0] == TWO52 * -(2 ** 53 - 1)
    assert r["im"][0] == TWO52 * (2 ** 53 - 1)
