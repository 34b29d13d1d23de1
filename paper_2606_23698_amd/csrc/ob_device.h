// gfx950 device building blocks of the Ozaki-Bailey kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "obfft_internal.h"

namespace obfft {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

// ---- residues (Sec. 2, Eq. ozaki: x~ mod m_i) ----

// Centred residue of an exact integer held in a double (|x| <= 2^54):
// x - m rne(x / m).  The quotient estimate errs by < 2/m, so |r| <= m/2 + 2.
__device__ __forceinline__ float residue_f64(double x, double m, double inv_m) {
  double qv = __builtin_rint(x * inv_m);
  return (float)__builtin_fma(-m, qv, x);
}

// Centred reduction of an exact FP32 integer (|x| < 2^24).
__device__ __forceinline__ float reduce_f32(float x, float m, float inv_m) {
  float qv = __builtin_rintf(x * inv_m);
  return __builtin_fmaf(-m, qv, x);
}

// Canonical residue in [0, m) of an exact FP32 integer (|x| < 2^24).  The
// centred step leaves |r| <= m/2 + 4; one conditional add makes it canonical.
__device__ __forceinline__ float canonical_f32(float x, float m, float inv_m) {
  float r = reduce_f32(x, m, inv_m);
  return r < 0.0f ? r + m : r;
}

// A centred residue of an exact FP32 integer (|x| <= 2^24) by the
// fold-and-add reduction of a friendly modulus m = 2^b - c (Sec. 2; rung H0
// of the co-design ladder, Sec. 8.3).  Since 2^b = c (mod m), t = 2^b h + l
// (h = t >> b arithmetic, l = t mod 2^b) is congruent to c h + l.  nf folds
// leave t in [-c, 2^b - 1 + c]; one conditional subtraction then gives
// [-floor(m/2), m - floor(m/2)).  m = 2^b (c = 0): the low b bits,
// sign-extended.
__device__ __forceinline__ float fold_reduce_f32(float x, int m, int b, int c, int nf) {
  int t = (int)x;
  if (c == 0) return (float)((int)((uint32_t)t << (32 - b)) >> (32 - b));
  const int mask = (1 << b) - 1;
  for (int f = 0; f < nf; f++) t = __mul24(c, t >> b) + (t & mask);  // |t >> b| < 2^23: one v_mad_i32_i24
  return (float)(t >= m - (m >> 1) ? t - m : t);
}

// ---- MFMA wrappers ----
__device__ __forceinline__ v4f mfma_fp8(long a, long b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}
// Scaled 16 x 16 x 128 FP8 (E4M3 x E4M3) MFMA: lane group h's 32-byte block
// of A is multiplied by 2^(sa - 127); B unscaled.
__device__ __forceinline__ v4f mfma_fp8_k128(v8i a, v8i b, v4f c, int sa) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, 127);
}
__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_f16_16(v8h a, v8h b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mfma_f16_32(v8h a, v8h b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Two E4M3 bytes from two small exact integers (|d| <= 16), written into the
// low (hi == false) or high half of `old`.
template <bool HI>
__device__ __forceinline__ uint32_t fp8_pack2(float a, float b, uint32_t old) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, (int)old, HI);
}

__device__ __forceinline__ uint32_t addc(uint32_t a, uint32_t b, uint32_t cin, uint32_t* cout) {
  return __builtin_addc(a, b, cin, cout);
}
__device__ __forceinline__ uint32_t subc(uint32_t a, uint32_t b, uint32_t bin, uint32_t* bout) {
  return __builtin_subc(a, b, bin, bout);
}

// ---- Phase B: Kulisch deposits, two-sided lift, correctly rounded pack ----
//
// Inputs are the Phase-A partials after the lane-half swap: register pair v
// holds (xv[v], yv[v]) = (partial 2v, partial 2v+1) of P for v < VP and of Z
// for VP <= v < VP + VZ.  Every partial is the FP32 value seed_j + P_j in the
// binade [2^23, 2^24), so its bit pattern is bits(seed_j) + P_j: the biased
// deposit of Alg. 2, whose bias (with every other additive constant of the
// lift) the host folds into the seeds.
template <int S, int TZ, int NW>
struct Epilogue {
  static constexpr int VP = (S + 1) / 2;
  static constexpr int VZ = (TZ + 1) / 2;
  static constexpr int NV = VP + VZ;
  static_assert(TZ == 6, "the lift sum reads six slices");

  __device__ __forceinline__ static uint32_t pbits(const float* xv, const float* yv, int s) {
    return __float_as_uint((s & 1) ? yv[s >> 1] : xv[s >> 1]);
  }
  __device__ __forceinline__ static uint32_t zbits(const float* xv, const float* yv, int t) {
    return __float_as_uint((t & 1) ? yv[VP + (t >> 1)] : xv[VP + (t >> 1)]);
  }

  // Column of the four patterns b0..b3 at bits 32c, 32c+8, 32c+16, 32c+24:
  // the low word L (mod 2^32) and the spill H into word c+1.  b1 << 8 fits
  // beside b0 (b0 < 2^31, (b1 << 8) mod 2^32 < 2^31) and drops b1's top byte,
  // which is the constant 0x4B of every pattern (put back by the seeds); the
  // spills of b2 and b3 are kept, with the two carries of L.
  template <int NB>
  __device__ __forceinline__ static void column(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, uint32_t& L,
                                                uint32_t& H) {
    uint32_t l = b0, h = 0, cy;
    if (NB > 1) l += b1 << 8;
    if (NB > 2) {
      l = addc(l, b2 << 16, 0u, &cy);
      h = (b2 >> 16) + cy;
    }
    if (NB > 3) {
      l = addc(l, b3 << 24, 0u, &cy);
      h = h + (b3 >> 8) + cy;
    }
    L = l;
    H = h;
  }

  // W = sum_s bits_s 256^s - dropped + khi 2^(32(NW-1))  (mod 2^(32 NW)).
  __device__ __forceinline__ static void deposits(const float* xv, const float* yv, uint32_t khi, uint32_t* w) {
    constexpr int NC = (S + 3) / 4;
    uint32_t L[NC], H[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      const int nb = S - 4 * c < 4 ? S - 4 * c : 4;
      uint32_t b0 = pbits(xv, yv, 4 * c);
      uint32_t b1 = nb > 1 ? pbits(xv, yv, 4 * c + 1) : 0u;
      uint32_t b2 = nb > 2 ? pbits(xv, yv, 4 * c + 2) : 0u;
      uint32_t b3 = nb > 3 ? pbits(xv, yv, 4 * c + 3) : 0u;
      if (nb == 4) column<4>(b0, b1, b2, b3, L[c], H[c]);
      else if (nb == 3) column<3>(b0, b1, b2, b3, L[c], H[c]);
      else if (nb == 2) column<2>(b0, b1, b2, b3, L[c], H[c]);
      else column<1>(b0, b1, b2, b3, L[c], H[c]);
    }
    w[0] = L[0];
    uint32_t cy = 0;
#pragma unroll
    for (int i = 1; i < NW; i++) {
      uint32_t a = i < NC ? L[i] : 0u;
      uint32_t b = i - 1 < NC ? H[i - 1] : 0u;
      w[i] = addc(a, b, cy, &cy);
    }
    w[NW - 1] += khi;
  }

  // zhat + zoff = round-half-up(2^-48 sum_t Z_t 256^t) + zoff (Sec. 5.1): word
  // 1 of the seeded sum (the seeds carry 2^47 and zoff 2^48), bits 16..31.
  __device__ __forceinline__ static uint32_t zhat(const float* xv, const float* yv, uint32_t zhi) {
    uint32_t L0, H0;
    column<4>(zbits(xv, yv, 0), zbits(xv, yv, 1), zbits(xv, yv, 2), zbits(xv, yv, 3), L0, H0);
    (void)L0;
    uint32_t w1 = H0 + zbits(xv, yv, 4) + (zbits(xv, yv, 5) << 8) + zhi;
    return w1 >> 16;
  }

  // Full pattern sum sum_s bits_s 256^s mod 2^160 (debug taps only).
  __device__ __forceinline__ static void deposits_full(const float* xv, const float* yv, uint32_t* w5) {
    uint64_t acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < S; s++) {
      int pos = 8 * s, wi = pos >> 5, sh = pos & 31;
      uint64_t v = (uint64_t)pbits(xv, yv, s) << sh;
      acc[wi] += (uint32_t)v;
      if (wi + 1 < 5) acc[wi + 1] += v >> 32;
    }
    uint64_t cy = 0;
#pragma unroll
    for (int i = 0; i < 5; i++) {
      uint64_t t = acc[i] + cy;
      w5[i] = (uint32_t)t;
      cy = t >> 32;
    }
  }

  // Lift constants held in registers for the whole epilogue (read once from
  // the plan's device copy, never re-read inside a round).
  struct LiftK {
    uint32_t M[NW], Mhalf[NW];
    uint32_t khi, zhi;
  };
  template <class CC>  // CrtConsts in any address space
  __device__ __forceinline__ static LiftK load_lift(const CC& C, bool exact) {
    LiftK k;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      k.M[i] = C.M[i];
      k.Mhalf[i] = C.Mhalf[i];
    }
    k.khi = exact ? C.khi_x : C.khi_c;
    k.zhi = C.zhi;
    return k;
  }

  __device__ __forceinline__ static void times_m(uint32_t zh, const LiftK& K, uint32_t* zm) {
    uint64_t p = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      p = (uint64_t)zh * K.M[i] + (p >> 32);
      zm[i] = (uint32_t)p;
    }
  }

  // Exact two-sided lift (Sec. 5.1, Alg. 2): with W = E + M/2 + zoff M,
  // X = W - (zhat + zoff) M = E - zhat M + M/2, corrected into [0, M) from
  // either side, and R = X - M/2 in [-M/2, M/2).
  __device__ __forceinline__ static void lift_exact(const uint32_t* w, uint32_t zh, const LiftK& K, uint32_t* R) {
    uint32_t zm[NW], X[NW], Y[NW], Z[NW], bw = 0, cy = 0;
    times_m(zh, K, zm);
#pragma unroll
    for (int i = 0; i < NW; i++) X[i] = subc(w[i], zm[i], bw, &bw);
    bw = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) Y[i] = subc(X[i], K.M[i], bw, &bw);
#pragma unroll
    for (int i = 0; i < NW; i++) Z[i] = addc(X[i], K.M[i], cy, &cy);
    bool xneg = (int32_t)X[NW - 1] < 0;
    bool ypos = (int32_t)Y[NW - 1] >= 0;
    bw = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      uint32_t s = xneg ? Z[i] : (ypos ? Y[i] : X[i]);
      R[i] = subc(s, K.Mhalf[i], bw, &bw);
    }
  }

  // The lift under the capacity bound (Eq. capacity): with W = E + zoff M,
  // X = W - (zhat + zoff) M = E - zhat M.  A stage output has |C| < 2^(cap-1)
  // (2^113 at K = 32), far below M/4, and E = C + z M, so E/M lies within 1/4
  // of the integer z; the fixed-point quotient differs from E/M by less than
  // r max|v| / 2^49 (about 2^-35), so zhat = z and X = C exactly: the
  // two-sided correction of the general lift is identically zero here.
  __device__ __forceinline__ static void lift_bounded(const uint32_t* w, uint32_t zh, const LiftK& K, uint32_t* R) {
    uint32_t zm[NW], bw = 0;
    times_m(zh, K, zm);
#pragma unroll
    for (int i = 0; i < NW; i++) R[i] = subc(w[i], zm[i], bw, &bw);
  }
};

// Correctly rounded R 2^e with R given as NW two's-complement words;
// binary64 result.  Single rounding (Sec. 5.1).
//
// Common case (four words, |R| >= 2^75, normal result): with R = H 2^64 + L
// (H signed, |H| < 2^53, L unsigned), L is rounded to odd at 2^21 (cut below
// 2^21, bit 21 set when anything was cut).  The rounding position of R is
// at least 2^23, so R and the rounded-to-odd R' lie strictly inside the same
// interval between consecutive even multiples of 2^21 and round alike; H and
// the 43-bit L' are exact doubles and one fma H 2^64 + L' rounds R' once.
// Otherwise the top 64 bits of |R| plus a sticky bit are converted by one
// fma, and subnormal results are rounded at 2^-1074 in integers.
template <int NW>
__device__ __forceinline__ double pack_f64(const uint32_t* R, int e) {
  if (NW == 4) {
    const int64_t H = (int64_t)(((uint64_t)R[NW - 1] << 32) | R[NW - 2]);
    if ((uint64_t)(H + 2048) >= 4096u && e >= -1097) {
      const uint32_t r0 = (R[0] & ~0x1FFFFFu) | ((R[0] & 0x1FFFFFu) ? 0x200000u : 0u);
      const double hd = __builtin_fma((double)(int32_t)R[NW - 1], 4294967296.0, (double)R[NW - 2]);
      const double ld = __builtin_fma((double)R[1], 4294967296.0, (double)r0);
      return __builtin_ldexp(__builtin_fma(hd, 18446744073709551616.0, ld), e);
    }
  }
  uint32_t sm = (uint32_t)((int32_t)R[NW - 1] >> 31);
  uint32_t a[4] = {0, 0, 0, 0};
  uint32_t cy = sm & 1u;
#pragma unroll
  for (int i = 0; i < NW; i++) a[i] = addc(R[i] ^ sm, 0u, cy, &cy);
  uint64_t hi = ((uint64_t)a[3] << 32) | a[2];
  uint64_t lo = ((uint64_t)a[1] << 32) | a[0];
  uint64_t t;
  int sh;
  if (hi) {
    int lz = __builtin_clzll(hi);
    sh = 64 - lz;
    t = (hi << lz) | (lo >> sh) | (uint64_t)((lo << lz) != 0);
  } else {
    t = lo;
    sh = 0;
  }
  int e2 = sh + e;
  double r;
  int top = 63 - (t ? __builtin_clzll(t) : 63) + e2;  // binary exponent of the result
  if (__builtin_expect(top >= -1022 || t == 0, 1)) {
    double d = __builtin_fma((double)(uint32_t)(t >> 32), 4294967296.0, (double)(uint32_t)t);
    r = __builtin_ldexp(d, e2);
  } else {
    // subnormal result: round once at the fixed position 2^-1074
    int drop = -1074 - e2;
    uint64_t qv;
    if (drop <= 0) {
      qv = t << (-drop);
    } else if (drop >= 64) {
      qv = 0;
    } else {
      qv = t >> drop;
      uint64_t rem = t - (qv << drop);
      uint64_t half = (uint64_t)1 << (drop - 1);
      if (rem > half || (rem == half && (qv & 1))) qv++;
    }
    r = __builtin_ldexp((double)qv, -1074);
  }
  return sm ? -r : r;
}

// binary32 result; |R| < 2^63 (the FP32 modulus set has log2 M = 62.6), so
// word 2 only repeats the sign of word 1.  Common case |R| >= 2^40: the
// rounding position is at least 2^17, R rounded to odd at 2^15 is an exact
// double (48 bits), and one conversion to binary32 rounds it as it would R.
template <int NW>
__device__ __forceinline__ float pack_f32(const uint32_t* R, int e) {
  if (NW == 3 && R[1] + 256u >= 512u && e >= -1000) {
    const uint32_t r0 = (R[0] & ~0x7FFFu) | ((R[0] & 0x7FFFu) ? 0x8000u : 0u);
    const double d = __builtin_fma((double)(int32_t)R[1], 4294967296.0, (double)r0);
    return (float)__builtin_ldexp(d, e);
  }
  uint32_t sm = (uint32_t)((int32_t)R[NW - 1] >> 31);
  uint32_t a[NW];
  uint32_t cy = sm & 1u;
#pragma unroll
  for (int i = 0; i < NW; i++) a[i] = addc(R[i] ^ sm, 0u, cy, &cy);
  uint64_t t = ((uint64_t)a[1] << 32) | a[0];
  int nb = t ? 64 - __builtin_clzll(t) : 0;
  int sh = nb > 32 ? nb - 32 : 0;
  uint32_t t32 = (uint32_t)(t >> sh) | (uint32_t)(sh && (t << (64 - sh)) != 0);
  int e2 = sh + e;
  float r;
  int top = (nb ? nb - 1 - sh : 0) + e2;
  if (__builtin_expect(top >= -126 || t32 == 0, 1)) {
    r = __builtin_ldexpf((float)t32, e2);
  } else {
    int drop = -149 - e2;
    uint32_t qv;
    if (drop <= 0) {
      qv = t32 << (-drop);
    } else if (drop >= 32) {
      qv = 0;
    } else {
      qv = t32 >> drop;
      uint32_t rem = t32 - (qv << drop);
      uint32_t half = 1u << (drop - 1);
      if (rem > half || (rem == half && (qv & 1))) qv++;
    }
    r = __builtin_ldexpf((float)qv, -149);
  }
  return sm ? -r : r;
}

}  // namespace obfft
