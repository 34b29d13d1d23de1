// gfx950 device building blocks of the Ozaki-Bailey kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "obfft_internal.h"

namespace obfft {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
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

// ---- MFMA wrappers ----
__device__ __forceinline__ v4f mfma_fp8(long a, long b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
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
// for VP <= v < VP + VZ.  Every partial is an FP32 value 2^23 + P exactly,
// i.e. its bit pattern is 0x4B000000 + P (the biased deposit of Alg. 2; the
// implicit bias is removed through the constant K0 / Czh).
template <int S, int TZ, int NW>
struct Epilogue {
  static constexpr int VP = (S + 1) / 2;
  static constexpr int VZ = (TZ + 1) / 2;
  static constexpr int NV = VP + VZ;

  __device__ __forceinline__ static uint32_t pbits(const float* xv, const float* yv, int s) {
    return __float_as_uint((s & 1) ? yv[s >> 1] : xv[s >> 1]);
  }
  __device__ __forceinline__ static uint32_t zbits(const float* xv, const float* yv, int t) {
    return __float_as_uint((t & 1) ? yv[VP + (t >> 1)] : xv[VP + (t >> 1)]);
  }

  // Biased deposits: E_b = sum_s bits(P_s) 2^{8s}, as 32-bit words (carry
  // sweep folded into 64-bit column sums of four slices each).
  __device__ __forceinline__ static void deposits(const float* xv, const float* yv, uint32_t* w,
                                                  uint32_t* w_top) {
    constexpr int NC = (S + 3) / 4;
    uint64_t col[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      uint64_t x = pbits(xv, yv, 4 * c);
#pragma unroll
      for (int j = 1; j < 4; j++)
        if (4 * c + j < S) x += (uint64_t)pbits(xv, yv, 4 * c + j) << (8 * j);
      col[c] = x;
    }
    uint64_t acc = col[0];
    w[0] = (uint32_t)acc;
#pragma unroll
    for (int c = 1; c < NC; c++) {
      acc = (acc >> 32) + col[c];
      w[c] = (uint32_t)acc;
    }
    *w_top = (uint32_t)(acc >> 32);
  }

  // zhat = round-half-up(2^-48 sum_t Z_t 256^t) (Sec. 5.1).
  __device__ __forceinline__ static uint32_t zhat(const float* xv, const float* yv, uint64_t czh) {
    uint64_t z = 0;
#pragma unroll
    for (int t = 0; t < TZ; t++) z += (uint64_t)zbits(xv, yv, t) << (8 * t);
    return (uint32_t)((z + czh) >> 48);
  }

  // X = E + M/2 - zhat M (mod 2^(32 NW)), then the two-sided correction into
  // [0, M) and R = X - M/2 in [-M/2, M/2) (Sec. 5.1, Alg. 2).
  __device__ __forceinline__ static void lift(const uint32_t* w, uint32_t zh, const CrtConsts& C,
                                              uint32_t* R) {
    uint32_t zm[NW];
    uint64_t p = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      p = (uint64_t)zh * C.M[i] + (p >> 32);
      zm[i] = (uint32_t)p;
    }
    uint32_t X[NW], cy = 0, bw = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) X[i] = addc(w[i], C.K0[i], cy, &cy);
#pragma unroll
    for (int i = 0; i < NW; i++) X[i] = subc(X[i], zm[i], bw, &bw);
    uint32_t Y[NW], Z[NW];
    bw = 0;
    cy = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) Y[i] = subc(X[i], C.M[i], bw, &bw);
#pragma unroll
    for (int i = 0; i < NW; i++) Z[i] = addc(X[i], C.M[i], cy, &cy);
    bool xneg = (int32_t)X[NW - 1] < 0;
    bool ypos = (int32_t)Y[NW - 1] >= 0;
    bw = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      uint32_t s = xneg ? Z[i] : (ypos ? Y[i] : X[i]);
      R[i] = subc(s, C.Mhalf[i], bw, &bw);
    }
  }
};

// Correctly rounded |R| 2^e with R given as NW two's-complement words;
// binary64 result.  Single rounding (Sec. 5.1): the top 64 bits plus a
// sticky bit are converted by one FP64 fma, whose rounding is exact RNE.
template <int NW>
__device__ __forceinline__ double pack_f64(const uint32_t* R, int e) {
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

// binary32 result; |R| < 2^63 (the FP32 modulus set has log2 M = 62.6).
template <int NW>
__device__ __forceinline__ float pack_f32(const uint32_t* R, int e) {
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
