// Pieces of the exact CRT reconstruction shared by the fused stage kernels
// and the standalone reconstruction kernels (device code, gfx950): the
// target-format traits, the split of a residue record between the two lane
// halves of the Phase-A MFMA, and Phase A itself (Sec. 4.2, Eqs. fcrt and
// slicing, on FP16 MFMA with FP32 accumulation).
#pragma once

#include "ob_device.h"

namespace obfft {

template <int TGT>
struct Tgt;
template <>
struct Tgt<0> {
  typedef double T;
  typedef double2 T2;
  typedef double V2 __attribute__((ext_vector_type(2)));  // one complex value as a plain vector
  static constexpr int PREC = 53, R = 12, S = 15, TZ = 6, NW = 4;
};
template <>
struct Tgt<1> {
  typedef float T;
  typedef float2 T2;
  typedef float V2 __attribute__((ext_vector_type(2)));
  static constexpr int PREC = 24, R = 6, S = 8, TZ = 6, NW = 3;
};

// Split of a residue record between the two lane halves of the Phase-A
// MFMA: the B operand of lane half h holds moduli ML h .. ML h + ML - 1 in
// its first ML slots (ML = 6 for r = 12, 4 for r = 6), zeros after.
template <int R>
struct RecSplit {
  static constexpr int RV = R / 2;              // packed FP16 pairs per output
  static constexpr int RH = (RV + 1) / 2;       // pairs supplied by the low half
  static constexpr int ML = 2 * RH;             // moduli per lane half
};

// Phase A for 64 scalar outputs (two 32x32x16 FP16 MFMAs) and the swap that
// gives every lane all partials of one output: lane l < 32 gets column l of
// b1's product, lane l >= 32 column l - 32 of b2's.  `seed` is the
// accumulator start 1.5 * 2^23 (the deposit bias), kept in VGPRs.
template <int NV>
__device__ __forceinline__ void phase_a(v8h aop, v8h b1, v8h b2, const v16f& seed, float* xv, float* yv) {
  v16f d1 = mfma_f16_32(aop, b1, seed);
  v16f d2 = mfma_f16_32(aop, b2, seed);
#pragma unroll
  for (int v = 0; v < NV; v++) {
    auto pr = __builtin_amdgcn_permlane32_swap(__float_as_uint(d1[v]), __float_as_uint(d2[v]),
                                               false, false);
    xv[v] = __uint_as_float(pr[0]);
    yv[v] = __uint_as_float(pr[1]);
  }
}

// Accumulator seeds of the Phase-A MFMA: register v of lane half h holds
// partial 2v + h, seeded with tbl[h][v] (1.5 * 2^23 plus the folded lift
// constants of that slice).
template <class TBL>  // float [2][16] in any address space
__device__ __forceinline__ v16f phase_a_seed(const TBL& tbl, int h) {
  v16f c;
  const auto* row = &tbl[h][0];
#pragma unroll
  for (int q = 0; q < 16; q++) c[q] = row[q];
  // opaque to the optimiser: the seed stays resident in 16 VGPRs instead of
  // being rematerialised before every MFMA
  asm volatile("" : "+v"(c));
  return c;
}

}  // namespace obfft
