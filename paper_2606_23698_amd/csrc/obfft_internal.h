// Internal definitions shared by the host plan code and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace obfft {

constexpr int kMaxModuli = 16;
constexpr int kMaxK = 32;          // longest contraction (p or q) of the fused stage kernel
constexpr int kThreads = 256;      // 4 waves of 64
constexpr int kTapStride = 40;     // uint32 words per output in the CRT debug taps

enum Substrate { SUB_FP8 = 0, SUB_INT8 = 1, SUB_FP16 = 2, SUB_AUTO = 3 };

// FP16 substrate: the first kFp16Split[precision] moduli of a set enter the
// residue GEMM as two radix-128 limbs per index; every later modulus as one
// FP16 slot per index, which needs 2 kMaxK floor(m/2) (floor(m/2) + 2) < 2^24
// (the largest possible partial sum of a 32-term, two-product accumulation,
// kept exact in FP32).  The default sets satisfy it from index 5 (r = 12:
// 961, 841, ...) and 4 (r = 6: 961, 841).
constexpr int kFp16Split[2] = {5, 4};

// Everything the CRT epilogue needs: Sec. 4.2 (Phase A over canonical
// residues, byte slices of u_k) and Sec. 5.1 (fractional lift, bias, M).
struct CrtConsts {
  int r;                 // number of moduli
  int S;                 // byte slices of u_k
  int T;                 // byte slices of w_k (f = 48)
  int nwords;            // 32-bit words of the lift arithmetic (4: FP64 set, 3: FP32 set)
  uint32_t M[4];         // M, little-endian words
  uint32_t Mhalf[4];     // M / 2
  uint32_t K0[4];        // (M/2 - Bp + zoff M) mod 2^128; Bp = implicit bias of the deposits
  uint64_t Czh;          // (2^47 - Bz + zoff 2^48) mod 2^64; Bz = implicit bias of the lift bytes
  uint32_t zoff;         // multiple of M added to E so that zhat stays unsigned
  uint32_t Bp5[5];       // Bp mod 2^160 (debug taps only)
};

// Per-modulus constants of the residue arithmetic.
struct ModConsts {
  int m[kMaxModuli];
  float inv_mf[kMaxModuli];
  double inv_md[kMaxModuli];
  int nd[kMaxModuli];    // digits per residue on the FP8 substrate (2 or 3)
  int sub[kMaxModuli];   // substrate of each modulus
};

// One Bailey stage of one axis, as launched.
struct StageParams {
  const void* in;
  void* out;
  int64_t ncols;        // stage 1: all columns; stage 2: columns per group
  int64_t inner;        // product of the faster extents
  int64_t N;            // axis length
  int64_t s_o;          // element stride between outer lines (N * inner)
  int64_t s_in_g, s_in_s, s_out_g, s_out_t;
  int K;                // contraction length (= output length)
  int G;                // number of column groups (p for stage 1, q for stage 2)
  int stage;
  int tiles_per_g;      // stage 2 only
  int extra_shift;      // added to the pack exponent
  const uint8_t* amat;  // MFMA A-operand planes of this stage / direction
  int64_t amat_g_stride;  // bytes per group g (0 for stage 1)
  int amat_fmax, amat_chmax, amat_mt;  // layout extents of the planes
  int64_t amat_mod_stride;  // bytes per modulus
  const uint16_t* phaseA;   // 64 lanes x 8 FP16 operand of the Phase-A MFMA
  uint16_t* dbg_res;        // canonical residues tap (may be null)
};

// Plan-time per-(N, p, q) operand set for one stage direction.
struct OperandPlanes {
  uint8_t* dev;          // device copy
  int64_t g_stride;      // bytes per group
  int64_t mod_stride;    // bytes per modulus
  int fmax, chmax, mt;
  int G;
};

}  // namespace obfft
