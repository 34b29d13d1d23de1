#pragma once
// Ozaki-Bailey stage kernels for gfx950 (MI355X).
//
// One launch computes one Bailey stage of one axis for every line of the
// array (Alg. 1): per contraction column it extracts the shared power-of-two
// scale, quantises Re and Im to k-bit integers, reduces them modulo every
// m_i (Sec. 2, Eq. ozaki), runs the complex residue GEMM per modulus on MFMA
// as four real products accumulated straight into R and I (Sec. 2; Sec. 4.1
// Eq. wmma; the paper's three Karatsuba products plus combines cost vector
// work that the matrix cores do not), reduces R and I to centred residues
// in the residue domain (Alg. 1), and reconstructs each
// output exactly by the Phase-A FP16 MFMA GEMM (Sec. 4.2) and the Kulisch
// Phase B with the two-sided lift and a correctly rounded pack (Sec. 5.1,
// Alg. 2).  The only FP64 arithmetic is the exponent/scale extraction and
// quantisation at the start and the single rounding at the end.
//
// Work decomposition: a workgroup of 4 waves owns 32 (K > 16) or 64
// contraction columns.  All columns of a workgroup share one stage matrix
// (stage 2: the same k2, so the same twiddle-fused F_p^(k2), Sec. 4.1).  Per
// modulus:
//   decon   every thread reduces K/TPC elements of one column and writes
//           their digit planes to LDS in the MFMA B-operand layout;
//   GEMM    each wave multiplies its 16-row M-tile of the matrix planes (held
//           in registers) with its 16-column N-tile from LDS;
//   combine the centred residues of R and I of the wave's 16 x 16 outputs
//           are packed as FP16 into registers: every lane keeps the residue
//           record of its own 8 outputs (4 rows x Re/Im) over all moduli.
// After the last modulus every lane reconstructs its own outputs: Phase A
// runs on 64 outputs at a time (two 32x32x16 FP16 MFMAs fed by a cross-half
// lane swap of the records, then one swap of the partials back), followed by
// the integer epilogue and one coalesced 16-byte store per complex output.
#include "ob_recon.h"

namespace obfft {

// K-chunks of one MFMA operand plane: INT8 64 slots (2 limbs per index),
// FP16 32 slots (2 limbs per index), FP8 32 slots (up to 4 digits per index).
__host__ __device__ constexpr int chunks_for(int sub, int K) {
  return sub == SUB_INT8 ? (2 * K + 63) / 64 : sub == SUB_FP16 ? (2 * K + 31) / 32 : (4 * K + 31) / 32;
}

__host__ __device__ constexpr int align16(int x) { return (x + 15) & ~15; }

// Workgroup shape for contraction length K (<= KMAX): MT 16-row M-tiles of
// the stage matrix and NT 16-column N-tiles, one (M-tile, N-tile) pair per
// wave, four waves.  K = 32 uses 32 columns so that two workgroups fit in
// one CU's LDS.
template <int KMAX>
struct Shape {
  static constexpr int MT = (KMAX + 15) / 16;
  static constexpr int NT = 4 / MT;
  static constexpr int NCOL = 16 * NT;
  static constexpr int TPC = kThreads / NCOL;           // threads per column in the decon
  static constexpr int KQ = (KMAX + TPC - 1) / TPC;     // elements per thread
};

// Data operand planes of one modulus: the two forms (a~, b~) of the
// four-product complex GEMM, FP8 room for three (the full-length tile adds
// -b~).
__host__ __device__ constexpr int dig_bytes(int sub, int kmax, int nt) {
  return (sub == SUB_FP8 ? 3 : 2) * chunks_for(sub, kmax) * nt * 64 * (sub == SUB_FP8 ? 8 : 16);
}

// LDS of one workgroup: two digit buffers (even / odd moduli), the column
// input and output offsets, the column exponents and the per-thread partial
// exponents.
template <int SUB, int TGT, int KMAX>
struct StageLds {
  typedef Shape<KMAX> SH;
  static constexpr int DIG = dig_bytes(SUB, KMAX, SH::NT);
  __host__ __device__ static int bytes(int) { return 2 * DIG + SH::NCOL * 20 + kThreads * 4; }
};

// Writes the digit planes of residue v (exact small integer) of column jc,
// contraction index s, data form `form` (0: a~, 1: b~).
// Byte offset of K-slot `slot` of column jc in one form's FP8 planes
// ([chunk][N-tile][lane][8 bytes]: slot kk of a chunk sits in lane
// (jc % 16) + 16 (kk / 8) at byte kk % 8).
template <int CHB, int NT>
__device__ __forceinline__ int fp8_slot(int form, int jc, int slot) {
  const int ch = slot >> 5, kk = slot & 31;
  return (((form * CHB + ch) * NT + (jc >> 4)) * 64 + (jc & 15) + 16 * (kk >> 3)) * 8 + (kk & 7);
}

// FP8 digit slots of index s: three slots 3s .. 3s + 2 for a 3-digit
// residue (they may straddle lanes and chunks, so bytes are written one by
// one), two slots 2s, 2s + 1 for a 2-digit one (one 16-bit store).
template <int SUB, int CHB, int NT>
__device__ __forceinline__ void put_digits_fp8(unsigned char* dig, int form, int jc, int s, float v, int nd) {
  if (nd == 3) {
    // balanced radix-32 digits, |d| <= 16, exact in E4M3
    float t1 = __builtin_rintf(v * 0.03125f);
    float d0 = __builtin_fmaf(-32.0f, t1, v);
    float t2 = __builtin_rintf(t1 * 0.03125f);
    float d1 = __builtin_fmaf(-32.0f, t2, t1);
    uint32_t wd = fp8_pack2<false>(d0, d1, 0u);
    wd = fp8_pack2<true>(t2, 0.0f, wd);
#pragma unroll
    for (int e = 0; e < 3; e++) dig[fp8_slot<CHB, NT>(form, jc, 3 * s + e)] = (unsigned char)(wd >> (8 * e));
  } else {
    float t1 = __builtin_rintf(v * 0.03125f);
    float d0 = __builtin_fmaf(-32.0f, t1, v);
    uint32_t wd = fp8_pack2<false>(d0, t1, 0u);
    *(uint16_t*)(dig + fp8_slot<CHB, NT>(form, jc, 2 * s)) = (uint16_t)wd;
  }
}

// Full-length FP8 tile on the scaled K = 128 MFMA: data digit e of indices
// s0 .. s0 + 3 (s0 % 4 == 0) of column jc in one form, one aligned word per
// digit, in planes [form][e][N-tile][column][32 indices]; NEG: also the
// negated digits (E4M3 sign bits flipped) as form + 1.
template <int NT, int ND, bool NEG = false>
__device__ __forceinline__ void put_digits_fp8_k128(unsigned char* dig, int form, int jc, int s0, const float* v) {
  float d[3][4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const float t1 = __builtin_rintf(v[u] * 0.03125f);
    d[0][u] = __builtin_fmaf(-32.0f, t1, v[u]);
    if (ND == 3) {
      const float t2 = __builtin_rintf(t1 * 0.03125f);
      d[1][u] = __builtin_fmaf(-32.0f, t2, t1);
      d[2][u] = t2;
    } else {
      d[1][u] = t1;
    }
  }
#pragma unroll
  for (int e = 0; e < ND; e++) {
    const uint32_t w = fp8_pack2<true>(d[e][2], d[e][3], fp8_pack2<false>(d[e][0], d[e][1], 0u));
    *(uint32_t*)(dig + ((form * 3 + e) * NT + (jc >> 4)) * 512 + (jc & 15) * 32 + s0) = w;
    if (NEG) *(uint32_t*)(dig + (((form + 1) * 3 + e) * NT + (jc >> 4)) * 512 + (jc & 15) * 32 + s0) = w ^ 0x80808080u;
  }
}

// INT8 limbs of a residue v (|v| <= 2043): v = d0 + 128 d1 with the low limb
// d0 = v mod 128 in [0, 127] and the high limb d1 = floor(v / 128) in
// [-16, 15], both valid signed bytes.  Returns the 16-bit pair (d0 | d1 << 8).
__device__ __forceinline__ uint32_t i8_limbs(int v) {
  return (((uint32_t)v << 1) & 0xFF00u) | ((uint32_t)v & 0x7Fu);
}

// Byte offset of contraction index s of column jc in one form's INT8 planes
// ([N-tile][lane][16 bytes]: lane (jc % 16) + 16 (s / 8), byte 2 (s % 8)).
__device__ __forceinline__ int i8_slot(int jc, int s) {
  return ((jc >> 4) * 64 + (jc & 15) + 16 * (s >> 3)) * 16 + 2 * (s & 7);
}

// Writes the limb pairs of KQ consecutive contraction indices s0.. of one
// column and one data form (KQ = 1, 2, 4 stay inside one lane's 16
// bytes and take one store; KQ = 3 may cross a lane and stores per index).
template <int KQ>
__device__ __forceinline__ void put_limbs(unsigned char* form_base, int jc, int s0, const uint32_t* w) {
  if (KQ == 4) {
    *(uint2*)(form_base + i8_slot(jc, s0)) = make_uint2(w[0] | (w[1] << 16), w[2] | (w[3] << 16));
  } else if (KQ == 2) {
    *(uint32_t*)(form_base + i8_slot(jc, s0)) = w[0] | (w[1] << 16);
  } else {
#pragma unroll
    for (int u = 0; u < KQ; u++) *(uint16_t*)(form_base + i8_slot(jc, s0 + u)) = (uint16_t)w[u];
  }
}

// FP16 limbs of a residue r (|r| <= 1022): r = d0 + 128 d1 with balanced
// d0 = r - 128 rne(r / 128) in [-64, 64] and d1 in [-8, 8], packed as two
// halves (d0 low).  Both are exact in FP16 (the conversion truncates, and
// small integers need no rounding).
__device__ __forceinline__ uint32_t f16_limbs(float r) {
  float t = __builtin_rintf(r * 0.0078125f);
  float d0 = __builtin_fmaf(-128.0f, t, r);
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(d0, t));
}

// Byte offset of contraction index s of column jc in one form's FP16 planes
// ([chunk][N-tile][lane][8 halves]; slots 2s, 2s + 1 of chunk s / 16 sit in
// lane (jc % 16) + 16 ((s % 16) / 4) at half 2 (s % 4)).
template <int NT>
__device__ __forceinline__ int f16_slot(int jc, int s) {
  return ((s >> 4) * NT + (jc >> 4)) * 1024 + ((jc & 15) + 16 * ((s & 15) >> 2)) * 16 + 4 * (s & 3);
}

// Byte offset of index s of column jc in one form's single-slot FP16 planes
// (moduli past the split: slot s of chunk s / 32 sits in lane
// (jc % 16) + 16 ((s % 32) / 8) at half s % 8).
template <int NT>
__device__ __forceinline__ int f16_slot1(int jc, int s) {
  return ((s >> 5) * NT + (jc >> 4)) * 1024 + ((jc & 15) + 16 * ((s & 31) >> 3)) * 16 + 2 * (s & 7);
}

// Writes the residues r[0..KQ) of indices s0.. as single FP16 slots (KQ = 4
// and 2 start on a multiple of KQ: one store inside one lane).
template <int KQ, int NT>
__device__ __forceinline__ void put_slots16(unsigned char* form_base, int jc, int s0, const float* r) {
  if (KQ == 4) {
    uint32_t w0 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(r[0], r[1]));
    uint32_t w1 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(r[2], r[3]));
    *(uint2*)(form_base + f16_slot1<NT>(jc, s0)) = make_uint2(w0, w1);
  } else if (KQ == 2) {
    *(uint32_t*)(form_base + f16_slot1<NT>(jc, s0)) =
        __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(r[0], r[1]));
  } else {
    // one 16-bit store per index (three indices may straddle two lanes).  The
    // conversion goes through the packing instruction: a plain cast of a value
    // computed in FP64 became a software double-to-half conversion of some
    // twenty instructions (the residues are small integers, exact either way).
#pragma unroll
    for (int u = 0; u < KQ; u += 2) {
      const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(r[u], u + 1 < KQ ? r[u + 1] : 0.0f));
      *(uint16_t*)(form_base + f16_slot1<NT>(jc, s0 + u)) = (uint16_t)w;
      if (u + 1 < KQ) *(uint16_t*)(form_base + f16_slot1<NT>(jc, s0 + u + 1)) = (uint16_t)(w >> 16);
    }
  }
}

// Writes the packed limb pairs of KQ consecutive indices s0.. (KQ = 4 starts
// on a multiple of 4 and KQ = 2 on an even index: one store inside one lane).
template <int KQ, int NT>
__device__ __forceinline__ void put_limbs16(unsigned char* form_base, int jc, int s0, const uint32_t* w) {
  if (KQ == 4) {
    *(uint4*)(form_base + f16_slot<NT>(jc, s0)) = make_uint4(w[0], w[1], w[2], w[3]);
  } else if (KQ == 2) {
    *(uint2*)(form_base + f16_slot<NT>(jc, s0)) = make_uint2(w[0], w[1]);
  } else {
#pragma unroll
    for (int u = 0; u < KQ; u++) *(uint32_t*)(form_base + f16_slot<NT>(jc, s0 + u)) = w[u];
  }
}

// Dynamic LDS of the stage and batch kernels.  Referenced directly (not
// through a pointer argument) so that every access keeps the LDS address
// space after inlining.
extern __shared__ __align__(16) unsigned char smem[];

// FULL: the contraction length equals KMAX (K = 8, 12, 16 or 32 on the FP16
// substrate: every power-of-two split from 64 on and the 12-point factors of
// 96 and 192), so every bound on K is known when compiling.
// Pointers read from a descriptor in memory (the batched launch) are
// generic to the compiler: every access through them would be a flat access
// and every constant a vector load.  The stage body therefore reads and
// writes through pointers typed with their address space: global (1) for
// data, constant (4) for the plan's read-only tables (scalar loads).
#define OB_GLOBAL __attribute__((address_space(1)))
#define OB_CONST __attribute__((address_space(4)))

// n / d for n < 2^31 by a multiply-high with the plan's magic number.
__device__ __forceinline__ uint32_t udiv31(uint32_t n, uint32_t magic, uint32_t shift) {
  return magic ? (__umulhi(n, magic) >> shift) : n;
}

// (column tile, group) of linear tile index `tile` of a stage.  Stage 2 on
// the contiguous axis (g_minor): a tile writes 16 bytes per output row at a
// stride of q elements; the 8 tiles of one column tile with k2 = 8b .. 8b + 7
// together fill whole 128-byte lines.  Workgroups go to the 8 XCDs round
// robin (workgroup w on XCD w % 8), each with its own L2: XCD x takes the
// column tiles c = 8 j + x, and for one block of gblock groups at a time
// runs those groups of a column tile back to back, so that the partial lines
// merge in that L2 while only gblock groups' matrix planes are live in it.
template <class PT>  // StageParams in any address space
__device__ __forceinline__ void decode_tile(const PT& P, int64_t tile, int64_t& c, int64_t& g) {
  if (P.stage == 1) {
    c = tile;
    g = 0;
  } else if (!P.g_minor) {
    g = tile / P.tiles_per_g;
    c = tile % P.tiles_per_g;
  } else {
    const int64_t T = P.tiles_per_g, G = P.G;
    const int64_t GB = P.gblock;
    if ((T & 7) == 0) {
      const int64_t x = tile & 7, slot = tile >> 3, per_blk = (T >> 3) * GB;
      const int64_t blk = slot / per_blk, rem = slot % per_blk;
      g = blk * GB + rem % GB;
      c = (rem / GB) * 8 + x;
    } else {
      const int64_t per_blk = T * GB, blk = tile / per_blk, rem = tile % per_blk;
      g = blk * GB + rem % GB;
      c = rem / GB;
    }
  }
}

// The same order read off a 1-, 2- or 3-D grid without divisions (grid_mode):
// the hardware's linear workgroup order is x fastest, then y, then z.
__device__ __forceinline__ void grid_tile(const StageParams& P, int64_t& c, int64_t& g) {
  const int64_t bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  switch (P.grid_mode) {
    case 1: c = bx; g = 0; break;
    case 2: c = bx; g = by; break;
    case 3: {
      const int64_t GB = P.gblock;
      c = by * 8 + (bx & 7);
      g = bz * GB + (bx >> 3);
      break;
    }
    case 4: {
      const int64_t GB = P.gblock;
      c = by;
      g = bz * GB + bx;
      break;
    }
    default: decode_tile(P, bx, c, g);
  }
}

// H0: the residue reduction after the GEMM takes the fold-and-add form for
// the friendly moduli (FP16 substrate; the reciprocal form otherwise).
// NP > 1: NP columns of a K <= 16 / NP stage per 16-row tile (fp16_pack): the
// tile runs as a full K = 16 contraction over block-diagonal planes with
// blocks of BR = 16 / NP rows; decon thread part p loads column p / (4 / NP)
// of its group and lanes 16 BR/4 b .. of the epilogue reconstruct column b.
// TAP: the debug variant, which also writes the canonical residues of every
// output (P.dbg_res) and the epilogue record of every output of one line
// (P.dbg_tap, P.dbg_line); the production kernels are built without it.
// PT: StageParams in any address space (a kernel argument, or a descriptor
// in the constant space read field by field where it is used).
template <int SUB, int TGT, int KMAX, bool FULL = false, bool H0 = false, int NP = 1, bool TAP = false,
          class PT = StageParams>
__device__ __forceinline__ void stage_tile(const PT& P, int64_t ctile, int64_t g) {
  typedef Tgt<TGT> TT;
  typedef Shape<KMAX> SH;
  typedef StageLds<SUB, TGT, KMAX> LY;
  typedef RecSplit<TT::R> RS;
  constexpr int R = TT::R;
  constexpr int MT = SH::MT, NT = SH::NT, NCOL = SH::NCOL, TPC = SH::TPC, KQ = SH::KQ;
  constexpr int CHB = chunks_for(SUB, KMAX);
  constexpr int DIG = LY::DIG;
  typedef Epilogue<TT::S, TT::TZ, TT::NW> EP;

  constexpr bool PK = NP > 1;
  constexpr int BR = 16 / NP;                // rows and contraction slots per packed column
  static_assert(NP == 1 || ((NP == 2 || NP == 4) && SUB == SUB_FP16 && KMAX == 16 && FULL && SH::TPC == 4),
                "packed columns: FP16, full 16-row tile, four parts per column");
  constexpr int NCR = NP * NCOL;             // columns of the stage per tile
  const int K = FULL ? KMAX : P.K;           // contraction length of the tile
  const int KR = PK ? P.K : K;               // of one column (packed: <= BR)
  int64_t* col_in = (int64_t*)(smem + 2 * DIG);
  int64_t* col_out = col_in + NCR;
  int* cexp = (int*)(col_out + NCR);
  int* pexp = cexp + NCR;

  // opaque to the optimiser: a persistent caller must not keep values derived
  // from the thread index live across its loop (they are cheap to recompute)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: tile addressing stays scalar
  const int64_t cstart = ctile * NCR;
  // Wave priority: a wave runs at priority 1 from here (column tables, input
  // loads, exponents) to the barrier after the exponents, and in every modulus
  // from the top of the iteration to its barrier (A-plane loads,
  // deconstruction, digit stores, the deferred combine); at priority 0 in the
  // GEMMs and the epilogue.  The issue arbiter then serves the waves of
  // workgroups that are starting, and of those that hold their next barrier,
  // first, while the waves past it fill the gaps: about 3 % off the 1024^3
  // transform, measured on several machines.  The start of the tile carries
  // most of it; priority in the epilogue instead costs 0.5-1.5 %.
  __builtin_amdgcn_s_setprio(1);
  if (tid < NCR) {
    // column c = (i, g, o) of the stage, i fastest (stage 2: g is the tile's)
    const int64_t c = cstart + tid;
    int64_t ci = -1, co = -1;
    if (c < P.ncols) {
      const uint32_t c32 = (uint32_t)c;  // ncols < 2^31 (checked by the plan)
      const uint32_t rest = udiv31(c32, P.inner_magic, P.inner_shift);
      const int64_t i = (int64_t)(c32 - rest * (uint32_t)P.inner);
      int64_t o, gg;
      if (P.stage == 1) {
        const uint32_t q = udiv31(rest, P.G_magic, P.G_shift);
        gg = rest - q * (uint32_t)P.G;
        o = q;
      } else {
        gg = g;
        o = rest;
      }
      ci = o * P.s_o + gg * P.s_in_g + i;
      co = o * P.s_o + gg * P.s_out_g + i;
    }
    col_in[tid] = ci;
    col_out[tid] = co;
  }
  // Digit slots that no index writes must read as zero (the FP16 planes must
  // not meet stale NaN patterns even against zero matrix slots).  Only the
  // full-length K = 32 tile writes every slot it reads (two limb chunks, or
  // the whole single-slot chunk, for all its columns), so it skips this.
  if (!(FULL && KMAX == 32))
    for (int x = tid * 16; x < 2 * DIG; x += kThreads * 16) *(uint4*)(smem + x) = make_uint4(0, 0, 0, 0);
  // (the full-length FP8 tile: every modulus writes every digit plane it reads)
  __syncthreads();

  // ---- load, column exponent, quantisation (Alg. 1 scaling invariant) ----
  const int jc = tid % NCOL, part = tid / NCOL;
  const int blk = PK ? part / (TPC / NP) : 0;  // packed: which column of the group
  const int rc = NP * jc + blk;                // this thread's column in the tables
  const int64_t cin = col_in[rc];
  double ar[KQ], br[KQ];
  int lmax = INT_MIN;
  bool nonfinite = false;
#pragma unroll
  for (int u = 0; u < KQ; u++) {
    const int s = part * KQ + u - blk * BR;  // index within the column
    double xr = 0.0, xi = 0.0;
    if (cin >= 0 && s < KR) {
      const typename TT::V2 v = ((const OB_GLOBAL typename TT::V2*)P.in)[cin + (int64_t)s * P.s_in_s];
      xr = (double)v.x;
      xi = (double)v.y;
    }
    nonfinite |= !__builtin_isfinite(xr) | !__builtin_isfinite(xi);
    if (xr != 0.0) lmax = max(lmax, __builtin_amdgcn_frexp_exp(xr) - 1);
    if (xi != 0.0) lmax = max(lmax, __builtin_amdgcn_frexp_exp(xi) - 1);
    ar[u] = xr;
    br[u] = xi;
  }
  // A non-finite value has no power-of-two scale: its column's outputs are
  // meaningless, and the plan's flag (read through obfft_last_error) says so.
  // One vector atomic per offending thread; the kernel runs on unchanged.
  if (__builtin_expect(nonfinite, 0))
    __hip_atomic_fetch_or((OB_GLOBAL uint32_t*)P.nf_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  pexp[part * NCOL + jc] = lmax;
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();
  int e = INT_MIN;
#pragma unroll
  for (int t = 0; t < TPC; t++)
    if (!PK || t / (TPC / NP) == blk) e = max(e, pexp[t * NCOL + jc]);
  if (e == INT_MIN) e = 0;  // all-zero column: every output is zero
  if (PK ? part % (TPC / NP) == 0 : part == 0) cexp[rc] = e;
#pragma unroll
  for (int u = 0; u < KQ; u++) {
    ar[u] = __builtin_rint(__builtin_ldexp(ar[u], TT::PREC - 1 - e));
    br[u] = __builtin_rint(__builtin_ldexp(br[u], TT::PREC - 1 - e));
  }
  // FP32 target: the quantised data are integers below 2^24, exact in FP32, so
  // their residues come from the FP32 reduction (|r| <= m/2 + 2 as in FP64)
  float arf[KQ], brf[KQ];
#pragma unroll
  for (int u = 0; u < KQ; u++) {
    arf[u] = (float)ar[u];
    brf[u] = (float)br[u];
  }

  const int mt = (MT == 2) ? (wave & 1) : 0;
  const int nt = (MT == 2) ? (wave >> 1) : wave;
  // A batched launch may run a K <= 16 stage on the two-M-tile shape: the
  // second M-tile then has no rows and no matrix planes.
  const bool mt_active = 16 * mt < K;
  const uint8_t* amat = ((SUB == SUB_FP8 && FULL) ? P.amat128 : P.amat) + g * P.amat_g_stride;
  const int col = nt * 16 + (lane & 15);
  // INT8 planes: [form][N-tile][lane][16 bytes]; contraction index s of
  // column jc sits in lane (jc % 16) + 16 (s / 8) at byte 2 (s % 8).
  constexpr int kI8FormBytes = NT * 64 * 16;
  const int s0 = part * KQ;
  constexpr int CH16 = chunks_for(SUB_FP16, KMAX);
  constexpr int kF16FormBytes = CH16 * NT * 1024;
  const int nch16 = (2 * K + 31) >> 5;

  // FP16 planes of this tile's matrix through a buffer resource: a scalar
  // base and byte count, the per-modulus offset in a scalar register and the
  // lane's 16 bytes as the vector offset (reads past the planes return 0)
  const __amdgpu_buffer_rsrc_t arsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)amat, 0, (int)min(P.amat_bytes - g * P.amat_g_stride, (int64_t)0x7FFFFFFF), 0x00020000);
  // residue records of this lane's outputs (row 16 mt + 4 (lane / 16) + v,
  // column col, Re / Im): rec[2 v + Re/Im][i / 2] packs moduli i (low half)
  // and i + 1 as FP16.  A pair is packed as soon as its odd modulus is done
  // and pinned in its register, so the records occupy 8 RV registers instead
  // of staying live as FP32 until the epilogue reads them.
  uint32_t rec[8][RS::RV];
  float rlo[8];  // the even modulus of the pair in progress
  // Combine of modulus i: centred residues of the GEMM sums into the records.
  auto combine = [&](const int i, const float* Dv, const float* Ev, const float* Fv, const float mf,
                     const float imf) {
    // ---- residue-domain combines, centred residues to the records ----
    // (Alg. 1 combines; the Phase-A carrier takes them signed, |v| <= m/2 + 2.
    // Rows past K hold zero products and are never stored.)
    float rrv[4], riv[4];
    int fm = 0, fb = 0, fc = 0, fn = 0;
    if (H0) {
      const OB_CONST ModConsts& MC = *(const OB_CONST ModConsts*)P.mc;
      fm = MC.m[i];
      fb = MC.fold_b[i];
      fc = MC.fold_c[i];
      fn = MC.fold_n[i];
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      if (SUB == SUB_FP16 && H0 && fb != 0) {
        rrv[v] = fold_reduce_f32(Dv[v], fm, fb, fc, fn);
        riv[v] = fold_reduce_f32(Fv[v], fm, fb, fc, fn);
      } else {
        rrv[v] = reduce_f32(Dv[v], mf, imf);
        riv[v] = reduce_f32(Fv[v], mf, imf);
      }
      if ((i & 1) == 0) {
        rlo[2 * v] = rrv[v];
        rlo[2 * v + 1] = riv[v];
      } else {
        // exact: |residue| <= m/2 + 2 < 2048
        rec[2 * v][i >> 1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(rlo[2 * v], rrv[v]));
        rec[2 * v + 1][i >> 1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(rlo[2 * v + 1], riv[v]));
        asm("" : "+v"(rec[2 * v][i >> 1]), "+v"(rec[2 * v + 1][i >> 1]));
      }
    }
    if (TAP && P.dbg_res) {  // canonical residue tap (tests only)
      const int eb = PK ? 4 * (lane >> 4) / BR : 0;  // the lane's column of the group
      const int64_t co = col_out[NP * col + eb];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int row = 16 * mt + 4 * (lane >> 4) + v - eb * BR;
        if (co >= 0 && row < KR) {
          int64_t el = co + (int64_t)row * P.s_out_t;
          ((OB_GLOBAL uint16_t*)P.dbg_res)[(el * 2) * R + i] = (uint16_t)(rrv[v] < 0.0f ? rrv[v] + mf : rrv[v]);
          ((OB_GLOBAL uint16_t*)P.dbg_res)[(el * 2 + 1) * R + i] = (uint16_t)(riv[v] < 0.0f ? riv[v] + mf : riv[v]);
        }
      }
    }
  };
  float pD[4] = {}, pE[4] = {}, pF[4] = {}, pmf = 1.0f, pimf = 1.0f;  // the GEMM sums awaiting their combine
#pragma unroll
  for (int i = 0; i < R; i++) {
    unsigned char* dig = smem + ((i & 1) ? DIG : 0);  // an offset, not a pointer select
    __builtin_amdgcn_s_setprio(1);
    const OB_CONST ModConsts& MC = *(const OB_CONST ModConsts*)P.mc;
    const double md = MC.md[i], imd = MC.inv_md[i];
    const float mf = MC.mf[i], imf = MC.inv_mf[i];
    // FP8 digits per residue: 3 for the moduli before the split (> 1052),
    // else 2; the full-length tile takes them from the position (the plan
    // checks that its modulus set follows this rule)
    const int nd = (SUB == SUB_FP8) ? (FULL ? (i < fp16_split(TGT, H0) ? 3 : 2) : MC.nd[i]) : 2;
    const uint8_t* amod = amat + i * P.amat_mod_stride;
    // A-operand planes of this modulus, issued before the deconstruction so
    // that their latency overlaps it (INT8: Re A, Im A, -Im A x 2 limbs, one chunk).
    v4i ai8[3][2];
    if (SUB == SUB_INT8 && mt_active) {
#pragma unroll
      for (int form = 0; form < 3; form++)
#pragma unroll
        for (int f = 0; f < 2; f++)
          ai8[form][f] = *(const v4i*)(amod + (((int64_t)form * P.amat_fmax + f) * P.amat_mt + mt) *
                                                  P.amat_chmax * 1024 + lane * 16);
    }
    // FP16: planes of Re A, Im A and -Im A, CH16 chunks of 32 slots each
    // (moduli past the split use chunk 0 only: one slot per index)
    const bool split16 = i < fp16_split(TGT, H0);
    const int nch = split16 ? nch16 : 1;
    v8h a16[3][CH16];
    if (SUB == SUB_FP16 && mt_active) {
#pragma unroll
      for (int form = 0; form < 3; form++)
#pragma unroll
        for (int ch = 0; ch < CH16; ch++)
          if (ch < nch)
            a16[form][ch] = __builtin_bit_cast(
                v8h, __builtin_amdgcn_raw_buffer_load_b128(
                         arsrc, (uint32_t)lane * 16u,
                         (uint32_t)(i * P.amat_mod_stride + ((form * P.amat_mt + mt) * P.amat_chmax + ch) * 1024), 0));
    }
    // ---- deconstruction: residues and digit planes (Sec. 2, Eq. ozaki) ----
    // indices past K (when KQ does not divide K) store zero limbs: the FP16
    // planes must not see stray NaN patterns even against zero matrix slots
    uint32_t la[KQ] = {}, lb[KQ] = {};
    float ra16[KQ] = {}, rb16[KQ] = {};
#pragma unroll
    for (int u = 0; u < KQ; u++) {
      int s = part * KQ + u;
      if (s < K) {
        if (SUB == SUB_FP16) {
          if (TGT == 1) {
            ra16[u] = reduce_f32(arf[u], mf, imf);
            rb16[u] = reduce_f32(brf[u], mf, imf);
          } else {
            ra16[u] = residue_f64(ar[u], md, imd);
            rb16[u] = residue_f64(br[u], md, imd);
          }
          if (split16) {
            la[u] = f16_limbs(ra16[u]);
            lb[u] = f16_limbs(rb16[u]);
          }
        } else if (SUB == SUB_INT8) {
          int ra = (int)__builtin_fma(-md, __builtin_rint(ar[u] * imd), ar[u]);
          int rb = (int)__builtin_fma(-md, __builtin_rint(br[u] * imd), br[u]);
          la[u] = i8_limbs(ra);
          lb[u] = i8_limbs(rb);
        } else if (!FULL) {
          // FP8: digit planes of a~ and b~ (four real products, as FP16)
          ra16[u] = TGT == 1 ? reduce_f32(arf[u], mf, imf) : residue_f64(ar[u], md, imd);
          rb16[u] = TGT == 1 ? reduce_f32(brf[u], mf, imf) : residue_f64(br[u], md, imd);
          put_digits_fp8<SUB, CHB, NT>(dig, 0, jc, s, ra16[u], nd);
          put_digits_fp8<SUB, CHB, NT>(dig, 1, jc, s, rb16[u], nd);
        }
      }
    }
    if (SUB == SUB_INT8 && s0 < K) {
      put_limbs<KQ>(dig, jc, s0, la);
      put_limbs<KQ>(dig + kI8FormBytes, jc, s0, lb);
    }
    if (SUB == SUB_FP8 && FULL) {
      // one form at a time: its four residues, then their digits
      static_assert(SUB != SUB_FP8 || !FULL || (KMAX == 32 && KQ == 4), "full-length FP8 tile: K = 32");
#pragma unroll
      for (int form = 0; form < 2; form++) {
        float rv[KQ];
#pragma unroll
        for (int u = 0; u < KQ; u++)
          rv[u] = TGT == 1 ? reduce_f32(form ? brf[u] : arf[u], mf, imf)
                           : residue_f64(form ? br[u] : ar[u], md, imd);
        // form 1 (b~) also as -b~ (form 2), so that the real part takes Im A x (-b~)
        if (nd == 3) {
          if (form) put_digits_fp8_k128<NT, 3, true>(dig, form, jc, s0, rv);
          else put_digits_fp8_k128<NT, 3>(dig, form, jc, s0, rv);
        } else {
          if (form) put_digits_fp8_k128<NT, 2, true>(dig, form, jc, s0, rv);
          else put_digits_fp8_k128<NT, 2>(dig, form, jc, s0, rv);
        }
      }
    }
    if (SUB == SUB_FP16 && s0 < K) {
      if (split16) {
        put_limbs16<KQ, NT>(dig, jc, s0, la);
        put_limbs16<KQ, NT>(dig + kF16FormBytes, jc, s0, lb);
      } else {
        put_slots16<KQ, NT>(dig, jc, s0, ra16);
        put_slots16<KQ, NT>(dig + kF16FormBytes, jc, s0, rb16);
      }
    }
    if (i > 0 && mt_active) combine(i - 1, pD, pE, pF, pmf, pimf);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    if (!mt_active) continue;
    // ---- residue GEMMs: R and I of the complex product (Sec. 2) ----
    float Dv[4], Ev[4], Fv[4];
    if (SUB == SUB_FP8) {
      // four real products on the digit planes.  General tile: R = Re A x~ -
      // Im A y~ and I = Im A x~ + Re A y~ on the K = 32 instruction, one
      // accumulator per matrix digit f (every partial sum is an integer of
      // magnitude <= 2 * 32 * 3 * 16 * 16 < 2^24); R = sum_f 32^f accR[f],
      // |R| < 2^22, exact in FP32.
      const int ndp = nd;  // K slots per index (3 digits: 96 slots, three chunks, at K = 32)
      const int nch = (ndp * K + 31) >> 5;
      v4f accR[3], accI[3];
#pragma unroll
      for (int f = 0; f < 3; f++) {
        accR[f] = (v4f){0.f, 0.f, 0.f, 0.f};
        accI[f] = (v4f){0.f, 0.f, 0.f, 0.f};
      }
      if (FULL) {
        // the scaled 16 x 16 x 128 MFMA: the nd^2 (matrix digit f, data digit
        // e) blocks of 32 slots, four per instruction (block b holds bytes
        // 16 (b / 2) .. + 15 of lane groups 2 (b % 2), 2 (b % 2) + 1); lane
        // group h scales its block of A by 32^f, so that one accumulator
        // takes sum_f 32^f (digit-f sum).  Every partial sum is an integer of
        // magnitude <= 2 * 32 * 3 * 16 * (16 + 32 * 16 + 1024) < 2^23: exact.
        const int h = lane >> 4;
        const int nins = nd == 3 ? 3 : 1;
#pragma unroll
        for (int ins = 0; ins < 3; ins++) {
          if (ins < nins) {
            // this lane group's two blocks of data digits of one form (a~, b~, -b~)
            auto bplane = [&](int form) {
              v8i bv;
#pragma unroll
              for (int pc = 0; pc < 2; pc++) {
                const int b = pc ? 2 + (h >> 1) : (h >> 1);
                const int idx = 4 * ins + b;
                const int e = idx < nd * nd ? idx % nd : 0;
                const uint4 w = *(const uint4*)(dig + ((form * 3 + e) * NT + nt) * 512 + (lane & 15) * 32 + 16 * (h & 1));
                bv[4 * pc] = w.x;
                bv[4 * pc + 1] = w.y;
                bv[4 * pc + 2] = w.z;
                bv[4 * pc + 3] = w.w;
              }
              return bv;
            };
            const int idxa = 4 * ins + h;
            const int sa = 127 + 5 * (idxa < nd * nd ? idxa / nd : 0);
            // the last instruction of a 3-digit modulus holds one block: only
            // the first 16 bytes of its A lanes can be non-zero
            const bool half = nd == 3 && ins == 2;
            auto aplane = [&](int pl) {
              const uint32_t so = (uint32_t)(i * P.amat_mod_stride + ((pl * 3 + ins) * 2 + mt) * 2048);
              const v4i lo = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(arsrc, (uint32_t)lane * 32u, so, 0));
              const v4i hi = half ? (v4i){0, 0, 0, 0}
                                  : __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(
                                                                arsrc, (uint32_t)lane * 32u + 16u, so, 0));
              return (v8i){lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            };
            // R = Re A x~ + Im A (-y~), I = Im A x~ + Re A y~
            const v8i bx = bplane(0);
            const v8i are = aplane(0);
            accR[0] = mfma_fp8_k128(are, bx, accR[0], sa);
            accI[0] = mfma_fp8_k128(are, bplane(1), accI[0], sa);
            const v8i aim = aplane(1);
            accI[0] = mfma_fp8_k128(aim, bx, accI[0], sa);
            accR[0] = mfma_fp8_k128(aim, bplane(2), accR[0], sa);
          }
        }
      } else {
        for (int ch = 0; ch < nch; ch++) {
          const long bx = *(const long*)(dig + (((0 * CHB + ch) * NT + nt) * 64 + lane) * 8);
          const long by = *(const long*)(dig + (((1 * CHB + ch) * NT + nt) * 64 + lane) * 8);
#pragma unroll
          for (int f = 0; f < 3; f++) {
            if (f < nd) {
              const uint8_t* ap = amod + ((int64_t)f * P.amat_mt + mt) * P.amat_chmax * 512 + ch * 512 + lane * 8;
              const int64_t pls = (int64_t)P.amat_fmax * P.amat_mt * P.amat_chmax * 512;  // bytes per plane
              const long ac = *(const long*)ap, as = *(const long*)(ap + pls), ams = *(const long*)(ap + 2 * pls);
              accR[f] = mfma_fp8(ac, bx, accR[f]);
              accI[f] = mfma_fp8(as, bx, accI[f]);
              accR[f] = mfma_fp8(ams, by, accR[f]);
              accI[f] = mfma_fp8(ac, by, accI[f]);
            }
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; v++) {
        Dv[v] = FULL ? accR[0][v] : __builtin_fmaf(1024.0f, accR[2][v], __builtin_fmaf(32.0f, accR[1][v], accR[0][v]));
        Ev[v] = 0.0f;
        Fv[v] = FULL ? accI[0][v] : __builtin_fmaf(1024.0f, accI[2][v], __builtin_fmaf(32.0f, accI[1][v], accI[0][v]));
      }
    } else if (SUB == SUB_FP16) {
      // four real products, accumulated exactly in FP32 (every partial sum
      // is an integer below 2^24): R = Re A x~ - Im A y~, I = Im A x~ + Re A y~
      v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ch = 0; ch < CH16; ch++) {
        if (ch < nch) {
          v8h bx = *(const v8h*)(dig + ((ch * NT + nt) * 64 + lane) * 16);
          v8h by = *(const v8h*)(dig + kF16FormBytes + ((ch * NT + nt) * 64 + lane) * 16);
          accR = mfma_f16_16(a16[0][ch], bx, accR);
          accI = mfma_f16_16(a16[1][ch], bx, accI);
          accR = mfma_f16_16(a16[2][ch], by, accR);
          accI = mfma_f16_16(a16[0][ch], by, accI);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; v++) {
        Dv[v] = accR[v];
        Ev[v] = 0.0f;
        Fv[v] = accI[v];
      }
    } else {
      // four real products per matrix limb f in INT32: R = Re A x~ + (-Im A) y~,
      // I = Im A x~ + Re A y~; R = accR[0] + 128 accR[1] is an integer of
      // magnitude <= 2 * 32 * 1019 * (127 + 16) < 2^24, exact in FP32
      const v4i bx = *(const v4i*)(dig + (nt * 64 + lane) * 16);
      const v4i by = *(const v4i*)(dig + kI8FormBytes + (nt * 64 + lane) * 16);
      v4i accR[2], accI[2];
#pragma unroll
      for (int f = 0; f < 2; f++) {
        accR[f] = mfma_i8(ai8[2][f], by, mfma_i8(ai8[0][f], bx, (v4i){0, 0, 0, 0}));
        accI[f] = mfma_i8(ai8[0][f], by, mfma_i8(ai8[1][f], bx, (v4i){0, 0, 0, 0}));
      }
#pragma unroll
      for (int v = 0; v < 4; v++) {
        Dv[v] = (float)(accR[0][v] + (accR[1][v] << 7));
        Ev[v] = 0.0f;
        Fv[v] = (float)(accI[0][v] + (accI[1][v] << 7));
      }
    }
    // the combine of this modulus runs after the next one's deconstruction,
    // so the GEMM's latency is covered by independent vector work
#pragma unroll
    for (int v = 0; v < 4; v++) {
      pD[v] = Dv[v];
      pE[v] = Ev[v];
      pF[v] = Fv[v];
    }
    pmf = mf;
    pimf = imf;
  }
  if (mt_active) combine(R - 1, pD, pE, pF, pmf, pimf);
  if (!mt_active) return;

  // ---- Phase A (FP16 MFMA) + Phase B (Kulisch, lift, pack) ----
  // Round (v, Re/Im): every lane reconstructs its own output of that row and
  // part.  The low lane half feeds moduli 0 .. ML-1 of its record and the
  // high half moduli ML .. r-1; one swap per packed pair hands each half the
  // other half's share (b1: the low lanes' outputs, b2: the high lanes').
  const v8h aop = *(const OB_GLOBAL v8h*)(P.phaseA + lane * 8);
  const OB_CONST CrtConsts& C = *(const OB_CONST CrtConsts*)P.crt;
  const v16f seed = phase_a_seed(C.seedT_c, lane >> 5);
  const typename EP::LiftK LK = EP::load_lift(C, false);
  // packed: lane l holds rows 4 (l / 16) .. + 3, i.e. column 4 (l / 16) / BR of the group
  // (NP = 2: lanes 0-31 rows 0-7, 32-63 rows 8-15; NP = 4: lanes 16 b .. 16 b + 15 column b)
  const int eb = PK ? 4 * (lane >> 4) / BR : 0;
  const int ecol = NP * col + eb;
  const int64_t co = col_out[ecol];
  const int ex = cexp[ecol] - 2 * (TT::PREC - 1) + P.extra_shift;
  typename TT::T re_part = 0;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const int v = j >> 1, prt = j & 1;
    if (16 * mt + v >= K) break;  // no lane of the wave has this row
    uint32_t b1w[4] = {0u, 0u, 0u, 0u}, b2w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < RS::RH; k++) {
      uint32_t x = rec[j][k];
      uint32_t y = RS::RH + k < RS::RV ? rec[j][RS::RH + k] : 0u;
      auto pr = __builtin_amdgcn_permlane32_swap(x, y, false, false);
      b1w[k] = pr[0];
      b2w[k] = pr[1];
    }
    v8h b1 = __builtin_bit_cast(v8h, make_uint4(b1w[0], b1w[1], b1w[2], b1w[3]));
    v8h b2 = __builtin_bit_cast(v8h, make_uint4(b2w[0], b2w[1], b2w[2], b2w[3]));
    float xv[EP::NV], yv[EP::NV];
    phase_a<EP::NV>(aop, b1, b2, seed, xv, yv);
    uint32_t wv[TT::NW];
    EP::deposits(xv, yv, LK.khi, wv);
    const uint32_t zh = EP::zhat(xv, yv, LK.zhi);
    uint32_t Rw[TT::NW];
    EP::lift_bounded(wv, zh, LK, Rw);
    typename TT::T y;
    if (TGT == 0)
      y = (typename TT::T)pack_f64<TT::NW>(Rw, ex);
    else
      y = (typename TT::T)pack_f32<TT::NW>(Rw, ex);
    if (TAP && P.dbg_tap) {
      // the raw epilogue record of this output when it lies on the tapped line
      // (layout in obfft_internal.h, kTapRec*; the host turns patterns into values)
      const int row = 16 * mt + 4 * (lane >> 4) + v - eb * BR;
      if (co >= 0 && row < KR) {
        const int64_t el = co + (int64_t)row * P.s_out_t;
        const int64_t line = (el / (P.N * P.inner)) * P.inner + el % P.inner;
        if (line == P.dbg_line) {
          const int64_t slot = (el / P.inner) % P.N;
          OB_GLOBAL uint32_t* t = (OB_GLOBAL uint32_t*)P.dbg_tap + (slot * 2 + prt) * kTapRecWords;
#pragma unroll
          for (int q = 0; q < EP::VP; q++) {
            t[kTapRecP + 2 * q] = __float_as_uint(xv[q]);
            t[kTapRecP + 2 * q + 1] = __float_as_uint(yv[q]);
          }
#pragma unroll
          for (int q = 0; q < EP::VZ; q++) {
            t[kTapRecZ + 2 * q] = __float_as_uint(xv[EP::VP + q]);
            t[kTapRecZ + 2 * q + 1] = __float_as_uint(yv[EP::VP + q]);
          }
#pragma unroll
          for (int w = 0; w < TT::NW; w++) {
            t[kTapRecW + w] = wv[w];
            t[kTapRecR + w] = Rw[w];
          }
          t[kTapRecZhat] = zh;
          t[kTapRecExp] = (uint32_t)ex;
          if (TGT == 0) {
            const uint64_t yb = __builtin_bit_cast(uint64_t, (double)y);
            t[kTapRecY] = (uint32_t)yb;
            t[kTapRecY + 1] = (uint32_t)(yb >> 32);
          } else {
            t[kTapRecY] = __builtin_bit_cast(uint32_t, (float)y);
          }
#pragma unroll
          for (int k = 0; k < R; k++) {
            const uint32_t pr = rec[j][k >> 1];
            const uint16_t hb = (uint16_t)((k & 1) ? pr >> 16 : pr);
            t[kTapRecRes + k] = (uint32_t)(int32_t)(float)__builtin_bit_cast(_Float16, hb);
          }
        }
      }
    }
    if (prt == 0) {
      re_part = y;
    } else {
      const int row = 16 * mt + 4 * (lane >> 4) + v - eb * BR;
      if (co >= 0 && row < KR) {
        typename TT::V2 z;
        z.x = re_part;
        z.y = y;
        ((OB_GLOBAL typename TT::V2*)P.out)[co + (int64_t)row * P.s_out_t] = z;
      }
    }
  }
}

template <int SUB, int TGT, int KMAX, bool FULL, bool H0, int NP, bool TAP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void ob_stage_kernel(
    const StageParams P) {
  int64_t c, g;
  grid_tile(P, c, g);
  stage_tile<SUB, TGT, KMAX, FULL, H0, NP, TAP>(P, c, g);
}

// Batched stage: one workgroup per tile of the members of one Bailey pass
// whose contraction length falls in this kernel's class.  tmember[t] is the
// member that owns tile t, descs[d] its stage and first[d] its first tile.
template <int SUB, int TGT, int KMAX, bool FULL, int NP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void ob_batch_kernel(const StageParams* __restrict__ descs,
                                                            const int64_t* __restrict__ first,
                                                            const uint16_t* __restrict__ tmember, int64_t total) {
  const int64_t t = blockIdx.x;
  if (t >= total) return;
  const int d = __builtin_amdgcn_readfirstlane((int)tmember[t]);  // uniform: scalar descriptor loads
  const StageParams P = descs[d];
  int64_t c, g;
  decode_tile(P, t - first[d], c, g);
  stage_tile<SUB, TGT, KMAX, FULL, false, NP>(P, c, g);
}


// Dynamic LDS of a stage tile: the packed variant holds column tables for
// twice the columns.
template <int SUB, int TGT, int KMAX, int NP>
static int stage_lds_bytes(int K) {
  return StageLds<SUB, TGT, KMAX>::bytes(K) + (NP - 1) * Shape<KMAX>::NCOL * 20;
}

template <int SUB, int TGT, int KMAX, bool FULL, bool H0, bool TAP, int NP = 1>
static hipError_t launch_stage_t(const StageParams& P, dim3 grid, hipStream_t st) {
  int lds = stage_lds_bytes<SUB, TGT, KMAX, NP>(P.K);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)ob_stage_kernel<SUB, TGT, KMAX, FULL, H0, NP, TAP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((ob_stage_kernel<SUB, TGT, KMAX, FULL, H0, NP, TAP>), grid, dim3(kThreads), lds, st, P);
  return hipGetLastError();
}

// Full-length variants for the default substrate at K = 12, 16 and 32 and
// the packed tiles for K <= 8 (four columns per tile up to K = 4, two up to
// K = 8), the full-length FP8 tile at K = 32 when the plan's modulus set
// follows its digit rule; everything else takes the general kernel.
template <int SUB, int TGT, bool H0, bool TAP>
static hipError_t launch_stage_k(const StageParams& P, dim3 grid, hipStream_t st) {
  constexpr bool F = SUB == SUB_FP16;
  int K = P.K;
  if (K <= 4) {
    if constexpr (F) return launch_stage_t<SUB, TGT, 16, true, H0, TAP, 4>(P, grid, st);
    else return launch_stage_t<SUB, TGT, 4, false, H0, TAP>(P, grid, st);
  }
  if (K <= 8) {
    if constexpr (F) return launch_stage_t<SUB, TGT, 16, true, H0, TAP, 2>(P, grid, st);
    else return launch_stage_t<SUB, TGT, 8, false, H0, TAP>(P, grid, st);
  }
  if (K <= 12) {
    if (F && K == 12) return launch_stage_t<SUB, TGT, 12, F, H0, TAP>(P, grid, st);
    return launch_stage_t<SUB, TGT, 12, false, H0, TAP>(P, grid, st);
  }
  if (K <= 16) {
    if (F && K == 16) return launch_stage_t<SUB, TGT, 16, F, H0, TAP>(P, grid, st);
    return launch_stage_t<SUB, TGT, 16, false, H0, TAP>(P, grid, st);
  }
  if (F && K == 32) return launch_stage_t<SUB, TGT, 32, F, H0, TAP>(P, grid, st);
  if constexpr (SUB == SUB_FP8)
    if (K == 32 && P.fp8_full && P.amat128) return launch_stage_t<SUB, TGT, 32, true, H0, TAP>(P, grid, st);
  return launch_stage_t<SUB, TGT, 32, false, H0, TAP>(P, grid, st);
}


}  // namespace obfft
