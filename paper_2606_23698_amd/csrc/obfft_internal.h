// Internal definitions shared by the host plan code and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace obfft {

constexpr int kMaxModuli = 16;
constexpr int kMaxK = 32;          // longest contraction (p or q) of the fused stage kernel
constexpr int kThreads = 256;      // 4 waves of 64
// A launch's x extent in work-items is a 32-bit field: tiles per x row < 2^32 / kThreads.
constexpr int64_t kMaxTiles = ((int64_t)1 << 32) / kThreads;
constexpr int kTapStride = 40;     // uint32 words per output in the CRT debug taps

enum Substrate { SUB_FP8 = 0, SUB_INT8 = 1, SUB_FP16 = 2, SUB_AUTO = 3 };

// Column packing of short contractions on the FP16 substrate: a stage with
// K <= 8 runs as a block-diagonal 16 x 16 product with np = 16 / 8 = 2
// (4 < K <= 8) or 16 / 4 = 4 (K <= 4) diagonal blocks, rows and contraction
// slots b 16/np .. (b+1) 16/np - 1 belonging to column b of the group, so that
// the 16-row MFMA tile and the per-row CRT epilogue carry np columns instead
// of one column and 16 - K dead rows.  1: no packing.
__host__ __device__ constexpr int fp16_pack(int sub, int K) {
  return sub != SUB_FP16 ? 1 : K <= 4 ? 4 : K <= 8 ? 2 : 1;
}

// FP16 substrate: the first fp16_split(...) moduli of a set enter the
// residue GEMM as two radix-128 limbs per index; every later modulus as one
// FP16 slot per index, which needs 2 kMaxK h (h + e) <= 2^24 with h =
// floor(m/2), e = 0 for a power of two (its residues are exact, |r| <= h)
// and 2 otherwise: the largest possible partial sum of a 32-term,
// two-product accumulation, kept exact in FP32 (every m <= 1024 passes).
// The paper's sets satisfy it from index 4 (r = 12: 1024, 961, 841, ...)
// and 3 (r = 6: 1024, 961, 841); the fold-and-add reduction, which needs the
// paper's reduction-friendly moduli, keeps that split.  The default stage
// sets have every modulus at most 1024, so the reciprocal-reduction kernels
// take every modulus as one slot (no limb split).
constexpr int kFp16Split[2] = {4, 3};
__host__ __device__ constexpr int fp16_split(int tgt, bool h0) { return h0 ? kFp16Split[tgt] : 0; }

// Everything the CRT epilogue needs: Sec. 4.2 (Phase A, byte slices of
// u_k) and Sec. 5.1 (fractional lift, bias, M).
//
// Phase A leaves partial j of an output in accumulator register j / 2 of
// lane half j % 2, as the FP32 value seed[j] + P_j with seed[j] =
// 1.5 * 2^23 + delta_j (delta_j < 2^16, |P_j| < 2^22: one binade), so its bit
// pattern is bits(seed[j]) + P_j.  The deltas fold every additive constant
// of the lift into the MFMA: the implicit bias of the bit patterns, the top
// byte that the fast deposit drops (see Epilogue), the offset zoff M that
// keeps zhat unsigned for centred residues, and M / 2 for the exact lift.
// Whatever does not fit in the last slice's 16 bits is added to the top word
// (khi, zhi).  Two seed sets: `x` for the exact two-sided lift, `c` for the
// lift of the stage kernels under the capacity bound (no M / 2).
struct CrtConsts {
  int r;                 // number of moduli
  int S;                 // byte slices of u_k
  int T;                 // byte slices of w_k (f = 48)
  int nwords;            // 32-bit words of the lift arithmetic (4: FP64 set, 3: FP32 set)
  uint32_t M[4];         // M, little-endian words
  uint32_t Mhalf[4];     // M / 2
  uint32_t negM[4];      // -M mod 2^128
  uint32_t khi_x, khi_c; // added to the top deposit word (exact / bounded lift)
  uint32_t zhi;          // added to word 1 of the lift sum
  uint32_t zoff;         // multiple of M added to E so that zhat stays unsigned
  float seed_x[32];      // Phase-A accumulator seeds per partial, exact lift
  float seed_c[32];      // same, bounded lift
  float seedT_x[2][16];  // seed_x[2 v + h] at [h][v]: one lane half's registers
  float seedT_c[2][16];  // same for seed_c
  uint32_t Bp5[5];       // sum_s bits(seed_x[s]) 256^s mod 2^160 (debug taps only)
  // Reconstruction ablations.  Recursive Garner (Eq. recursive-garner): m_k,
  // the Barrett multiplier ceil(2^32 / m_k), (prod_{i<k} m_i)^-1 mod m_k and,
  // at [k][j] for j < k, m_k - (prod_{i<j} m_i mod m_k).  Plain FP64 sum:
  // M rounded to binary64.
  uint32_t gm[16], gmagic[16], ginv[16];
  uint32_t gneg[16][16];
  double Mf;
};

// Per-modulus constants of the residue arithmetic.
struct ModConsts {
  int m[kMaxModuli];
  float inv_mf[kMaxModuli];
  double inv_md[kMaxModuli];
  float mf[kMaxModuli];   // m as FP32 and FP64 (no conversions in the kernels)
  double md[kMaxModuli];
  int nd[kMaxModuli];    // digits per residue on the FP8 substrate (2 or 3)
  int sub[kMaxModuli];   // substrate of each modulus
  // Fold-and-add form of a reduction-friendly modulus m = 2^b - c (Sec. 2,
  // Sec. 8.3 rung H0: a power of two, or a small complement
  // c <= kH0MaxComplement): fold_n
  // folds t <- c (t >> b) + (t mod 2^b) take any |t| <= 2^24 into
  // [-c, 2^b - 1 + c].  fold_b = 0 marks a modulus that keeps the reciprocal
  // reduction.  Used only by plans that ask for the fold (OBFFT_RED_H0).
  int fold_b[kMaxModuli], fold_c[kMaxModuli], fold_n[kMaxModuli];
};

// Largest complement 2^b - m of a modulus reduced by folds.  The seven
// friendly members of the FP64 set have c <= 25; the next one, 961, has 63.
constexpr int kH0MaxComplement = 31;

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
  int g_minor;          // stage 2: tile order (0: group-major; 1: blocks of gblock groups
                        // of a column tile on one XCD back to back, see stage_tile)
  int gblock;           // groups per block of the group-minor order (divides G)
  int grid_mode;        // how the stage kernel reads (column tile, group) off blockIdx:
                        // 0 linear index, 1 stage 1 (x), 2 group-major (x, y),
                        // 3 group-minor (8 GB, T / 8, G / GB), 4 group-minor (GB, T, G / GB)
  uint32_t inner_magic, inner_shift, G_magic, G_shift;  // n / d = mulhi(n, magic) >> shift
                                                        // for n < 2^31 (magic 0: d = 1)
  int extra_shift;      // added to the pack exponent
  const uint8_t* amat;  // MFMA A-operand planes of this stage / direction
  const uint8_t* amat128;  // the full-length FP8 tile's planes (same strides), or null
  int64_t amat_g_stride;  // bytes per group g (0 for stage 1)
  int amat_fmax, amat_chmax, amat_mt;  // layout extents of the planes
  int64_t amat_bytes;                  // bytes of the planes from amat on (all groups)
  int64_t amat_mod_stride;  // bytes per modulus
  const uint16_t* phaseA;   // 64 lanes x 8 FP16 operand of the Phase-A MFMA
  uint16_t* dbg_res;        // canonical residues tap (debug kernels only; may be null)
  const ModConsts* mc;      // device copies of the plan constants (read per use,
  const CrtConsts* crt;     // so that they do not occupy scalar registers)
  uint32_t* nf_flag;        // set (bit 0) when a non-finite input value is read
  uint32_t* dbg_tap;        // epilogue records of one line (debug kernels only; may be null)
  int64_t dbg_line;         // the tapped line: outer * inner + inner index
  int fp8_full;             // FP8: the modulus set has 3 digits per residue for the moduli
                            // before the split and 2 after it (the full-length tile's rule)
  int pad_;
};

// One output's epilogue record in the debug tap of a stage, as the debug
// kernel writes it (32-bit words): the Phase-A partial patterns of the P and
// Z slices (bits of seed_c[j] + P_j), the deposit words W = E + zoff M, the
// lift quotient zhat + zoff, the lifted words R, the pack exponent, the
// packed value's bits and the (centred) residues that entered Phase A.
constexpr int kTapRecWords = 64;
constexpr int kTapRecP = 0, kTapRecZ = 16, kTapRecW = 24, kTapRecZhat = 29, kTapRecR = 30,
              kTapRecExp = 34, kTapRecY = 35, kTapRecRes = 40;

// The persistent batched launch: one kernel over the tiles of every Bailey
// pass of every member.  Work items are numbered pass-major (all tiles of
// pass 0 of every member, then pass 1, ...); a segment is the tiles of one
// (pass, member), and a segment may start only when the same member's
// previous pass (its dependency) has completed every tile.
struct PersistParams {
  const StageParams* descs;  // [nseg] stage of each segment (pass-major: pass * count + member)
  const int64_t* seg_start;  // [nseg + 1] first item of each segment; seg_start[nseg] = total
  const int* seg_dep;        // [nseg] the segment that must be complete first, or -1
  const int* seg_cls;        // [nseg] tile variant (kPersist* below)
  int nseg;
  int spin_limit;            // polls of a dependency before the kernel gives up
  int claim;                 // items a workgroup claims at once (>= 1)
  int pad_;
  int64_t total;             // items
  uint32_t* ctl;             // [0] item counter, [1] give-up flag, [2 + seg] tiles completed
  uint32_t* flags;           // the plan's status word: bit 1 = a dependency wait gave up
};

// Tile variants of the persistent kernel (FP16 substrate, FP64 target).
enum {
  kPersistK4Packed = 0,   // K <= 4: four columns per 16-row tile
  kPersistK8Packed = 1,   // 4 < K <= 8: two columns per tile
  kPersistK12Full = 2, kPersistK12 = 3,
  kPersistK16Full = 4, kPersistK16 = 5,
  kPersistK32Full = 6, kPersistK32 = 7,
  kPersistVariants = 8
};
constexpr unsigned kPersistMaskFull = (1u << kPersistK4Packed) | (1u << kPersistK8Packed) | (1u << kPersistK12Full) |
                                      (1u << kPersistK16Full) | (1u << kPersistK32Full);
constexpr unsigned kPersistMaskAll = (1u << kPersistVariants) - 1;

// Plan-time per-(N, p, q) operand set for one stage direction.
struct OperandPlanes {
  uint8_t* dev;          // device copy
  uint8_t* dev128;       // FP8, K = 32, full-length tile: the same planes laid out for the
                         // scaled K = 128 MFMA (null otherwise)
  int64_t g_stride;      // bytes per group
  int64_t mod_stride;    // bytes per modulus
  int fmax, chmax, mt;
  int G;
};

}  // namespace obfft
