// Standalone CRT reconstruction kernels for gfx950 (MI355X): canonical
// residues in HBM in, one rounded value per output out.
//
//  * crt_kernel: the method's route, Phase A on FP16 MFMA (Sec. 4.2) and the
//    Kulisch Phase B with the two-sided lift and the correctly rounded pack
//    (Sec. 5.1, Alg. 2), with optional checkpoint taps;
//  * garner_kernel and slice_fp64_kernel: two of the reconstructions the
//    paper ranks the Kulisch route against (Sec. 4.1, Eq. recursive-garner;
//    Sec. 4.2 and App. C, the plain FP64 Phase B);
//  * crt_int8_kernel: the Kulisch route with Phase A moved to the INT8
//    matrix cores (Sec. 8.2, the B200 cross-check; Sec. 8.3, Eq. h1-group);
//  * crt_int16_kernel: the Kulisch accumulator in 16-bit words (Sec. 6.3,
//    Eq. kulisch-width; Sec. 6.4, Strategy A).
#include "crt_methods.h"
#include "ob_recon.h"

namespace obfft {

// ---- standalone CRT reconstruction (unit-level access to Phase A / B) ----

// The Phase-A operand of output o for lane half h: its moduli ML h ..
// ML h + ML - 1 (those below R) as FP16, read as 32-bit residue pairs (R and
// ML are even, so every pair is 4-byte aligned and inside row o); zero for
// o >= n.
template <int R>
__device__ __forceinline__ v8h residue_operand(const uint16_t* residues, int64_t n, int64_t o, int h) {
  constexpr int ML = RecSplit<R>::ML;
  static_assert(R % 2 == 0 && ML % 2 == 0, "pairs of residues");
  v8h b;
#pragma unroll
  for (int j = 0; j < 8; j++) b[j] = (_Float16)0.0f;
  if (o < n) {
    const uint32_t* row = (const uint32_t*)(residues + o * R + ML * h);
#pragma unroll
    for (int j = 0; j < ML / 2; j++) {
      if (ML * h + 2 * j < R) {
        const uint32_t pr = row[j];
        b[2 * j] = (_Float16)(float)(pr & 0xFFFFu);
        b[2 * j + 1] = (_Float16)(float)(pr >> 16);
      }
    }
  }
  return b;
}
template <int TGT>
__global__ __launch_bounds__(256) void crt_kernel(int64_t n, const uint16_t* residues, const int* exps,
                                                  void* out, uint32_t* taps, const uint16_t* phaseA,
                                                  const CrtConsts* crt) {
  const CrtConsts& C = *crt;
  typedef Tgt<TGT> TT;
  constexpr int R = TT::R;
  typedef Epilogue<TT::S, TT::TZ, TT::NW> EP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (base >= n) return;
  const int h = lane >> 5;
  v8h aop = *(const v8h*)(phaseA + lane * 8);
  const int64_t o1 = base + (lane & 31), o2 = o1 + 32;
  const v8h b1 = residue_operand<R>(residues, n, o1, h), b2 = residue_operand<R>(residues, n, o2, h);
  float xv[EP::NV], yv[EP::NV];
  phase_a<EP::NV>(aop, b1, b2, phase_a_seed(C.seedT_x, h), xv, yv);
  uint32_t wv[TT::NW];
  const typename EP::LiftK LK = EP::load_lift(C, true);
  EP::deposits(xv, yv, LK.khi, wv);
  const uint32_t zh = EP::zhat(xv, yv, LK.zhi);
  uint32_t Rw[TT::NW];
  EP::lift_exact(wv, zh, LK, Rw);
  const int64_t o = base + lane;
  if (o < n) {
    const int ex = exps[o];
    if (TGT == 0)
      ((double*)out)[o] = pack_f64<TT::NW>(Rw, ex);
    else
      ((float*)out)[o] = pack_f32<TT::NW>(Rw, ex);
    if (taps) {
      uint32_t* tp = taps + o * kTapStride;
      constexpr int VP = EP::VP;
      for (int s2 = 0; s2 < TT::S; s2++) tp[s2] = EP::pbits(xv, yv, s2) - __float_as_uint(C.seed_x[s2]);
      for (int t = 0; t < TT::TZ; t++) tp[16 + t] = EP::zbits(xv, yv, t) - __float_as_uint(C.seed_x[2 * VP + t]);
      // E = sum_s bits_s 256^s - sum_s bits(seed_s) 256^s  (mod 2^160)
      uint32_t Ef[5], E[5], bw = 0;
      EP::deposits_full(xv, yv, Ef);
      for (int i = 0; i < 5; i++) E[i] = subc(Ef[i], C.Bp5[i], bw, &bw);
      for (int i = 0; i < 5; i++) tp[24 + i] = E[i];
      tp[29] = zh - C.zoff;
      for (int i = 0; i < 4; i++) tp[30 + i] = i < TT::NW ? Rw[i] : (uint32_t)((int32_t)Rw[TT::NW - 1] >> 31);
      tp[34] = (uint32_t)ex;
    }
  }
}

// ---- reconstruction ablations: the lineage the Kulisch Phase B replaces ----

// x mod m for x < 2^26 with magic = ceil(2^32 / m): the quotient estimate is
// floor(x / m) or one more (x (magic m - 2^32) < 2^32), so one correction.
__device__ __forceinline__ uint32_t barrett_mod(uint32_t x, uint32_t m, uint32_t magic) {
  const uint32_t q = __umulhi(x, magic);
  const int32_t r = (int32_t)(x - q * m);
  return (uint32_t)(r + ((r >> 31) & (int32_t)m));
}

// Recursive Garner (Sec. 4.1, Eq. recursive-garner; App. C), one output per
// lane.  Digit k is (v_k - sum_{j<k} d_j prod_{i<j} m_i) (prod_{i<k} m_i)^-1
// mod m_k; with the weights stored negated the inner sum stays unsigned and
// below 2^26, so each digit takes one reduction before and one after its
// inverse.  The positional value d_0 + m_0 (d_1 + m_1 (...)) is then built by
// Horner in NW words, centred into [-M/2, M/2) and packed once, so the output
// equals the Kulisch route's bit for bit.
template <int TGT>
__global__ __launch_bounds__(256) void garner_kernel(int64_t n, const uint16_t* residues, const int* exps,
                                                     void* out, const CrtConsts* crt) {
  typedef Tgt<TGT> TT;
  constexpr int R = TT::R, NW = TT::NW;
  static_assert(R % 2 == 0, "residue rows are read as 32-bit pairs");
  const CrtConsts& C = *crt;
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= n) return;
  uint32_t v[R];
  const uint32_t* rp = (const uint32_t*)(residues + o * R);  // 4-byte aligned: R even
#pragma unroll
  for (int k = 0; k < R / 2; k++) {
    const uint32_t pr = rp[k];
    v[2 * k] = pr & 0xFFFFu;
    v[2 * k + 1] = pr >> 16;
  }
  uint32_t d[R];
#pragma unroll
  for (int k = 0; k < R; k++) {
    uint32_t acc = v[k];
#pragma unroll
    for (int j = 0; j < k; j++) acc += d[j] * C.gneg[k][j];
    acc = barrett_mod(acc, C.gm[k], C.gmagic[k]);
    d[k] = barrett_mod(acc * C.ginv[k], C.gm[k], C.gmagic[k]);
  }
  uint32_t w[NW];
  w[0] = d[R - 1];
#pragma unroll
  for (int i = 1; i < NW; i++) w[i] = 0;
#pragma unroll
  for (int k = R - 2; k >= 0; k--) {
    uint64_t t = (uint64_t)w[0] * C.gm[k] + d[k];
    w[0] = (uint32_t)t;
#pragma unroll
    for (int i = 1; i < NW; i++) {
      t = (uint64_t)w[i] * C.gm[k] + (t >> 32);
      w[i] = (uint32_t)t;
    }
  }
  uint32_t b = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) (void)subc(w[i], C.Mhalf[i], b, &b);
  if (!b) {  // value >= M/2: subtract M
    uint32_t cy = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) w[i] = addc(w[i], C.negM[i], cy, &cy);
  }
  if (TGT == 0)
    ((double*)out)[o] = pack_f64<NW>(w, exps[o]);
  else
    ((float*)out)[o] = pack_f32<NW>(w, exps[o]);
}

// Slicing direct CRT with a plain FP64 Phase B (Sec. 4.2, Phase B on the FP
// vector pipe; App. C, the fp64-sum option): the Phase-A slice sums P_s as in
// crt_kernel, then T = sum_s P_s 256^s in FP64 with a rounding after every
// addition (s ascending), the lift T - zhat * fl(M) in FP64 (zhat from the
// same lift columns as the exact route, the product rounded before the
// subtraction), and one scaling by 2^exp.  The accuracy baseline: the sum
// spans about 120 bits while the result needs its top 53.
template <int TGT>
__global__ __launch_bounds__(256) void slice_fp64_kernel(int64_t n, const uint16_t* residues, const int* exps,
                                                         void* out, const uint16_t* phaseA, const CrtConsts* crt) {
#pragma clang fp contract(off)
  const CrtConsts& C = *crt;
  typedef Tgt<TGT> TT;
  constexpr int R = TT::R;
  typedef Epilogue<TT::S, TT::TZ, TT::NW> EP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (base >= n) return;
  const int h = lane >> 5;
  v8h aop = *(const v8h*)(phaseA + lane * 8);
  const int64_t o1 = base + (lane & 31), o2 = o1 + 32;
  const v8h b1 = residue_operand<R>(residues, n, o1, h), b2 = residue_operand<R>(residues, n, o2, h);
  float xv[EP::NV], yv[EP::NV];
  phase_a<EP::NV>(aop, b1, b2, phase_a_seed(C.seedT_x, h), xv, yv);
  const typename EP::LiftK LK = EP::load_lift(C, true);
  const uint32_t zh = EP::zhat(xv, yv, LK.zhi) - C.zoff;
  const int64_t o = base + lane;
  if (o >= n) return;
  double T = 0.0, scale = 1.0;
#pragma unroll
  for (int s = 0; s < TT::S; s++) {
    // both in the binade [2^23, 2^24): the difference is P_s exactly
    const float ps = __uint_as_float(EP::pbits(xv, yv, s)) - C.seed_x[s];
    T = T + (double)ps * scale;
    scale *= 256.0;
  }
  const double lift = (double)zh * C.Mf;
  const double y = ldexp(T - lift, exps[o]);
  if (TGT == 0)
    ((double*)out)[o] = y;
  else
    ((float*)out)[o] = (float)y;
}

// ---- Phase A on INT8 MFMA: two limbs, shifted columns ----

// The B operand of one 32x32x32 INT8 MFMA for output o and lane half h:
// limb q = 16 h + j of the output, where limbs 0 .. R-1 are the low bytes
// v0_k = v_k - 256 v1_k (as two's-complement bytes: v_k mod 256) and limbs
// R .. 2R-1 the high limbs v1_k = (v_k + 128) >> 8 in [0, 8]; zeros beyond,
// and for o >= n.
template <int R>
__device__ __forceinline__ v4i_t limb_operand(const uint16_t* residues, int64_t n, int64_t o, int h) {
  static_assert(R % 2 == 0 && 2 * R <= 32, "limb layout");
  uint32_t lo[R], hi[R];
#pragma unroll
  for (int k = 0; k < R; k++) lo[k] = hi[k] = 0;
  if (o < n) {
    const uint32_t* row = (const uint32_t*)(residues + o * R);
#pragma unroll
    for (int k = 0; k < R / 2; k++) {
      const uint32_t pr = row[k];
      lo[2 * k] = pr & 0xFFu;
      lo[2 * k + 1] = (pr >> 16) & 0xFFu;
      hi[2 * k] = ((pr & 0xFFFFu) + 128u) >> 8;
      hi[2 * k + 1] = ((pr >> 16) + 128u) >> 8;
    }
  }
  auto limb = [&](int q) -> uint32_t { return q < R ? lo[q] : (q < 2 * R ? hi[q - R] : 0u); };
  v4i_t b0, b1;
#pragma unroll
  for (int w = 0; w < 4; w++) {
    b0[w] = (int)(limb(4 * w) | (limb(4 * w + 1) << 8) | (limb(4 * w + 2) << 16) | (limb(4 * w + 3) << 24));
    b1[w] = (int)(limb(16 + 4 * w) | (limb(17 + 4 * w) << 8) | (limb(18 + 4 * w) << 16) |
                  (limb(19 + 4 * w) << 24));
  }
  return h ? b1 : b0;
}

// Column j of the Phase-A product after the lane-half swap: rows
// 8a + b (b < 4) sit in xv[4a + b], rows 8a + 4 + b in yv[4a + b].
__device__ __forceinline__ uint32_t i8_part(const uint32_t* xv, const uint32_t* yv, int j) {
  const int a = j >> 3, b = j & 7;
  return b < 4 ? xv[4 * a + b] : yv[4 * a + b - 4];
}

// Four biased column sums (each in (0, 2^19)) deposited at bits 0, 8, 16, 24
// of one word: the low word L and the spill H into the next word.
__device__ __forceinline__ void i8_column(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, uint32_t& L,
                                          uint32_t& H) {
  uint32_t c1, c2;
  uint32_t l = b0 + (b1 << 8);
  l = addc(l, b2 << 16, 0u, &c1);
  l = addc(l, b3 << 24, 0u, &c2);
  L = l;
  H = (b2 >> 16) + (b3 >> 8) + c1 + c2;
}

// One output per lane, 64 per wave: Phase A as two 32x32x32 INT8 MFMAs (the
// matrix rows are the S + 2 raw and T + 2 lift columns of balanced-digit
// slices, the contraction runs over the 2r limbs; INT32 accumulation is
// exact: |column| <= r 128 136), the accumulators started at the bias; then
// W = sum_s col_s 256^s + wadd = E + M/2 + zoff M (mod 2^(32 NW)) and
// zhat + zoff from the lift columns, the exact two-sided lift and the pack.
template <int TGT>
__global__ __launch_bounds__(256) void crt_int8_kernel(int64_t n, const uint16_t* residues, const int* exps,
                                                       void* out, const int8_t* aop_tab, const CrtConsts* crt,
                                                       const CrtAltConsts* i8) {
  typedef Tgt<TGT> TT;
  constexpr int R = TT::R, S = TT::S, NW = TT::NW;
  typedef Epilogue<TT::S, TT::TZ, TT::NW> EP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (base >= n) return;
  const int h = lane >> 5;
  const v4i_t aop = ((const v4i_t*)aop_tab)[lane];
  const int64_t o1 = base + (lane & 31), o2 = o1 + 32;
  const v4i_t b1 = limb_operand<R>(residues, n, o1, h), b2 = limb_operand<R>(residues, n, o2, h);
  v16i_t seed;
#pragma unroll
  for (int v = 0; v < 16; v++) seed[v] = kI8PhaseABias;
  const v16i_t d1 = mfma_i8_32(aop, b1, seed), d2 = mfma_i8_32(aop, b2, seed);
  uint32_t xv[16], yv[16];
#pragma unroll
  for (int v = 0; v < 16; v++) {
    auto pr = __builtin_amdgcn_permlane32_swap((uint32_t)d1[v], (uint32_t)d2[v], false, false);
    xv[v] = pr[0];
    yv[v] = pr[1];
  }
  // raw columns s < S + 2; those at bit 32 NW or above vanish mod 2^(32 NW)
  constexpr int NS = (S + 2 < 4 * NW) ? S + 2 : 4 * NW;
  constexpr int NC = (NS + 3) / 4;
  uint32_t L[NC], H[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const uint32_t p0 = i8_part(xv, yv, 4 * c);
    const uint32_t p1 = 4 * c + 1 < NS ? i8_part(xv, yv, 4 * c + 1) : 0u;
    const uint32_t p2 = 4 * c + 2 < NS ? i8_part(xv, yv, 4 * c + 2) : 0u;
    const uint32_t p3 = 4 * c + 3 < NS ? i8_part(xv, yv, 4 * c + 3) : 0u;
    i8_column(p0, p1, p2, p3, L[c], H[c]);
  }
  const CrtAltConsts& K = *i8;
  // two interleaved carry chains: (L + H shifted one word), then + wadd
  uint32_t W[NW], ca = 0, cb = 0;
  W[0] = addc(L[0], K.wadd[0], 0u, &cb);
#pragma unroll
  for (int i = 1; i < NW; i++) {
    const uint32_t t = addc(i < NC ? L[i] : 0u, H[i - 1], ca, &ca);
    W[i] = addc(t, K.wadd[i], cb, &cb);
  }
  // lift columns t = 0 .. 7 at rows S + 2 + t: bits 48 .. 63 of their sum
  // plus zadd (mod 2^64) are zhat + zoff
  constexpr int Z0 = S + 2;
  uint32_t ZL0, ZH0, ZL1, ZH1;
  i8_column(i8_part(xv, yv, Z0), i8_part(xv, yv, Z0 + 1), i8_part(xv, yv, Z0 + 2), i8_part(xv, yv, Z0 + 3), ZL0,
            ZH0);
  i8_column(i8_part(xv, yv, Z0 + 4), i8_part(xv, yv, Z0 + 5), i8_part(xv, yv, Z0 + 6), i8_part(xv, yv, Z0 + 7),
            ZL1, ZH1);
  (void)ZH1;
  uint32_t zc;
  (void)addc(ZL0, K.zadd[0], 0u, &zc);
  const uint32_t z1 = ZL1 + ZH0 + K.zadd[1] + zc;
  const uint32_t zh = z1 >> 16;
  const typename EP::LiftK LK = EP::load_lift(*crt, true);
  uint32_t Rw[NW];
  EP::lift_exact(W, zh, LK, Rw);
  const int64_t o = base + lane;
  if (o < n) {
    if (TGT == 0)
      ((double*)out)[o] = pack_f64<NW>(Rw, exps[o]);
    else
      ((float*)out)[o] = pack_f32<NW>(Rw, exps[o]);
  }
}

// ---- Kulisch accumulation in 16-bit words (Strategy A) ----

// One output per lane after the FP16 Phase A of crt_kernel: the slice sums
// P_s (below 2^23, the exact differences of the partials and their seeds)
// are deposited at bit 8 s into 16-bit words of radix 2^12, two words per
// register; each slice spreads over the three words its bits touch, and a
// word collects at most four pieces, so it stays below 2^14 and the two
// words of a register are added by one 32-bit add with no carry between
// them.  A carry sweep resolves the redundant form into 32-bit words, then
// the lift and the pack are the 32-bit route's.
template <int TGT>
__global__ __launch_bounds__(256) void crt_int16_kernel(int64_t n, const uint16_t* residues, const int* exps,
                                                        void* out, const uint16_t* phaseA, const CrtConsts* crt,
                                                        const CrtAltConsts* alt) {
  const CrtConsts& C = *crt;
  typedef Tgt<TGT> TT;
  constexpr int R = TT::R, S = TT::S, NW = TT::NW;
  typedef Epilogue<TT::S, TT::TZ, TT::NW> EP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (base >= n) return;
  const int h = lane >> 5;
  v8h aop = *(const v8h*)(phaseA + lane * 8);
  const int64_t o1 = base + (lane & 31), o2 = o1 + 32;
  const v8h b1 = residue_operand<R>(residues, n, o1, h), b2 = residue_operand<R>(residues, n, o2, h);
  float xv[EP::NV], yv[EP::NV];
  phase_a<EP::NV>(aop, b1, b2, phase_a_seed(C.seedT_x, h), xv, yv);
  // words of radix 2^12 covering the 32 NW bits the lift needs
  constexpr int NQ = (32 * NW + 11) / 12, NR = (NQ + 1) / 2;
  uint32_t acc[NR + 1];
#pragma unroll
  for (int i = 0; i <= NR; i++) acc[i] = 0;
#pragma unroll
  for (int s = 0; s < S; s++) {
    const uint32_t p = EP::pbits(xv, yv, s) - __float_as_uint(C.seed_x[s]);
    const int q = (8 * s) / 12, o = (8 * s) % 12;
    const uint32_t a0 = (p << o) & 0xFFFu;
    const uint32_t a1 = (p >> (12 - o)) & 0xFFFu;
    const uint32_t a2 = p >> (24 - o);
    if ((q & 1) == 0) {
      if (q / 2 < NR) acc[q / 2] += a0 | (a1 << 16);
      if (q / 2 + 1 < NR) acc[q / 2 + 1] += a2;
    } else {
      if (q / 2 < NR) acc[q / 2] += a0 << 16;
      if (q / 2 + 1 < NR) acc[q / 2 + 1] += a1 | (a2 << 16);
    }
  }
  // carry sweep over the NQ words, then the 12-bit digits into 32-bit words
  uint32_t d[NQ];
#pragma unroll
  for (int i = 0; i < NQ; i++) d[i] = (i & 1) ? acc[i / 2] >> 16 : acc[i / 2] & 0xFFFFu;
#pragma unroll
  for (int i = 0; i + 1 < NQ; i++) {
    d[i + 1] += d[i] >> 12;
    d[i] &= 0xFFFu;
  }
  uint32_t E[NW];
#pragma unroll
  for (int j = 0; j < NW; j++) E[j] = 0;
#pragma unroll
  for (int i = 0; i < NQ; i++) {
    const int bit = 12 * i, j = bit / 32, sh = bit % 32;
    if (j < NW) E[j] |= d[i] << sh;
    if (sh > 20 && j + 1 < NW) E[j + 1] |= d[i] >> (32 - sh);
  }
  const CrtAltConsts& K = *alt;
  uint32_t W[NW], cy = 0;
#pragma unroll
  for (int j = 0; j < NW; j++) W[j] = addc(E[j], K.kadd[j], cy, &cy);
  const typename EP::LiftK LK = EP::load_lift(C, true);
  const uint32_t zh = EP::zhat(xv, yv, LK.zhi);
  uint32_t Rw[NW];
  EP::lift_exact(W, zh, LK, Rw);
  const int64_t o = base + lane;
  if (o < n) {
    if (TGT == 0)
      ((double*)out)[o] = pack_f64<NW>(Rw, exps[o]);
    else
      ((float*)out)[o] = pack_f32<NW>(Rw, exps[o]);
  }
}

hipError_t launch_crt(int tgt, int64_t n, const uint16_t* residues, const int* exps, void* out,
                      uint32_t* taps, const uint16_t* phaseA, const CrtConsts* C, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (tgt == 0)
    hipLaunchKernelGGL(crt_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, st, n, residues, exps, out, taps,
                       phaseA, C);
  else
    hipLaunchKernelGGL(crt_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, n, residues, exps, out, taps,
                       phaseA, C);
  return hipGetLastError();
}

hipError_t launch_crt_ablation(int tgt, int method, int64_t n, const uint16_t* residues, const int* exps,
                              void* out, const uint16_t* phaseA, const CrtConsts* C, const int8_t* phaseA_i8,
                              const CrtAltConsts* i8, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (method == 4) {
    if (tgt == 0)
      hipLaunchKernelGGL(crt_int16_kernel<0>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA, C, i8);
    else
      hipLaunchKernelGGL(crt_int16_kernel<1>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA, C, i8);
  } else if (method == 3) {
    if (tgt == 0)
      hipLaunchKernelGGL(crt_int8_kernel<0>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA_i8, C,
                         i8);
    else
      hipLaunchKernelGGL(crt_int8_kernel<1>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA_i8, C,
                         i8);
  } else if (method == 1) {
    if (tgt == 0)
      hipLaunchKernelGGL(garner_kernel<0>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, C);
    else
      hipLaunchKernelGGL(garner_kernel<1>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, C);
  } else {
    if (tgt == 0)
      hipLaunchKernelGGL(slice_fp64_kernel<0>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA, C);
    else
      hipLaunchKernelGGL(slice_fp64_kernel<1>, dim3(blocks), dim3(256), 0, st, n, residues, exps, out, phaseA, C);
  }
  return hipGetLastError();
}

}  // namespace obfft
