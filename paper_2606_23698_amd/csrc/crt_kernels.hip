// Standalone CRT reconstruction kernels for gfx950 (MI355X): canonical
// residues in HBM in, one rounded value per output out.
//
//  * crt_kernel: the method's route, Phase A on FP16 MFMA (Sec. 4.2) and the
//    Kulisch Phase B with the two-sided lift and the correctly rounded pack
//    (Sec. 5.1, Alg. 2), with optional checkpoint taps;
//  * garner_kernel and slice_fp64_kernel: two of the reconstructions the
//    paper ranks the Kulisch route against (Sec. 4.1, Eq. recursive-garner;
//    Sec. 4.2 and App. C, the plain FP64 Phase B).
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
                              void* out, const uint16_t* phaseA, const CrtConsts* C, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (method == 1) {
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
