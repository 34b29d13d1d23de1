// Instantiations and host launchers of the Ozaki-Bailey stage kernels
// (single transforms and the batched launches) for gfx950.
#include "ob_stage.h"

namespace obfft {

// ---- plan-time conversion of signed digit planes to E4M3 ----
__global__ void digits_to_fp8_kernel(uint8_t* p, int64_t n4) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  uint32_t w = ((const uint32_t*)p)[i];
  float d0 = (float)(int8_t)(w & 0xFF), d1 = (float)(int8_t)((w >> 8) & 0xFF);
  float d2 = (float)(int8_t)((w >> 16) & 0xFF), d3 = (float)(int8_t)(w >> 24);
  uint32_t o = fp8_pack2<false>(d0, d1, 0u);
  o = fp8_pack2<true>(d2, d3, o);
  ((uint32_t*)p)[i] = o;
}


// ---- host-side launch helpers ----
// h0: the fold-and-add reduction of the friendly moduli (FP16 substrate,
// FP64 target only; the plan checks it).
hipError_t launch_stage(int sub, int tgt, bool h0, const StageParams& P, dim3 grid, hipStream_t st) {
  if (sub == SUB_FP16) {
    if (h0) return tgt == 0 ? launch_stage_k<SUB_FP16, 0, true, false>(P, grid, st) : hipErrorInvalidValue;
    return tgt == 0 ? launch_stage_k<SUB_FP16, 0, false, false>(P, grid, st)
                    : launch_stage_k<SUB_FP16, 1, false, false>(P, grid, st);
  }
  if (h0) return hipErrorInvalidValue;
  if (sub == SUB_INT8)
    return tgt == 0 ? launch_stage_k<SUB_INT8, 0, false, false>(P, grid, st)
                    : launch_stage_k<SUB_INT8, 1, false, false>(P, grid, st);
  return tgt == 0 ? launch_stage_k<SUB_FP8, 0, false, false>(P, grid, st)
                  : launch_stage_k<SUB_FP8, 1, false, false>(P, grid, st);
}

template <int SUB, int KMAX, bool FULL, int NP = 1>
static hipError_t launch_batch_t(const StageParams* descs, const int64_t* first, const uint16_t* tmember,
                                 int64_t total, hipStream_t st) {
  int lds = stage_lds_bytes<SUB, 0, KMAX, NP>(KMAX);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)ob_batch_kernel<SUB, 0, KMAX, FULL, NP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((ob_batch_kernel<SUB, 0, KMAX, FULL, NP>), dim3((unsigned)total), dim3(kThreads), lds, st,
                     descs, first, tmember, total);
  return hipGetLastError();
}

// K classes of the batched launches: the stage kernel's compile-time tile
// shapes (K <= 4, 8, 12, 16, 32).
int kclass_of(int K) { return K <= 4 ? 0 : K <= 8 ? 1 : K <= 12 ? 2 : K <= 16 ? 3 : 4; }
int kclass_kmax(int c) {
  static const int kmax[5] = {4, 8, 12, 16, 32};
  return kmax[c];
}

// full: every member of the launch has K equal to the class's KMAX (the
// FP16 substrate then takes the full-length variant).
template <int SUB>
static hipError_t launch_batch_s(int kmax, bool full, const StageParams* descs, const int64_t* first,
                                 const uint16_t* tmember, int64_t total, hipStream_t st) {
  constexpr bool F = SUB == SUB_FP16;
  switch (kmax) {
    case 4:  // FP16: the packed four-column tile
      if constexpr (F) return launch_batch_t<SUB, 16, true, 4>(descs, first, tmember, total, st);
      else return launch_batch_t<SUB, 4, false>(descs, first, tmember, total, st);
    case 8:  // FP16: the packed two-column tile for every K of the class
      if constexpr (F) return launch_batch_t<SUB, 16, true, 2>(descs, first, tmember, total, st);
      else return launch_batch_t<SUB, 8, false>(descs, first, tmember, total, st);
    case 12:
      return F && full ? launch_batch_t<SUB, 12, F>(descs, first, tmember, total, st)
                       : launch_batch_t<SUB, 12, false>(descs, first, tmember, total, st);
    case 16:
      return F && full ? launch_batch_t<SUB, 16, F>(descs, first, tmember, total, st)
                       : launch_batch_t<SUB, 16, false>(descs, first, tmember, total, st);
    default:
      return F && full ? launch_batch_t<SUB, 32, F>(descs, first, tmember, total, st)
                       : launch_batch_t<SUB, 32, false>(descs, first, tmember, total, st);
  }
}

// FP64-target batched launch over the members of one pass and K class.
hipError_t launch_batch(int sub, int kmax, bool full, const StageParams* descs, const int64_t* first,
                        const uint16_t* tmember, int64_t total, hipStream_t st) {
  if (sub == SUB_FP16) return launch_batch_s<SUB_FP16>(kmax, full, descs, first, tmember, total, st);
  if (sub == SUB_INT8) return launch_batch_s<SUB_INT8>(kmax, false, descs, first, tmember, total, st);
  return launch_batch_s<SUB_FP8>(kmax, false, descs, first, tmember, total, st);
}

// Columns per workgroup of the stage kernel for contraction length K.
int stage_cols_per_wg(int K, int sub) {
  if (fp16_pack(sub, K) > 1) return fp16_pack(sub, K) * Shape<16>::NCOL;
  return K <= 16 ? Shape<16>::NCOL : Shape<32>::NCOL;
}

hipError_t launch_digits_to_fp8(uint8_t* p, int64_t bytes, hipStream_t st) {
  int64_t n4 = bytes / 4;
  hipLaunchKernelGGL(digits_to_fp8_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, p, n4);
  return hipGetLastError();
}

}  // namespace obfft
