// Instruction-contract probes for gfx950 (tests only): one wave runs one
// MFMA (or lane permutation, or conversion) on operands laid out one register
// set per lane, so a test can check the register layout and the exact
// integer accumulation the kernels rely on.
#include "crt_methods.h"
#include "ob_device.h"

namespace obfft {

// ---- MFMA contract probes (layout and exact integer accumulation) ----
__global__ void mfma_probe_kernel(int kind, const void* a, const void* b, void* d) {
  const int lane = threadIdx.x;
  if (kind == 0) {
    long av = ((const long*)a)[lane], bv = ((const long*)b)[lane];
    v4f c = {0.f, 0.f, 0.f, 0.f};
    ((v4f*)d)[lane] = mfma_fp8(av, bv, c);
  } else if (kind == 1) {
    v4i av = ((const v4i*)a)[lane], bv = ((const v4i*)b)[lane];
    v4i c = {0, 0, 0, 0};
    ((v4i*)d)[lane] = mfma_i8(av, bv, c);
  } else if (kind == 2) {
    v8h av = ((const v8h*)a)[lane], bv = ((const v8h*)b)[lane];
    v16f c;
    for (int v = 0; v < 16; v++) c[v] = 0.f;
    ((v16f*)d)[lane] = mfma_f16_32(av, bv, c);
  } else if (kind == 3) {
    uint32_t x = ((const uint32_t*)a)[lane], y = ((const uint32_t*)b)[lane];
    auto pr = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    ((uint32_t*)d)[lane] = pr[0];
    ((uint32_t*)d)[64 + lane] = pr[1];
  } else if (kind == 5) {
    v8h av = ((const v8h*)a)[lane], bv = ((const v8h*)b)[lane];
    v4f c = {0.f, 0.f, 0.f, 0.f};
    ((v4f*)d)[lane] = mfma_f16_16(av, bv, c);
  } else if (kind == 6) {
    v4i_t av = ((const v4i_t*)a)[lane], bv = ((const v4i_t*)b)[lane];
    v16i_t c;
    for (int v = 0; v < 16; v++) c[v] = 0;
    ((v16i_t*)d)[lane] = mfma_i8_32(av, bv, c);
  } else if (kind == 7) {
    // scaled K = 128 FP8 MFMA: a = 64 lanes x 32 bytes, then 64 E8M0 scales of A (one int each);
    // b = 64 lanes x 32 bytes (unscaled)
    const v8i av = ((const v8i*)a)[lane], bv = ((const v8i*)b)[lane];
    const int sa = ((const int*)a)[64 * 8 + lane];
    v4f c = {0.f, 0.f, 0.f, 0.f};
    ((v4f*)d)[lane] = mfma_fp8_k128(av, bv, c, sa);
  } else if (kind == 4) {
    // E4M3 conversion of small integers: a = 64 floats, d = 64 bytes
    float x = ((const float*)a)[lane];
    uint32_t w = fp8_pack2<false>(x, 0.0f, 0u);
    ((uint8_t*)d)[lane] = (uint8_t)(w & 0xFF);
  }
}


hipError_t launch_mfma_probe(int kind, const void* a, const void* b, void* d, hipStream_t st) {
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, st, kind, a, b, d);
  return hipGetLastError();
}

}  // namespace obfft
