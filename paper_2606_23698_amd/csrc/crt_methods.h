// Constants and MFMA helper of the alternative exact reconstruction routes
// (host and device): Phase A on signed-byte MFMA with the two-limb
// shifted-column layout (Sec. 8.2, the B200 cross-check; Sec. 8.3, Eq.
// h1-group), and the Kulisch accumulation in 16-bit words (Sec. 6.3, Eq.
// kulisch-width; Sec. 6.4, Strategy A).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace obfft {

// Every Phase-A accumulator starts at this bias so that each column sum
// (|P'| <= r 128 (128 + 8) = 208896 for r = 12) is deposited as a
// non-negative value below 2^19.
constexpr int32_t kI8PhaseABias = 1 << 18;

struct CrtAltConsts {
  // INT8 Phase A
  int raw;             // raw columns S + 2 (balanced slices of u_k, shifted high limb)
  int frac;            // lift columns T + 2
  uint32_t wadd[4];    // M/2 + zoff M - sum_s bias 256^s  (mod 2^(32 NW))
  uint32_t zadd[2];    // 2^47 + zoff 2^48 - sum_t bias 256^t  (mod 2^64)
  // 16-bit Kulisch words: added to the swept accumulator E
  uint32_t kadd[4];    // M/2 + zoff M  (mod 2^(32 NW))
};

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16i_t mfma_i8_32(v4i_t a, v4i_t b, v16i_t c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

}  // namespace obfft
