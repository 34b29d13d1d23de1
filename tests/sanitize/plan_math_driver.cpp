// Host driver of the plan-time mathematics for the sanitizer test: builds
// every constant table of both modulus sets and the MFMA operand planes of
// several factorisations, stages, directions and substrates, and prints a
// checksum.  Built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host (no device code runs).
#include <cstdio>
#include <string>
#include <vector>

#include "plan_math.h"

using namespace obfft;

static const int32_t kFP64[12] = {2039, 2029, 2027, 1089, 1024, 961, 841, 625, 529, 511, 491, 487};
static const int32_t kFP32[6] = {2039, 2029, 2027, 1024, 961, 841};
// the default sets of the transform plans (every modulus at most 1024, no limb split)
static const int32_t kStageFP64[12] = {1024, 1023, 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967};
static const int32_t kStageFP32[6] = {1024, 1023, 1021, 1019, 1013, 1009};

int main() {
  uint64_t sum = 0;
  for (int cfg = 0; cfg < 4; cfg++) {
    const int prec = cfg & 1, stage_set = cfg >> 1;
    const int split = stage_set ? 0 : (prec ? 3 : 4);
    ModSet H;
    std::string err;
    const int32_t* mods = stage_set ? (prec ? kStageFP32 : kStageFP64) : (prec ? kFP32 : kFP64);
    if (!build_modset(mods, prec ? 6 : 12, H, err)) {
      std::printf("build_modset: %s\n", err.c_str());
      return 1;
    }
    CrtConsts C;
    build_crt_consts(H, C);
    CrtAltConsts A;
    std::vector<int8_t> aop;
    build_crt_alt(H, C, A, aop);
    std::vector<uint16_t> pa;
    int npairs = 0;
    build_phaseA_operand(H, pa, &npairs);
    for (int8_t v : aop) sum += (uint8_t)v;
    for (uint16_t v : pa) sum += v;
    sum += C.M[0] + C.khi_c + (uint64_t)(capacity_bits(32, prec ? 24 : 53) * 1000);
    const int bits = prec ? 23 : 52;
    const int64_t shapes[][3] = {{32, 4, 8}, {1024, 32, 32}, {96, 8, 12}, {12, 3, 4}, {7, 7, 1}, {1, 1, 1}};
    for (const auto& s : shapes) {
      std::vector<int64_t> roots;
      quantised_roots(s[0], bits, roots);
      for (int64_t v : roots) sum += (uint64_t)v;
      for (int sub = 0; sub < 3; sub++)
        for (int stage = 1; stage <= 2; stage++)
          for (int dir = 0; dir < 2; dir++) {
            std::vector<uint8_t> bytes;
            OperandPlanes L;
            build_operand_planes(H, roots, s[0], s[1], s[2], stage, dir, sub, split, bytes, L);
            for (uint8_t b : bytes) sum = sum * 31 + b;
            // the full-length FP8 tile's layout (K = 32 stages)
            build_operand_planes(H, roots, s[0], s[1], s[2], stage, dir, sub, split, bytes, L, 1);
            for (uint8_t b : bytes) sum = sum * 31 + b;
          }
    }
  }
  for (int m = 2; m < 2048; m++) {
    int b, c, nf;
    h0_fold_form(m, &b, &c, &nf);
    sum += b + c + nf + fp8_digits(m) + fp16_single_slot_ok(m);
  }
  for (int d = -16; d <= 16; d++) sum += e4m3_encode(d);
  for (int v = -2048; v <= 2048; v++) sum += f16_encode_int(v);
  std::printf("plan math checksum %llu\n", (unsigned long long)sum);
  return 0;
}
