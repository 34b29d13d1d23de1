// Plan-time mathematics (host only): modulus-set constants, quantised roots,
// MFMA operand planes.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "crt_methods.h"
#include "obfft_internal.h"

namespace obfft {

typedef unsigned __int128 u128;

constexpr int kFracBits = 48;                  // f of the fractional lift (Sec. 5.1)
constexpr uint32_t kFloatBiasBits = 0x4B400000u; // bit pattern of 1.5 * 2^23 as FP32
constexpr uint32_t kLiftOffset = 16384;          // > max |zhat| for centred residues (12,252)
constexpr int kFp8TwoDigitMax = 1052;          // moduli up to here need 2 radix-32 digits

struct ModSet {
  int r;
  int32_t m[kMaxModuli];
  u128 M;
  u128 u[kMaxModuli];     // CRT idempotents (Eq. fcrt)
  uint64_t w[kMaxModuli]; // round(2^48 u_k / M) (Sec. 5.1)
  int S, T;               // byte slices of u_k and w_k
  double log2M;
};

bool build_modset(const int32_t* mods, int r, ModSet& H, std::string& err);
double capacity_bits(int64_t Kmax, int kbits);
void build_crt_consts(const ModSet& H, CrtConsts& C);
void build_crt_alt(const ModSet& H, const CrtConsts& C, CrtAltConsts& K, std::vector<int8_t>& aop);
void quantised_roots(int64_t N, int bits, std::vector<int64_t>& out);
int fp8_digits(int m);
uint8_t e4m3_encode(int d);
uint16_t f16_encode_int(int v);
void build_operand_planes(const ModSet& H, const std::vector<int64_t>& roots, int64_t N,
                          int64_t p, int64_t q, int stage, int direction, int substrate,
                          int fp16_split, std::vector<uint8_t>& bytes, OperandPlanes& L, int layout128 = 0);
// True when residues mod m may enter the FP16 residue GEMM as one slot per
// index (no limb split) with an exact FP32 accumulation.
bool fp16_single_slot_ok(int m);
// Fold-and-add form of m for the H0 reduction of exact sums |t| <= 2^24:
// m = 2^b - c and the number of folds that take every such t into
// [-c, 2^b - 1 + c] (nf = 0 for a power of two).  *b = 0 when m is not
// friendly (complement above kH0MaxComplement).
void h0_fold_form(int m, int* b, int* c, int* nf);
void build_phaseA_operand(const ModSet& H, std::vector<uint16_t>& out, int* npairs);

}  // namespace obfft
