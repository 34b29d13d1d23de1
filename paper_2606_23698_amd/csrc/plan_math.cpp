// Plan-time mathematics of the Ozaki-Bailey FFT (host only).
//
//  * modulus set, M, CRT idempotents u_k, byte slices, lift weights w_k
//    (Sec. 2, Eq. capacity; Sec. 4.2, Eqs. fcrt and slicing; Sec. 5.1);
//  * quantised roots of unity Q(w_N^t) = RNE(2^B (cos, -sin)(2 pi t / N)),
//    evaluated in double-double arithmetic (Sec. 4.1, Eq. twiddle-fusion:
//    the fused coefficient is one quantised root);
//  * the MFMA operand planes of the residue GEMMs and of the Phase-A GEMM.
#include "plan_math.h"

#include <cmath>
#include <cstring>
#include <stdexcept>

namespace obfft {

static int bitlen(u128 x) {
  int n = 0;
  while (x) { n++; x >>= 1; }
  return n;
}

static int64_t modinv(int64_t a, int64_t m) {
  int64_t t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr) {
    int64_t qq = r / nr;
    int64_t tmp = t - qq * nt; t = nt; nt = tmp;
    tmp = r - qq * nr; r = nr; nr = tmp;
  }
  if (r != 1) return -1;
  return t < 0 ? t + m : t;
}

static int64_t gcd64(int64_t a, int64_t b) {
  while (b) { int64_t t = a % b; a = b; b = t; }
  return a;
}

bool build_modset(const int32_t* mods, int r, ModSet& H, std::string& err) {
  if (r < 2 || r > kMaxModuli) { err = "modulus count out of range"; return false; }
  H.r = r;
  H.M = 1;
  H.log2M = 0.0;
  for (int k = 0; k < r; k++) {
    if (mods[k] < 2 || mods[k] >= 2048) { err = "modulus out of range [2, 2048)"; return false; }
    for (int j = 0; j < k; j++)
      if (gcd64(mods[j], mods[k]) != 1) { err = "moduli not pairwise coprime"; return false; }
    H.m[k] = mods[k];
    H.M *= (u128)mods[k];
    H.log2M += std::log2((double)mods[k]);
  }
  if (bitlen(H.M) > 124) { err = "modulus product too large"; return false; }
  for (int k = 0; k < r; k++) {
    u128 Mk = H.M / (u128)H.m[k];
    int64_t inv = modinv((int64_t)(Mk % (u128)H.m[k]), H.m[k]);
    H.u[k] = Mk * (u128)inv;   // < M since inv < m_k
  }
  H.S = (bitlen(H.M) + 7) / 8;
  // w_k = round(2^48 u_k / M): 48 steps of binary long division of u_k / M.
  H.T = 0;
  for (int k = 0; k < r; k++) {
    u128 rem = H.u[k];
    uint64_t qv = 0;
    for (int i = 0; i < kFracBits; i++) {
      rem <<= 1;
      qv <<= 1;
      if (rem >= H.M) { rem -= H.M; qv |= 1; }
    }
    if (2 * rem == H.M) { err = "tie in lift weight"; return false; }
    if (2 * rem > H.M) qv++;
    H.w[k] = qv;
    int nb = 0;
    for (uint64_t x = qv; x; x >>= 8) nb++;
    if (nb > H.T) H.T = nb;
  }
  return true;
}

double capacity_bits(int64_t Kmax, int kbits) {
  return 1.0 + std::log2((double)Kmax) + 2.0 * (kbits + 1);
}

// ---- 160-bit helpers (little-endian 32-bit words) ----
static void add_shifted(uint32_t* acc, int nw, uint64_t v, int bitpos) {
  // acc += v << bitpos (mod 2^(32 nw))
  int w = bitpos / 32, o = bitpos % 32;
  u128 x = (u128)v << o;
  uint64_t carry = 0;
  for (int i = w; i < nw; i++) {
    uint64_t s = (uint64_t)acc[i] + (uint64_t)(uint32_t)x + carry;
    acc[i] = (uint32_t)s;
    carry = s >> 32;
    x >>= 32;
  }
}

static void sub_words(uint32_t* a, const uint32_t* b, int nw) {
  int64_t borrow = 0;
  for (int i = 0; i < nw; i++) {
    int64_t d = (int64_t)a[i] - (int64_t)b[i] - borrow;
    borrow = d < 0;
    a[i] = (uint32_t)d;
  }
}

// Splits delta (mod 2^bits) into per-slice seed offsets: bytes for slices
// 0 .. n-2, 16 bits for slice n-1 (all < 2^16, so seed + P stays in one
// binade); returns the remainder above bit 8 (n - 1) + 16.
static u128 split_delta(u128 delta, int n, int* d) {
  for (int s = 0; s < n; s++) {
    int width = s < n - 1 ? 8 : 16;
    d[s] = (int)((delta >> (8 * s)) & ((1u << width) - 1));
  }
  int top = 8 * (n - 1) + 16;
  return top >= 128 ? 0 : (delta >> top) << top;
}

void build_crt_consts(const ModSet& H, CrtConsts& C) {
  memset(&C, 0, sizeof(C));
  C.r = H.r;
  C.S = H.S;
  C.T = H.T;
  C.nwords = (bitlen(H.M) + 2 <= 96) ? 3 : 4;
  const int NW = C.nwords;
  const u128 mask = NW == 4 ? ~(u128)0 : (((u128)1 << (32 * NW)) - 1);
  u128 M = H.M, Mh = H.M >> 1, nM = (~H.M + 1);
  for (int i = 0; i < 4; i++) {
    C.M[i] = (uint32_t)(M >> (32 * i));
    C.Mhalf[i] = (uint32_t)(Mh >> (32 * i));
    C.negM[i] = (uint32_t)(nM >> (32 * i));
  }
  C.zoff = kLiftOffset;

  // Bit patterns of the partials: bits(seed) + P with bits(seed) = kFloatBiasBits
  // + delta.  The fast deposit adds pattern s at bit 8 s but drops the top
  // byte (0x4B) of the pattern of every slice s = 4 c + 1 that lands at bit
  // 32 c + 8; that constant is put back through the deltas.
  const int S = H.S, T = H.T, VP = (S + 1) / 2;
  u128 base = 0, dropped = 0;
  for (int s = 0; s < S; s++) base += (u128)kFloatBiasBits << (8 * s);
  for (int s = 1; s < S && 8 * s + 24 < 32 * NW; s += 4)
    dropped += (u128)(kFloatBiasBits >> 24) << (8 * s + 24);
  const u128 zM = H.M * (u128)kLiftOffset;
  for (int variant = 0; variant < 2; variant++) {
    // target: W = E + (exact ? M/2 : 0) + zoff M  (mod 2^(32 NW))
    u128 want = (variant == 0 ? Mh : 0) + zM;
    u128 delta = (want - base + dropped) & mask;
    int d[16];
    u128 rest = split_delta(delta, S, d);
    // the remainder must sit inside the top word
    if ((rest & (((u128)1 << (32 * (NW - 1))) - 1)) != 0) throw std::runtime_error("seed split");
    uint32_t hi = (uint32_t)(rest >> (32 * (NW - 1)));
    float* seed = variant == 0 ? C.seed_x : C.seed_c;
    for (int j = 0; j < 32; j++) seed[j] = 12582912.0f;  // 1.5 * 2^23
    for (int s2 = 0; s2 < S; s2++) seed[s2] = 12582912.0f + (float)d[s2];
    if (variant == 0) C.khi_x = hi; else C.khi_c = hi;
    if (variant == 0) {
      // taps: the full (undropped) pattern sum of the seeds, mod 2^160
      uint32_t Bp[5] = {0, 0, 0, 0, 0};
      for (int s2 = 0; s2 < S; s2++) add_shifted(Bp, 5, kFloatBiasBits + (uint32_t)d[s2], 8 * s2);
      memcpy(C.Bp5, Bp, sizeof(Bp));
    }
  }
  // (the transposed copies are filled after the lift-sum seeds below)
  // lift sum Z = sum_t bits(seed) 256^t (mod 2^64) + 2^47 (round half up) +
  // zoff 2^48; only word 1 is read, and the fast sum drops the top byte of
  // slice 1 (bit 32) as above
  {
    uint64_t zbase = 0, zdrop = 0;
    for (int t = 0; t < T; t++) zbase += (uint64_t)kFloatBiasBits << (8 * t);
    for (int t = 1; t < T && 8 * t + 24 < 64; t += 4) zdrop += (uint64_t)(kFloatBiasBits >> 24) << (8 * t + 24);
    uint64_t want = ((uint64_t)1 << (kFracBits - 1)) + ((uint64_t)kLiftOffset << kFracBits);
    uint64_t delta = want - zbase + zdrop;
    int d[16];
    u128 rest = split_delta((u128)delta, T, d) & (((u128)1 << 64) - 1);
    if ((rest & 0xFFFFFFFFull) != 0) throw std::runtime_error("seed split");
    C.zhi = (uint32_t)(rest >> 32);
    for (int t = 0; t < T; t++) {
      C.seed_x[2 * VP + t] = 12582912.0f + (float)d[t];
      C.seed_c[2 * VP + t] = 12582912.0f + (float)d[t];
    }
  }
  for (int h = 0; h < 2; h++)
    for (int v = 0; v < 16; v++) {
      C.seedT_x[h][v] = C.seed_x[2 * v + h];
      C.seedT_c[h][v] = C.seed_c[2 * v + h];
    }
  // recursive Garner: mixed-radix weights prod_{i<j} m_i reduced mod m_k
  for (int k = 0; k < H.r; k++) {
    const uint64_t mk = (uint64_t)H.m[k];
    C.gm[k] = (uint32_t)mk;
    C.gmagic[k] = (uint32_t)((((uint64_t)1 << 32) + mk - 1) / mk);
    uint64_t radix = 1 % mk;  // prod_{i<j} m_i mod m_k
    for (int j = 0; j < k; j++) {
      C.gneg[k][j] = (uint32_t)(mk - radix);
      radix = radix * (uint64_t)H.m[j] % mk;
    }
    C.ginv[k] = (uint32_t)modinv((int64_t)radix, (int64_t)mk);
  }
  // nearest binary64 to M: the top 53 significant bits, ties to even
  {
    const int nb = bitlen(H.M);
    u128 q = H.M;
    int e = 0;
    if (nb > 53) {
      const int sh = nb - 53;
      q = H.M >> sh;
      const u128 rem = H.M & ((((u128)1) << sh) - 1), half = ((u128)1) << (sh - 1);
      if (rem > half || (rem == half && (q & 1))) q += 1;
      e = sh;
    }
    C.Mf = std::ldexp((double)(uint64_t)q, e);
  }
}

// INT8 Phase-A route (Sec. 8.3, Eq. h1-group, on signed bytes).  The A
// operand is 32 rows x 32 limb columns of int8: row s < S + 2 is raw column s,
// row S + 2 + t lift column t; column k < r multiplies the low limb of
// modulus k by the balanced base-256 digit s of u_k, column r + k its high
// limb by digit s - 1 (the shifted column); lift rows use the digits of w_k.
// Lane l holds row l % 32, columns 16 (l / 32) .. + 15.
static void balanced_digits(u128 x, int count, int* d) {
  for (int i = 0; i < count; i++) {
    int b = (int)(x & 0xFF);
    if (b >= 128) b -= 256;
    d[i] = b;
    x = (b >= 0 ? x - (u128)b : x + (u128)(-b)) >> 8;
  }
  if (x != 0) throw std::runtime_error("balanced digits");
}

void build_crt_alt(const ModSet& H, const CrtConsts& C, CrtAltConsts& K, std::vector<int8_t>& aop) {
  const int r = H.r, S = H.S, T = H.T, NW = C.nwords;
  K.raw = S + 2;
  K.frac = T + 2;
  if (K.raw + K.frac > 32 || 2 * r > 32) throw std::runtime_error("int8 phase A shape");
  int A[32][32];
  memset(A, 0, sizeof(A));
  for (int k = 0; k < r; k++) {
    int du[17], dw[8];
    balanced_digits(H.u[k], S + 1, du);
    balanced_digits((u128)H.w[k], T + 1, dw);
    for (int s = 0; s < S + 2; s++) {
      A[s][k] = s <= S ? du[s] : 0;
      A[s][r + k] = s >= 1 ? du[s - 1] : 0;
    }
    for (int t = 0; t < T + 2; t++) {
      A[S + 2 + t][k] = t <= T ? dw[t] : 0;
      A[S + 2 + t][r + k] = t >= 1 ? dw[t - 1] : 0;
    }
  }
  aop.assign(64 * 16, 0);
  for (int l = 0; l < 64; l++)
    for (int j = 0; j < 16; j++) aop[l * 16 + j] = (int8_t)A[l % 32][16 * (l / 32) + j];
  // bias of every accumulator, weighted by its column position
  const u128 mask = NW == 4 ? ~(u128)0 : (((u128)1 << (32 * NW)) - 1);
  u128 braw = 0, bz = 0;
  for (int s = 0; s < S + 2 && 8 * s < 128; s++) braw += (u128)kI8PhaseABias << (8 * s);
  for (int t = 0; t < T + 2; t++) bz += (u128)kI8PhaseABias << (8 * t);
  const u128 wadd = ((H.M >> 1) + H.M * (u128)kLiftOffset - braw) & mask;
  const u128 zadd = ((((u128)1) << (kFracBits - 1)) + ((u128)kLiftOffset << kFracBits) - bz) &
                    ((((u128)1) << 64) - 1);
  for (int i = 0; i < 4; i++) K.wadd[i] = (uint32_t)(wadd >> (32 * i));
  K.zadd[0] = (uint32_t)zadd;
  K.zadd[1] = (uint32_t)(zadd >> 32);
  const u128 kadd = ((H.M >> 1) + H.M * (u128)kLiftOffset) & mask;
  for (int i = 0; i < 4; i++) K.kadd[i] = (uint32_t)(kadd >> (32 * i));
}

// ---- double-double trigonometry ----
namespace {
struct DD {
  double hi, lo;
};
inline DD two_sum(double a, double b) {
  double s = a + b, v = s - a;
  return {s, (a - (s - v)) + (b - v)};
}
inline DD fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
inline DD operator+(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
  double lo = s.lo + t.hi;
  DD u = fast_two_sum(s.hi, lo);
  lo = u.lo + t.lo;
  return fast_two_sum(u.hi, lo);
}
inline DD operator-(DD a) { return {-a.hi, -a.lo}; }
inline DD operator-(DD a, DD b) { return a + (-b); }
inline DD operator*(DD a, DD b) {
  double p = a.hi * b.hi;
  double e = std::fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p, e);
}
inline DD div_int(DD a, double d) {
  // (a / d) to double-double accuracy, d a small exact integer
  double q1 = a.hi / d;
  double p = q1 * d;
  double pe = std::fma(q1, d, -p);
  DD rem = (a - DD{p, pe});
  double q2 = rem.hi / d;
  return fast_two_sum(q1, q2);
}
const DD kHalfPi = {1.5707963267948966, 6.123233995736766e-17};

// sin and cos of x in [0, pi/4] by Taylor series in double-double.
void sincos_small(DD x, DD& s, DD& c) {
  DD x2 = x * x;
  DD term = x;
  s = x;
  for (int n = 1; n < 16; n++) {
    term = div_int(term * x2, (double)((2 * n) * (2 * n + 1)));
    s = (n & 1) ? s - term : s + term;
  }
  term = {1.0, 0.0};
  c = term;
  for (int n = 1; n < 16; n++) {
    term = div_int(term * x2, (double)((2 * n - 1) * (2 * n)));
    c = (n & 1) ? c - term : c + term;
  }
}

int64_t rne_dd(DD v) {
  double n = std::nearbyint(v.hi);
  double frac = (v.hi - n) + v.lo;
  if (frac > 0.5) return (int64_t)n + 1;
  if (frac < -0.5) return (int64_t)n - 1;
  if (frac == 0.5 || frac == -0.5) {
    int64_t a = (int64_t)n, b = frac > 0 ? a + 1 : a - 1;
    return (a % 2 == 0) ? a : b;
  }
  return (int64_t)n;
}
}  // namespace

void quantised_roots(int64_t N, int bits, std::vector<int64_t>& out) {
  out.assign(2 * N, 0);
  double scale = std::ldexp(1.0, bits);
  for (int64_t t = 0; t < N; t++) {
    // angle 2 pi t / N = (pi/2) (Q + f), Q = floor(4t/N), f = (4t - QN)/N
    int64_t q4 = 4 * t;
    int64_t Q = q4 / N;
    int64_t r4 = q4 - Q * N;
    bool flip = 2 * r4 > N;        // use the complementary angle for f > 1/2
    int64_t num = flip ? N - r4 : r4;
    double fh = (double)num / (double)N;
    double fl = std::fma(-fh, (double)N, (double)num) / (double)N;
    DD psi = kHalfPi * DD{fh, fl};
    DD s, c;
    sincos_small(psi, s, c);
    if (flip) { DD tmp = s; s = c; c = tmp; }
    DD cs, sn;   // cos and sin of the full angle
    switch (Q & 3) {
      case 0: cs = c; sn = s; break;
      case 1: cs = -s; sn = c; break;
      case 2: cs = -c; sn = -s; break;
      default: cs = s; sn = -c; break;
    }
    DD a = cs * DD{scale, 0.0};
    DD b = (-sn) * DD{scale, 0.0};
    out[2 * t] = rne_dd(a);
    out[2 * t + 1] = rne_dd(b);
  }
}

// ---- MFMA operand planes ----

static int centred(int64_t v, int m) {
  int64_t r = v % m;
  if (r < 0) r += m;
  if (r > m / 2) r -= m;
  return (int)r;
}

static int rne_div(int c, int R) {
  // nearest integer to c / R, ties to even
  double x = (double)c / (double)R;
  return (int)std::nearbyint(x);
}

int fp8_digits(int m) { return m <= kFp8TwoDigitMax ? 2 : 3; }

// Balanced radix-R digits of a centred residue (the same rule the kernels use
// on the data side: d0 = v - R rne(v/R), then recurse on rne(v/R)).
static void balanced_digits(int c, int R, int nd, int* d) {
  for (int i = 0; i < nd - 1; i++) {
    int q = rne_div(c, R);
    d[i] = c - R * q;
    c = q;
  }
  d[nd - 1] = c;
}

uint8_t e4m3_encode(int d) {
  if (d == 0) return 0;
  int sign = d < 0;
  int a = sign ? -d : d;
  int e = 31 - __builtin_clz((unsigned)a);
  int mant = ((a << 3) >> e) - 8;
  if ((((mant + 8) << e) >> 3) != a) throw std::runtime_error("digit not representable in E4M3");
  return (uint8_t)((sign << 7) | ((e + 7) << 3) | mant);
}

uint16_t f16_encode_int(int v) {
  if (v == 0) return 0;
  int sign = v < 0;
  int a = sign ? -v : v;
  if (a > 2048) throw std::runtime_error("integer not FP16-exact");
  int e = 31 - __builtin_clz((unsigned)a);
  int mant = (a << 10 >> e) - 1024;
  return (uint16_t)((sign << 15) | ((e + 15) << 10) | mant);
}

// Matrix entry (integer) of a stage: stage 1 F_q[t][s] = w_N^{p s t}; stage 2
// F_p^(g)[t][s] = w_N^{s (g + q t)} -- one quantised root (Eq. twiddle-fusion).
static void matrix_entry(const std::vector<int64_t>& roots, int64_t N, int64_t p, int64_t q,
                         int stage, int64_t g, int64_t t, int64_t s, int direction,
                         int64_t* c, int64_t* sn) {
  int64_t idx = stage == 1 ? (p * s * t) % N : (s * (g + q * t)) % N;
  *c = roots[2 * idx];
  *sn = roots[2 * idx + 1] * (direction ? -1 : 1);
}

bool fp16_single_slot_ok(int m) {
  const int64_t h = m / 2, e = (m & (m - 1)) == 0 ? 0 : 2;
  return 2LL * kMaxK * h * (h + e) <= (1LL << 24);
}

static int64_t floor_div(int64_t a, int64_t d) { return a >= 0 ? a / d : -((-a + d - 1) / d); }

void h0_fold_form(int m, int* b, int* c, int* nf) {
  int bb = 0;
  while ((1 << bb) < m) bb++;
  const int cc = (1 << bb) - m;
  *b = 0;
  *c = cc;
  *nf = 0;
  if (m < 2 || cc > kH0MaxComplement) return;
  // interval of t after each fold: t' = c h + l, h in [floor(lo / 2^b),
  // floor(hi / 2^b)], l in [0, 2^b)
  int64_t lo = -(1LL << 24), hi = 1LL << 24;
  const int64_t B = 1LL << bb;
  int n = 0;
  while (cc > 0 && (lo < -cc || hi > B - 1 + cc)) {
    const int64_t hl = floor_div(lo, B), hh = floor_div(hi, B);
    lo = cc * hl;
    hi = cc * hh + B - 1;
    if (++n > 32) return;  // no convergence: keep the reciprocal reduction
  }
  *b = bb;
  *nf = n;
}

void build_operand_planes(const ModSet& H, const std::vector<int64_t>& roots, int64_t N,
                          int64_t p, int64_t q, int stage, int direction, int substrate,
                          int fp16_split, std::vector<uint8_t>& bytes, OperandPlanes& L, int layout128) {
  int K = stage == 1 ? (int)q : (int)p;
  // layout128: the planes of the full-length FP8 tile (K = 32) on the scaled
  // K = 128 MFMA instead of the general tile's
  const bool k128 = substrate == SUB_FP8 && K == 32 && layout128;
  int G = stage == 1 ? 1 : (int)q;
  // packed FP16 tiles: the planes are the block-diagonal diag(F, ..., F) of
  // np blocks of 16 / np rows and slots in a 16 x 16 matrix
  const int np = fp16_pack(substrate, K);
  const bool pk = np > 1;
  const int BR = 16 / np;
  const int KV = pk ? 16 : K;
  int MT = (KV + 15) / 16;
  int bpl, fmax, chmax;
  if (substrate == SUB_INT8) { bpl = 16; fmax = 2; chmax = (2 * K + 63) / 64; }
  else if (substrate == SUB_FP16) { bpl = 16; fmax = 1; chmax = (2 * KV + 31) / 32; }
  else { bpl = 8; fmax = 3; chmax = (4 * K + 31) / 32; }
  int64_t chunk_bytes = 64 * bpl;
  L.fmax = fmax; L.chmax = chmax; L.mt = MT; L.G = G;
  L.mod_stride = 3LL * fmax * MT * chmax * chunk_bytes;
  L.g_stride = (int64_t)H.r * L.mod_stride;
  bytes.assign((size_t)(L.g_stride * G), 0);
  std::vector<int> cval(3 * K * K);
  for (int g = 0; g < G; g++) {
    for (int i = 0; i < H.r; i++) {
      int m = H.m[i];
      for (int t = 0; t < K; t++)
        for (int s = 0; s < K; s++) {
          int64_t c, sn;
          matrix_entry(roots, N, p, q, stage, g, t, s, direction, &c, &sn);
          cval[(0 * K + t) * K + s] = centred(c, m);
          cval[(1 * K + t) * K + s] = centred(sn, m);
          // four real products on every substrate: Re A, Im A, -Im A
          cval[(2 * K + t) * K + s] = centred(-sn, m);
        }
      if (substrate == SUB_FP16) {
        // [form][M-tile][chunk][lane][8 halves]; slot 32 ch + 8 (lane / 16) + j
        // holds limb weight 128^(slot % 2) of index slot / 2, folded mod m,
        // for the first fp16_split moduli, and index `slot` itself (one FP16
        // slot per index, chunk 0 only) for the others.
        const bool split = i < fp16_split;
        int pw128 = 128 % m;
        for (int form = 0; form < 3; form++)
          for (int mt = 0; mt < MT; mt++)
            for (int ch = 0; ch < chmax; ch++)
              for (int lane = 0; lane < 64; lane++)
                for (int j = 0; j < 8; j++) {
                  int t = 16 * mt + lane % 16;
                  int slot = 32 * ch + 8 * (lane / 16) + j;
                  int s = split ? slot / 2 : slot, e = split ? slot % 2 : 0;
                  int val = 0;
                  if (pk) {  // block (t / BR, s / BR) is F on the diagonal, else 0
                    const bool diag = t / BR == s / BR;
                    t %= BR;
                    s = diag ? s % BR : K;
                  }
                  if (t < K && s < K) {
                    int a = cval[(form * K + t) * K + s];
                    val = e ? centred((int64_t)a * pw128, m) : a;
                  }
                  uint16_t h = f16_encode_int(val);
                  int64_t off = g * L.g_stride + i * L.mod_stride +
                                (((int64_t)form * MT + mt) * chmax + ch) * chunk_bytes + lane * bpl + 2 * j;
                  bytes[off] = (uint8_t)(h & 0xFF);
                  bytes[off + 1] = (uint8_t)(h >> 8);
                }
        continue;
      }
      if (k128) {
        // Full-length FP8 tile on the scaled 16 x 16 x 128 MFMA: the
        // products (matrix digit f, data digit e) of one modulus form nd^2
        // blocks of 32 slots (index s), taken four to an instruction in the
        // order idx = f nd + e; block b of an instruction sits at bytes
        // 16 (b / 2) .. + 15 of lane groups 2 (b % 2) and 2 (b % 2) + 1, the
        // first 16 indices in the first group.  [form][instr][M-tile][lane][32 bytes];
        // forms Re A and Im A only (the kernel negates the data instead of Im A).
        const int nd = fp8_digits(m);
        const int pw[3] = {1, 32 % m, (32 * 32) % m};
        for (int form = 0; form < 2; form++)
          for (int ins = 0; ins < 3; ins++)
            for (int mt = 0; mt < MT; mt++)
              for (int lane = 0; lane < 64; lane++)
                for (int j = 0; j < 32; j++) {
                  const int h = lane / 16, t = 16 * mt + lane % 16;
                  const int b = j < 16 ? h / 2 : 2 + h / 2;
                  const int idx = 4 * ins + b;
                  const int s = 16 * (h % 2) + j % 16;
                  int digit = 0;
                  if (idx < nd * nd && t < K && s < K) {
                    const int f = idx / nd, e = idx % nd;
                    int d[3];
                    balanced_digits(centred((int64_t)cval[(form * K + t) * K + s] * pw[e], m), 32, nd, d);
                    digit = d[f];
                  }
                  const int64_t off = g * L.g_stride + i * L.mod_stride +
                                      (((int64_t)form * 3 + ins) * MT + mt) * 2048 + lane * 32 + j;
                  bytes[off] = (uint8_t)(int8_t)digit;
                }
        continue;
      }
      int R = substrate == SUB_INT8 ? 128 : 32;
      int nd = substrate == SUB_INT8 ? 2 : fp8_digits(m);
      int ndp = substrate == SUB_INT8 ? 2 : nd;  // FP8: nd slots per index
      int nf = nd;
      int pw[3] = {1, R % m, (R * R) % m};
      for (int form = 0; form < 3; form++)
        for (int f = 0; f < fmax; f++)
          for (int mt = 0; mt < MT; mt++)
            for (int ch = 0; ch < chmax; ch++)
              for (int lane = 0; lane < 64; lane++)
                for (int j = 0; j < bpl; j++) {
                  int t = 16 * mt + lane % 16;
                  int kk = (substrate == SUB_INT8 ? 16 : 8) * (lane / 16) + j;
                  int slot = (substrate == SUB_INT8 ? 64 : 32) * ch + kk;
                  int s = slot / ndp, e = slot % ndp;
                  int digit = 0;
                  if (t < K && s < K && e < nd && f < nf) {
                    int a = cval[(form * K + t) * K + s];
                    int ce = centred((int64_t)a * pw[e], m);
                    int d[3];
                    balanced_digits(ce, R, nd, d);
                    digit = d[f];
                  }
                  int64_t off = g * L.g_stride + i * L.mod_stride +
                                ((((int64_t)form * fmax + f) * MT + mt) * chmax + ch) * chunk_bytes +
                                lane * bpl + j;
                  // FP8 planes hold the signed digit as int8 here; they are
                  // converted to E4M3 on the device by the same instruction
                  // the kernels use for the data digits.
                  bytes[off] = (uint8_t)(int8_t)digit;
                }
    }
  }
}

// Phase-A operand of v_mfma_f32_32x32x16_f16: A[row][slot], row = partial
// placement, slot = modulus.  Lane l holds row l % 32, slots 8 (l / 32) + j;
// slot 8 h + j carries modulus ML h + j for j < ML (ML = 2 ceil(r / 4): 6 for
// r = 12, 4 for r = 6), so that each lane half takes one share of a residue
// record.  Row rho is read back in register v = (rho % 4) + 4 (rho / 8) of
// lane half (rho / 4) % 2; register pair v carries P_{2v}, P_{2v+1} for
// v < ceil(S/2) and then the lift bytes Z_{2u}, Z_{2u+1}.
void build_phaseA_operand(const ModSet& H, std::vector<uint16_t>& out, int* npairs) {
  out.assign(64 * 8, 0);
  int vp = (H.S + 1) / 2, vz = (H.T + 1) / 2;
  int ML = 2 * ((H.r / 2 + 1) / 2);
  *npairs = vp + vz;
  for (int lane = 0; lane < 64; lane++)
    for (int j = 0; j < 8; j++) {
      int rho = lane % 32, k = ML * (lane / 32) + j;
      int v = (rho % 4) + 4 * (rho / 8), half = (rho / 4) % 2;
      int val = 0;
      if (j < ML && k < H.r) {
        if (v < vp) {
          int s = 2 * v + half;
          if (s < H.S) val = (int)((H.u[k] >> (8 * s)) & 0xFF);
        } else if (v < vp + vz) {
          int t = 2 * (v - vp) + half;
          if (t < H.T) val = (int)((H.w[k] >> (8 * t)) & 0xFF);
        }
      }
      out[lane * 8 + j] = f16_encode_int(val);
    }
}

}  // namespace obfft
