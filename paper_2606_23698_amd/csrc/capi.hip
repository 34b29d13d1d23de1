// C ABI of libobfft: plans, the six-step driver and the unit-level entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "obfft.h"
#include "plan_math.h"

namespace obfft {
hipError_t launch_stage(int sub, int tgt, bool h0, const StageParams& P, dim3 grid, hipStream_t st);
hipError_t launch_stage_tap(int sub, int tgt, bool h0, const StageParams& P, dim3 grid, hipStream_t st);
hipError_t launch_crt(int tgt, int64_t n, const uint16_t* residues, const int* exps, void* out,
                      uint32_t* taps, const uint16_t* phaseA, const CrtConsts* C, hipStream_t st);
hipError_t launch_crt_ablation(int tgt, int method, int64_t n, const uint16_t* residues, const int* exps,
                              void* out, const uint16_t* phaseA, const CrtConsts* C, const int8_t* phaseA_i8,
                              const CrtAltConsts* i8, hipStream_t st);
hipError_t launch_digits_to_fp8(uint8_t* p, int64_t bytes, hipStream_t st);
hipError_t launch_mfma_probe(int kind, const void* a, const void* b, void* d, hipStream_t st);
hipError_t launch_scale(void* data, int64_t n_scalars, double factor, int tgt, hipStream_t st);
int stage_cols_per_wg(int K, int sub);
hipError_t launch_batch(int sub, int kmax, bool full, const StageParams* descs, const int64_t* first,
                        const uint16_t* tmember, int64_t total, hipStream_t st);
int kclass_of(int K);
int kclass_kmax(int c);
int persist_lds_bytes(unsigned cls_mask);
int persist_variant(int K);
int persist_grid(unsigned mask, int lds);
hipError_t launch_persist(unsigned mask, const PersistParams* Q, uint32_t* ctl, int64_t ctl_words, int grid, int lds,
                          hipStream_t st);
struct NativePlan;
NativePlan* native_plan_create(const int64_t* n, std::string& err);
void native_plan_destroy(NativePlan* np);
hipError_t native_execute(NativePlan* np, const void* in, void* out, void* ws, int inverse, hipStream_t st);
}  // namespace obfft

using namespace obfft;

// The paper's modulus sets (Sec. 2): the standalone CRT entry points and the
// fold-and-add reduction use them.
static const int32_t kModFP64[12] = {2039, 2029, 2027, 1089, 1024, 961, 841, 625, 529, 511, 491, 487};
static const int32_t kModFP32[6] = {2039, 2029, 2027, 1024, 961, 841};
// Default sets of the transform plans: pairwise coprime, every modulus at
// most 1024, so each residue is one FP16 slot of the residue GEMM (no limb
// split of the data).  log2 M = 119.58 (FP64 target, above the 114 bits that
// K = 32 needs) and 59.95 (FP32 target, above 56); the epilogue shape is the
// same as with the paper's sets (15 / 8 byte slices of u_k, 6 of w_k).  The
// stage results are exact integers, so the outputs do not depend on the set.
static const int32_t kModStageFP64[12] = {1024, 1023, 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967};
static const int32_t kModStageFP32[6] = {1024, 1023, 1021, 1019, 1013, 1009};

struct DevPlanes {
  OperandPlanes L;
};

struct obfft_plan_s {
  int64_t n[3] = {0, 0, 0};
  int p[3] = {0, 0, 0}, q[3] = {0, 0, 0};
  int precision = 0, substrate = SUB_FP8, kbits = 53;
  int reduction = OBFFT_RED_RECIPROCAL;
  int group_block = 0;  // 0: the library's choice
  int fp8_full = 0;     // the modulus set follows the full-length FP8 tile's digit rule
  int order[3] = {2, 1, 0};  // axes in execution order (0 = n1)
  ModSet H;
  CrtConsts C;
  ModConsts MC;
  std::vector<int64_t> roots[3];
  DevPlanes planes[3][2][2];  // axis, stage-1, direction
  std::vector<void*> dev_allocs;
  uint16_t* d_phaseA = nullptr;
  const ModConsts* d_mc = nullptr;    // device copies of MC and C
  const CrtConsts* d_crt = nullptr;
  uint32_t* d_flags = nullptr;        // device word: bit 0 = a non-finite input was read
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  obfft_status_t last = OBFFT_SUCCESS;
  NativePlan* native = nullptr;
  int device = 0;
  // batch plans
  int batch_count = 0;
  std::vector<obfft_plan_t> members;          // owned, one per distinct shape
  std::vector<obfft_plan_t> members_of_batch; // per batch entry (borrowed)
  StageParams* d_desc = nullptr;      // device [6][count]
  StageParams* h_desc = nullptr;      // pinned host staging [6][count]
  int64_t* d_first = nullptr;         // device [6][count]: a member's first tile in its class launch
  uint16_t* d_tmember = nullptr;      // device: member of every tile, launches concatenated
  int64_t tmember_off[6][5] = {};     // per pass and K class: offset into d_tmember
  int64_t batch_total[6][5] = {};     // per pass and K class: tiles (= grid of that launch)
  int batch_full[6][5] = {};          // per pass and K class: every member has K = the class's KMAX
  void* batch_ws = nullptr;
  std::vector<size_t> ws_off;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  hipEvent_t desc_done = nullptr;     // the last descriptor upload has left the pinned buffer
  bool use_graph = true;
  // persistent batched launch (FP16 substrate): one kernel over every pass
  int batch_mode = OBFFT_BATCH_PASSES;
  int persist_ok = 0;                 // the plan's substrate has the persistent kernel
  int persist_nseg = 0, persist_grid_size = 0, persist_lds = 0, persist_spin = 1 << 21;
  int persist_claim = 1;              // items a workgroup claims at once
  unsigned persist_mask = 0;          // tile variants the batch's stages need
  int64_t persist_items = 0;
  PersistParams* d_persist = nullptr; // device copy of the kernel's parameter block
  int64_t* d_seg_start = nullptr;
  int* d_seg_dep = nullptr;
  int* d_seg_cls = nullptr;
  uint32_t* d_ctl = nullptr;          // [2 + nseg]: item counter, give-up flag, completed tiles
};

static obfft_status_t fail(obfft_plan_t plan, obfft_status_t s) {
  if (plan) plan->last = s;
  return s;
}

static bool device_is_gfx950() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  return strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

extern "C" void obfft_options_default(obfft_options_t* opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->precision = OBFFT_PREC_FP64;
  opt->substrate = OBFFT_SUB_AUTO;
}

// Library default factorisation N = p q with p <= q <= 32: the most balanced
// split with both factors even if there is one (32 = 4 x 8, 256 = 16 x 16,
// 1024 = 32 x 32, 12 = 2 x 6), else the most balanced split of any parity
// (9 = 3 x 3, 18 = 3 x 6, 1 = 1 x 1: a length-1 axis is an exact identity).
static bool default_split(int64_t N, int* p, int* q) {
  for (int pass = 0; pass < 2; pass++) {
    int best = -1;
    for (int a = 1; a <= kMaxK; a++) {
      if (N % a) continue;
      int64_t b = N / a;
      if (b < a || b > kMaxK) continue;
      if (pass == 0 && ((a & 1) || (b & 1))) continue;
      best = a;
    }
    if (best > 0) {
      *p = best;
      *q = (int)(N / best);
      return true;
    }
  }
  return false;
}

static void build_modconsts(const ModSet& H, ModConsts& MC, int substrate) {
  memset(&MC, 0, sizeof(MC));
  for (int i = 0; i < H.r; i++) {
    MC.m[i] = H.m[i];
    MC.inv_mf[i] = 1.0f / (float)H.m[i];
    MC.inv_md[i] = 1.0 / (double)H.m[i];
    MC.mf[i] = (float)H.m[i];
    MC.md[i] = (double)H.m[i];
    MC.nd[i] = fp8_digits(H.m[i]);
    MC.sub[i] = substrate;
    h0_fold_form(H.m[i], &MC.fold_b[i], &MC.fold_c[i], &MC.fold_n[i]);
  }
}

static obfft_status_t upload(obfft_plan_t plan, const void* host, size_t bytes, void** dev) {
  void* d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return OBFFT_ALLOC_FAILED;
  plan->dev_allocs.push_back(d);
  if (hipMemcpy(d, host, bytes, hipMemcpyHostToDevice) != hipSuccess) return OBFFT_HIP_ERROR;
  *dev = d;
  return OBFFT_SUCCESS;
}

static obfft_status_t plan_build(obfft_plan_t plan, const obfft_options_t* opt) {
  plan->precision = opt->precision;
  int sub = opt->substrate;
  plan->substrate = sub;
  plan->kbits = plan->precision == OBFFT_PREC_FP32 ? 24 : 53;
  const bool h0 = opt->reduction == OBFFT_RED_H0;
  const int32_t* mods = plan->precision == OBFFT_PREC_FP32 ? kModStageFP32 : (h0 ? kModFP64 : kModStageFP64);
  int r = plan->precision == OBFFT_PREC_FP32 ? 6 : 12;
  if (opt->n_moduli_override) {
    if (!opt->moduli_override) return OBFFT_INVALID_VALUE;
    mods = opt->moduli_override;
    r = opt->n_moduli_override;
  }
  std::string err;
  if (!build_modset(mods, r, plan->H, err)) return OBFFT_INVALID_VALUE;
  // FP16 needs every modulus past the split to fit one slot per index; AUTO
  // takes FP16 when the set allows it, else INT8
  const int fp16_split = obfft::fp16_split(plan->precision == OBFFT_PREC_FP32 ? 1 : 0, h0);
  bool fp16_ok = true;
  for (int i = fp16_split; i < plan->H.r; i++) fp16_ok = fp16_ok && fp16_single_slot_ok(plan->H.m[i]);
  if (sub == OBFFT_SUB_AUTO) sub = fp16_ok ? OBFFT_SUB_FP16 : OBFFT_SUB_INT8;
  if (sub == OBFFT_SUB_FP16 && !fp16_ok) return OBFFT_UNSUPPORTED_SIZE;
  plan->substrate = sub;
  // the full-length FP8 tile takes 3 digits per residue for the moduli before
  // the split and 2 after it
  plan->fp8_full = 1;
  for (int i = 0; i < plan->H.r; i++)
    if (fp8_digits(plan->H.m[i]) != (i < fp16_split ? 3 : 2)) plan->fp8_full = 0;
  // the fold-and-add reduction is an ablation of the default FP64 path
  plan->reduction = opt->reduction;
  plan->group_block = opt->group_block;
  if (opt->axis_order[0] | opt->axis_order[1] | opt->axis_order[2])
    for (int k = 0; k < 3; k++) plan->order[k] = opt->axis_order[k];
  if (opt->reduction == OBFFT_RED_H0 && (sub != OBFFT_SUB_FP16 || plan->precision != OBFFT_PREC_FP64))
    return OBFFT_INVALID_VALUE;
  int64_t kmax = 0;
  for (int a = 0; a < 3; a++) {
    int64_t N = plan->n[a];
    int pp = opt->p[a], qq = opt->q[a];
    if (pp == 0 && qq == 0) {
      if (!default_split(N, &pp, &qq)) return OBFFT_UNSUPPORTED_SIZE;
    } else if ((int64_t)pp * qq != N) {
      return OBFFT_INVALID_VALUE;
    }
    if (pp < 1 || qq < 1 || pp > kMaxK || qq > kMaxK) return OBFFT_UNSUPPORTED_SIZE;
    plan->p[a] = pp;
    plan->q[a] = qq;
    kmax = std::max<int64_t>(kmax, std::max(pp, qq));
    // the stage kernels index contraction columns in 31 bits, and a launch
    // holds fewer than kMaxTiles workgroups
    const int64_t n_all = plan->n[0] * plan->n[1] * plan->n[2];
    if (n_all / qq >= ((int64_t)1 << 31)) return OBFFT_UNSUPPORTED_SIZE;
    const int64_t c1 = stage_cols_per_wg(qq, sub), c2 = stage_cols_per_wg(pp, sub);
    if ((n_all / qq + c1 - 1) / c1 >= kMaxTiles || qq * ((n_all / N + c2 - 1) / c2) >= kMaxTiles)
      return OBFFT_UNSUPPORTED_SIZE;
  }
  // Eq. capacity: log2 M > 1 + log2 K + 2(k+1)
  if (!(plan->H.log2M > capacity_bits(kmax, plan->kbits))) return OBFFT_CAPACITY_EXCEEDED;
  int expect_r = plan->precision == OBFFT_PREC_FP32 ? 6 : 12, expect_S = plan->precision ? 8 : 15;
  if (plan->H.r != expect_r || plan->H.S != expect_S || plan->H.T != 6) return OBFFT_UNSUPPORTED_SIZE;
  build_crt_consts(plan->H, plan->C);
  build_modconsts(plan->H, plan->MC, sub);
  if (!device_is_gfx950()) return OBFFT_UNSUPPORTED_DEVICE;
  hipGetDevice(&plan->device);
  int bits = plan->kbits - 1;
  std::map<std::tuple<int64_t, int, int, int, int>, OperandPlanes> cache;
  for (int a = 0; a < 3; a++) {
    quantised_roots(plan->n[a], bits, plan->roots[a]);
    for (int st = 1; st <= 2; st++)
      for (int d = 0; d < 2; d++) {
        auto key = std::make_tuple(plan->n[a], plan->p[a], plan->q[a], st, d);
        auto it = cache.find(key);
        if (it != cache.end()) {
          plan->planes[a][st - 1][d].L = it->second;
          continue;
        }
        std::vector<uint8_t> bytes;
        OperandPlanes L;
        build_operand_planes(plan->H, plan->roots[a], plan->n[a], plan->p[a], plan->q[a], st, d, sub, fp16_split,
                             bytes, L);
        void* dptr = nullptr;
        obfft_status_t s = upload(plan, bytes.data(), bytes.size(), &dptr);
        if (s != OBFFT_SUCCESS) return s;
        L.dev = (uint8_t*)dptr;
        L.dev128 = nullptr;
        if (sub == SUB_FP8) {
          if (launch_digits_to_fp8(L.dev, (int64_t)bytes.size(), 0) != hipSuccess) return OBFFT_HIP_ERROR;
          // K = 32 with the full-length digit rule: also the full tile's layout
          const int64_t K = st == 1 ? plan->q[a] : plan->p[a];
          if (K == 32 && plan->fp8_full) {
            OperandPlanes L2;
            build_operand_planes(plan->H, plan->roots[a], plan->n[a], plan->p[a], plan->q[a], st, d, sub,
                                 fp16_split, bytes, L2, 1);
            if (L2.mod_stride != L.mod_stride || L2.g_stride != L.g_stride) return OBFFT_HIP_ERROR;
            if ((s = upload(plan, bytes.data(), bytes.size(), &dptr)) != OBFFT_SUCCESS) return s;
            L.dev128 = (uint8_t*)dptr;
            if (launch_digits_to_fp8(L.dev128, (int64_t)bytes.size(), 0) != hipSuccess) return OBFFT_HIP_ERROR;
          }
        }
        cache[key] = L;
        plan->planes[a][st - 1][d].L = L;
      }
  }
  std::vector<uint16_t> pa;
  int npairs = 0;
  build_phaseA_operand(plan->H, pa, &npairs);
  void* dpa = nullptr;
  obfft_status_t s = upload(plan, pa.data(), pa.size() * 2, &dpa);
  if (s != OBFFT_SUCCESS) return s;
  plan->d_phaseA = (uint16_t*)dpa;
  void* dmc = nullptr;
  void* dcr = nullptr;
  s = upload(plan, &plan->MC, sizeof(ModConsts), &dmc);
  if (s != OBFFT_SUCCESS) return s;
  s = upload(plan, &plan->C, sizeof(CrtConsts), &dcr);
  if (s != OBFFT_SUCCESS) return s;
  plan->d_mc = (const ModConsts*)dmc;
  plan->d_crt = (const CrtConsts*)dcr;
  const uint32_t zero_flags[64] = {};
  void* dfl = nullptr;
  s = upload(plan, zero_flags, sizeof(zero_flags), &dfl);
  if (s != OBFFT_SUCCESS) return s;
  plan->d_flags = (uint32_t*)dfl;
  plan->ws_bytes = (size_t)(plan->n[0] * plan->n[1] * plan->n[2]) * (plan->precision ? 8 : 16);
  if (hipDeviceSynchronize() != hipSuccess) return OBFFT_HIP_ERROR;
  if (plan->precision == OBFFT_PREC_FP64) {
    std::string nerr;
    plan->native = native_plan_create(plan->n, nerr);
  }
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_plan_create(obfft_plan_t* out, int64_t n1, int64_t n2, int64_t n3,
                                            const obfft_options_t* opt) {
  if (!out) return OBFFT_INVALID_VALUE;
  *out = nullptr;
  if (n1 < 1 || n2 < 1 || n3 < 1) return OBFFT_INVALID_VALUE;
  obfft_options_t def;
  obfft_options_default(&def);
  if (!opt) opt = &def;
  if (opt->precision != OBFFT_PREC_FP64 && opt->precision != OBFFT_PREC_FP32) return OBFFT_INVALID_VALUE;
  if (opt->substrate < 0 || opt->substrate > OBFFT_SUB_AUTO) return OBFFT_INVALID_VALUE;
  if (opt->reduction != OBFFT_RED_RECIPROCAL && opt->reduction != OBFFT_RED_H0) return OBFFT_INVALID_VALUE;
  if (opt->group_block < 0 || opt->group_block > 32 || (opt->group_block & (opt->group_block - 1)))
    return OBFFT_INVALID_VALUE;
  if (opt->axis_order[0] | opt->axis_order[1] | opt->axis_order[2]) {
    int seen = 0;
    for (int k = 0; k < 3; k++) {
      if (opt->axis_order[k] < 0 || opt->axis_order[k] > 2) return OBFFT_INVALID_VALUE;
      seen |= 1 << opt->axis_order[k];
    }
    if (seen != 7) return OBFFT_INVALID_VALUE;
  }
  obfft_plan_t plan = new (std::nothrow) obfft_plan_s();
  if (!plan) return OBFFT_ALLOC_FAILED;
  plan->n[0] = n1;
  plan->n[1] = n2;
  plan->n[2] = n3;
  obfft_status_t s;
  try {
    s = plan_build(plan, opt);
  } catch (...) {
    s = OBFFT_INVALID_VALUE;
  }
  if (s != OBFFT_SUCCESS) {
    obfft_plan_destroy(plan);
    return s;
  }
  *out = plan;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_plan_destroy(obfft_plan_t plan) {
  if (!plan) return OBFFT_INVALID_VALUE;
  for (auto m : plan->members) obfft_plan_destroy(m);
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
  if (plan->desc_done) (void)hipEventDestroy(plan->desc_done);
  if (plan->d_desc) (void)hipFree(plan->d_desc);
  if (plan->d_first) (void)hipFree(plan->d_first);
  if (plan->d_tmember) (void)hipFree(plan->d_tmember);
  if (plan->h_desc) (void)hipHostFree(plan->h_desc);
  if (plan->batch_ws) (void)hipFree(plan->batch_ws);
  if (plan->d_persist) (void)hipFree(plan->d_persist);
  if (plan->d_seg_start) (void)hipFree(plan->d_seg_start);
  if (plan->d_seg_dep) (void)hipFree(plan->d_seg_dep);
  if (plan->d_seg_cls) (void)hipFree(plan->d_seg_cls);
  if (plan->d_ctl) (void)hipFree(plan->d_ctl);
  for (void* d : plan->dev_allocs) hipFree(d);
  if (plan->ws_owned && plan->ws) hipFree(plan->ws);
  if (plan->native) native_plan_destroy(plan->native);
  delete plan;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_plan_info(obfft_plan_t plan, obfft_plan_info_t* info) {
  if (!plan || !info) return OBFFT_INVALID_VALUE;
  memset(info, 0, sizeof(*info));
  info->precision = plan->precision;
  info->substrate = plan->substrate;
  info->r = plan->H.r;
  for (int i = 0; i < plan->H.r; i++) info->moduli[i] = plan->H.m[i];
  info->log2M = plan->H.log2M;
  int64_t kmax = 0;
  for (int a = 0; a < 3; a++) {
    info->p[a] = plan->p[a];
    info->q[a] = plan->q[a];
    info->n[a] = plan->n[a];
    kmax = std::max<int64_t>(kmax, std::max(plan->p[a], plan->q[a]));
  }
  info->budget_bits = kmax ? capacity_bits(kmax, plan->kbits) : 0.0;
  info->S = plan->H.S;
  info->S_frac = plan->H.T;
  info->workspace_bytes = plan->ws_bytes;
  return OBFFT_SUCCESS;
}

extern "C" size_t obfft_workspace_size(obfft_plan_t plan) { return plan ? plan->ws_bytes : 0; }

extern "C" obfft_status_t obfft_set_workspace(obfft_plan_t plan, void* ptr, size_t bytes) {
  if (!plan || !ptr || bytes < plan->ws_bytes) return fail(plan, OBFFT_INVALID_VALUE);
  if (plan->ws_owned && plan->ws) hipFree(plan->ws);
  plan->ws = ptr;
  plan->ws_owned = false;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_plan_roots(obfft_plan_t plan, int axis, int64_t* host_out) {
  if (!plan || !host_out || axis < 0 || axis > 2) return fail(plan, OBFFT_INVALID_VALUE);
  memcpy(host_out, plan->roots[axis].data(), plan->roots[axis].size() * sizeof(int64_t));
  return OBFFT_SUCCESS;
}

static obfft_status_t ensure_ws(obfft_plan_t plan) {
  if (plan->ws) return OBFFT_SUCCESS;
  if (hipMalloc(&plan->ws, plan->ws_bytes) != hipSuccess) {
    plan->ws = nullptr;
    return OBFFT_ALLOC_FAILED;
  }
  plan->ws_owned = true;
  return OBFFT_SUCCESS;
}

static bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x != y && x < y + bytes && y < x + bytes;
}

// n / d = mulhi(n, magic) >> shift for every n < 2^31 (magic = ceil(2^(31+l) / d),
// l = ceil(log2 d), shift = l - 1; magic 0 encodes d = 1).
static void div_magic(int64_t d, uint32_t* magic, uint32_t* shift) {
  if (d <= 1) {
    *magic = 0;
    *shift = 0;
    return;
  }
  int l = 0;
  while (((int64_t)1 << l) < d) l++;
  unsigned __int128 num = (unsigned __int128)1 << (31 + l);
  *magic = (uint32_t)((num + (unsigned __int128)d - 1) / (unsigned __int128)d);
  *shift = (uint32_t)(l - 1);
}

// The stage kernel's grid for `tiles` tiles: a 1-, 2- or 3-D shape that spells
// out (column tile, group) without divisions when every extent fits.
// Groups of one column tile run back to back on one XCD (stage 2 of the
// contiguous axis): their partial output lines merge in that XCD's L2.
static const int kGroupBlock = 8;
static const int kMaxClaim = 256;   // items per claim of the persistent batched launch

static dim3 stage_grid(StageParams& P, int64_t tiles) {
  const int64_t kMaxYZ = 65535;
  if (P.stage == 1) {
    if (tiles < kMaxTiles) {
      P.grid_mode = 1;
      return dim3((unsigned)tiles);
    }
  } else if (!P.g_minor) {
    if (P.tiles_per_g < kMaxTiles && P.G <= kMaxYZ) {
      P.grid_mode = 2;
      return dim3((unsigned)P.tiles_per_g, (unsigned)P.G);
    }
  } else {
    const int64_t T = P.tiles_per_g, G = P.G, GB = P.gblock;
    if ((T & 7) == 0 && T / 8 <= kMaxYZ && G / GB <= kMaxYZ) {
      P.grid_mode = 3;
      return dim3((unsigned)(8 * GB), (unsigned)(T / 8), (unsigned)(G / GB));
    }
    if ((T & 7) != 0 && T <= kMaxYZ && G / GB <= kMaxYZ) {
      P.grid_mode = 4;
      return dim3((unsigned)GB, (unsigned)T, (unsigned)(G / GB));
    }
  }
  P.grid_mode = 0;
  return dim3((unsigned)tiles);
}

static void stage_params(obfft_plan_t plan, int axis, int stage, int direction, const void* in, void* out,
                         StageParams& P, int64_t& grid) {
  memset(&P, 0, sizeof(P));
  int64_t N = plan->n[axis];
  int64_t inner = 1, outer = 1;
  for (int b = axis + 1; b < 3; b++) inner *= plan->n[b];
  for (int b = 0; b < axis; b++) outer *= plan->n[b];
  int64_t p = plan->p[axis], q = plan->q[axis];
  P.in = in;
  P.out = out;
  P.inner = inner;
  P.N = N;
  P.s_o = N * inner;
  P.stage = stage;
  const OperandPlanes& L = plan->planes[axis][stage - 1][direction].L;
  P.amat = L.dev;
  P.amat128 = L.dev128;
  P.amat_g_stride = stage == 1 ? 0 : L.g_stride;
  P.amat_mod_stride = L.mod_stride;
  P.amat_fmax = L.fmax;
  P.amat_chmax = L.chmax;
  P.amat_mt = L.mt;
  P.amat_bytes = (int64_t)std::max(L.G, 1) * L.g_stride;
  P.phaseA = plan->d_phaseA;
  div_magic(inner, &P.inner_magic, &P.inner_shift);
  div_magic(stage == 1 ? p : q, &P.G_magic, &P.G_shift);
  P.mc = plan->d_mc;
  P.crt = plan->d_crt;
  P.nf_flag = plan->d_flags;
  P.fp8_full = plan->fp8_full;
  if (stage == 1) {
    P.K = (int)q;
    P.G = (int)p;
    P.ncols = outer * p * inner;
    P.s_in_g = inner;
    P.s_in_s = p * inner;
    P.s_out_g = inner;
    P.s_out_t = p * inner;
    int ncw = stage_cols_per_wg(P.K, plan->substrate);
    grid = (P.ncols + ncw - 1) / ncw;
  } else {
    P.K = (int)p;
    P.G = (int)q;
    P.ncols = outer * inner;
    P.s_in_g = p * inner;
    P.s_in_s = inner;
    P.s_out_g = inner;
    P.s_out_t = q * inner;
    int ncw = stage_cols_per_wg(P.K, plan->substrate);
    P.tiles_per_g = (int)((P.ncols + ncw - 1) / ncw);
    P.g_minor = inner == 1;
    const int gb = plan->group_block > 0 && q % plan->group_block == 0 ? plan->group_block : kGroupBlock;
    P.gblock = (q % gb) == 0 ? gb : (int)q;
    grid = (int64_t)P.tiles_per_g * q;
  }
}

// dbg / tap: the debug kernels' residue tap and the epilogue records of line
// tap_line (either may be null; both null selects the production kernel).
static obfft_status_t run_stage(obfft_plan_t plan, int axis, int stage, int direction, const void* in,
                                void* out, int extra_shift, uint16_t* dbg, hipStream_t st,
                                uint32_t* tap = nullptr, int64_t tap_line = -1) {
  StageParams P;
  int64_t tiles;
  stage_params(plan, axis, stage, direction, in, out, P, tiles);
  const dim3 grid = stage_grid(P, tiles);
  P.extra_shift = extra_shift;
  P.dbg_res = dbg;
  P.dbg_tap = tap;
  P.dbg_line = tap_line;
  if (tiles <= 0) return OBFFT_SUCCESS;
  const bool h0 = plan->reduction == OBFFT_RED_H0;
  const hipError_t e = (dbg || tap) ? launch_stage_tap(plan->substrate, plan->precision, h0, P, grid, st)
                                    : launch_stage(plan->substrate, plan->precision, h0, P, grid, st);
  return e == hipSuccess ? OBFFT_SUCCESS : OBFFT_HIP_ERROR;
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// ws: the Y' workspace to use instead of the plan's (null: the plan's,
// allocated on first use).
static obfft_status_t run_transform(obfft_plan_t plan, const void* in, void* out, int direction,
                                    bool normalise, void* stream, void* ws = nullptr) {
  if (!in || !out) return OBFFT_INVALID_VALUE;
  int64_t total = plan->n[0] * plan->n[1] * plan->n[2];
  size_t bytes = (size_t)total * (plan->precision ? 8 : 16);
  if (overlaps(in, out, bytes)) return OBFFT_INVALID_VALUE;
  obfft_status_t s = OBFFT_SUCCESS;
  if (!ws) {
    s = ensure_ws(plan);
    if (s != OBFFT_SUCCESS) return s;
    ws = plan->ws;
  }
  hipStream_t st = (hipStream_t)stream;
  int shift = 0;
  bool post_scale = false;
  if (normalise) {
    if (is_pow2(total)) {
      int l = 0;
      while (((int64_t)1 << l) < total) l++;
      shift = -l;
    } else {
      post_scale = true;
    }
  }
  const void* cur = in;
  for (int k = 0; k < 3; k++) {
    int a = plan->order[k];
    s = run_stage(plan, a, 1, direction, cur, ws, 0, nullptr, st);
    if (s != OBFFT_SUCCESS) return s;
    s = run_stage(plan, a, 2, direction, ws, out, k == 2 ? shift : 0, nullptr, st);
    if (s != OBFFT_SUCCESS) return s;
    cur = out;
  }
  if (post_scale) {
    if (launch_scale(out, 2 * total, 1.0 / (double)total, plan->precision, st) != hipSuccess)
      return OBFFT_HIP_ERROR;
  }
  return OBFFT_SUCCESS;
}

#define CHECK_PLAN(prec)                                   \
  if (!plan) return OBFFT_INVALID_VALUE;                   \
  if (plan->batch_count) return fail(plan, OBFFT_INVALID_VALUE); \
  if (plan->precision != (prec)) return fail(plan, OBFFT_WRONG_PRECISION);

extern "C" obfft_status_t fft3d_z2z_forward(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP64);
  return fail(plan, run_transform(plan, in, out, 0, false, stream));
}
// ---- forward transform without any allocation ----
//
// The Y' workspace between the two stages of each axis lives in a file-scope
// device array.  Each device that runs the library holds its own copy (at
// its own address) from module load until the process ends; host code uses
// only the address hipGetSymbolAddress returns for the current device, never
// the array's name, which on the host is a stand-in and not a device address.
// Every call on one device shares that device's array; the workspace is
// written in full by stage 1 before stage 2 reads it, so nothing has to be
// cleared between calls, but calls that overlap in time on one device race.
static constexpr size_t kScratchBytes = (size_t)256 << 20;  // 2^24 complex128 elements, e.g. 256^3
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices];

static obfft_status_t scratch_for_current_device(void** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OBFFT_HIP_ERROR;
  if (dev < 0 || dev >= kScratchDevices) return OBFFT_UNSUPPORTED_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OBFFT_HIP_ERROR;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return OBFFT_SUCCESS;
}

extern "C" size_t obfft_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" obfft_status_t fft3d_z2z_forward_noalloc(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP64);
  if (plan->ws_bytes > kScratchBytes) return fail(plan, OBFFT_SCRATCH_EXCEEDED);
  void* ws = nullptr;
  const obfft_status_t s = scratch_for_current_device(&ws);
  if (s != OBFFT_SUCCESS) return fail(plan, s);
  return fail(plan, run_transform(plan, in, out, 0, false, stream, ws));
}

extern "C" obfft_status_t fft3d_z2z_inverse(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP64);
  return fail(plan, run_transform(plan, in, out, 1, true, stream));
}
extern "C" obfft_status_t fft3d_z2z_adjoint(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP64);
  return fail(plan, run_transform(plan, in, out, 1, false, stream));
}
extern "C" obfft_status_t fft3d_c2c_forward(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP32);
  return fail(plan, run_transform(plan, in, out, 0, false, stream));
}
extern "C" obfft_status_t fft3d_c2c_inverse(obfft_plan_t plan, const void* in, void* out, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP32);
  return fail(plan, run_transform(plan, in, out, 1, true, stream));
}

static obfft_status_t run_native(obfft_plan_t plan, const void* in, void* out, int inverse, void* stream) {
  CHECK_PLAN(OBFFT_PREC_FP64);
  if (!plan->native) return fail(plan, OBFFT_UNSUPPORTED_SIZE);
  if (!in || !out) return fail(plan, OBFFT_INVALID_VALUE);
  int64_t total = plan->n[0] * plan->n[1] * plan->n[2];
  if (overlaps(in, out, (size_t)total * 16)) return fail(plan, OBFFT_INVALID_VALUE);
  obfft_status_t s = ensure_ws(plan);
  if (s != OBFFT_SUCCESS) return fail(plan, s);
  if (native_execute(plan->native, in, out, plan->ws, inverse, (hipStream_t)stream) != hipSuccess)
    return fail(plan, OBFFT_HIP_ERROR);
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t fft3d_z2z_native_forward(obfft_plan_t plan, const void* in, void* out, void* stream) {
  return run_native(plan, in, out, 0, stream);
}
extern "C" obfft_status_t fft3d_z2z_native_inverse(obfft_plan_t plan, const void* in, void* out, void* stream) {
  return run_native(plan, in, out, 1, stream);
}

extern "C" obfft_status_t obfft_stage(obfft_plan_t plan, int axis, int stage, int direction, const void* in,
                                      void* out, void* residues_out, void* stream) {
  if (!plan || plan->batch_count) return OBFFT_INVALID_VALUE;
  if (axis < 0 || axis > 2 || (stage != 1 && stage != 2) || (direction != 0 && direction != 1) || !in ||
      !out || in == out)
    return fail(plan, OBFFT_INVALID_VALUE);
  return fail(plan, run_stage(plan, axis, stage, direction, in, out, 0, (uint16_t*)residues_out,
                              (hipStream_t)stream));
}

static uint32_t float_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, sizeof(u));
  return u;
}

// Epilogue records of one line of one stage (debug entry point): runs the
// debug variant of the stage kernel, copies the raw records of the line to the
// host and turns the seeded bit patterns into the values they encode.
extern "C" obfft_status_t obfft_debug_tap(obfft_plan_t plan, int axis, int stage, int direction, int64_t line,
                                          const void* in, void* out, void* host_dump, void* stream) {
  if (!plan || plan->batch_count) return OBFFT_INVALID_VALUE;
  if (axis < 0 || axis > 2 || (stage != 1 && stage != 2) || (direction != 0 && direction != 1) || !in ||
      !out || in == out || !host_dump)
    return fail(plan, OBFFT_INVALID_VALUE);
  const int64_t N = plan->n[axis], total = plan->n[0] * plan->n[1] * plan->n[2];
  if (line < 0 || line >= total / N) return fail(plan, OBFFT_INVALID_VALUE);
  const size_t bytes = (size_t)N * 2 * kTapRecWords * sizeof(uint32_t);
  uint32_t* d_tap = nullptr;
  if (hipMalloc(&d_tap, bytes) != hipSuccess) return fail(plan, OBFFT_ALLOC_FAILED);
  hipStream_t st = (hipStream_t)stream;
  std::vector<uint32_t> raw((size_t)N * 2 * kTapRecWords);
  obfft_status_t s = OBFFT_SUCCESS;
  if (hipMemsetAsync(d_tap, 0xFF, bytes, st) != hipSuccess) s = OBFFT_HIP_ERROR;
  if (s == OBFFT_SUCCESS) s = run_stage(plan, axis, stage, direction, in, out, 0, nullptr, st, d_tap, line);
  if (s == OBFFT_SUCCESS &&
      (hipMemcpyAsync(raw.data(), d_tap, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    s = OBFFT_HIP_ERROR;
  (void)hipFree(d_tap);
  if (s != OBFFT_SUCCESS) return fail(plan, s);
  const CrtConsts& C = plan->C;
  const int NW = C.nwords, VP = (C.S + 1) / 2;
  const int wbits = 32 * NW;
  const unsigned __int128 mask = NW == 4 ? ~(unsigned __int128)0 : (((unsigned __int128)1 << wbits) - 1);
  unsigned __int128 M = 0;
  for (int i = 0; i < NW; i++) M |= (unsigned __int128)C.M[i] << (32 * i);
  uint32_t* dump = (uint32_t*)host_dump;
  for (int64_t rcd = 0; rcd < 2 * N; rcd++) {
    const uint32_t* t = &raw[(size_t)rcd * kTapRecWords];
    uint32_t* o = dump + (size_t)rcd * kTapRecWords;
    memset(o, 0, kTapRecWords * sizeof(uint32_t));
    for (int q = 0; q < C.S; q++) o[kTapRecP + q] = t[kTapRecP + q] - float_bits(C.seed_c[q]);
    for (int q = 0; q < C.T; q++) o[kTapRecZ + q] = t[kTapRecZ + q] - float_bits(C.seed_c[2 * VP + q]);
    // E = W - zoff M (mod 2^(32 NW)): the kernel's accumulator holds only the
    // low 32 NW bits of E (R = E - zhat M is all it needs, |R| < 2^113)
    unsigned __int128 W = 0, Rv = 0;
    for (int i = 0; i < NW; i++) {
      W |= (unsigned __int128)t[kTapRecW + i] << (32 * i);
      Rv |= (unsigned __int128)t[kTapRecR + i] << (32 * i);
    }
    unsigned __int128 E = (W - (unsigned __int128)C.zoff * M) & mask;
    const bool rneg = (Rv >> (wbits - 1)) & 1;
    for (int i = 0; i < 5; i++) o[kTapRecW + i] = i < NW ? (uint32_t)(E >> (32 * i)) : 0u;
    for (int i = 0; i < 4; i++) o[kTapRecR + i] = i < NW ? (uint32_t)(Rv >> (32 * i)) : (rneg ? ~0u : 0u);
    o[kTapRecZhat] = t[kTapRecZhat] - C.zoff;
    o[kTapRecExp] = t[kTapRecExp];
    o[kTapRecY] = t[kTapRecY];
    o[kTapRecY + 1] = plan->precision == OBFFT_PREC_FP64 ? t[kTapRecY + 1] : 0u;
    for (int k = 0; k < C.r; k++) o[kTapRecRes + k] = t[kTapRecRes + k];
  }
  return OBFFT_SUCCESS;
}

// ---- unit-level CRT reconstruction (cached constants per precision) ----
struct CrtCache {
  bool ready = false;
  CrtConsts C;
  uint16_t* d_phaseA = nullptr;
  CrtConsts* d_C = nullptr;
  int8_t* d_phaseA_i8 = nullptr;  // INT8 Phase-A operand (64 lanes x 16 bytes)
  CrtAltConsts* d_i8 = nullptr;
};
static std::mutex g_crt_mu;
static std::map<std::pair<int, int>, CrtCache> g_crt;

// Constants of the standalone reconstruction for one precision on the
// current device, built on first use.
static obfft_status_t crt_cache(int precision, CrtCache** out) {
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_crt_mu);
  CrtCache* cc = &g_crt[std::make_pair(dev, precision)];
  if (!cc->ready) {
    ModSet H;
    std::string err;
    if (!build_modset(precision ? kModFP32 : kModFP64, precision ? 6 : 12, H, err)) return OBFFT_INVALID_VALUE;
    build_crt_consts(H, cc->C);
    std::vector<uint16_t> pa;
    int npairs = 0;
    build_phaseA_operand(H, pa, &npairs);
    if (!cc->d_phaseA && hipMalloc(&cc->d_phaseA, pa.size() * 2) != hipSuccess) return OBFFT_ALLOC_FAILED;
    if (hipMemcpy(cc->d_phaseA, pa.data(), pa.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
      return OBFFT_HIP_ERROR;
    if (!cc->d_C && hipMalloc(&cc->d_C, sizeof(CrtConsts)) != hipSuccess) return OBFFT_ALLOC_FAILED;
    if (hipMemcpy(cc->d_C, &cc->C, sizeof(CrtConsts), hipMemcpyHostToDevice) != hipSuccess)
      return OBFFT_HIP_ERROR;
    CrtAltConsts K;
    std::vector<int8_t> a8;
    build_crt_alt(H, cc->C, K, a8);
    if (!cc->d_phaseA_i8 && hipMalloc(&cc->d_phaseA_i8, a8.size()) != hipSuccess) return OBFFT_ALLOC_FAILED;
    if (hipMemcpy(cc->d_phaseA_i8, a8.data(), a8.size(), hipMemcpyHostToDevice) != hipSuccess)
      return OBFFT_HIP_ERROR;
    if (!cc->d_i8 && hipMalloc(&cc->d_i8, sizeof(CrtAltConsts)) != hipSuccess) return OBFFT_ALLOC_FAILED;
    if (hipMemcpy(cc->d_i8, &K, sizeof(CrtAltConsts), hipMemcpyHostToDevice) != hipSuccess)
      return OBFFT_HIP_ERROR;
    cc->ready = true;
  }
  *out = cc;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_crt_reconstruct(int precision, int64_t n, const void* residues, const void* exps,
                                                void* out, void* taps, void* stream) {
  if ((precision != 0 && precision != 1) || n < 0 || (n > 0 && (!residues || !exps || !out)))
    return OBFFT_INVALID_VALUE;
  if (n >= ((int64_t)1 << 31)) return OBFFT_UNSUPPORTED_SIZE;
  if (n == 0) return OBFFT_SUCCESS;
  if (!device_is_gfx950()) return OBFFT_UNSUPPORTED_DEVICE;
  CrtCache* cc = nullptr;
  obfft_status_t st = crt_cache(precision, &cc);
  if (st != OBFFT_SUCCESS) return st;
  if (launch_crt(precision, n, (const uint16_t*)residues, (const int*)exps, out, (uint32_t*)taps, cc->d_phaseA,
                 cc->d_C, (hipStream_t)stream) != hipSuccess)
    return OBFFT_HIP_ERROR;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_crt_reconstruct_method(int precision, int method, int64_t n, const void* residues,
                                                       const void* exps, void* out, void* stream) {
  if ((precision != 0 && precision != 1) || method < OBFFT_CRT_KULISCH || method > OBFFT_CRT_KULISCH_INT16 ||
      n < 0 || (n > 0 && (!residues || !exps || !out)))
    return OBFFT_INVALID_VALUE;
  if (n >= ((int64_t)1 << 31)) return OBFFT_UNSUPPORTED_SIZE;
  if (method == OBFFT_CRT_KULISCH) return obfft_crt_reconstruct(precision, n, residues, exps, out, nullptr, stream);
  if (n == 0) return OBFFT_SUCCESS;
  if (!device_is_gfx950()) return OBFFT_UNSUPPORTED_DEVICE;
  CrtCache* cc = nullptr;
  obfft_status_t st = crt_cache(precision, &cc);
  if (st != OBFFT_SUCCESS) return st;
  if (launch_crt_ablation(precision, method, n, (const uint16_t*)residues, (const int*)exps, out, cc->d_phaseA,
                          cc->d_C, cc->d_phaseA_i8, cc->d_i8, (hipStream_t)stream) != hipSuccess)
    return OBFFT_HIP_ERROR;
  return OBFFT_SUCCESS;
}

extern "C" void obfft_taps_layout(obfft_taps_layout_t* t) {
  if (!t) return;
  t->P = 0;
  t->Z = 16;
  t->E = 24;
  t->n_E = 5;
  t->zhat = 29;
  t->R = 30;
  t->n_R = 4;
  t->stride = kTapStride;
}

// Runs one MFMA (or lane-swap / conversion) probe on device buffers; used by
// the hardware-contract tests.  kind: 0 fp8 16x16x32, 1 i8 16x16x64,
// 2 f16 32x32x16, 3 permlane32 swap, 4 E4M3 conversion, 5 f16 16x16x32.
extern "C" obfft_status_t obfft_mfma_probe(int kind, const void* a, const void* b, void* d, void* stream) {
  if (kind < 0 || kind > 7 || !a || !d || (kind != 4 && !b)) return OBFFT_INVALID_VALUE;
  if (!device_is_gfx950()) return OBFFT_UNSUPPORTED_DEVICE;
  return launch_mfma_probe(kind, a, b, d, (hipStream_t)stream) == hipSuccess ? OBFFT_SUCCESS : OBFFT_HIP_ERROR;
}

// ---- batched transforms ----
//
// All member transforms of a batch run pass by pass (axis n3 stage 1, n3
// stage 2, n2 ..., n1 stage 2).  In every pass the members are grouped by the
// contraction length K of their stage (K <= 4, 8, 12, 16, 32: the kernel's
// compile-time tile shape), and each group is ONE launch over the tiles of
// all its members (a workgroup per tile), driven by a device table of stage
// descriptors.  The launches are captured once in a hipGraph and replayed;
// only the table (with the callers' pointers) is re-uploaded per call.
static const int kPassStage[6] = {1, 2, 1, 2, 1, 2};

// opts: one options struct for every member (per_member == 0) or an array of
// `count` (per_member == 1).
static obfft_status_t batch_plan_create(obfft_plan_t* out, int count, const int64_t* shapes,
                                        const obfft_options_t* opts, int per_member) {
  if (!out || count <= 0 || count > 65535 || !shapes) return OBFFT_INVALID_VALUE;
  *out = nullptr;
  obfft_options_t def;
  obfft_options_default(&def);
  if (!opts) {
    opts = &def;
    per_member = 0;
  }
  for (int i = 0; i < (per_member ? count : 1); i++)
    if (opts[i].precision != OBFFT_PREC_FP64 || opts[i].reduction != OBFFT_RED_RECIPROCAL ||
        opts[i].substrate != opts[0].substrate || opts[i].n_moduli_override || opts[i].moduli_override)
      return OBFFT_INVALID_VALUE;
  obfft_plan_t bp = new (std::nothrow) obfft_plan_s();
  if (!bp) return OBFFT_ALLOC_FAILED;
  bp->batch_count = count;
  // members share planes when their shapes and options coincide: plan each
  // distinct (shape, factorisation, axis order, tile order) once
  typedef std::tuple<int64_t, int64_t, int64_t, std::vector<int>> Key;
  std::map<Key, obfft_plan_t> uniq;
  std::vector<obfft_plan_t> per(count);
  for (int i = 0; i < count; i++) {
    const obfft_options_t* opt = per_member ? &opts[i] : opts;
    std::vector<int> ok = {opt->p[0], opt->p[1], opt->p[2], opt->q[0], opt->q[1], opt->q[2],
                           opt->axis_order[0], opt->axis_order[1], opt->axis_order[2], opt->group_block};
    Key key = std::make_tuple(shapes[3 * i], shapes[3 * i + 1], shapes[3 * i + 2], ok);
    auto it = uniq.find(key);
    if (it == uniq.end()) {
      obfft_plan_t m = nullptr;
      obfft_status_t s = obfft_plan_create(&m, shapes[3 * i], shapes[3 * i + 1], shapes[3 * i + 2], opt);
      if (s != OBFFT_SUCCESS) {
        obfft_plan_destroy(bp);
        return s;
      }
      bp->members.push_back(m);
      it = uniq.emplace(key, m).first;
    }
    per[i] = it->second;
  }
  for (int i = 1; i < count; i++)
    if (per[i]->substrate != per[0]->substrate) {
      obfft_plan_destroy(bp);
      return OBFFT_INVALID_VALUE;
    }
  bp->substrate = per[0]->substrate;
  bp->precision = OBFFT_PREC_FP64;
  for (int k = 0; k < 3; k++) bp->order[k] = per[0]->order[k];
  {
    const uint32_t zero_flags[64] = {};
    void* dfl = nullptr;
    if (upload(bp, zero_flags, sizeof(zero_flags), &dfl) != OBFFT_SUCCESS) {
      obfft_plan_destroy(bp);
      return OBFFT_ALLOC_FAILED;
    }
    bp->d_flags = (uint32_t*)dfl;
  }
  bp->MC = per[0]->MC;
  bp->C = per[0]->C;
  // workspace offsets (256-byte aligned)
  size_t off = 0;
  bp->ws_off.resize(count);
  for (int i = 0; i < count; i++) {
    bp->ws_off[i] = off;
    off += (per[i]->ws_bytes + 255) & ~(size_t)255;
  }
  bp->ws_bytes = off;
  // descriptors without pointers; per pass and K class, the members' tiles
  size_t dbytes = sizeof(StageParams) * 6 * count;
  if (hipHostMalloc((void**)&bp->h_desc, dbytes, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&bp->d_desc, dbytes) != hipSuccess ||
      hipMalloc((void**)&bp->d_first, sizeof(int64_t) * 6 * count) != hipSuccess) {
    obfft_plan_destroy(bp);
    return OBFFT_ALLOC_FAILED;
  }
  std::vector<int64_t> first(6 * count), tiles(6 * count);
  std::vector<int> cls(6 * count);
  for (int pass = 0; pass < 6; pass++) {
    for (int i = 0; i < count; i++) {
      StageParams& P = bp->h_desc[pass * count + i];
      int64_t grid;
      stage_params(per[i], per[i]->order[pass / 2], kPassStage[pass], 0, nullptr, nullptr, P, grid);
      P.nf_flag = bp->d_flags;
      cls[pass * count + i] = kclass_of(P.K);
      tiles[pass * count + i] = grid;  // the single-transform tiling is the class's
    }
    for (int c = 0; c < 5; c++) {
      int64_t acc = 0;
      int full = 1;
      for (int i = 0; i < count; i++) {
        if (cls[pass * count + i] != c) continue;
        first[pass * count + i] = acc;
        acc += tiles[pass * count + i];
        full &= bp->h_desc[pass * count + i].K == kclass_kmax(c) &&
                (bp->substrate != SUB_FP8 || (bp->h_desc[pass * count + i].fp8_full && bp->h_desc[pass * count + i].amat128));
      }
      bp->batch_full[pass][c] = full;
      bp->batch_total[pass][c] = acc;
      if (acc >= kMaxTiles) {
        obfft_plan_destroy(bp);
        return OBFFT_UNSUPPORTED_SIZE;
      }
    }
  }
  int64_t ttot = 0;
  for (int pass = 0; pass < 6; pass++)
    for (int c = 0; c < 5; c++) {
      bp->tmember_off[pass][c] = ttot;
      ttot += bp->batch_total[pass][c];
    }
  std::vector<uint16_t> tm((size_t)std::max<int64_t>(ttot, 1));
  for (int pass = 0; pass < 6; pass++)
    for (int i = 0; i < count; i++) {
      int64_t base = bp->tmember_off[pass][cls[pass * count + i]] + first[pass * count + i];
      for (int64_t t = 0; t < tiles[pass * count + i]; t++) tm[base + t] = (uint16_t)i;
    }
  if (hipMalloc((void**)&bp->d_tmember, tm.size() * sizeof(uint16_t)) != hipSuccess) {
    obfft_plan_destroy(bp);
    return OBFFT_ALLOC_FAILED;
  }
  if (hipMemcpy(bp->d_first, first.data(), sizeof(int64_t) * first.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bp->d_tmember, tm.data(), tm.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreateWithFlags(&bp->desc_done, hipEventDisableTiming) != hipSuccess) {
    obfft_plan_destroy(bp);
    return OBFFT_HIP_ERROR;
  }
  bp->members_of_batch = per;
  // segments of the persistent launch: (pass, member) pass-major, each
  // depending on the same member's previous pass
  if (bp->substrate == SUB_FP16) {
    const int nseg = 6 * count;
    std::vector<int64_t> seg_start(nseg + 1, 0);
    std::vector<int> seg_dep(nseg), seg_cls(nseg);
    unsigned mask = 0;
    for (int sg = 0; sg < nseg; sg++) {
      seg_start[sg + 1] = seg_start[sg] + tiles[sg];
      seg_dep[sg] = sg >= count ? sg - count : -1;
      seg_cls[sg] = persist_variant(bp->h_desc[sg].K);
      mask |= 1u << seg_cls[sg];
    }
    bp->persist_nseg = nseg;
    bp->persist_items = seg_start[nseg];
    bp->persist_lds = persist_lds_bytes(mask);
    bp->persist_mask = mask;
    bp->persist_grid_size = persist_grid(mask, bp->persist_lds);
    // claim size: about four chunks per workgroup over the batch, at most 64
    // items (one publication, i.e. one L2 write-back, per chunk and segment)
    bp->persist_claim = (int)std::max<int64_t>(
        1, std::min<int64_t>(64, seg_start[nseg] / (4 * (int64_t)std::max(bp->persist_grid_size, 1))));
    if (bp->persist_grid_size <= 0 ||
        seg_start[nseg] >= ((int64_t)1 << 32) - (int64_t)bp->persist_grid_size * kMaxClaim) {
      obfft_plan_destroy(bp);
      return OBFFT_HIP_ERROR;
    }
    if (hipMalloc((void**)&bp->d_seg_start, sizeof(int64_t) * (nseg + 1)) != hipSuccess ||
        hipMalloc((void**)&bp->d_seg_dep, sizeof(int) * nseg) != hipSuccess ||
        hipMalloc((void**)&bp->d_seg_cls, sizeof(int) * nseg) != hipSuccess ||
        hipMalloc((void**)&bp->d_ctl, sizeof(uint32_t) * (2 + nseg)) != hipSuccess ||
        hipMalloc((void**)&bp->d_persist, sizeof(PersistParams)) != hipSuccess) {
      obfft_plan_destroy(bp);
      return OBFFT_ALLOC_FAILED;
    }
    PersistParams Q;
    memset(&Q, 0, sizeof(Q));
    Q.descs = bp->d_desc;
    Q.seg_start = bp->d_seg_start;
    Q.seg_dep = bp->d_seg_dep;
    Q.seg_cls = bp->d_seg_cls;
    Q.nseg = nseg;
    Q.spin_limit = bp->persist_spin;
    Q.claim = bp->persist_claim;
    Q.total = seg_start[nseg];
    Q.ctl = bp->d_ctl;
    Q.flags = bp->d_flags;
    if (hipMemcpy(bp->d_seg_start, seg_start.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(bp->d_seg_dep, seg_dep.data(), sizeof(int) * nseg, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bp->d_seg_cls, seg_cls.data(), sizeof(int) * nseg, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bp->d_persist, &Q, sizeof(Q), hipMemcpyHostToDevice) != hipSuccess) {
      obfft_plan_destroy(bp);
      return OBFFT_HIP_ERROR;
    }
    bp->persist_ok = 1;
  }
  *out = bp;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_batch_plan_create(obfft_plan_t* out, int count, const int64_t* shapes,
                                                  const obfft_options_t* opt) {
  return batch_plan_create(out, count, shapes, opt, 0);
}

extern "C" obfft_status_t obfft_batch_plan_create_each(obfft_plan_t* out, int count, const int64_t* shapes,
                                                       const obfft_options_t* opts) {
  if (!opts) return OBFFT_INVALID_VALUE;
  return batch_plan_create(out, count, shapes, opts, 1);
}

static obfft_status_t batch_launch_passes(obfft_plan_t bp, hipStream_t st) {
  int count = bp->batch_count;
  if (bp->batch_mode == OBFFT_BATCH_PERSISTENT)
    return launch_persist(bp->persist_mask, bp->d_persist, bp->d_ctl, 2 + bp->persist_nseg, bp->persist_grid_size, bp->persist_lds,
                          st) == hipSuccess
               ? OBFFT_SUCCESS
               : OBFFT_HIP_ERROR;
  for (int pass = 0; pass < 6; pass++)
    for (int c = 0; c < 5; c++) {
      int64_t total = bp->batch_total[pass][c];
      if (total <= 0) continue;
      if (launch_batch(bp->substrate, kclass_kmax(c), bp->batch_full[pass][c] != 0, bp->d_desc + pass * count,
                       bp->d_first + pass * count,
                       bp->d_tmember + bp->tmember_off[pass][c], total, st) != hipSuccess)
        return OBFFT_HIP_ERROR;
    }
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_batch_forward(obfft_plan_t plan, const void* const* ins, void* const* outs,
                                              void* stream) {
  if (!plan || !plan->batch_count || !ins || !outs) return OBFFT_INVALID_VALUE;
  int count = plan->batch_count;
  hipStream_t st = (hipStream_t)stream;
  if (!plan->batch_ws) {
    if (hipMalloc(&plan->batch_ws, std::max<size_t>(plan->ws_bytes, 256)) != hipSuccess)
      return fail(plan, OBFFT_ALLOC_FAILED);
  }
  // the previous call's upload must have left the pinned staging buffer
  if (hipEventSynchronize(plan->desc_done) != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
  for (int i = 0; i < count; i++) {
    obfft_plan_t m = plan->members_of_batch[i];
    size_t bytes = (size_t)(m->n[0] * m->n[1] * m->n[2]) * 16;
    if (!ins[i] || !outs[i] || overlaps(ins[i], outs[i], bytes)) return fail(plan, OBFFT_INVALID_VALUE);
    void* ws = (char*)plan->batch_ws + plan->ws_off[i];
    const void* cur = ins[i];
    for (int pass = 0; pass < 6; pass++) {
      StageParams& P = plan->h_desc[pass * count + i];
      bool s1 = kPassStage[pass] == 1;
      P.in = s1 ? cur : ws;
      P.out = s1 ? ws : outs[i];
      if (!s1) cur = outs[i];
    }
  }
  if (hipMemcpyAsync(plan->d_desc, plan->h_desc, sizeof(StageParams) * 6 * count, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipEventRecord(plan->desc_done, st) != hipSuccess)
    return fail(plan, OBFFT_HIP_ERROR);
  if (!plan->use_graph) return fail(plan, batch_launch_passes(plan, st));
  if (!plan->graph_exec) {
    if (!plan->capture_stream && hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(plan, OBFFT_HIP_ERROR);
    if (hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(plan, OBFFT_HIP_ERROR);
    obfft_status_t s = batch_launch_passes(plan, plan->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(plan->capture_stream, &g);
    if (s != OBFFT_SUCCESS || e != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
    plan->graph = g;
    if (hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0) != hipSuccess)
      return fail(plan, OBFFT_HIP_ERROR);
  }
  if (hipGraphLaunch(plan->graph_exec, st) != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
  return OBFFT_SUCCESS;
}

static void drop_graph(obfft_plan_t plan) {
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->graph_exec = nullptr;
  plan->graph = nullptr;
}

// Selects graph replay (1, default) or direct launches (0) for a batch plan.
extern "C" obfft_status_t obfft_batch_set_graph(obfft_plan_t plan, int use_graph) {
  if (!plan || !plan->batch_count) return OBFFT_INVALID_VALUE;
  plan->use_graph = use_graph != 0;
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_batch_set_mode(obfft_plan_t plan, int mode) {
  if (!plan || !plan->batch_count) return OBFFT_INVALID_VALUE;
  if (mode != OBFFT_BATCH_PASSES && mode != OBFFT_BATCH_PERSISTENT) return fail(plan, OBFFT_INVALID_VALUE);
  if (mode == OBFFT_BATCH_PERSISTENT && !plan->persist_ok) return fail(plan, OBFFT_INVALID_VALUE);
  if (mode != plan->batch_mode) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
    drop_graph(plan);
    plan->batch_mode = mode;
  }
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_batch_set_poll_limit(obfft_plan_t plan, int polls) {
  if (!plan || !plan->batch_count || polls < 0) return OBFFT_INVALID_VALUE;
  if (!plan->persist_ok) return fail(plan, OBFFT_INVALID_VALUE);
  if (hipDeviceSynchronize() != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
  plan->persist_spin = polls;
  const size_t off = offsetof(PersistParams, spin_limit);
  if (hipMemcpy((char*)plan->d_persist + off, &polls, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return fail(plan, OBFFT_HIP_ERROR);
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_batch_set_claim(obfft_plan_t plan, int items) {
  if (!plan || !plan->batch_count || items < 1 || items > kMaxClaim) return OBFFT_INVALID_VALUE;
  if (!plan->persist_ok) return fail(plan, OBFFT_INVALID_VALUE);
  if (hipDeviceSynchronize() != hipSuccess) return fail(plan, OBFFT_HIP_ERROR);
  plan->persist_claim = items;
  const size_t off = offsetof(PersistParams, claim);
  if (hipMemcpy((char*)plan->d_persist + off, &items, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return fail(plan, OBFFT_HIP_ERROR);
  return OBFFT_SUCCESS;
}

extern "C" int obfft_batch_get_claim(obfft_plan_t plan) {
  return plan && plan->batch_count && plan->persist_ok ? plan->persist_claim : 0;
}

// Workspace of the batch (sum of the members', 256-byte aligned).
// ---- host-only introspection (no device needed) ----
extern "C" obfft_status_t obfft_quantised_roots(int64_t N, int bits, int64_t* host_out) {
  if (N < 1 || bits < 1 || bits > 61 || !host_out) return OBFFT_INVALID_VALUE;
  std::vector<int64_t> q;
  quantised_roots(N, bits, q);
  memcpy(host_out, q.data(), q.size() * sizeof(int64_t));
  return OBFFT_SUCCESS;
}

extern "C" obfft_status_t obfft_crt_constants(int precision, obfft_crt_constants_t* out) {
  if ((precision != 0 && precision != 1) || !out) return OBFFT_INVALID_VALUE;
  ModSet H;
  std::string err;
  if (!build_modset(precision ? kModFP32 : kModFP64, precision ? 6 : 12, H, err)) return OBFFT_INVALID_VALUE;
  memset(out, 0, sizeof(*out));
  out->r = H.r;
  out->S = H.S;
  out->S_frac = H.T;
  out->log2M = H.log2M;
  for (int i = 0; i < 4; i++) out->M[i] = (uint32_t)(H.M >> (32 * i));
  for (int k = 0; k < H.r; k++) {
    out->moduli[k] = H.m[k];
    for (int i = 0; i < 4; i++) out->u[k][i] = (uint32_t)(H.u[k] >> (32 * i));
    out->w[k] = H.w[k];
  }
  return OBFFT_SUCCESS;
}

extern "C" const char* obfft_status_string(obfft_status_t s) {
  switch (s) {
    case OBFFT_SUCCESS: return "OBFFT_SUCCESS";
    case OBFFT_INVALID_VALUE: return "OBFFT_INVALID_VALUE";
    case OBFFT_UNSUPPORTED_SIZE: return "OBFFT_UNSUPPORTED_SIZE";
    case OBFFT_CAPACITY_EXCEEDED: return "OBFFT_CAPACITY_EXCEEDED";
    case OBFFT_NONFINITE_INPUT: return "OBFFT_NONFINITE_INPUT";
    case OBFFT_ALLOC_FAILED: return "OBFFT_ALLOC_FAILED";
    case OBFFT_HIP_ERROR: return "OBFFT_HIP_ERROR";
    case OBFFT_UNSUPPORTED_DEVICE: return "OBFFT_UNSUPPORTED_DEVICE";
    case OBFFT_WRONG_PRECISION: return "OBFFT_WRONG_PRECISION";
    case OBFFT_BATCH_ABORTED: return "OBFFT_BATCH_ABORTED";
    case OBFFT_SCRATCH_EXCEEDED: return "OBFFT_SCRATCH_EXCEEDED";
  }
  return "unknown status";
}

extern "C" obfft_status_t obfft_last_error(obfft_plan_t plan) {
  if (!plan) return OBFFT_INVALID_VALUE;
  if (plan->d_flags) {
    // the device word the kernels raise on a non-finite input; reading clears it
    uint32_t f = 0;
    if (hipMemcpy(&f, plan->d_flags, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) return OBFFT_HIP_ERROR;
    if (f) {
      const uint32_t zero = 0;
      if (hipMemcpy(plan->d_flags, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return OBFFT_HIP_ERROR;
      plan->last = (f & 2u) ? OBFFT_BATCH_ABORTED : OBFFT_NONFINITE_INPUT;
    }
  }
  return plan->last;
}

// Clears the recorded status (and the device flag) of a plan.
extern "C" obfft_status_t obfft_clear_error(obfft_plan_t plan) {
  if (!plan) return OBFFT_INVALID_VALUE;
  (void)obfft_last_error(plan);
  plan->last = OBFFT_SUCCESS;
  return OBFFT_SUCCESS;
}
