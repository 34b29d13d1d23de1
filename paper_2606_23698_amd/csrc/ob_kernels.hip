// Instantiations and host launchers of the Ozaki-Bailey stage kernels
// (single transforms and the batched launches) for gfx950.
#include <algorithm>

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
      // FP8: `full` also says that the modulus set follows the full-length tile's digit rule
      if constexpr (F || SUB == SUB_FP8)
        if (full) return launch_batch_t<SUB, 32, true>(descs, first, tmember, total, st);
      return launch_batch_t<SUB, 32, false>(descs, first, tmember, total, st);
  }
}

// Persistent batched stage kernel (FP16 substrate, FP64 target): every
// workgroup claims work items in order from a global counter until none are
// left; an item is one tile of one (pass, member) segment.  Before a tile
// whose segment depends on the member's previous pass, one thread polls that
// pass's completion count with acquire semantics at agent scope (the tiles of
// the previous pass were written by other workgroups, possibly on other
// XCDs); after a tile, one thread adds 1 to its segment's count with release
// semantics.  Items are claimed in increasing order and every dependency
// points to smaller items, so the smallest unfinished item can always run:
// the launch cannot deadlock, whatever the grid.  A wait that exceeds the
// plan's poll limit raises the give-up flag, and every workgroup then leaves
// at its next poll or claim, so the kernel always ends.
// MASK: the tile variants (bit v = kPersist* v) the kernel carries.  One
// body holding all eight spills registers, so the plan launches the
// instantiation with the fewest variants that covers its members.
template <unsigned MASK, class PT>
__device__ __forceinline__ void persist_run_tile(int cls, const PT& P, int64_t c, int64_t g) {
  if ((MASK >> kPersistK4Packed & 1) && cls == kPersistK4Packed) stage_tile<SUB_FP16, 0, 16, true, false, 4>(P, c, g);
  else if ((MASK >> kPersistK8Packed & 1) && cls == kPersistK8Packed) stage_tile<SUB_FP16, 0, 16, true, false, 2>(P, c, g);
  else if ((MASK >> kPersistK12Full & 1) && cls == kPersistK12Full) stage_tile<SUB_FP16, 0, 12, true>(P, c, g);
  else if ((MASK >> kPersistK12 & 1) && cls == kPersistK12) stage_tile<SUB_FP16, 0, 12, false>(P, c, g);
  else if ((MASK >> kPersistK16Full & 1) && cls == kPersistK16Full) stage_tile<SUB_FP16, 0, 16, true>(P, c, g);
  else if ((MASK >> kPersistK16 & 1) && cls == kPersistK16) stage_tile<SUB_FP16, 0, 16, false>(P, c, g);
  else if ((MASK >> kPersistK32Full & 1) && cls == kPersistK32Full) stage_tile<SUB_FP16, 0, 32, true>(P, c, g);
  else if (MASK >> kPersistK32 & 1) stage_tile<SUB_FP16, 0, 32, false>(P, c, g);
}

// The parameters live in device memory and are re-read per item (scalar
// loads) rather than held in registers across the tile body.
//
// Claims: a workgroup takes `claim` consecutive items at a time.  Making a
// tile's stores visible to the other XCDs takes an agent-scope release,
// which on this part writes back the XCD's L2; one such release per tile
// costs more than the tile itself, so a workgroup publishes its finished
// tiles of a segment together: when the chunk ends, and whenever the next
// item belongs to another segment (before waiting for that segment's
// dependency, so that no tile is held unpublished while its workgroup
// waits).  Every wave fences its own stores at agent scope (release) before
// the barrier, because the barrier does not wait for outstanding vector
// stores; thread 0 then adds the count with a release add.  A waiter polls
// with relaxed loads and, once the dependency is complete, every wave takes
// one acquire fence before the tile reads its input.  A workgroup remembers
// the last dependency it has seen complete (it stays complete for the rest
// of the launch).
//
// Deadlock freedom: chunks are claimed in increasing item order, a wait is
// entered only with nothing unpublished, and every dependency lies in an
// earlier pass (smaller items); the workgroup holding the smallest
// unpublished item is therefore never waiting, and the launch drains
// whatever the grid.
__device__ __forceinline__ void persist_publish(const PersistParams* Qp, int seg, uint32_t n) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    OB_GLOBAL uint32_t* ctl = (OB_GLOBAL uint32_t*)((const OB_CONST PersistParams*)Qp)->ctl;
    __hip_atomic_fetch_add(&ctl[2 + seg], n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <unsigned MASK>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void ob_persist_kernel(
    const PersistParams* __restrict__ Qp) {
  __shared__ int64_t s_item;
  __shared__ int s_go, s_ready;
  if (threadIdx.x == 0) s_ready = -1;
  bool stop = false;
  while (!stop) {
    const PersistParams* Qg = Qp;
    asm volatile("" : "+s"(Qg));  // the parameter block is re-read after every tile
    const OB_CONST PersistParams* Q = (const OB_CONST PersistParams*)Qg;  // scalar loads
    OB_GLOBAL uint32_t* ctl = (OB_GLOBAL uint32_t*)Q->ctl;
    const int64_t total = Q->total;
    const int claim = Q->claim;
    if (threadIdx.x == 0) {
      const bool gave_up = __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      s_item = gave_up ? total
                       : (int64_t)__hip_atomic_fetch_add(&ctl[0], (uint32_t)claim, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int64_t base = s_item;
    if (base >= total) break;
    const int64_t end = min(base + (int64_t)claim, total);
    // the segment of item `base`: the last d with seg_start[d] <= base
    const OB_CONST int64_t* seg_start = (const OB_CONST int64_t*)Q->seg_start;
    int lo = 0, hi = Q->nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (seg_start[mid] <= base) lo = mid;
      else hi = mid - 1;
    }
    int d = __builtin_amdgcn_readfirstlane(lo);
    int cur = -1;          // segment whose finished tiles await publication
    uint32_t pending = 0;  // how many
    for (int64_t it = base; it < end; it++) {
      while (seg_start[d + 1] <= it) d++;  // items ascend: the segment only moves forward
      d = __builtin_amdgcn_readfirstlane(d);
      if (d != cur) {
        if (pending) persist_publish(Qp, cur, pending);
        pending = 0;
        cur = d;
        if (threadIdx.x == 0) {
          int go = 1;  // 0: leave, 1: run, 2: run after an acquire fence
          const int dep = ((const OB_CONST int*)Q->seg_dep)[d];
          if (dep >= 0 && dep != s_ready) {
            const uint32_t need = (uint32_t)(seg_start[dep + 1] - seg_start[dep]);
            const int limit = Q->spin_limit;
            for (int k = 0;; k++) {
              if (__hip_atomic_load(&ctl[2 + dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
                go = 2;
                s_ready = dep;
                break;
              }
              if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                go = 0;
                break;
              }
              if (k >= limit) {
                __hip_atomic_store(&ctl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or((OB_GLOBAL uint32_t*)Q->flags, 2u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                go = 0;
                break;
              }
              __builtin_amdgcn_s_sleep(4);
            }
          }
          s_go = go;
        }
        __syncthreads();
        const int go = s_go;
        if (!go) {
          stop = true;
          break;
        }
        if (go == 2) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      const int64_t local = it - seg_start[d];
      const int cls = ((const OB_CONST int*)Q->seg_cls)[d];
      // the descriptor stays in memory: its fields are scalar loads where used
      const OB_CONST StageParams& P = ((const OB_CONST StageParams*)Q->descs)[d];
      int64_t c, g;
      decode_tile(P, local, c, g);
      persist_run_tile<MASK>(cls, P, c, g);
      pending++;
      // the next tile rewrites the LDS column tables and digit buffers that
      // slower waves of this one may still read (its epilogue reads the
      // output columns and exponents)
      __syncthreads();
    }
    if (pending) persist_publish(Qp, cur, pending);
  }
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// LDS of the persistent kernel: the largest tile variant among `cls_mask`.
int persist_lds_bytes(unsigned cls_mask) {
  const int b[kPersistVariants] = {
      stage_lds_bytes<SUB_FP16, 0, 16, 4>(16), stage_lds_bytes<SUB_FP16, 0, 16, 2>(16),
      stage_lds_bytes<SUB_FP16, 0, 12, 1>(12), stage_lds_bytes<SUB_FP16, 0, 12, 1>(12),
      stage_lds_bytes<SUB_FP16, 0, 16, 1>(16), stage_lds_bytes<SUB_FP16, 0, 16, 1>(16),
      stage_lds_bytes<SUB_FP16, 0, 32, 1>(32), stage_lds_bytes<SUB_FP16, 0, 32, 1>(32)};
  int m = 0;
  for (int v = 0; v < kPersistVariants; v++)
    if (cls_mask & (1u << v)) m = std::max(m, b[v]);
  return m;
}

// Tile variant of a stage with contraction length K (the same choice as the
// single-transform launch).
int persist_variant(int K) {
  if (K <= 4) return kPersistK4Packed;
  if (K <= 8) return kPersistK8Packed;
  if (K <= 12) return K == 12 ? kPersistK12Full : kPersistK12;
  if (K <= 16) return K == 16 ? kPersistK16Full : kPersistK16;
  return K == 32 ? kPersistK32Full : kPersistK32;
}

// Instantiations of the persistent kernel: the full-length and packed
// variants only (every member's contraction lengths are <= 8, 12, 16 or 32:
// all power-of-two extents and the 12-point factors), and all eight.
static const void* persist_kernel(unsigned mask) {
  return (mask & ~kPersistMaskFull) == 0 ? (const void*)ob_persist_kernel<kPersistMaskFull>
                                         : (const void*)ob_persist_kernel<kPersistMaskAll>;
}

// Workgroups of the persistent launch: what the device holds at once.  The
// kernel has a few bytes of static LDS of its own, so the dynamic maximum is
// raised only to what the tile variants need (at most 20 KB), never to the
// whole 160 KB of the CU.
int persist_grid(unsigned mask, int lds) {
  static int attr_lds[2] = {0, 0};
  const void* k = persist_kernel(mask);
  const int ki = k == (const void*)ob_persist_kernel<kPersistMaskFull> ? 0 : 1;
  if (lds > attr_lds[ki]) {
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
    attr_lds[ki] = lds;
  }
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  return std::max(1, per_cu) * std::max(1, cus);
}

// The control block is cleared by a kernel (not a memset), so that the pair
// can be captured in a graph and replayed.
hipError_t launch_persist(unsigned mask, const PersistParams* Q, uint32_t* ctl, int64_t ctl_words, int grid, int lds,
                          hipStream_t st) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((ctl_words + 255) / 256)), dim3(256), 0, st, ctl, ctl_words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((mask & ~kPersistMaskFull) == 0)
    hipLaunchKernelGGL(ob_persist_kernel<kPersistMaskFull>, dim3((unsigned)grid), dim3(kThreads), lds, st, Q);
  else
    hipLaunchKernelGGL(ob_persist_kernel<kPersistMaskAll>, dim3((unsigned)grid), dim3(kThreads), lds, st, Q);
  return hipGetLastError();
}

// FP64-target batched launch over the members of one pass and K class.
hipError_t launch_batch(int sub, int kmax, bool full, const StageParams* descs, const int64_t* first,
                        const uint16_t* tmember, int64_t total, hipStream_t st) {
  if (sub == SUB_FP16) return launch_batch_s<SUB_FP16>(kmax, full, descs, first, tmember, total, st);
  if (sub == SUB_INT8) return launch_batch_s<SUB_INT8>(kmax, false, descs, first, tmember, total, st);
  return launch_batch_s<SUB_FP8>(kmax, full && kmax == 32, descs, first, tmember, total, st);
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
