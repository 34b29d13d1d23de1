/*
 * obfft -- Ozaki-Bailey full-FP64 complex 3-D FFT for AMD MI355X (gfx950).
 *
 * C ABI of the library libobfft.so.  Every transform is a Bailey six-step FFT
 * per axis (Sec. 2, "The Bailey six-step FFT": input index j = j1 + p j2,
 * output index k = k2 + q k1) whose two DFT stages are Ozaki-II residue GEMMs
 * on MFMA (Sec. 2, Eq. ozaki) with the twiddles fused into the second-stage
 * operands (Sec. 4.1, Eq. twiddle-fusion), complex products as four real
 * GEMMs accumulated into R and I (the paper's Karatsuba split, Alg. 1, trades
 * one product for combines that cost more on this part), and an exact CRT
 * reconstruction: a Phase-A GEMM on FP16 MFMA over canonical residues
 * (Sec. 4.2, Eqs. fcrt, slicing, phaseAcost) followed by a Kulisch fixed-point
 * accumulation, a two-sided modulo-M lift and one correctly rounded pack
 * (Sec. 5.1, Alg. 2).
 *
 * Conventions (all entry points)
 *   - Data are complex interleaved (re, im), C order, n3 fastest: the memory
 *     layout of a contiguous torch.complex128 (FP64 target) or complex64
 *     (FP32 target) tensor of shape (n1, n2, n3).
 *   - Forward transform: Y[k] = sum_j X[j] exp(-2 pi i j.k / n), unnormalised.
 *     Inverse: exp(+2 pi i ...) and the factor 1/(n1 n2 n3).  Adjoint:
 *     exp(+2 pi i ...), unnormalised (the Hermitian adjoint of forward).
 *   - Axes are processed n3, then n2, then n1 unless the plan's axis_order
 *     says otherwise; stage 1 contracts over j2 (length q), stage 2 over j1
 *     (length p).  Factorisation and axis order change output bits; both are
 *     fixed by the plan.
 *   - `in`/`out` are DEVICE pointers owned by the caller; in == out is
 *     allowed, partial overlap is rejected with OBFFT_INVALID_VALUE.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls are stream-ordered and asynchronous; errors detectable on the host
 *     are returned immediately; nothing is allocated on the device inside an
 *     execute call except the plan workspace on its first use (see
 *     obfft_set_workspace).
 *   - No exception crosses the ABI.  A plan may be used from one stream at a
 *     time unless each concurrent user has its own workspace.
 */
#ifndef OBFFT_H
#define OBFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct obfft_plan_s* obfft_plan_t;

typedef enum {
  OBFFT_SUCCESS = 0,
  OBFFT_INVALID_VALUE = 1,        /* bad pointer, size, option or overlap */
  OBFFT_UNSUPPORTED_SIZE = 2,     /* an extent with no admissible p x q split, or
                                     n1 n2 n3 / q >= 2^31 on some axis */
  OBFFT_CAPACITY_EXCEEDED = 3,    /* log2 M <= 1 + log2 K + 2(k+1) (Sec. 2, Eq. capacity) */
  OBFFT_NONFINITE_INPUT = 4,      /* a kernel read an Inf or NaN input value (reported by
                                     obfft_last_error after the stream has synchronised) */
  OBFFT_ALLOC_FAILED = 5,         /* device or host allocation failed */
  OBFFT_HIP_ERROR = 6,            /* a HIP runtime call failed */
  OBFFT_UNSUPPORTED_DEVICE = 7,   /* the current device is not gfx950 */
  OBFFT_WRONG_PRECISION = 8,      /* z2z call on an FP32 plan or c2c on an FP64 plan */
  OBFFT_BATCH_ABORTED = 9,        /* a dependency wait of the persistent batched launch reached its
                                     poll limit; every workgroup then left and the batch outputs are
                                     incomplete (reported by obfft_last_error) */
  OBFFT_SCRATCH_EXCEEDED = 10     /* the allocation-free entry point was called on a plan whose
                                     workspace exceeds the library's fixed scratch array */
} obfft_status_t;

/* Precision target.  FP64: r = 12 moduli, k = 53; FP32: r = 6 moduli,
 * k = 24, S = 8 (Sec. 7, "Ozaki-II for FP32").  The transform plans default
 * to pairwise coprime sets with every modulus at most 1024 (FP64: 1024, 1023,
 * 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967, log2 M = 119.6;
 * FP32: 1024, 1023, 1021, 1019, 1013, 1009, log2 M = 60.0), which the FP16
 * residue GEMM takes whole.  The paper's sets (Sec. 2: 2039, 2029, 2027, 1089,
 * 1024, 961, 841, 625, 529, 511, 491, 487, log2 M = 117.9; Sec. 7: 2039, 2029,
 * 2027, 1024, 961, 841, log2 M = 62.6) serve the standalone CRT entry points
 * and the H0 reduction, and any plan through moduli_override.  Transform
 * outputs do not depend on the set: the stage results are exact integers. */
enum { OBFFT_PREC_FP64 = 0, OBFFT_PREC_FP32 = 1 };

/* MFMA substrate of the residue GEMMs.  All substrates produce bit-identical
 * outputs (the residues of an exact integer product are unique).
 *   FP8  : E4M3 radix-32 digit planes, FP32 accumulation, four real
 *          products; at K = 32 the scaled v_mfma_scale_f32_16x16x128_f8f6f4
 *          with the matrix-digit weights in its block scales, otherwise
 *          v_mfma_f32_16x16x32_fp8_fp8 with one accumulator per digit
 *   INT8 : 8-bit limbs (radix 128), v_mfma_i32_16x16x64_i8, INT32
 *          accumulation, four real products
 *   FP16 : whole FP16 matrix residues against one FP16 data residue per
 *          index (every modulus must satisfy 64 h (h + e) <= 2^24, h =
 *          floor(m/2), e = 0 for a power of two and 2 otherwise, i.e.
 *          m <= 1024, else OBFFT_UNSUPPORTED_SIZE); with the H0 reduction
 *          the first 4 moduli of its set enter as radix-128 data limbs
 *          instead.  v_mfma_f32_16x16x32_f16, exact FP32 accumulation of
 *          the four real products straight into Re and Im
 *   AUTO : FP16 when the modulus set allows it (both default sets do), else
 *          INT8 */
enum { OBFFT_SUB_FP8 = 0, OBFFT_SUB_INT8 = 1, OBFFT_SUB_FP16 = 2, OBFFT_SUB_AUTO = 3 };

/* Residue reduction of the GEMM sums (exact integers |t| <= 2^24) in the
 * stage kernels.
 *   RECIPROCAL : t - m rne(t / m) in FP32, three vector instructions for any
 *                modulus (default)
 *   H0         : fold-and-add for the reduction-friendly moduli m = 2^b - c
 *                with c <= 31 or c = 0 (Sec. 2; rung H0 of the co-design
 *                ladder, Sec. 8.3: 2039, 2029, 2027, 1024, 511, 491, 487 of
 *                the FP64 set), the reciprocal form for the rest.  An
 *                ablation: FP16 substrate and FP64 target only, single
 *                transforms only (else OBFFT_INVALID_VALUE); outputs are
 *                bit-identical to RECIPROCAL (residues are unique). */
enum { OBFFT_RED_RECIPROCAL = 0, OBFFT_RED_H0 = 1 };

typedef struct {
  int precision;            /* OBFFT_PREC_* */
  int substrate;            /* OBFFT_SUB_* */
  int p[3];                 /* per axis (n1, n2, n3); 0 = library default */
  int q[3];                 /* per axis; p*q must equal the extent */
  int n_moduli_override;    /* 0 = the default set of the precision (and reduction);
                               else use moduli_override */
  const int32_t* moduli_override; /* host pointer, pairwise coprime, each < 2048 */
  int reduction;            /* OBFFT_RED_* (0 = default) */
  int group_block;          /* tile order of stage 2 on the contiguous axis: the number of
                               twiddle groups k2 whose tiles of one column block run back to
                               back on one XCD, so that their partial output lines merge in
                               its L2.  0 = library default (8 when it divides q); else one of
                               1, 2, 4, 8, 16, 32 (else OBFFT_INVALID_VALUE), used where it
                               divides q of that axis.  Changes speed only, never results. */
  int axis_order[3];        /* the axes in execution order (0 = n1), a permutation of
                               {0, 1, 2}; all zero = library default {2, 1, 0} (n3, then n2,
                               then n1).  Changes output bits (every axis pass rounds once
                               per stage), so the plan records it. */
  int reserved[3];
} obfft_options_t;

typedef struct {
  int precision, substrate;
  int r;                    /* number of moduli */
  int32_t moduli[16];
  double log2M;             /* log2 of the modulus product */
  double budget_bits;       /* 1 + log2 Kmax + 2(k+1) of Eq. capacity */
  int p[3], q[3];
  int S, S_frac;            /* byte slices of u_k and of w_k (Sec. 4.2, Sec. 5.1) */
  int64_t n[3];
  size_t workspace_bytes;
} obfft_plan_info_t;

/* Fills `opt` with defaults: FP64, AUTO substrate, library factorisation. */
void obfft_options_default(obfft_options_t* opt);

/* Creates a plan for an n1 x n2 x n3 transform.  Computes every constant of
 * Sec. 2 / Sec. 4.2 / Sec. 5.1 for the modulus set, checks the capacity
 * budget for Kmax = max over axes of max(p, q) (Eq. capacity; rejects with
 * OBFFT_CAPACITY_EXCEEDED), quantises the roots of unity, builds the MFMA
 * operand planes and uploads them to the current device.  opt may be NULL.
 * On failure *plan is set to NULL.  Host and device memory is owned by the
 * plan until obfft_plan_destroy. */
obfft_status_t obfft_plan_create(obfft_plan_t* plan, int64_t n1, int64_t n2, int64_t n3,
                                 const obfft_options_t* opt);
obfft_status_t obfft_plan_destroy(obfft_plan_t plan);
obfft_status_t obfft_plan_info(obfft_plan_t plan, obfft_plan_info_t* info);

/* Bytes of device workspace an execute call needs (one array of the
 * transform's size for the six-step ping-pong).  If the caller supplies
 * none, the plan allocates it on first use and frees it on destroy. */
size_t obfft_workspace_size(obfft_plan_t plan);
obfft_status_t obfft_set_workspace(obfft_plan_t plan, void* device_ptr, size_t bytes);

/* Copies the plan's quantised roots Q(w_N^t) = (RNE(2^B cos 2 pi t/N),
 * RNE(-2^B sin 2 pi t/N)), t < N, for `axis` (0 = n1) into host memory
 * (2 N int64).  B = 52 (FP64) or 23 (FP32).  Introspection only. */
obfft_status_t obfft_plan_roots(obfft_plan_t plan, int axis, int64_t* host_out);

/* FP64-target transforms (complex128 in/out). */
obfft_status_t fft3d_z2z_forward(obfft_plan_t plan, const void* in, void* out, void* stream);
obfft_status_t fft3d_z2z_inverse(obfft_plan_t plan, const void* in, void* out, void* stream);
obfft_status_t fft3d_z2z_adjoint(obfft_plan_t plan, const void* in, void* out, void* stream);

/* Forward transform that allocates nothing, for callers that cannot
 * allocate device memory (code under stream or graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same result, bit for bit, as
 * fft3d_z2z_forward on the same plan.  The Y' workspace is a fixed device
 * array inside the library (obfft_noalloc_scratch_bytes() bytes, 256 MiB:
 * every transform of at most 2^24 complex128 elements, e.g. 256^3); each
 * device that loads the library holds its own copy until the process ends.
 * A plan whose workspace_bytes exceeds it is rejected with
 * OBFFT_SCRATCH_EXCEEDED before anything is launched.  The call does not
 * allocate: no hipMalloc/hipFree, and the plan's own workspace is neither
 * used nor created.  Every call on one device shares that device's array
 * (its contents are not carried between calls), so calls that overlap in
 * time on one device -- on different streams, or from different threads
 * -- race and must be serialised by the caller. */
obfft_status_t fft3d_z2z_forward_noalloc(obfft_plan_t plan, const void* in, void* out, void* stream);
size_t obfft_noalloc_scratch_bytes(void);

/* FP32-target transforms (complex64 in/out) on a plan made with
 * precision = OBFFT_PREC_FP32 (Sec. 7). */
obfft_status_t fft3d_c2c_forward(obfft_plan_t plan, const void* in, void* out, void* stream);
obfft_status_t fft3d_c2c_inverse(obfft_plan_t plan, const void* in, void* out, void* stream);

/* The comparator: a native FP64 FFT (radix butterflies in FP64 registers,
 * FP64 twiddles; no emulation) of the same size on the same device.
 * Works on any FP64 plan; uses the plan's workspace. */
obfft_status_t fft3d_z2z_native_forward(obfft_plan_t plan, const void* in, void* out, void* stream);
obfft_status_t fft3d_z2z_native_inverse(obfft_plan_t plan, const void* in, void* out, void* stream);

/* Debug tap of the fused stage kernel (the checkpoints of Alg. 2 for one
 * line).  Runs stage `stage` (1 or 2) of axis `axis` (0 = n1), direction 0
 * (forward) or 1 (conjugate), on the device array `in` (natural order for
 * stage 1, Y' slots for stage 2, as obfft_stage) into the device array `out`
 * (not aliasing in), with the debug variant of the kernel, then copies the
 * epilogue records of every output of line `line` to host memory and returns
 * after synchronising `stream`.  A line of axis a is (outer o, inner i) with
 * line = o * inner + i, inner = product of the faster extents,
 * 0 <= line < n1 n2 n3 / n_a.  host_dump: uint32 [n_a][2 (Re, Im)][64]; the
 * record of output slot t (the slot order of the stage, as obfft_stage) is:
 *   [0, S)      Phase-A slice sums P_s (int32, Eq. slicing)
 *   [16, 16+T)  Phase-A lift sums Z_t (int32, Sec. 5.1)
 *   [24, 29)    E = sum_s 256^s P_s modulo 2^(32 w), little-endian words, w = 4
 *               (FP64 target) or 3 (FP32), higher words zero: the kernel's
 *               Kulisch accumulator keeps only these low bits of E (|E| may
 *               reach 2^131), all that R = E - zhat M (|R| < 2^113) needs
 *   29          zhat = round-half-up(2^-48 sum_t 256^t Z_t) (int32)
 *   [30, 34)    R = E - zhat M, the exact stage integer (two's complement)
 *   34          the pack exponent: the output is RNE(R 2^exp) (int32)
 *   35, 36      the output value's bits (binary64 low/high word; binary32 in 35)
 *   [40, 40+r)  the residues v_k that entered Phase A (int32; the stage
 *               kernels take centred residues, |v_k| <= m_k/2 + 2)
 * The stage output is written to `out` as by obfft_stage.  Allocates a small
 * device buffer per call.  Bad arguments return OBFFT_INVALID_VALUE. */
obfft_status_t obfft_debug_tap(obfft_plan_t plan, int axis, int stage, int direction, int64_t line,
                               const void* in, void* out, void* host_dump, void* stream);

/* One Bailey stage of one axis (unit-level access to the fused kernel).
 * stage 1 reads natural order and writes Y' with Y'_{j1,k2} at slot
 * j1 + p k2; stage 2 reads those slots and writes Z_{k1,k2} at k2 + q k1
 * (Alg. 1).  direction: 0 forward, 1 conjugate.  out must not alias in.
 * If residues_out (device) is not NULL, the canonical residues of every
 * output's real and imaginary integer are written as uint16
 * [slot][re/im][r] (debug tap; slows the kernel). */
obfft_status_t obfft_stage(obfft_plan_t plan, int axis, int stage, int direction,
                           const void* in, void* out, void* residues_out, void* stream);

/* Exact CRT reconstruction of n scalars from canonical residues: the Phase-A
 * GEMM on FP16 MFMA (Sec. 4.2, Eqs. fcrt and slicing) and the Kulisch Phase B
 * with the two-sided modulo-M lift and the correctly rounded pack (Sec. 5.1,
 * Alg. 2), exposed for unit-level parity.  precision selects the modulus set
 * (12 moduli for FP64, 6 for FP32).
 *   residues: device uint16 [n][r], residue k of output i in [0, m_k);
 *             larger values are a caller error (results undefined, no fault).
 *   exps:     device int32 [n]; output i is RNE(R_i * 2^exps[i]).
 *   out:      device double [n] (FP64) or float [n] (FP32).
 *   taps:     device uint32 [n][layout.stride] or NULL; see obfft_taps_layout.
 * n >= 2^31 returns OBFFT_UNSUPPORTED_SIZE. */
obfft_status_t obfft_crt_reconstruct(int precision, int64_t n, const void* residues,
                                     const void* exps, void* out, void* taps, void* stream);

/* Reconstruction methods for obfft_crt_reconstruct_method: the Kulisch
 * route above and two of the reconstructions the paper ranks it against. */
enum {
  OBFFT_CRT_KULISCH = 0,    /* Phase A on FP16 MFMA + Kulisch Phase B (as obfft_crt_reconstruct) */
  OBFFT_CRT_GARNER = 1,     /* recursive Garner (Sec. 4.1, Eq. recursive-garner; App. C): mixed-
                               radix digits in 32-bit integer arithmetic, the positional value in
                               multiword integers, one correctly rounded pack.  Exact: the same
                               output bits as OBFFT_CRT_KULISCH for every residue tuple. */
  OBFFT_CRT_SLICE_FP64 = 2, /* slicing direct CRT with a plain FP64 Phase B (Sec. 4.2; App. C,
                               Table precision): the exact Phase-A slice sums P_s, then
                               T = sum_s P_s 256^s in FP64 (s ascending, one rounding per
                               addition), y = T - fl(zhat * fl(M)) with zhat the lift of Sec. 5.1,
                               scaled by 2^exps[i]; FP32 target: y rounded to binary32.  The
                               accuracy baseline: not exact, it keeps about the top 53 of the
                               sum's ~120 bits. */
  OBFFT_CRT_KULISCH_INT8 = 3, /* the Kulisch route with Phase A on INT8 MFMA (Sec. 8.2, the B200
                               cross-check; Sec. 8.3, Eq. h1-group): residues split into two
                               signed-byte limbs v = v0 + 256 v1, the high limb against the next
                               lower slice, slices of u_k and w_k as balanced base-256 digits,
                               exact INT32 accumulation.  Same output bits as OBFFT_CRT_KULISCH. */
  OBFFT_CRT_KULISCH_INT16 = 4 /* the Kulisch accumulator in 16-bit words (Sec. 6.3, Eq.
                               kulisch-width; Sec. 6.4, Strategy A): slice sums deposited into
                               radix-2^12 words with four guard bits, one carry sweep at the
                               end.  Same output bits as OBFFT_CRT_KULISCH. */
};

/* The standalone reconstruction by one of the methods above, for timing and
 * accuracy comparisons on the same residues.  Arguments as for
 * obfft_crt_reconstruct (no taps).  An unknown method or precision returns
 * OBFFT_INVALID_VALUE; n >= 2^31 returns OBFFT_UNSUPPORTED_SIZE; residues at
 * or above their modulus give undefined values (no fault). */
obfft_status_t obfft_crt_reconstruct_method(int precision, int method, int64_t n, const void* residues,
                                            const void* exps, void* out, void* stream);

/* Word offsets inside one output's taps record of obfft_crt_reconstruct:
 *   P    [P, P+S)        Phase-A slice sums P_s (Eq. slicing)
 *   Z    [Z, Z+S_frac)   Phase-A lift sums Z_t (Sec. 5.1)
 *   E    [E, E+n_E)      E = sum_k v_k u_k, little-endian words (mod 2^160)
 *   zhat                 round-half-up(2^-48 sum_t 256^t Z_t)
 *   R    [R, R+n_R)      the lifted value in [-M/2, M/2), two's complement
 *   stride               words per output (the power-of-two exponent is at
 *                        R + n_R) */
typedef struct { int P, Z, E, n_E, zhat, R, n_R, stride; } obfft_taps_layout_t;
void obfft_taps_layout(obfft_taps_layout_t* layout);

/* Hardware-contract probe (tests only): one wave runs one instruction on
 * device operands laid out one register set per lane.  kind 0: FP8
 * 16x16x32 MFMA (a, b: 64 x 8 bytes, d: 64 x 4 float); 1: INT8 16x16x64
 * (64 x 16 bytes, d: 64 x 4 int32); 2: FP16 32x32x16 (64 x 8 half, d: 64 x
 * 16 float); 3: permlane32 swap (a, b: 64 uint32, d: 2 x 64 uint32); 4: E4M3
 * conversion of 64 floats in a (b unused) into 64 bytes of d; 5: FP16
 * 16x16x32 (64 x 8 half, d: 64 x 4 float); 6: INT8 32x32x32 (64 x 16 bytes,
 * d: 64 x 16 int32); 7: scaled FP8 16x16x128 (a: 64 x 32 bytes followed by
 * 64 int32 E8M0 scales of A, b: 64 x 32 bytes unscaled, d: 64 x 4 float). */
obfft_status_t obfft_mfma_probe(int kind, const void* a, const void* b, void* d, void* stream);

/* Host-only introspection (no device needed). */
/* Q(w_N^t) scaled by 2^bits, t < N, into host int64 [N][2] (bits <= 61). */
obfft_status_t obfft_quantised_roots(int64_t N, int bits, int64_t* host_out);

typedef struct {
  int r, S, S_frac;
  double log2M;
  int32_t moduli[16];
  uint32_t M[4];            /* little-endian words of M */
  uint32_t u[16][4];        /* CRT idempotents u_k (Sec. 4.2, Eq. fcrt) */
  uint64_t w[16];           /* lift weights round(2^48 u_k / M) (Sec. 5.1) */
} obfft_crt_constants_t;
obfft_status_t obfft_crt_constants(int precision, obfft_crt_constants_t* out);

/* Batched transforms: `count` independent FP64 forward transforms of possibly
 * different shapes (host int64 [count][3]).  By default each of the six Bailey
 * passes (axis n3 stage 1, n3 stage 2, n2 ..., n1 stage 2) runs as one launch
 * per contraction class over the tiles of every member (one workgroup per
 * tile, each finding its member in a device descriptor table); on the FP16
 * substrate the whole batch may instead run as one persistent launch
 * (obfft_batch_set_mode).  The launches are captured once in a hipGraph and
 * replayed.  Members with
 * equal shapes share one plan.
 * Outputs are bit-identical to fft3d_z2z_forward on each member.  The batch
 * owns a workspace of the summed member sizes, allocated on first use.
 * 1 <= count <= 65535, else OBFFT_INVALID_VALUE.
 * ins/outs: host arrays of `count` device pointers. */
obfft_status_t obfft_batch_plan_create(obfft_plan_t* plan, int count, const int64_t* shapes,
                                       const obfft_options_t* opt);
/* The same with options per member (host array of `count`): each member may
 * take its own factorisation, axis order and tile order (an autotuner's
 * choice per shape; the tile variant of every stage follows from its
 * contraction length).  Every member's output is bit-identical to
 * fft3d_z2z_forward on a plan made with that member's options.  All members
 * must share precision (FP64), substrate and reduction, and take no modulus
 * override, else OBFFT_INVALID_VALUE. */
obfft_status_t obfft_batch_plan_create_each(obfft_plan_t* plan, int count, const int64_t* shapes,
                                            const obfft_options_t* opts);
obfft_status_t obfft_batch_forward(obfft_plan_t plan, const void* const* ins, void* const* outs,
                                   void* stream);
/* use_graph = 0 launches the batch directly instead of replaying the graph. */
obfft_status_t obfft_batch_set_graph(obfft_plan_t plan, int use_graph);

/* How a batch runs.
 *   OBFFT_BATCH_PERSISTENT : one persistent launch over the tiles of every pass
 *     of every member (FP16 substrate).  Workgroups (as many as the device
 *     holds at once) claim tiles in pass-major order from a global counter, a
 *     few at a time (obfft_batch_set_claim); a tile of pass s of a member waits
 *     until the member's pass s - 1 has completed every tile (per-(member,
 *     pass) counters with release and acquire at device scope), so passes of
 *     different members overlap.  On this 8-XCD part each release writes back
 *     an XCD's L2 and each acquire invalidates it, which costs more than the
 *     kernel boundaries of the per-pass launches, so it is not the default.  Each
 *     wait polls at most the plan's poll limit (obfft_batch_set_poll_limit)
 *     before the launch gives up: every workgroup then leaves, and
 *     obfft_last_error reports OBFFT_BATCH_ABORTED.  A small clearing kernel
 *     resets the counters before each launch; both are captured in the graph.
 *   OBFFT_BATCH_PASSES : one launch per Bailey pass and contraction class (the
 *     default; the other substrates always run this way).
 * Outputs are bit-identical in both modes.  OBFFT_INVALID_VALUE for a mode the
 * plan cannot run. */
enum { OBFFT_BATCH_PASSES = 0, OBFFT_BATCH_PERSISTENT = 1 };
obfft_status_t obfft_batch_set_mode(obfft_plan_t plan, int mode);
/* Polls of one dependency wait before the persistent launch gives up (default
 * 2^21, a few seconds; 0 gives up at the first unmet dependency). */
obfft_status_t obfft_batch_set_poll_limit(obfft_plan_t plan, int polls);

/* Items (tiles) a workgroup of the persistent launch claims at once, 1..256
 * (else OBFFT_INVALID_VALUE).  A workgroup publishes the finished tiles of
 * one segment together, and each publication makes its XCD write back its
 * L2, so larger claims mean fewer write-backs and coarser load balance.
 * The plan picks about four claims per workgroup over the batch, at most 64;
 * obfft_batch_get_claim returns the current value (0 for a plan without a
 * persistent launch).  Changes speed only, never results. */
obfft_status_t obfft_batch_set_claim(obfft_plan_t plan, int items);
int obfft_batch_get_claim(obfft_plan_t plan);

const char* obfft_status_string(obfft_status_t status);
/* The status of the last failed call on this plan (OBFFT_SUCCESS if none),
 * or OBFFT_NONFINITE_INPUT when a kernel of this plan has read an Inf or NaN
 * input value since the flag was last read: the kernels raise a device flag
 * and run to completion (the affected outputs are meaningless), and this
 * call reads the flag with a blocking copy, so call it after synchronising
 * the stream.  Reading clears the device flag; the status stays until
 * obfft_clear_error. */
obfft_status_t obfft_last_error(obfft_plan_t plan);
/* Resets the plan's recorded status and device flag to OBFFT_SUCCESS. */
obfft_status_t obfft_clear_error(obfft_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* OBFFT_H */
