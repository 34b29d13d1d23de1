// Native FP64 3-D FFT for gfx950: the comparator of the emulated transform.
//
// One kernel pass per axis reads every element from HBM once and writes it
// once (the traffic model Q = 96 N^3 bytes of Sec. 4.1, Eq. Q-fft).  A
// workgroup stages B lines in LDS and runs a self-sorting (Stockham) mixed
// radix-8/4/3/2 FFT on them: each pass reads R values per butterfly into
// registers, multiplies by FP64 twiddles from a table of w_N^t, applies the
// length-R DFT in registers and writes the results back to LDS in the
// expanded (autosorted) positions.  No emulation: this is the plain FP64
// path the Ozaki-Bailey kernel is measured against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

namespace obfft {

void quantised_roots(int64_t N, int bits, std::vector<int64_t>& out);

constexpr int kNatThreads = 256;
constexpr int kNatLdsComplex = 8192;   // 128 KiB of complex data per workgroup
constexpr int kMaxPasses = 12;
constexpr int kNatRegs = 32;           // complex values a thread holds during a pass
// Arrays from this size on are streamed with nontemporal loads and stores by
// the 4-step kernels.  Measured on gfx950: every axis of the 4, 8 and 16 GiB
// shapes gets faster (1024^3: 21.7 -> 19.3 ms), while at 2 GiB (512^3) and
// below the default cache policy is faster.
constexpr int64_t kNatStreamBytes = int64_t(4) << 30;

struct NatAxis {
  int64_t N, inner, outer;
  int B;                       // lines per workgroup
  int npass;
  int radix[kMaxPasses];
  const double2* tw;           // w_N^t, t < N (forward sign)
};

struct NativePlan {
  int64_t n[3];
  NatAxis ax[3];
  std::vector<void*> allocs;
};

template <int R, int DIR>
__device__ __forceinline__ void dft_r(double2* v) {
  // DIR = +1 forward (exp(-2 pi i / R)), -1 inverse
  if (R == 2) {
    double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
  } else if (R == 3) {
    const double c1 = -0.5, s1 = 0.86602540378443864676 * DIR;
    double2 a = v[0], b = v[1], c = v[2];
    double2 t = make_double2(b.x + c.x, b.y + c.y);
    double2 d = make_double2(b.x - c.x, b.y - c.y);
    v[0] = make_double2(a.x + t.x, a.y + t.y);
    double2 m = make_double2(a.x + c1 * t.x, a.y + c1 * t.y);
    // -i s1 d
    v[1] = make_double2(m.x + s1 * d.y, m.y - s1 * d.x);
    v[2] = make_double2(m.x - s1 * d.y, m.y + s1 * d.x);
  } else if (R == 4) {
    double2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    double2 t0 = make_double2(a0.x + a2.x, a0.y + a2.y);
    double2 t1 = make_double2(a0.x - a2.x, a0.y - a2.y);
    double2 t2 = make_double2(a1.x + a3.x, a1.y + a3.y);
    double2 t3 = make_double2(a1.x - a3.x, a1.y - a3.y);
    // -i DIR t3
    double2 u3 = make_double2(DIR * t3.y, -DIR * t3.x);
    v[0] = make_double2(t0.x + t2.x, t0.y + t2.y);
    v[2] = make_double2(t0.x - t2.x, t0.y - t2.y);
    v[1] = make_double2(t1.x + u3.x, t1.y + u3.y);
    v[3] = make_double2(t1.x - u3.x, t1.y - u3.y);
  } else if (R == 8) {
    const double h = 0.70710678118654752440;
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    dft_r<4, DIR>(e);
    dft_r<4, DIR>(o);
    // o[k] *= w_8^{k DIR}
    double2 o1 = make_double2(h * (o[1].x + DIR * o[1].y), h * (o[1].y - DIR * o[1].x));
    double2 o2 = make_double2(DIR * o[2].y, -DIR * o[2].x);
    double2 o3 = make_double2(h * (-o[3].x + DIR * o[3].y), h * (-o[3].y - DIR * o[3].x));
    double2 oo[4] = {o[0], o1, o2, o3};
#pragma unroll
    for (int k = 0; k < 4; k++) {
      v[k] = make_double2(e[k].x + oo[k].x, e[k].y + oo[k].y);
      v[k + 4] = make_double2(e[k].x - oo[k].x, e[k].y - oo[k].y);
    }
  }
}

template <int R, int DIR>
__device__ __forceinline__ void stockham_pass(double2* lds, int B, int64_t N, int Ns, const double2* tw) {
  const int nb = (int)(N / R);        // butterflies per line
  const int total = nb * B;
  constexpr int MAXB = kNatRegs;      // complex values per thread per pass
  // The plan sizes B so that one round covers every butterfly of the pass:
  // all reads complete (barrier) before any write, so the pass is in place.
  for (int base = 0; base < total; base += kNatThreads * (MAXB / R)) {
    double2 reg[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB / R; q++) {
      int idx = base + q * kNatThreads + threadIdx.x;
      if (idx < total) {
        int line = idx / nb, j = idx % nb;
        double2* src = lds + (int64_t)line * N;
#pragma unroll
        for (int r = 0; r < R; r++) reg[q * R + r] = src[j + r * nb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB / R; q++) {
      int idx = base + q * kNatThreads + threadIdx.x;
      if (idx < total) {
        int line = idx / nb, j = idx % nb;
        int jm = j % Ns;
        double2* x = &reg[q * R];
        if (Ns > 1) {
          // twiddle w_{Ns R}^{r jm} = w_N^{r jm N/(Ns R)}
          int64_t step = N / ((int64_t)Ns * R) * jm;
#pragma unroll
          for (int r = 1; r < R; r++) {
            double2 w = tw[(r * step) % N];
            double wy = DIR * w.y;
            double2 a = x[r];
            x[r] = make_double2(a.x * w.x - a.y * wy, a.x * wy + a.y * w.x);
          }
        }
        dft_r<R, DIR>(x);
        int idxd = (j / Ns) * Ns * R + jm;
        double2* dst = lds + (int64_t)line * N;
#pragma unroll
        for (int r = 0; r < R; r++) dst[idxd + r * Ns] = x[r];
      }
    }
    __syncthreads();
  }
}

template <int DIR>
__global__ __launch_bounds__(kNatThreads) void native_axis_kernel(const double2* in, double2* out, NatAxis A,
                                                                  double post_scale) {
  extern __shared__ __align__(16) double2 lds[];
  const int64_t N = A.N, inner = A.inner;
  const int B = A.B;
  const int64_t nlines = A.outer * inner;
  const int64_t line0 = (int64_t)blockIdx.x * B;
  const int nl = (int)min((int64_t)B, nlines - line0);
  // load: element (line, n) of line id L = o inner + i at o N inner + n inner + i
  for (int64_t e = threadIdx.x; e < (int64_t)nl * N; e += kNatThreads) {
    int b, n;
    if (inner >= B) {
      b = (int)(e % nl);
      n = (int)(e / nl);
    } else {
      b = (int)(e / N);
      n = (int)(e % N);
    }
    int64_t L = line0 + b;
    int64_t o = L / inner, i = L % inner;
    lds[(int64_t)b * N + n] = in[o * N * inner + (int64_t)n * inner + i];
  }
  __syncthreads();
  int Ns = 1;
  for (int p = 0; p < A.npass; p++) {
    int R = A.radix[p];
    if (R == 8) stockham_pass<8, DIR>(lds, nl, N, Ns, A.tw);
    else if (R == 4) stockham_pass<4, DIR>(lds, nl, N, Ns, A.tw);
    else if (R == 3) stockham_pass<3, DIR>(lds, nl, N, Ns, A.tw);
    else stockham_pass<2, DIR>(lds, nl, N, Ns, A.tw);
    Ns *= R;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)nl * N; e += kNatThreads) {
    int b, n;
    if (inner >= B) {
      b = (int)(e % nl);
      n = (int)(e / nl);
    } else {
      b = (int)(e / N);
      n = (int)(e % N);
    }
    int64_t L = line0 + b;
    int64_t o = L / inner, i = L % inner;
    double2 v = lds[(int64_t)b * N + n];
    if (post_scale != 1.0) v = make_double2(v.x * post_scale, v.y * post_scale);
    out[o * N * inner + (int64_t)n * inner + i] = v;
  }
}

// ---- register-resident four-step kernel: N = R1 x R2, R1 <= R2 <= 32 ----
//
// Line element n = n1 R2 + n2, output k = k1 + R1 k2 (Cooley-Tukey):
//   step 1: thread (line, n2) loads x[n1 R2 + n2], n1 < R1, does DFT_R1 over n1
//           in registers and multiplies by w_N^{n2 k1};
//   exchange through LDS (real plane, then imaginary plane);
//   step 2: thread (line, k1) does DFT_R2 over n2 in registers and stores
//           X[k1 + R1 k2], k2 < R2.
// STRIDED selects the lane mapping: false (contiguous axis) puts neighbouring
// lanes along a line, true puts them on neighbouring lines, so that global
// loads and stores are coalesced in both cases.

// Length-R DFT in registers, in place, decimation in frequency: one radix-r
// step (r = 4, 2 or 3) turns v[j + m a] (m = R / r) into the r blocks
// y_b[j] = w_R^{j b} sum_a v[j + m a] w_r^{a b} stored at v[m b + j], and
// block b then holds, after its own length-m transform, X[b + r k'].  No
// copies: the output X[k] is left at position pos(k), a digit reversal known
// at compile time.  Twiddles w_R^t come from the axis table at stride N / R.
template <int R, int DIR>
struct RegDft {
  static constexpr int r = (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : 3;
  static constexpr int m = R / r;

  __host__ __device__ static constexpr int pos(int k) {
    if constexpr (R == 1) {
      return 0;
    } else {
      return m * (k % r) + RegDft<m, DIR>::pos(k / r);
    }
  }

  __device__ __forceinline__ static void run(double2* v, const double2* tw, int tstride) {
    if constexpr (R > 1) {
#pragma unroll
      for (int j = 0; j < m; j++) {
        double2 t[r];
#pragma unroll
        for (int a = 0; a < r; a++) t[a] = v[j + m * a];
        dft_r<r, DIR>(t);
#pragma unroll
        for (int b = 0; b < r; b++) {
          const int e = j * b;  // twiddle w_R^e, e < R
          double2 x = t[b];
          if (e == 0) {
          } else if (2 * e == R) {
            x = make_double2(-x.x, -x.y);
          } else if (4 * e == R) {
            x = make_double2(DIR * x.y, -DIR * x.x);
          } else if (4 * e == 3 * R) {
            x = make_double2(-DIR * x.y, DIR * x.x);
          } else {
            const double2 w = tw[e * tstride];
            const double wy = DIR * w.y;
            x = make_double2(__builtin_fma(x.x, w.x, -x.y * wy), __builtin_fma(x.x, wy, x.y * w.x));
          }
          v[j + m * b] = x;
        }
      }
#pragma unroll
      for (int b = 0; b < r; b++) RegDft<m, DIR>::run(v + m * b, tw, tstride * r);
    }
  }
};

// Global loads and stores of the 4-step kernel; SM marks them nontemporal
// (streaming: the lines are read once and written once).
typedef double nat_d2 __attribute__((ext_vector_type(2)));
template <bool SM>
__device__ __forceinline__ double2 nat_load(const double2* p) {
  if constexpr (SM) {
    const nat_d2 t = __builtin_nontemporal_load((const nat_d2*)p);
    return make_double2(t.x, t.y);
  } else {
    return *p;
  }
}
template <bool SM>
__device__ __forceinline__ void nat_store(double2* p, double2 v) {
  if constexpr (SM) __builtin_nontemporal_store((nat_d2){v.x, v.y}, (nat_d2*)p);
  else *p = v;
}

// NT threads per workgroup: 256, or 512 on a strided axis with R2 = 32, so
// that a workgroup holds 16 lines and every global access of a wave covers
// 16 neighbouring lines (256-byte runs instead of 128).  SM: nontemporal
// global accesses, taken for arrays of at least kNatStreamBytes.
template <int R1, int R2, bool STRIDED, int DIR, int NT = kNatThreads, bool SM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void native_4step_kernel(const double2* in, double2* out, int64_t inner,
                                                                   int64_t nlines, const double2* tw,
                                                                   double post_scale) {
  constexpr int N = R1 * R2;
  constexpr int LPW = NT / R2;                    // lines per workgroup
  constexpr int LS = ((R1 * (R2 + 1)) | 1);      // padded line stride in LDS (doubles, odd)
  __shared__ double plane[LPW * LS];
  const int tid = threadIdx.x;
  const int64_t line0 = (int64_t)blockIdx.x * LPW;
  // step 1 mapping
  int l1, n2;
  if (STRIDED) {
    l1 = tid % LPW;
    n2 = tid / LPW;
  } else {
    n2 = tid % R2;
    l1 = tid / R2;
  }
  const int64_t L = line0 + l1;
  const bool valid1 = L < nlines;
  const int64_t o1 = L / inner, i1 = L % inner;
  const double2* src = in + o1 * N * inner + i1;
  double2 v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; n1++)
    v[n1] = valid1 ? nat_load<SM>(&src[(int64_t)(n1 * R2 + n2) * inner]) : make_double2(0.0, 0.0);
  RegDft<R1, DIR>::run(v, tw, N / R1);
  // X1[k1] sits at v[pos(k1)]; twiddle w_N^{n2 k1}
#pragma unroll
  for (int k1 = 1; k1 < R1; k1++) {
    const int pk = RegDft<R1, DIR>::pos(k1);
    double2 w = tw[(n2 * k1) % N];
    double wy = DIR * w.y;
    double2 a = v[pk];
    v[pk] = make_double2(__builtin_fma(a.x, w.x, -a.y * wy), __builtin_fma(a.x, wy, a.y * w.x));
  }
  // step 2 mapping: task (line, k1); R1 <= R2 so LPW * R1 <= threads
  int l2, k1t;
  if (STRIDED) {
    l2 = tid % LPW;
    k1t = tid / LPW;
  } else {
    k1t = tid % R1;
    l2 = tid / R1;
  }
  const bool active2 = STRIDED ? (k1t < R1) : (l2 < LPW);
  double2 u[R2];
  // exchange: real plane, then imaginary plane
#pragma unroll
  for (int c = 0; c < 2; c++) {
#pragma unroll
    for (int k1 = 0; k1 < R1; k1++) {
      const int pk = RegDft<R1, DIR>::pos(k1);
      plane[l1 * LS + k1 * (R2 + 1) + n2] = c ? v[pk].y : v[pk].x;
    }
    __syncthreads();
    if (active2) {
#pragma unroll
      for (int j = 0; j < R2; j++) {
        double x = plane[l2 * LS + k1t * (R2 + 1) + j];
        if (c) u[j].y = x;
        else u[j].x = x;
      }
    }
    __syncthreads();
  }
  if (!active2) return;
  RegDft<R2, DIR>::run(u, tw, N / R2);
  const int64_t L2 = line0 + l2;
  if (L2 >= nlines) return;
  const int64_t o2 = L2 / inner, i2 = L2 % inner;
  double2* dst = out + o2 * N * inner + i2;
#pragma unroll
  for (int k2 = 0; k2 < R2; k2++) {
    double2 x = u[RegDft<R2, DIR>::pos(k2)];
    if (post_scale != 1.0) x = make_double2(x.x * post_scale, x.y * post_scale);
    nat_store<SM>(&dst[(int64_t)(k1t + R1 * k2) * inner], x);
  }
}

template <int R1, int R2, bool STRIDED, int NT, bool SM>
static void launch_4step_k(const double2* in, double2* out, const NatAxis& A, int inverse, double ps, hipStream_t st) {
  const int64_t nlines = A.outer * A.inner;
  const int64_t grid = (nlines + NT / R2 - 1) / (NT / R2);
  if (inverse)
    hipLaunchKernelGGL((native_4step_kernel<R1, R2, STRIDED, -1, NT, SM>), dim3((unsigned)grid), dim3(NT), 0, st, in,
                       out, A.inner, nlines, A.tw, ps);
  else
    hipLaunchKernelGGL((native_4step_kernel<R1, R2, STRIDED, 1, NT, SM>), dim3((unsigned)grid), dim3(NT), 0, st, in,
                       out, A.inner, nlines, A.tw, ps);
}

template <int R1, int R2>
static hipError_t launch_4step(const double2* in, double2* out, const NatAxis& A, int inverse, double ps, bool stream,
                               hipStream_t st) {
  constexpr int NTS = R2 == 32 ? 2 * kNatThreads : kNatThreads;  // strided axes
  if (A.inner > 1) {
    if (stream) launch_4step_k<R1, R2, true, NTS, true>(in, out, A, inverse, ps, st);
    else launch_4step_k<R1, R2, true, NTS, false>(in, out, A, inverse, ps, st);
  } else {
    if (stream) launch_4step_k<R1, R2, false, kNatThreads, true>(in, out, A, inverse, ps, st);
    else launch_4step_k<R1, R2, false, kNatThreads, false>(in, out, A, inverse, ps, st);
  }
  return hipGetLastError();
}

// Returns hipErrorNotSupported when N has no register split.
static hipError_t launch_native_axis(const double2* in, double2* out, const NatAxis& A, int inverse, double ps,
                                     bool stream, hipStream_t st) {
  switch (A.N) {
    case 1024: return launch_4step<32, 32>(in, out, A, inverse, ps, stream, st);
    case 512: return launch_4step<16, 32>(in, out, A, inverse, ps, stream, st);
    case 256: return launch_4step<16, 16>(in, out, A, inverse, ps, stream, st);
    case 192: return launch_4step<12, 16>(in, out, A, inverse, ps, stream, st);
    case 128: return launch_4step<8, 16>(in, out, A, inverse, ps, stream, st);
    case 96: return launch_4step<6, 16>(in, out, A, inverse, ps, stream, st);
    case 64: return launch_4step<8, 8>(in, out, A, inverse, ps, stream, st);
    case 48: return launch_4step<6, 8>(in, out, A, inverse, ps, stream, st);
    case 32: return launch_4step<4, 8>(in, out, A, inverse, ps, stream, st);
    case 24: return launch_4step<3, 8>(in, out, A, inverse, ps, stream, st);
    case 16: return launch_4step<4, 4>(in, out, A, inverse, ps, stream, st);
    case 12: return launch_4step<3, 4>(in, out, A, inverse, ps, stream, st);
    case 8: return launch_4step<2, 4>(in, out, A, inverse, ps, stream, st);
    case 4: return launch_4step<2, 2>(in, out, A, inverse, ps, stream, st);
    default: return hipErrorNotSupported;
  }
}

__global__ void scale_kernel(void* data, int64_t n, double f, int tgt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (tgt == 0) ((double*)data)[i] *= f;
    else ((float*)data)[i] = (float)((double)((float*)data)[i] * f);
  }
}

hipError_t launch_scale(void* data, int64_t n_scalars, double factor, int tgt, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n_scalars + 255) / 256, (int64_t)1 << 20);
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, data, n_scalars, factor, tgt);
  return hipGetLastError();
}

static bool factor_radices(int64_t N, NatAxis& A) {
  int np = 0;
  int64_t m = N;
  while (m > 1) {
    int r;
    if (m % 8 == 0) r = 8;
    else if (m % 4 == 0) r = 4;
    else if (m % 2 == 0) r = 2;
    else if (m % 3 == 0) r = 3;
    else return false;
    if (np >= kMaxPasses) return false;
    A.radix[np++] = r;
    m /= r;
  }
  A.npass = np;
  return true;
}

void native_plan_destroy(NativePlan* np);

NativePlan* native_plan_create(const int64_t* n, std::string& err) {
  NativePlan* np = new NativePlan();
  for (int a = 0; a < 3; a++) {
    np->n[a] = n[a];
    NatAxis& A = np->ax[a];
    A.N = n[a];
    A.inner = 1;
    A.outer = 1;
    for (int b = a + 1; b < 3; b++) A.inner *= n[b];
    for (int b = 0; b < a; b++) A.outer *= n[b];
    if (A.N > kNatLdsComplex || !factor_radices(A.N, A)) {
      err = "unsupported native length";
      delete np;
      return nullptr;
    }
    int64_t B = kNatLdsComplex / A.N;
    if (B > 64) B = 64;
    for (int p = 0; p < A.npass; p++) {
      int64_t cap = (int64_t)kNatThreads * (kNatRegs / A.radix[p]) * A.radix[p] / A.N;
      if (B > cap) B = cap;
    }
    if (B < 1) {
      err = "native length too long";
      delete np;
      return nullptr;
    }
    A.B = (int)B;
    // twiddles: nearest doubles of (cos, -sin)(2 pi t / N), from a 2^62-scaled
    // double-double evaluation rounded to 53 bits
    std::vector<int64_t> q;
    quantised_roots(A.N, 61, q);
    std::vector<double2> tw(A.N);
    for (int64_t t = 0; t < A.N; t++) tw[t] = make_double2(std::ldexp((double)q[2 * t], -61),
                                                          std::ldexp((double)q[2 * t + 1], -61));
    void* d = nullptr;
    if (hipMalloc(&d, A.N * sizeof(double2)) != hipSuccess ||
        hipMemcpy(d, tw.data(), A.N * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
      err = "twiddle upload failed";
      native_plan_destroy(np);
      return nullptr;
    }
    np->allocs.push_back(d);
    A.tw = (const double2*)d;
  }
  return np;
}

void native_plan_destroy(NativePlan* np) {
  if (!np) return;
  for (void* d : np->allocs) hipFree(d);
  delete np;
}

hipError_t native_execute(NativePlan* np, const void* in, void* out, void* /*ws*/, int inverse, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)native_axis_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        kNatLdsComplex * 16);
    hipFuncSetAttribute((const void*)native_axis_kernel<-1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        kNatLdsComplex * 16);
    attr = true;
  }
  int64_t total = np->n[0] * np->n[1] * np->n[2];
  const bool stream = total * (int64_t)sizeof(double2) >= kNatStreamBytes;
  const double2* src = (const double2*)in;
  for (int k = 0; k < 3; k++) {
    int a = 2 - k;
    NatAxis A = np->ax[a];
    double ps = (inverse && k == 2) ? 1.0 / (double)total : 1.0;
    if (A.N == 1) {
      if (src != (const double2*)out || ps != 1.0) {
        hipError_t e = hipMemcpyAsync(out, src, total * sizeof(double2), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        if (ps != 1.0) {
          e = launch_scale(out, 2 * total, ps, 0, st);
          if (e != hipSuccess) return e;
        }
      }
      src = (const double2*)out;
      continue;
    }
    hipError_t e = launch_native_axis(src, (double2*)out, A, inverse, ps, stream, st);
    if (e == hipErrorNotSupported) {
      (void)hipGetLastError();
      int64_t nlines = A.outer * A.inner;
      int64_t grid = (nlines + A.B - 1) / A.B;
      size_t lds = (size_t)A.B * A.N * sizeof(double2);
      if (inverse)
        hipLaunchKernelGGL(native_axis_kernel<-1>, dim3((unsigned)grid), dim3(kNatThreads), lds, st, src,
                           (double2*)out, A, ps);
      else
        hipLaunchKernelGGL(native_axis_kernel<1>, dim3((unsigned)grid), dim3(kNatThreads), lds, st, src,
                           (double2*)out, A, ps);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    src = (const double2*)out;
  }
  return hipSuccess;
}

}  // namespace obfft
