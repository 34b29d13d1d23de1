/*
 * Double-double DFT oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * The accuracy reference: the separable 3-D DFT
 *     X[k1,k2,k3] = sum_j x[j1,j2,j3] w_n1^{j1 k1} w_n2^{j2 k2} w_n3^{j3 k3}
 * (the problem statement of Sec. 2, "The Bailey six-step FFT", applied per
 * axis), evaluated in double-double arithmetic (about 106 significand bits)
 * with twiddles supplied as double-double values of exp(-+2 pi i t / n).
 *
 * Each 1-D transform is a textbook recursive mixed-radix decimation in time:
 * n = r m with r the smallest prime factor; r sub-transforms of length m on
 * the decimated sequences, then the direct length-r combination with the
 * twiddles w_n^{a (k + m b)}.  Nothing else is reordered or fused.
 *
 * Compile with -ffp-contract=off: the error-free transformations rely on it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } ddc;

static inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  dd r = {s, (a - (s - bb)) + (b - bb)};
  return r;
}

static inline dd quick_two_sum(double a, double b) {
  double s = a + b;
  dd r = {s, b - (s - a)};
  return r;
}

static inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

static inline dd dd_neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }

static inline dd dd_mul(dd a, dd b) {
  double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p, e);
}

static inline ddc ddc_mul(ddc a, ddc b) {
  ddc r;
  r.re = dd_add(dd_mul(a.re, b.re), dd_neg(dd_mul(a.im, b.im)));
  r.im = dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re));
  return r;
}

static inline ddc ddc_add(ddc a, ddc b) {
  ddc r = {dd_add(a.re, b.re), dd_add(a.im, b.im)};
  return r;
}

static int64_t smallest_factor(int64_t n) {
  for (int64_t r = 2; r * r <= n; r++)
    if (n % r == 0) return r;
  return n;
}

/* out[0..n) = DFT_n of in[0], in[stride], ...; tw holds w_twN^t, n | twN. */
static void fft_rec(const ddc* in, int64_t stride, ddc* out, int64_t n, const ddc* tw,
                    int64_t twN, ddc* scratch) {
  if (n == 1) { out[0] = in[0]; return; }
  int64_t r = smallest_factor(n), m = n / r;
  for (int64_t a = 0; a < r; a++) fft_rec(in + a * stride, stride * r, out + a * m, m, tw, twN, scratch);
  int64_t step = twN / n;
  for (int64_t k = 0; k < m; k++) {
    for (int64_t b = 0; b < r; b++) {
      ddc acc = {{0.0, 0.0}, {0.0, 0.0}};
      for (int64_t a = 0; a < r; a++) {
        int64_t t = (a * (k + m * b)) % n;
        acc = ddc_add(acc, ddc_mul(tw[t * step], out[a * m + k]));
      }
      scratch[k + m * b] = acc;
    }
  }
  memcpy(out, scratch, sizeof(ddc) * n);
}

typedef struct {
  ddc* data;
  int64_t N, inner;
  int64_t line_begin, line_end;
  const ddc* tw;
} dd_job;

static void* dd_worker(void* arg) {
  dd_job* J = (dd_job*)arg;
  int64_t N = J->N;
  ddc* x = (ddc*)malloc(sizeof(ddc) * N * 3);
  ddc* y = x + N;
  ddc* s = y + N;
  for (int64_t line = J->line_begin; line < J->line_end; line++) {
    int64_t o = line / J->inner, i = line % J->inner;
    ddc* base = J->data + o * N * J->inner + i;
    for (int64_t j = 0; j < N; j++) x[j] = base[j * J->inner];
    fft_rec(x, 1, y, N, J->tw, N, s);
    for (int64_t j = 0; j < N; j++) base[j * J->inner] = y[j];
  }
  free(x);
  return NULL;
}

/* in: complex double interleaved; out: (re_hi, re_lo, im_hi, im_lo) per element;
 * tw[a]: n[a] x 4 doubles (re_hi, re_lo, im_hi, im_lo) of w_{n[a]}^t. */
int oracle_dd_fft3(const double* in, double* out, const int64_t* n, const double* const* tw,
                   int nthreads) {
  int64_t total = n[0] * n[1] * n[2];
  ddc* d = (ddc*)out;
  for (int64_t e = 0; e < total; e++) {
    d[e].re.hi = in[2 * e];
    d[e].re.lo = 0.0;
    d[e].im.hi = in[2 * e + 1];
    d[e].im.lo = 0.0;
  }
  if (nthreads < 1) nthreads = 1;
  for (int a = 2; a >= 0; a--) {
    int64_t inner = 1, outer = 1;
    for (int b = a + 1; b < 3; b++) inner *= n[b];
    for (int b = 0; b < a; b++) outer *= n[b];
    int64_t lines = inner * outer;
    int nt = nthreads;
    if (nt > lines) nt = (int)lines;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
    dd_job* jobs = (dd_job*)malloc(sizeof(dd_job) * nt);
    for (int t = 0; t < nt; t++) {
      jobs[t].data = d;
      jobs[t].N = n[a];
      jobs[t].inner = inner;
      jobs[t].line_begin = lines * t / nt;
      jobs[t].line_end = lines * (t + 1) / nt;
      jobs[t].tw = (const ddc*)tw[a];
      pthread_create(&th[t], NULL, dd_worker, &jobs[t]);
    }
    for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
    free(th); free(jobs);
  }
  return 0;
}

/* ---- exported: sampled lines (the cost cone of a few outputs of a large transform) ----
 * Both routines take and return double-double complex values, four doubles
 * per element (re_hi, re_lo, im_hi, im_lo), so that a chain of them (one
 * output position of every line of the first axis, then of the second, then
 * the whole third-axis line) never rounds to binary64 in between.  The
 * definition is the same separable DFT as above; only the outputs that the
 * sampled line depends on are evaluated. */

typedef struct {
  const double* in;
  int in_z;  /* input is complex binary64 (re, im) rather than double-double */
  ddc* out;
  int64_t N, k, begin, end;
  const ddc* tw;
} dd_cone_job;

static void* dd_cone_worker(void* arg) {
  dd_cone_job* J = (dd_cone_job*)arg;
  int64_t N = J->N;
  for (int64_t line = J->begin; line < J->end; line++) {
    ddc acc = {{0.0, 0.0}, {0.0, 0.0}};
    for (int64_t j = 0; j < N; j++) {
      ddc x;
      if (J->in_z) {
        const double* z = J->in + 2 * (line * N + j);
        x.re.hi = z[0]; x.re.lo = 0.0; x.im.hi = z[1]; x.im.lo = 0.0;
      } else {
        x = ((const ddc*)J->in)[line * N + j];
      }
      acc = ddc_add(acc, ddc_mul(J->tw[(j * J->k) % N], x));
    }
    J->out[line] = acc;
  }
  return NULL;
}

/* out[l] = sum_j in[l N + j] w_N^{j k}: output position k of the DFT of every
 * contiguous length-N line (direct sum, j ascending).  in_z = 1: the input is
 * complex binary64 (two doubles per element), else double-double. */
int oracle_dd_lines_at(const double* in, int in_z, double* out, int64_t nlines, int64_t N, int64_t k,
                       const double* tw, int nthreads) {
  if (N < 1 || k < 0 || k >= N) return -1;
  if (nthreads < 1) nthreads = 1;
  int nt = nthreads;
  if (nt > nlines) nt = (int)nlines;
  if (nt < 1) return 0;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
  dd_cone_job* jobs = (dd_cone_job*)malloc(sizeof(dd_cone_job) * nt);
  for (int t = 0; t < nt; t++) {
    jobs[t].in = in;
    jobs[t].in_z = in_z;
    jobs[t].out = (ddc*)out;
    jobs[t].N = N;
    jobs[t].k = k;
    jobs[t].begin = nlines * t / nt;
    jobs[t].end = nlines * (t + 1) / nt;
    jobs[t].tw = (const ddc*)tw;
    pthread_create(&th[t], NULL, dd_cone_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th); free(jobs);
  return 0;
}

/* The whole length-N DFT of every contiguous line, double-double in and out. */
int oracle_dd_lines(const double* in, double* out, int64_t nlines, int64_t N, const double* tw) {
  if (N < 1) return -1;
  ddc* s = (ddc*)malloc(sizeof(ddc) * N);
  for (int64_t line = 0; line < nlines; line++)
    fft_rec((const ddc*)in + line * N, 1, (ddc*)out + line * N, N, (const ddc*)tw, N, s);
  free(s);
  return 0;
}
