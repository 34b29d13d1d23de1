/*
 * Exact-pipeline oracle of the Ozaki-Bailey 3-D FFT -- TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain definition of what the emulated transform computes.  The
 * method (residue GEMMs + CRT + Kulisch) reaches exactly this result; here it
 * is reached directly with 128-bit integers, so a reader can check it against
 * the paper by eye:
 *
 *   Bailey six-step with j = j1 + p*j2, k = k2 + q*k1 (Sec. 2, "The Bailey
 *   six-step FFT").  Stage 1 contracts over j2 for each column j1 with the
 *   length-q DFT matrix; stage 2 contracts over j1 for each column k2 with the
 *   twiddle-fused matrix F_p^(k2), whose entries are ONE quantised root
 *   omega_N^{j1 (k2 + q k1)} each (Sec. 4.1, Eq. twiddle-fusion).
 *
 *   Per column: one power-of-two scale shared by Re and Im (Alg. 1, scaling
 *   invariant): e = max ilogb over the nonzero parts, x~ = RNE(x 2^{(k-1)-e})
 *   with k = 53 (FP64 target) or 24 (FP32 target) (Sec. 2, Eq. ozaki and
 *   Eq. capacity).  Twiddles are integers scaled by 2^B, B = k - 1.
 *
 *   Complex product by the 3-real-GEMM Karatsuba split D = sum c a~,
 *   E = sum s b~, F = sum (c+s)(a~+b~); Re = D - E, Im = F - D - E (Sec. 2,
 *   complex CRT paragraph; Alg. 1).
 *
 *   The only rounding: y = RNE(Re * 2^{e-(k-1)-B}) in the target format
 *   (Sec. 5.1, correctly rounded pack).  The inverse normalisation by a
 *   power of two is an extra exponent on the last pack.
 *
 * Axes run in the order given (the product runs n3, n2, n1).  Data is complex
 * interleaved, C order, held in doubles for both targets (FP32-target values
 * are exactly representable).
 */
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

typedef struct {
  int prec;   /* significand bits of the target format: 53 or 24 */
  int tbits;  /* twiddle scale bits B = prec - 1 */
  int emin_q; /* exponent of the smallest subnormal: -1074 or -149 */
} fmt_t;

static fmt_t make_fmt(int precision) {
  fmt_t f;
  if (precision == 1) { f.prec = 24; f.tbits = 23; f.emin_q = -149; }
  else { f.prec = 53; f.tbits = 52; f.emin_q = -1074; }
  return f;
}

static int bitlen128(u128 a) {
  int n = 0;
  while (a) { a >>= 1; n++; }
  return n;
}

/* Correctly rounded R * 2^exp, significand `prec` bits, ties to even
 * (Sec. 5.1: the single rounding of the pipeline). */
double oracle_pack(i128 R, int exp, const fmt_t* f) {
  if (R == 0) return 0.0;
  int neg = R < 0;
  u128 a = neg ? (u128)(-(R + 1)) + 1 : (u128)R;
  int nb = bitlen128(a);
  int top = nb - 1 + exp;
  int qe = top - (f->prec - 1);
  if (qe < f->emin_q) qe = f->emin_q;
  int shift = qe - exp;
  u128 q;
  if (shift <= 0) {
    q = a << (-shift);
  } else if (shift > nb) {
    q = 0;
  } else {
    q = a >> shift;
    u128 r = a - (q << shift);
    u128 half = (u128)1 << (shift - 1);
    if (r > half || (r == half && (q & 1))) q++;
  }
  double v = ldexp((double)(uint64_t)q, qe);
  return neg ? -v : v;
}

/* Column exponent: max ilogb over the nonzero real and imaginary parts. */
static int column_exponent(const double* x, int64_t n, int64_t stride, int* e) {
  int best = INT_MIN;
  for (int64_t j = 0; j < n; j++) {
    const double* z = x + 2 * j * stride;
    if (z[0] != 0.0) { int t = ilogb(z[0]); if (t > best) best = t; }
    if (z[1] != 0.0) { int t = ilogb(z[1]); if (t > best) best = t; }
  }
  *e = best;
  return best != INT_MIN;
}

static int64_t quantise(double x, int shift) {
  return (int64_t)nearbyint(ldexp(x, shift));
}

/* One complex contraction column: out[t] = sum_s root(t, s) * x[s].
 * `rootidx(t, s)` is the exponent of the quantised root; `roots` holds
 * (cos, sin) integer pairs.  Writes the exact Re/Im integers when asked. */
typedef struct {
  const int64_t* roots; /* [N][2] */
  int64_t N, p, q;
  fmt_t f;
} line_ctx;

static void contract(const line_ctx* L, int stage, int64_t g, const double* col, int64_t K,
                     double* out, int64_t out_stride_c, int extra_shift,
                     i128* re_int, i128* im_int, int* exp_out) {
  int e;
  int64_t T = K; /* square DFT blocks */
  if (!column_exponent(col, K, 1, &e)) {
    for (int64_t t = 0; t < T; t++) {
      out[2 * t * out_stride_c] = 0.0;
      out[2 * t * out_stride_c + 1] = 0.0;
      if (re_int) { re_int[t] = 0; im_int[t] = 0; }
    }
    if (exp_out) *exp_out = INT_MIN;
    return;
  }
  if (exp_out) *exp_out = e;
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * 2 * K);
  int64_t* b = a + K;
  int qshift = (L->f.prec - 1) - e;
  for (int64_t s = 0; s < K; s++) {
    a[s] = quantise(col[2 * s], qshift);
    b[s] = quantise(col[2 * s + 1], qshift);
  }
  int pexp = e - (L->f.prec - 1) - L->f.tbits + extra_shift;
  for (int64_t t = 0; t < T; t++) {
    i128 D = 0, E = 0, F = 0;
    for (int64_t s = 0; s < K; s++) {
      int64_t idx;
      if (stage == 1) idx = (L->p * s * t) % L->N;               /* F_q[k2][j2] = w_N^{p j2 k2} */
      else idx = (s * (g + L->q * t)) % L->N;                     /* F_p^(k2)[k1][j1] = w_N^{j1 (k2 + q k1)} */
      int64_t c = L->roots[2 * idx], sn = L->roots[2 * idx + 1];
      D += (i128)c * a[s];
      E += (i128)sn * b[s];
      F += (i128)(c + sn) * (i128)(a[s] + b[s]);
    }
    i128 re = D - E, im = F - D - E;
    if (re_int) { re_int[t] = re; im_int[t] = im; }
    out[2 * t * out_stride_c] = oracle_pack(re, pexp, &L->f);
    out[2 * t * out_stride_c + 1] = oracle_pack(im, pexp, &L->f);
  }
  free(a);
}

/* Stage 1 of one contiguous line X[N] -> Y'[N] (slot j1 + p*k2 holds Y'_{j1,k2}). */
static void stage1(const line_ctx* L, const double* X, double* Y, i128* ri, i128* ii, int* ex) {
  int64_t p = L->p, q = L->q;
  double* col = (double*)malloc(sizeof(double) * 2 * q);
  double* res = (double*)malloc(sizeof(double) * 2 * q);
  i128* rr = ri ? (i128*)malloc(sizeof(i128) * 2 * q) : NULL;
  for (int64_t j1 = 0; j1 < p; j1++) {
    for (int64_t j2 = 0; j2 < q; j2++) {
      col[2 * j2] = X[2 * (j1 + p * j2)];
      col[2 * j2 + 1] = X[2 * (j1 + p * j2) + 1];
    }
    contract(L, 1, j1, col, q, res, 1, 0, rr, rr ? rr + q : NULL, ex ? ex + j1 : NULL);
    for (int64_t k2 = 0; k2 < q; k2++) {
      Y[2 * (j1 + p * k2)] = res[2 * k2];
      Y[2 * (j1 + p * k2) + 1] = res[2 * k2 + 1];
      if (ri) { ri[j1 + p * k2] = rr[k2]; ii[j1 + p * k2] = rr[q + k2]; }
    }
  }
  free(col); free(res); free(rr);
}

/* Stage 2 of one line Y'[N] -> Z[N] (slot k2 + q*k1 holds Z_{k1,k2}). */
static void stage2(const line_ctx* L, const double* Y, double* Z, int extra_shift,
                   i128* ri, i128* ii, int* ex) {
  int64_t p = L->p, q = L->q;
  double* res = (double*)malloc(sizeof(double) * 2 * p);
  i128* rr = ri ? (i128*)malloc(sizeof(i128) * 2 * p) : NULL;
  for (int64_t k2 = 0; k2 < q; k2++) {
    contract(L, 2, k2, Y + 2 * p * k2, p, res, 1, extra_shift, rr, rr ? rr + p : NULL,
             ex ? ex + k2 : NULL);
    for (int64_t k1 = 0; k1 < p; k1++) {
      Z[2 * (k2 + q * k1)] = res[2 * k1];
      Z[2 * (k2 + q * k1) + 1] = res[2 * k1 + 1];
      if (ri) { ri[k2 + q * k1] = rr[k1]; ii[k2 + q * k1] = rr[p + k1]; }
    }
  }
  free(res); free(rr);
}

/* ---- exported: one line, one stage, with the exact integers (checkpoints) ---- */

static void split128(i128 v, int64_t* hi, uint64_t* lo) {
  *lo = (uint64_t)v;
  *hi = (int64_t)(v >> 64);
}

/* stage = 1: input X (natural order), output Y' slots; stage = 2: input Y',
 * output Z slots.  Exact integers returned as (hi, lo) 64-bit halves. */
int oracle_line_stage(const double* in, double* out, int64_t N, int64_t p, int64_t q,
                      const int64_t* roots, int precision, int stage, int extra_shift,
                      int64_t* re_hi, uint64_t* re_lo, int64_t* im_hi, uint64_t* im_lo,
                      int* col_exp) {
  if (p * q != N || p < 1 || q < 1) return -1;
  line_ctx L = {roots, N, p, q, make_fmt(precision)};
  i128* ri = (i128*)malloc(sizeof(i128) * 2 * N);
  i128* ii = ri + N;
  if (stage == 1) stage1(&L, in, out, ri, ii, col_exp);
  else stage2(&L, in, out, extra_shift, ri, ii, col_exp);
  for (int64_t t = 0; t < N; t++) {
    if (re_hi) split128(ri[t], re_hi + t, re_lo + t);
    if (im_hi) split128(ii[t], im_hi + t, im_lo + t);
  }
  free(ri);
  return 0;
}

/* ---- exported: the whole 3-D transform ---- */

typedef struct {
  double* data;
  int64_t N, inner, outer;
  int64_t line_begin, line_end;
  line_ctx L;
  int extra_shift;
} axis_job;

static void* axis_worker(void* arg) {
  axis_job* J = (axis_job*)arg;
  int64_t N = J->N;
  double* X = (double*)malloc(sizeof(double) * 2 * N);
  double* Y = (double*)malloc(sizeof(double) * 2 * N);
  for (int64_t line = J->line_begin; line < J->line_end; line++) {
    int64_t o = line / J->inner, i = line % J->inner;
    double* base = J->data + 2 * (o * N * J->inner + i);
    for (int64_t j = 0; j < N; j++) {
      X[2 * j] = base[2 * j * J->inner];
      X[2 * j + 1] = base[2 * j * J->inner + 1];
    }
    stage1(&J->L, X, Y, NULL, NULL, NULL);
    stage2(&J->L, Y, X, J->extra_shift, NULL, NULL, NULL);
    for (int64_t j = 0; j < N; j++) {
      base[2 * j * J->inner] = X[2 * j];
      base[2 * j * J->inner + 1] = X[2 * j + 1];
    }
  }
  free(X); free(Y);
  return NULL;
}

/* n[3] = (n1, n2, n3); p[a], q[a] factor n[a]; order[] lists axes (0 = n1);
 * roots[a] = quantised roots for length n[a]; final_shift is added to the
 * exponent of the last pack (e.g. -log2(n1 n2 n3) for the inverse). */
int oracle_fft3(const double* in, double* out, const int64_t* n, const int64_t* p,
                const int64_t* q, const int* order, const int64_t* const* roots,
                int precision, int final_shift, int nthreads) {
  int64_t total = n[0] * n[1] * n[2];
  if (in != out) memcpy(out, in, sizeof(double) * 2 * total);
  if (nthreads < 1) nthreads = 1;
  for (int step = 0; step < 3; step++) {
    int a = order[step];
    if (p[a] * q[a] != n[a]) return -1;
    int64_t inner = 1, outer = 1;
    for (int b = a + 1; b < 3; b++) inner *= n[b];
    for (int b = 0; b < a; b++) outer *= n[b];
    int64_t lines = inner * outer;
    int nt = nthreads;
    if (nt > lines) nt = (int)lines;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
    axis_job* jobs = (axis_job*)malloc(sizeof(axis_job) * nt);
    for (int t = 0; t < nt; t++) {
      jobs[t].data = out;
      jobs[t].N = n[a];
      jobs[t].inner = inner;
      jobs[t].outer = outer;
      jobs[t].line_begin = lines * t / nt;
      jobs[t].line_end = lines * (t + 1) / nt;
      jobs[t].L.roots = roots[a];
      jobs[t].L.N = n[a];
      jobs[t].L.p = p[a];
      jobs[t].L.q = q[a];
      jobs[t].L.f = make_fmt(precision);
      jobs[t].extra_shift = (step == 2) ? final_shift : 0;
      pthread_create(&th[t], NULL, axis_worker, &jobs[t]);
    }
    for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
    free(th); free(jobs);
  }
  return 0;
}

/* Packs one exact integer (given as hi/lo halves) -- exposed so tests can pin
 * the rounding against Python's correctly rounded int -> float. */
double oracle_pack_hilo(int64_t hi, uint64_t lo, int exp, int precision) {
  i128 v = ((i128)hi << 64) | (i128)lo;
  fmt_t f = make_fmt(precision);
  return oracle_pack(v, exp, &f);
}

/* ---- exported: independent contiguous lines (both stages of one axis pass) ----
 * Used to time a bounded sample of a large transform: every axis pass of the
 * 3-D transform is exactly this per-line work on N^2 lines. */
int oracle_lines(const double* in, double* out, int64_t nlines, int64_t N, int64_t p, int64_t q,
                 const int64_t* roots, int precision, int nthreads) {
  if (p * q != N) return -1;
  if (in != out) memcpy(out, in, sizeof(double) * 2 * nlines * N);
  if (nthreads < 1) nthreads = 1;
  int nt = nthreads;
  if (nt > nlines) nt = (int)nlines;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
  axis_job* jobs = (axis_job*)malloc(sizeof(axis_job) * nt);
  for (int t = 0; t < nt; t++) {
    jobs[t].data = out;
    jobs[t].N = N;
    jobs[t].inner = 1;
    jobs[t].outer = nlines;
    jobs[t].line_begin = nlines * t / nt;
    jobs[t].line_end = nlines * (t + 1) / nt;
    jobs[t].L.roots = roots;
    jobs[t].L.N = N;
    jobs[t].L.p = p;
    jobs[t].L.q = q;
    jobs[t].L.f = make_fmt(precision);
    jobs[t].extra_shift = 0;
    pthread_create(&th[t], NULL, axis_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th); free(jobs);
  return 0;
}

/* ---- exported: one output position k of every line (the cost cone) ----
 * Output k = k2 + q k1 of a line needs, from stage 1, the k2-th output of
 * every column j1 (each column still needs all its elements for its
 * exponent), then one stage-2 contraction.  Same definitions as above,
 * evaluated only where the sampled output depends on them. */
typedef struct {
  const double* in;
  double* out;
  int64_t N, k, begin, end;
  line_ctx L;
} cone_job;

static void contract_one(const line_ctx* L, int stage, int64_t g, const double* col, int64_t K,
                         int64_t t, double* out2) {
  int e;
  if (!column_exponent(col, K, 1, &e)) { out2[0] = 0.0; out2[1] = 0.0; return; }
  int qshift = (L->f.prec - 1) - e;
  int pexp = e - (L->f.prec - 1) - L->f.tbits;
  i128 D = 0, E = 0, F = 0;
  for (int64_t s = 0; s < K; s++) {
    int64_t a = quantise(col[2 * s], qshift), b = quantise(col[2 * s + 1], qshift);
    int64_t idx = stage == 1 ? (L->p * s * t) % L->N : (s * (g + L->q * t)) % L->N;
    int64_t c = L->roots[2 * idx], sn = L->roots[2 * idx + 1];
    D += (i128)c * a;
    E += (i128)sn * b;
    F += (i128)(c + sn) * (i128)(a + b);
  }
  out2[0] = oracle_pack(D - E, pexp, &L->f);
  out2[1] = oracle_pack(F - D - E, pexp, &L->f);
}

static void* cone_worker(void* arg) {
  cone_job* J = (cone_job*)arg;
  const line_ctx* L = &J->L;
  int64_t N = J->N, p = L->p, q = L->q;
  int64_t k2 = J->k % q, k1 = J->k / q;
  double* col = (double*)malloc(sizeof(double) * 2 * (p > q ? p : q));
  double* y = (double*)malloc(sizeof(double) * 2 * p);
  for (int64_t line = J->begin; line < J->end; line++) {
    const double* X = J->in + 2 * N * line;
    for (int64_t j1 = 0; j1 < p; j1++) {
      for (int64_t j2 = 0; j2 < q; j2++) {
        col[2 * j2] = X[2 * (j1 + p * j2)];
        col[2 * j2 + 1] = X[2 * (j1 + p * j2) + 1];
      }
      contract_one(L, 1, j1, col, q, k2, y + 2 * j1);
    }
    contract_one(L, 2, k2, y, p, k1, J->out + 2 * line);
  }
  free(col); free(y);
  return NULL;
}

int oracle_lines_at(const double* in, double* out, int64_t nlines, int64_t N, int64_t p, int64_t q,
                    const int64_t* roots, int precision, int64_t k, int nthreads) {
  if (p * q != N || k < 0 || k >= N) return -1;
  if (nthreads < 1) nthreads = 1;
  int nt = nthreads;
  if (nt > nlines) nt = (int)nlines;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nt);
  cone_job* jobs = (cone_job*)malloc(sizeof(cone_job) * nt);
  for (int t = 0; t < nt; t++) {
    jobs[t].in = in;
    jobs[t].out = out;
    jobs[t].N = N;
    jobs[t].k = k;
    jobs[t].begin = nlines * t / nt;
    jobs[t].end = nlines * (t + 1) / nt;
    jobs[t].L.roots = roots;
    jobs[t].L.N = N;
    jobs[t].L.p = p;
    jobs[t].L.q = q;
    jobs[t].L.f = make_fmt(precision);
    pthread_create(&th[t], NULL, cone_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th); free(jobs);
  return 0;
}
