/*
 * oracle_fft.c -- plain, slow, FP64 CPU oracle for the FFT -> filter -> IFFT path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * Every routine works in double precision (the paper does not state its own
 * precision) on interleaved (re, im) arrays.  The arithmetic follows the paper
 * ("Construction of an algorithm in parallel for the Fast Fourier Transform",
 * Higuera, Sarria, Fonseca, Idarraga):
 *
 *   orc_dft_direct   the definition, eq. (E2) / (coefFourier) with the sign and
 *                    scale as arguments: out[k] = s * sum_j in[j] e^{sgn 2 pi i kj/N}.
 *                    O(N^2); twiddle angle from the exact integer (j*k) mod N.
 *   orc_fft_fwd      Section 2: the radix-2 tree of interpolating polynomials
 *                    P_k^(n).  Leaves in bit-reversed order, levels 1..m merge
 *                    two half-length polynomials with the factors Z of Table 2,
 *                    then the 1/N of eq. (E2).
 *   orc_fft_inv      Section 3: the inverse evaluated through the forward
 *                    transform, p(2 pi - x_k) = N * FFT(c)[k], read "in
 *                    contrary order" k -> (N - k) mod N.  Unscaled, eq. (E3).
 *   orc_fft2_fwd     Section 5, eq. (5): FFT on rows, multiply by M, FFT on
 *                    columns (factor 1/N, N = number of rows).
 *   orc_fft2_inv     Section 5, 2D-IDFT: unscaled inverse on columns and rows,
 *                    then the factor 1/M.
 *   orc_filter2      Section 6: multiply a real filter into the real and the
 *                    imaginary part of the spectrum, then the 2D-IDFT.
 *   orc_mask_*       the masks, evaluated in FP64 (Gaussian and Butterworth on
 *                    fftfreq radii; the paper's disc filter, eq. (filtro)).
 *   orc_loss_grad    mean |y - c|^2 of y = 2D-IDFT(m * 2D-DFT(x)) and its exact
 *                    gradient with respect to the real mask m (not in the paper;
 *                    derived from eq. (5) and the 2D-IDFT definition).
 *
 * Threads (pthreads) only split independent rows, columns or batch entries; the
 * arithmetic order inside one transform never depends on the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_SIZE -2
#define ORC_ERR_NOMEM -6

static const double ORC_TWO_PI = 6.28318530717958647692528676655900577;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static int ilog2(int64_t n) {
  int m = 0;
  while (((int64_t)1 << m) < n) ++m;
  return m;
}

/* Z[t] = e^{-2 pi i t / n} (Table 2), from the exact integer t in [0, n). */
static void z_factor(int64_t t, int64_t n, double* re, double* im) {
  double a = ORC_TWO_PI * (double)t / (double)n;
  *re = cos(a);
  *im = -sin(a);
}

/* ------------------------------------------------------------------------- */
/* Definition: direct O(N^2) sum.                                             */
/* ------------------------------------------------------------------------- */
int orc_dft_direct(int64_t n, const double* in, double* out, int sign, double scale) {
  if (n < 1 || !in || !out || (sign != 1 && sign != -1)) return ORC_ERR_ARG;
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      int64_t t = (int64_t)(((unsigned __int128)j * (unsigned __int128)k) % (unsigned __int128)n);
      double wr, wi;
      z_factor(t, n, &wr, &wi); /* e^{-2 pi i t/n} */
      if (sign > 0) wi = -wi;   /* e^{+2 pi i t/n} */
      double xr = in[2 * j], xi = in[2 * j + 1];
      sr += xr * wr - xi * wi;
      si += xr * wi + xi * wr;
    }
    out[2 * k] = scale * sr;
    out[2 * k + 1] = scale * si;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Section 2: the tree of interpolating polynomials.                          */
/* ------------------------------------------------------------------------- */

/* Bit reversal of p over m bits: the leaf order of the tree (N=8 gives
 * C(0),C(4),C(2),C(6),C(1),C(5),C(3),C(7)). */
static int64_t bitrev(int64_t p, int m) {
  int64_t r = 0;
  for (int b = 0; b < m; ++b) r |= ((p >> b) & 1) << (m - 1 - b);
  return r;
}

/* Runs the tree on c (length n = 2^m, in place, interleaved) up to level
 * `levels` (0..m).  After level n the array is made of blocks of 2^n values;
 * each block holds the 2^n coefficients of one polynomial P^(n) (unscaled).
 * No 1/N scaling is applied here. */
static void tree_levels(int64_t n, double* c, int levels) {
  int m = ilog2(n);
  /* level 0: the leaves, bit-reversed order */
  for (int64_t p = 0; p < n; ++p) {
    int64_t q = bitrev(p, m);
    if (q > p) {
      double tr = c[2 * p], ti = c[2 * p + 1];
      c[2 * p] = c[2 * q];
      c[2 * p + 1] = c[2 * q + 1];
      c[2 * q] = tr;
      c[2 * q + 1] = ti;
    }
  }
  /* levels 1..levels: merge pairs of half-length polynomials */
  for (int lev = 1; lev <= levels; ++lev) {
    int64_t s = (int64_t)1 << lev; /* length of a merged block */
    int64_t h = s >> 1;
    for (int64_t b = 0; b < n; b += s) {
      for (int64_t j = 0; j < h; ++j) {
        double wr, wi;
        z_factor(j * (n / s), n, &wr, &wi); /* Z[j N/s] = e^{-2 pi i j/s} */
        double* lo = c + 2 * (b + j);
        double* hi = c + 2 * (b + j + h);
        double tr = wr * hi[0] - wi * hi[1];
        double ti = wr * hi[1] + wi * hi[0];
        hi[0] = lo[0] - tr;
        hi[1] = lo[1] - ti;
        lo[0] = lo[0] + tr;
        lo[1] = lo[1] + ti;
      }
    }
  }
}

/* Exposed for the structural test of the worked 8-point example: copies in to
 * out and stops the tree after `levels` levels. */
int orc_tree_partial(int64_t n, const double* in, double* out, int levels) {
  if (!is_pow2(n)) return ORC_ERR_SIZE;
  if (!in || !out || levels < 0 || levels > ilog2(n)) return ORC_ERR_ARG;
  memcpy(out, in, sizeof(double) * 2 * (size_t)n);
  tree_levels(n, out, levels);
  return ORC_OK;
}

/* eq. (E2): H(k) = (1/N) sum_j f_j e^{-2 pi i kj/N}, batch of contiguous rows. */
int orc_fft_fwd(int64_t n, int64_t batch, const double* in, double* out) {
  if (!is_pow2(n)) return ORC_ERR_SIZE;
  if (batch < 0 || (batch > 0 && (!in || !out))) return ORC_ERR_ARG;
  for (int64_t b = 0; b < batch; ++b) {
    double* o = out + 2 * b * n;
    memmove(o, in + 2 * b * n, sizeof(double) * 2 * (size_t)n);
    tree_levels(n, o, ilog2(n));
    for (int64_t k = 0; k < 2 * n; ++k) o[k] /= (double)n;
  }
  return ORC_OK;
}

/* Section 3: f[(N-k) mod N] = N * FFT(c)[k]; unscaled inverse of eq. (E3). */
int orc_fft_inv(int64_t n, int64_t batch, const double* in, double* out) {
  if (!is_pow2(n)) return ORC_ERR_SIZE;
  if (batch < 0 || (batch > 0 && (!in || !out))) return ORC_ERR_ARG;
  double* g = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  if (!g) return ORC_ERR_NOMEM;
  for (int64_t b = 0; b < batch; ++b) {
    memcpy(g, in + 2 * b * n, sizeof(double) * 2 * (size_t)n);
    tree_levels(n, g, ilog2(n));
    for (int64_t k = 0; k < 2 * n; ++k) g[k] /= (double)n; /* FFT(c) */
    double* o = out + 2 * b * n;
    for (int64_t k = 0; k < n; ++k) {
      int64_t d = (n - k) % n; /* contrary order */
      o[2 * d] = (double)n * g[2 * k];
      o[2 * d + 1] = (double)n * g[2 * k + 1];
    }
  }
  free(g);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* A minimal range splitter over pthreads.                                    */
/* ------------------------------------------------------------------------- */
typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi);
typedef struct {
  range_fn fn;
  void* ctx;
  int64_t lo, hi;
} range_job;

static void* range_thread(void* p) {
  range_job* j = (range_job*)p;
  j->fn(j->ctx, j->lo, j->hi);
  return NULL;
}

static void parallel_range(int nthreads, int64_t count, range_fn fn, void* ctx) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((int64_t)nthreads > count) nthreads = (int)(count > 0 ? count : 1);
  if (nthreads == 1) {
    fn(ctx, 0, count);
    return;
  }
  pthread_t th[256];
  range_job jobs[256];
  int started[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].fn = fn;
    jobs[t].ctx = ctx;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
    started[t] = pthread_create(&th[t], NULL, range_thread, &jobs[t]) == 0;
    if (!started[t]) range_thread(&jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t)
    if (started[t]) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Section 5: 2D transforms on row-major [rows N][cols M] matrices.           */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t rows, cols;
  double* a; /* in/out, row-major interleaved */
  int inverse;
} pass_ctx;

/* FFT on rows, then multiplication by M (forward); unscaled inverse on rows. */
static void rows_range(void* p, int64_t lo, int64_t hi) {
  pass_ctx* c = (pass_ctx*)p;
  int64_t M = c->cols;
  for (int64_t x = lo; x < hi; ++x) {
    double* row = c->a + 2 * x * M;
    if (c->inverse) {
      orc_fft_inv(M, 1, row, row);
    } else {
      orc_fft_fwd(M, 1, row, row);
      for (int64_t k = 0; k < 2 * M; ++k) row[k] *= (double)M;
    }
  }
}

/* FFT (with its 1/N) or unscaled inverse on columns. */
static void cols_range(void* p, int64_t lo, int64_t hi) {
  pass_ctx* c = (pass_ctx*)p;
  int64_t N = c->rows, M = c->cols;
  double* col = (double*)malloc(sizeof(double) * 2 * (size_t)N);
  if (!col) return;
  for (int64_t v = lo; v < hi; ++v) {
    for (int64_t x = 0; x < N; ++x) {
      col[2 * x] = c->a[2 * (x * M + v)];
      col[2 * x + 1] = c->a[2 * (x * M + v) + 1];
    }
    if (c->inverse)
      orc_fft_inv(N, 1, col, col);
    else
      orc_fft_fwd(N, 1, col, col);
    for (int64_t x = 0; x < N; ++x) {
      c->a[2 * (x * M + v)] = col[2 * x];
      c->a[2 * (x * M + v) + 1] = col[2 * x + 1];
    }
  }
  free(col);
}

static int check2(int64_t N, int64_t M) {
  if (!is_pow2(N) || !is_pow2(M)) return ORC_ERR_SIZE;
  return ORC_OK;
}

/* eq. (5): F(u,v) = (1/N) sum_x sum_y f(x,y) e^{-2 pi i (ux/N + vy/M)},
 * evaluated as FFT on rows -> x M -> FFT on columns. */
static void fft2_fwd_one(int64_t N, int64_t M, double* a, int nthreads) {
  pass_ctx c = {N, M, a, 0};
  parallel_range(nthreads, N, rows_range, &c);
  parallel_range(nthreads, M, cols_range, &c);
}

/* 2D-IDFT: f(x,y) = (1/M) sum_u sum_v F(u,v) e^{+2 pi i (ux/N + vy/M)}. */
static void fft2_inv_one(int64_t N, int64_t M, double* a, int nthreads) {
  pass_ctx c = {N, M, a, 1};
  parallel_range(nthreads, M, cols_range, &c);
  parallel_range(nthreads, N, rows_range, &c);
  for (int64_t i = 0; i < 2 * N * M; ++i) a[i] /= (double)M;
}

int orc_fft2_fwd(int64_t N, int64_t M, int64_t batch, const double* in, double* out, int nthreads) {
  int e = check2(N, M);
  if (e) return e;
  if (batch < 0 || (batch > 0 && (!in || !out))) return ORC_ERR_ARG;
  for (int64_t b = 0; b < batch; ++b) {
    double* o = out + 2 * b * N * M;
    memmove(o, in + 2 * b * N * M, sizeof(double) * 2 * (size_t)(N * M));
    fft2_fwd_one(N, M, o, nthreads);
  }
  return ORC_OK;
}

int orc_fft2_inv(int64_t N, int64_t M, int64_t batch, const double* in, double* out, int nthreads) {
  int e = check2(N, M);
  if (e) return e;
  if (batch < 0 || (batch > 0 && (!in || !out))) return ORC_ERR_ARG;
  for (int64_t b = 0; b < batch; ++b) {
    double* o = out + 2 * b * N * M;
    memmove(o, in + 2 * b * N * M, sizeof(double) * 2 * (size_t)(N * M));
    fft2_inv_one(N, M, o, nthreads);
  }
  return ORC_OK;
}

/* Section 6: g = 2D-IDFT(H . 2D-DFT(f)) with a real mask H [N][M] shared by
 * the whole batch; H scales the real and the imaginary part alike. */
int orc_filter2(int64_t N, int64_t M, int64_t batch, const double* in, const double* mask, double* out,
                int nthreads) {
  int e = check2(N, M);
  if (e) return e;
  if (batch < 0 || (batch > 0 && (!in || !out || !mask))) return ORC_ERR_ARG;
  for (int64_t b = 0; b < batch; ++b) {
    double* o = out + 2 * b * N * M;
    memmove(o, in + 2 * b * N * M, sizeof(double) * 2 * (size_t)(N * M));
    fft2_fwd_one(N, M, o, nthreads);
    for (int64_t i = 0; i < N * M; ++i) {
      o[2 * i] *= mask[i];
      o[2 * i + 1] *= mask[i];
    }
    fft2_inv_one(N, M, o, nthreads);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Masks, FP64.  Frequencies on fftfreq's grid: k/n for k < (n+1)/2, else (k-n)/n. */
/* ------------------------------------------------------------------------- */
static double freq(int64_t k, int64_t n) { return (double)(k < (n + 1) / 2 ? k : k - n) / (double)n; }

int orc_mask_gaussian(int64_t N, int64_t M, double sigma_f, double* out) {
  if (N < 1 || M < 1 || !out || !(sigma_f > 0.0)) return ORC_ERR_ARG;
  for (int64_t u = 0; u < N; ++u)
    for (int64_t v = 0; v < M; ++v) {
      double fu = freq(u, N), fv = freq(v, M);
      double r2 = fu * fu + fv * fv;
      out[u * M + v] = exp(-r2 / (2.0 * sigma_f * sigma_f));
    }
  return ORC_OK;
}

int orc_mask_butterworth(int64_t N, int64_t M, double cutoff, int order, double* out) {
  if (N < 1 || M < 1 || !out || !(cutoff > 0.0) || order < 1) return ORC_ERR_ARG;
  for (int64_t u = 0; u < N; ++u)
    for (int64_t v = 0; v < M; ++v) {
      double fu = freq(u, N), fv = freq(v, M);
      double r = sqrt(fu * fu + fv * fv);
      out[u * M + v] = 1.0 / (1.0 + pow(r / cutoff, 2.0 * (double)order));
    }
  return ORC_OK;
}

/* eq. (filtro): 0 where sqrt((u-c1)^2 + (v-c2)^2) <= b, 1 elsewhere. */
int orc_mask_disc(int64_t N, int64_t M, double b, double c1, double c2, double* out) {
  if (N < 1 || M < 1 || !out || !(b > 0.0)) return ORC_ERR_ARG;
  for (int64_t u = 0; u < N; ++u)
    for (int64_t v = 0; v < M; ++v) {
      double du = (double)u - c1, dv = (double)v - c2;
      out[u * M + v] = (sqrt(du * du + dv * dv) <= b) ? 0.0 : 1.0;
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Learnable mask: loss and gradient.                                          */
/*   X_b = 2D-DFT(x_b),  y_b = 2D-IDFT(m . X_b),  r_b = y_b - c_b               */
/*   L   = (1/K) sum_b sum_xy |r_b|^2,  K = B N M                               */
/* y_b is linear in m with d y_b[x,y] / d m[u,v] = (1/M) X_b[u,v] e^{+...}, so   */
/*   dL/dm[u,v] = (2/K) sum_b Re( conj(X_b[u,v]) * D_b[u,v] ),                  */
/*   D_b[u,v]   = (1/M) sum_xy r_b[x,y] e^{-2 pi i (ux/N + vy/M)}               */
/*              = (N/M) * 2D-DFT(r_b)[u,v]   (eq. (5) carries 1/N).             */
/* The batch sum runs in order b = 0..B-1.                                     */
/* ------------------------------------------------------------------------- */
int orc_loss_grad(int64_t N, int64_t M, int64_t batch, const double* x, const double* clean_re,
                  const double* mask, double* y_out, double* loss_out, double* grad_out, int nthreads) {
  int e = check2(N, M);
  if (e) return e;
  if (batch < 1 || !x || !clean_re || !mask || !grad_out || !loss_out) return ORC_ERR_ARG;
  int64_t P = N * M;
  double* X = (double*)malloc(sizeof(double) * 2 * (size_t)P);
  double* r = (double*)malloc(sizeof(double) * 2 * (size_t)P);
  if (!X || !r) {
    free(X);
    free(r);
    return ORC_ERR_NOMEM;
  }
  double K = (double)batch * (double)P;
  double loss = 0.0;
  for (int64_t i = 0; i < P; ++i) grad_out[i] = 0.0;
  for (int64_t b = 0; b < batch; ++b) {
    memcpy(X, x + 2 * b * P, sizeof(double) * 2 * (size_t)P);
    fft2_fwd_one(N, M, X, nthreads);
    for (int64_t i = 0; i < P; ++i) {
      r[2 * i] = mask[i] * X[2 * i];
      r[2 * i + 1] = mask[i] * X[2 * i + 1];
    }
    fft2_inv_one(N, M, r, nthreads);
    if (y_out) memcpy(y_out + 2 * b * P, r, sizeof(double) * 2 * (size_t)P);
    for (int64_t i = 0; i < P; ++i) {
      r[2 * i] -= clean_re[b * P + i];
      loss += r[2 * i] * r[2 * i] + r[2 * i + 1] * r[2 * i + 1];
    }
    fft2_fwd_one(N, M, r, nthreads);
    for (int64_t i = 0; i < P; ++i) {
      double dr = r[2 * i] * (double)N / (double)M, di = r[2 * i + 1] * (double)N / (double)M;
      grad_out[i] += (2.0 / K) * (X[2 * i] * dr + X[2 * i + 1] * di);
    }
  }
  *loss_out = loss / K;
  free(X);
  free(r);
  return ORC_OK;
}

/* Threaded batch of 1D transforms (forward with 1/N, or unscaled inverse). */
typedef struct {
  int64_t n;
  const double* in;
  double* out;
  int inverse;
} batch1_ctx;

static void batch1_range(void* p, int64_t lo, int64_t hi) {
  batch1_ctx* c = (batch1_ctx*)p;
  if (c->inverse)
    orc_fft_inv(c->n, hi - lo, c->in + 2 * lo * c->n, c->out + 2 * lo * c->n);
  else
    orc_fft_fwd(c->n, hi - lo, c->in + 2 * lo * c->n, c->out + 2 * lo * c->n);
}

int orc_fft_batch(int64_t n, int64_t batch, const double* in, double* out, int inverse, int nthreads) {
  if (!is_pow2(n)) return ORC_ERR_SIZE;
  if (batch < 0 || (batch > 0 && (!in || !out))) return ORC_ERR_ARG;
  batch1_ctx c = {n, in, out, inverse};
  parallel_range(nthreads, batch, batch1_range, &c);
  return ORC_OK;
}
