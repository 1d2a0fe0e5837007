/* oracle_checks.c -- the FP64 oracle's entry points on small and edge-case
 * inputs (lengths 1 and 2, non-square and one-row images, batches of one and
 * several, every mask kind, the gradient), for a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer.  Results are checked against the direct
 * definition where one applies; the sanitizers abort on a memory or UB error.
 * Exit status 0 when every check passed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_dft_direct(int64_t n, const double* in, double* out, int sign, double scale);
int orc_tree_partial(int64_t n, const double* in, double* out, int levels);
int orc_fft_fwd(int64_t n, int64_t batch, const double* in, double* out);
int orc_fft_inv(int64_t n, int64_t batch, const double* in, double* out);
int orc_fft2_fwd(int64_t N, int64_t M, int64_t batch, const double* in, double* out, int nthreads);
int orc_fft2_inv(int64_t N, int64_t M, int64_t batch, const double* in, double* out, int nthreads);
int orc_filter2(int64_t N, int64_t M, int64_t batch, const double* in, const double* mask, double* out,
                int nthreads);
int orc_mask_gaussian(int64_t N, int64_t M, double sigma_f, double* out);
int orc_mask_butterworth(int64_t N, int64_t M, double cutoff, int order, double* out);
int orc_mask_disc(int64_t N, int64_t M, double b, double c1, double c2, double* out);
int orc_loss_grad(int64_t N, int64_t M, int64_t batch, const double* x, const double* clean_re,
                  const double* mask, double* y_out, double* loss_out, double* grad_out, int nthreads);
int orc_fft_batch(int64_t n, int64_t batch, const double* in, double* out, int inverse, int nthreads);

static int failures = 0;

static void fill(double* a, int64_t count, unsigned seed) {
  for (int64_t i = 0; i < count; ++i) {
    seed = seed * 1664525u + 1013904223u;
    a[i] = (double)(seed >> 8) / (double)(1u << 24) - 0.5;
  }
}

static double max_abs_diff(const double* a, const double* b, int64_t count) {
  double m = 0.0;
  for (int64_t i = 0; i < count; ++i) m = fmax(m, fabs(a[i] - b[i]));
  return m;
}

static void check(int ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

int main(void) {
  /* 1D: tree vs the definition, both directions, lengths 1 .. 256 */
  for (int64_t n = 1; n <= 256; n *= 2) {
    const int64_t B = 3;
    double* x = malloc(sizeof(double) * 2 * n * B);
    double* y = malloc(sizeof(double) * 2 * n * B);
    double* r = malloc(sizeof(double) * 2 * n);
    fill(x, 2 * n * B, (unsigned)n);
    check(orc_fft_fwd(n, B, x, y) == 0, "orc_fft_fwd");
    for (int64_t b = 0; b < B; ++b) {
      check(orc_dft_direct(n, x + 2 * n * b, r, -1, 1.0 / (double)n) == 0, "orc_dft_direct");
      check(max_abs_diff(r, y + 2 * n * b, 2 * n) < 1e-12, "forward tree vs definition");
    }
    check(orc_fft_inv(n, B, x, y) == 0, "orc_fft_inv");
    check(orc_dft_direct(n, x, r, +1, 1.0) == 0, "orc_dft_direct inverse");
    check(max_abs_diff(r, y, 2 * n) < 1e-12 * (double)n, "inverse vs definition");
    check(orc_fft_batch(n, B, x, y, 0, 2) == 0, "orc_fft_batch");
    for (int lv = 0; lv <= 8 && (1 << lv) <= n; ++lv) check(orc_tree_partial(n, x, r, lv) == 0, "orc_tree_partial");
    free(x);
    free(y);
    free(r);
  }
  /* argument errors */
  {
    double a[8] = {0};
    check(orc_fft_fwd(3, 1, a, a) != 0, "length 3 refused");
    check(orc_fft2_fwd(4, 6, 1, a, a, 1) != 0, "2D 4x6 refused");
    check(orc_fft_batch(8, -1, a, a, 0, 1) != 0, "negative batch refused");
    check(orc_fft_batch(8, 0, NULL, NULL, 0, 1) == 0, "empty batch");
  }
  /* 2D and the filter on non-square and degenerate shapes */
  {
    const int64_t shapes[][2] = {{1, 1}, {1, 8}, {8, 1}, {4, 16}, {16, 4}, {32, 32}};
    for (unsigned s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
      const int64_t N = shapes[s][0], M = shapes[s][1], P = N * M, B = 2;
      double* x = malloc(sizeof(double) * 2 * P * B);
      double* X = malloc(sizeof(double) * 2 * P * B);
      double* y = malloc(sizeof(double) * 2 * P * B);
      double* mask = malloc(sizeof(double) * P);
      double* grad = malloc(sizeof(double) * P);
      double* clean = malloc(sizeof(double) * P * B);
      fill(x, 2 * P * B, (unsigned)(7 * s + 1));
      fill(clean, P * B, (unsigned)(9 * s + 2));
      check(orc_fft2_fwd(N, M, B, x, X, 3) == 0, "orc_fft2_fwd");
      check(orc_fft2_inv(N, M, B, X, y, 3) == 0, "orc_fft2_inv");
      check(max_abs_diff(x, y, 2 * P * B) < 1e-12, "2D round trip");
      for (int64_t i = 0; i < P; ++i) mask[i] = 1.0;
      check(orc_filter2(N, M, B, x, mask, y, 2) == 0, "orc_filter2");
      check(max_abs_diff(x, y, 2 * P * B) < 1e-12, "all-ones filter is the identity");
      check(orc_mask_gaussian(N, M, 0.1, mask) == 0, "orc_mask_gaussian");
      check(orc_mask_butterworth(N, M, 0.15, 4, mask) == 0, "orc_mask_butterworth");
      check(orc_mask_disc(N, M, 2.0, (double)N / 2, (double)M / 2, mask) == 0, "orc_mask_disc");
      double loss = 0.0;
      check(orc_loss_grad(N, M, B, x, clean, mask, y, &loss, grad, 2) == 0, "orc_loss_grad");
      check(isfinite(loss), "finite loss");
      free(x);
      free(X);
      free(y);
      free(mask);
      free(grad);
      free(clean);
    }
  }
  printf("oracle_checks: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
