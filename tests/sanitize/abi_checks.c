/* abi_checks.c -- every argument-validation path of libfftmi's C-ABI that runs
 * without a GPU, for a build of the host sources with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every call returned the
 * status include/fftmi.h documents; the sanitizers abort on a memory or UB
 * error.  With no device present, plan creation past the argument checks
 * reports FFT_ERR_HIP. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fftmi.h"

static int failures = 0;

#define EXPECT(call, want)                                                              \
  do {                                                                                  \
    int got_ = (call);                                                                  \
    if (got_ != (want)) {                                                               \
      fprintf(stderr, "%s:%d %s returned %d, expected %d\n", __FILE__, __LINE__, #call, \
              got_, (want));                                                            \
      ++failures;                                                                       \
    }                                                                                   \
  } while (0)

int main(void) {
  fft_plan_t h = (fft_plan_t)0;
  fft_plan_t bogus = (fft_plan_t)(uintptr_t)0x1234;
  void* p = (void*)(uintptr_t)0x100;
  size_t n = 0;
  int64_t d1[1] = {1024}, d2[2] = {64, 64};

  /* plan creation: arguments first, then the device */
  EXPECT(fft_plan(NULL, 1, d1, 1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 1, NULL, 1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 0, d1, 1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 3, d2, 1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 1, d1, -1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 1, d1, 1, 0x80u), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 1, d1, 1, FFT_REAL_EVEN), FFT_ERR_ARG);
  EXPECT(fft_plan(&h, 2, d2, 1, FFT_REAL_EVEN), FFT_ERR_ARG);
  {
    int64_t bad[][2] = {{12, 8}, {0, 8}, {-8, 8}, {8, 6}, {(int64_t)1 << 15, 8}, {8, (int64_t)1 << 15}};
    for (unsigned i = 0; i < sizeof bad / sizeof bad[0]; ++i) EXPECT(fft_plan(&h, 2, bad[i], 1, 0), FFT_ERR_SIZE);
    int64_t big1[1] = {(int64_t)1 << 25}, odd1[1] = {1000};
    EXPECT(fft_plan(&h, 1, big1, 1, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan(&h, 1, odd1, 1, 0), FFT_ERR_SIZE);
  }
  EXPECT(fft_plan(&h, 1, d1, 4, 0), FFT_ERR_HIP); /* valid request, no device here */
  if (h != (fft_plan_t)0) {
    fprintf(stderr, "failed fft_plan left a handle\n");
    ++failures;
  }

  /* padded plans */
  {
    int64_t ok[2] = {460, 506}, z[2] = {0, 5}, big[2] = {17000, 5};
    EXPECT(fft_plan_padded(NULL, ok, 1, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_padded(&h, NULL, 1, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_padded(&h, ok, -1, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_padded(&h, z, 1, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan_padded(&h, big, 1, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan_padded(&h, ok, 1, 0), FFT_ERR_HIP);
  }

  /* ragged plans */
  {
    int64_t sizes[4] = {64, 128, 2048, 1}, bad[2] = {64, 96}, big[1] = {4096}, zero[1] = {0};
    EXPECT(fft_plan_ragged(NULL, 4, sizes, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_ragged(&h, 4, NULL, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_ragged(&h, -1, sizes, 0), FFT_ERR_ARG);
    EXPECT(fft_plan_ragged(&h, 4, sizes, 0x80u), FFT_ERR_ARG);
    EXPECT(fft_plan_ragged(&h, 2, bad, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan_ragged(&h, 1, big, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan_ragged(&h, 1, zero, 0), FFT_ERR_SIZE);
    EXPECT(fft_plan_ragged(&h, 4, sizes, 0), FFT_ERR_HIP);
  }

  /* tree plans (Section 2's processes) */
  EXPECT(fft_plan_tree(NULL, 64, 2, 0), FFT_ERR_ARG);
  EXPECT(fft_plan_tree(&h, 64, 2, FFT_IN_REAL_F32), FFT_ERR_ARG);
  EXPECT(fft_plan_tree(&h, 64, -1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan_tree(&h, 64, FFT_TREE_MAX_LOG2_PROCS + 1, 0), FFT_ERR_ARG);
  EXPECT(fft_plan_tree(&h, 96, 2, 0), FFT_ERR_SIZE);
  EXPECT(fft_plan_tree(&h, 2, 2, 0), FFT_ERR_SIZE);
  EXPECT(fft_plan_tree(&h, (int64_t)1 << (FFT_TREE_MAX_LOG2 + 1), 0, 0), FFT_ERR_SIZE);
  EXPECT(fft_plan_tree(&h, 64, 2, 0), FFT_ERR_HIP);
  EXPECT(fft_tree_exec(bogus, p, (char*)p + 8, p, (fft_tree_stats*)p, 10, NULL), FFT_ERR_ARG);

  /* every call on a handle that is not a live plan */
  EXPECT(fft_plan_destroy(NULL), FFT_OK);
  EXPECT(fft_plan_destroy(bogus), FFT_ERR_ARG);
  EXPECT(fft_workspace_size(NULL, &n), FFT_ERR_ARG);
  EXPECT(fft_workspace_size(bogus, &n), FFT_ERR_ARG);
  EXPECT(fft_spectrum_size(bogus, &n), FFT_ERR_ARG);
  EXPECT(fft_exec(bogus, p, p, p, FFT_FORWARD, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter(bogus, p, p, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_noalloc(bogus, p, p, NULL, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_noalloc(NULL, p, p, NULL, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_stage(bogus, 0, p, p, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_stage(bogus, 3, p, p, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_save(bogus, p, p, NULL, p, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_save(bogus, p, p, NULL, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_mask_grad(bogus, p, p, (float*)p, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse_grad(bogus, p, p, p, (const float*)p, 1.0f, (float*)p, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse_grad(NULL, p, NULL, p, (const float*)p, 1.0f, (float*)p, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse(bogus, (const float*)p, (const float*)p, (const float*)p, 1.0f, p, (float*)p, p, NULL),
         FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse_spectral(bogus, (const float*)p, (const float*)p, (const float*)p, 1.0f, p, (float*)p, p,
                                   NULL),
         FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse_spectral_grad(bogus, p, (const float*)p, 1.0f, (float*)p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_mse_spectral_grad(NULL, p, (const float*)p, 1.0f, (float*)p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_filter_ragged(bogus, p, p, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft_plan_tune(bogus, p, p, NULL, p, NULL), FFT_ERR_ARG);
  EXPECT(fft2d_spectrum(bogus, p, (float*)p, p, NULL), FFT_ERR_ARG);
  {
    int b = 0, c = 0, o = 0, rb = 0, w = 0, g = 0;
    int64_t ch = 0;
    EXPECT(fft_plan_schedule(bogus, &b, &c, &ch, &o, &rb), FFT_ERR_ARG);
    EXPECT(fft_plan_layout(NULL, &rb, &w, &ch, &g), FFT_ERR_ARG);
    EXPECT(fft_plan_layout(bogus, NULL, NULL, NULL, NULL), FFT_ERR_ARG);
  }

  /* status texts for every code, and an unknown one */
  {
    int codes[] = {FFT_OK, FFT_ERR_ARG, FFT_ERR_SIZE, FFT_ERR_UNSUPPORTED, FFT_ERR_WORKSPACE, FFT_ERR_HIP,
                   FFT_ERR_NOMEM, FFT_ERR_STATE, FFT_ERR_SCRATCH, -99, 12345};
    for (unsigned i = 0; i < sizeof codes / sizeof codes[0]; ++i) {
      const char* s = fft_strerror(codes[i]);
      if (!s || !strlen(s)) {
        fprintf(stderr, "empty text for status %d\n", codes[i]);
        ++failures;
      }
    }
  }
  if (fft_version() <= 0) ++failures;

  printf("abi_checks: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
