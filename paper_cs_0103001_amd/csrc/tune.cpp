// tune.cpp -- launch-shape choices of rank-2 plans: the column tile width W.
//
// A column tile reads W*RB*8 contiguous bytes per row block; wider tiles give
// longer runs but fewer workgroups per CU (LDS: W * N * 8.5 bytes).  The
// default gives 256-thread workgroups, several of which share a CU (their
// neighbouring tiles' runs meet in the XCD's L2); an autotuned value
// recorded for the shape takes precedence.
#include <algorithm>
#include <cstdlib>

#include "fft_schedule.hpp"
#include "launch.hpp"
#include "plan.hpp"

#ifndef FFTMI_MSE_TARGET_DEFAULT
#define FFTMI_MSE_TARGET_DEFAULT 512
#endif

namespace fftmi {

int widest_cols_tile(int log2L, int cols, int wmax, int max_threads) {
  const int tpt = threads_per_transform(1 << log2L);
  const int cap = max_threads > 0 ? max_threads : max_block_threads(log2L);
  int w = 1;
  while (w * 2 <= wmax && w * 2 <= cols && (w * 2) * tpt <= cap && lds_bytes_cols(log2L, w * 2) <= kLdsBytes)
    w *= 2;
  return w;
}

int tuned_cols_width(const fftmi_plan* p, int cols) {
  // one 256-thread transform per workgroup for long columns, more for short
  const int tpt = threads_per_transform(1 << p->log_n);
  int w = std::max(1, 256 / tpt);
  if (const char* env = std::getenv("FFTMI_COLS_W")) {
    const int v = std::atoi(env);
    if (v >= 1 && (v & (v - 1)) == 0) w = v;
  }
  return widest_cols_tile(p->log_n, cols, w);
}

int64_t filter_chunk(int64_t N, int64_t M, int64_t batch) {
  int64_t mib = 128;
  if (const char* env = std::getenv("FFTMI_CHUNK_MB")) mib = std::atoll(env);
  if (batch <= 1 || mib <= 0) return std::max<int64_t>(batch, 1);
  const int64_t per_image = N * M * 8;
  const int64_t c = (mib << 20) / std::max<int64_t>(per_image, 1);
  return std::max<int64_t>(1, std::min(batch, c));
}

// Runs of consecutive images such that runs * col_tiles work items come to
// at most `target` (an environment variable may set it), every run but the
// last of the same length.
static int run_groups(int64_t col_tiles, int64_t batch, int64_t target, const char* env_name) {
  if (const char* env = std::getenv(env_name)) {
    const long long v = std::atoll(env);
    if (v >= 1 && v <= (1 << 20)) target = v;
  }
  if (batch <= 1 || col_tiles <= 0) return 1;
  int64_t g = std::max<int64_t>(1, std::min<int64_t>(batch, target / col_tiles));
  const int64_t per = (batch + g - 1) / g;
  return (int)((batch + per - 1) / per);
}

int grad_groups(int64_t col_tiles, int64_t batch) {
  // work items (column tile, run of images): about two per CU, each over a
  // long run.  Fewer, longer runs keep fewer images in flight at a time:
  // batch 64 of 1024^2 took 304 / 258 / 246 / 293 us with runs of 8 / 16 /
  // 32 / 64 images (non-temporal loads then took 32-image runs to 194 us).
  return run_groups(col_tiles, batch, 512, "FFTMI_GRAD_TARGET");
}

int mse_groups(int64_t col_tiles, int64_t batch) {
  // the frequency-domain MSE's column pass: as many work items as fit on the
  // chip in one round (its column tiles per run, M / (2w) + 1, are not a
  // power of two)
  return run_groups(col_tiles, batch, FFTMI_MSE_TARGET_DEFAULT, "FFTMI_MSE_TARGET");
}

}  // namespace fftmi
