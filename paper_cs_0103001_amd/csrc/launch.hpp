// launch.hpp -- host-side entry points of the HIP kernels (internal to libfftmi).
//
// Layouts used between passes of the 2D path:
//   row-major   image b, element (u, v) at  b*N*M + u*M + v
//   blocked     image b, element (u, v) at  (b*(N/RB) + u/RB) * BS + v*RB + u % RB
// RB rows are interleaved per column so that a column tile of W columns reads
// W*RB*8 contiguous bytes per row block, while a row pass over one block reads
// and writes RB*M*8 contiguous bytes.  The block stride BS is RB*M plus a
// small pad (a multiple of 32 elements), so that the strided accesses of a
// column tile do not all fall on the same memory channels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftmi {

// Real mask over the (u, v) bins, evaluated inside the column kernels.
struct MaskArgs {
  int kind;             // FFT_MASK_* from fftmi.h
  const float* data;    // tensor mask, row-major [N][M]
  float gauss_coef;     // -1 / (2 sigma^2)
  float inv_fc2;        // 1 / cutoff^2
  int order;            // Butterworth order n (exponent 2n)
  double disc_b2;       // b^2
  double c1, c2;        // disc centre (bin units)
  float inv_n, inv_m;   // 1/N and 1/M (exact powers of two) for the frequency grid
  float tensor_bias;    // added to every tensor-mask value (-1: the fused MSE form's m - 1)
  int tensor_cm;        // the tensor mask is stored transposed, [M][N] (column v contiguous)
};

struct Launch {
  hipStream_t stream;
  const float2* tw;      // twiddle tables of the launch's transform length, [stage][k][r]
  const float2* tw_lds;  // the same in the layout copied to LDS, [stage][r-1][k]
};

// Batched transforms along contiguous rows of length L = 2^log2L, row-major in
// and out (1D path, L <= 2^14).  rows = number of transforms.
hipError_t launch_rows_rm(int log2L, bool inv, const void* in, bool in_f32, void* out, bool out_f32,
                          int64_t rows, float scale, const Launch& lc);

// Row pass into the blocked layout: `blocks` groups of RB consecutive rows of
// length L.  pair = pack two real rows into one complex transform (in_f32 and
// RB even).
hipError_t launch_rows_to_blk(int log2L, bool inv, bool pair, const void* in, bool in_f32, float2* ws,
                              int64_t blocks, int rb, unsigned bs, float scale, const Launch& lc);

// Pass one of the fused MSE gradient: real rows in - in2 (pairs, rb even).
hipError_t launch_rows_to_blk_diff(int log2L, const float* in, const float* in2, float2* ws, int64_t blocks, int rb,
                                   unsigned bs, float scale, const Launch& lc);

// Last pass of the fused MSE forward: inverse row transforms of the blocked
// workspace (the filtered spectrum of (m - 1) X), plus x - c, squared and
// summed per tile into part[0 .. *ntiles).
hipError_t launch_rows_loss(int log2L, const float2* ws, const float* x, const float* c, float* part, int64_t blocks,
                            int rb, unsigned bs, float scale, int64_t* ntiles, const Launch& lc);

// out[0] = weight * sum of part[0 .. n), double precision, fixed order; mid
// holds sum_partials_scratch(n) doubles of intermediate sums.
int64_t sum_partials_scratch(int64_t n);
hipError_t launch_sum_partials(const float* part, int64_t n, float weight, float* out, double* mid, hipStream_t st);

// Half-spectrum path for real rows (pass one): rows in pairs, columns
// 0 .. L/2-1 of each row's spectrum into blocks of L/2 columns, column 0
// holding A[0] + i A[L/2].  rb even.
hipError_t launch_rows_to_blk_half(int log2L, const float* in, float2* ws, int64_t blocks, int rb, unsigned bs,
                                   float scale, const Launch& lc);

// Half-spectrum path, last pass: inverse row transforms of the blocked half
// spectra (two rows per complex transform) into real rows (float32, or
// complex64 with zero imaginary parts).  rb even.
hipError_t launch_rows_c2r(int log2L, const float2* ws, void* out, bool out_f32, int64_t blocks, int rb, unsigned bs,
                           float scale, const Launch& lc);

// Row pass out of the blocked layout into row-major output.
hipError_t launch_rows_from_blk(int log2L, bool inv, const float2* ws, void* out, bool out_f32, int64_t blocks,
                                int rb, unsigned bs, float scale, const Launch& lc);

// Column pass on the blocked layout (column length L = N): forward transform,
// mask multiply, inverse transform, in place.  save != nullptr also stores the
// forward spectrum (blocked layout).  half: the workspace holds M columns of a
// half spectrum (see launch_rows_to_blk_half; analytic masks only).
hipError_t launch_cols_filter(int log2L, float2* ws, float2* save, int64_t nimg, int M, int rb, unsigned bs, int w,
                              bool half, const MaskArgs& mask, const Launch& lc);

// Column pass on the blocked layout: one unscaled transform, in place.
hipError_t launch_cols_fft(int log2L, bool inv, float2* ws, int64_t nimg, int M, int rb, unsigned bs, int w,
                           const Launch& lc);

// out[v][u] = in[u][v] for a float32 [N][M] array (tiles through LDS).
hipError_t launch_transpose_f32(const float* in, float* out, int64_t N, int64_t M, hipStream_t st);

// Blocked workspace (rows rows in blocks of rb) -> row-major out, times scale;
// complex64 or, with out_f32, the real parts.
hipError_t launch_unblock(const float2* ws, void* out, bool out_f32, int64_t rows, int M, int rb, unsigned bs,
                          float scale, hipStream_t st);

// |z| * scale of the blocked workspace into row-major float32.
hipError_t launch_unblock_mag(const float2* ws, float* out, int64_t rows, int M, int rb, unsigned bs, float scale,
                              hipStream_t st);

// Zero padding [nimg][n0][m0] -> [nimg][2^log2N][2^log2M] and cropping back
// (float32 or complex64 elements).
hipError_t launch_pad(const void* in, void* out, bool f32, int64_t nimg, int n0, int m0, int log2N, int log2M,
                      hipStream_t st);
hipError_t launch_crop(const void* in, void* out, bool f32, int64_t nimg, int n0, int m0, int log2N, int log2M,
                       hipStream_t st);

// Column pass for the mask gradient over images split into `groups` runs of
// consecutive images: for every (group, column tile), forward-transform the
// blocked rows of each image in order, multiply by conj(saved spectrum X) and
// accumulate the real part; part[g] = w_lin * sum + (mask ? w_sq * (m - 1) *
// sum |X|^2 : 0).  With groups == 1, part may be the final gradient.
// The filtered MSE in the frequency domain for real images: columns
// 0 .. M/2 of the row spectra of x and of x - c from one complex transform
// per row (rb rows per tile, rb * TPT <= 1024), in a blocked layout of mh
// columns (block stride bs); then per run of images the column transforms,
// the loss terms of each stored bin and its mirror (one sum per tile in
// part[]) and the per-bin sums of |X|^2 and Re(conj X . R) ([N][mh] per
// run); the mask gradient w * ((m - 1) sum|X|^2 + sum Re(conj X . R)) from
// those sums, mirrored for v > M/2.
hipError_t launch_rows_xd(int log2L, const float* x, const float* c, float2* wsx, float2* wsd, int64_t blocks, int rb,
                          unsigned bs, const Launch& lc);
hipError_t launch_cols_mse(int log2L, const float2* wsx, const float2* wsd, const float* mask, float* sumx,
                           float* sumxr, float* part, int64_t nimg, int groups, int M, int mh, int rb, unsigned bs,
                           int w, int64_t* ntiles, const Launch& lc);
hipError_t launch_mse_grad_sums(const float* sumx, const float* sumxr, const float* mask, float* grad, int N, int M,
                                int mh, int groups, float w, hipStream_t stream);
hipError_t launch_cols_grad(int log2L, const float2* ws, const float2* save, const float* mask, float* part,
                            int64_t nimg, int groups, int M, int rb, unsigned bs, int w, float w_lin, float w_sq,
                            const Launch& lc);

// grad = sum over g of part[g] (n floats each, n % 4 == 0), in group order.
hipError_t launch_sum_groups(const float* part, float* grad, int64_t n, int groups, hipStream_t stream);

// Strided column pass of the four-step long 1D transform over an [L][C]
// matrix per batch entry (row r of entry b at in + b*in_bstride +
// r*in_rstride), tiles of w columns.  twiddle_transpose: pass one (multiply by
// W_N^{k1 n2}, N = L*C, from tw_fs[n2*L + k1], and store column c as the
// contiguous row out + b*out_bstride + c*out_rstride); otherwise pass two
// (store [L][C] with row stride out_rstride; tw_fs unused).  nt: bit 1
// non-temporal loads (pass one: 1024-thread tiles only), bit 2 (pass two)
// non-temporal stores.
hipError_t launch_cols_strided(int log2L, bool inv, bool twiddle_transpose, const float2* in, float2* out,
                               int64_t batch, int C, int w, float scale, const float2* tw_fs, int64_t in_bstride,
                               int in_rstride, int64_t out_bstride, int out_rstride, int nt, const Launch& lc);

// Workgroups of a persistent launch.  With k = ceil(ntiles / resident) tiles
// for the busiest workgroup, ceil(ntiles / k) workgroups finish in the same
// number of rounds as a full grid but keep every round equally populated, so
// a bandwidth-bound pass does not end with a round run by a fraction of the
// chip.  The count is rounded up to a multiple of 8 where that still fits, so
// that a workgroup keeps its XCD's slot of the tile order on every round.
inline int64_t persistent_grid(int64_t ntiles, int64_t resident) {
  if (ntiles <= resident) return ntiles;
  const int64_t k = (ntiles + resident - 1) / resident;
  int64_t g = (ntiles + k - 1) / k;
  const int64_t g8 = (g + 7) & ~int64_t(7);
  return g >= 16 && g8 <= resident ? g8 : g;
}

// ---------------------------------------------------------------- ragged
constexpr int kRaggedMaxLog2 = 11;  // sides 1 .. 2048

// One image of a ragged batch: element offset in the packed input/output and
// in the workspace, log2 of its side, the rows per block of its blocked
// workspace layout and that layout's block stride (elements).
struct RaggedImage {
  int64_t off;
  int64_t ws_off;
  int lg;
  int rb;
  int64_t bs;
};

// FP32 twiddle tables (global layout) per log2 side.
struct TwTable {
  const float2* p[kRaggedMaxLog2 + 1];
};

// Dynamic LDS of a ragged pass with workgroups of `block` threads (any side).
int ragged_lds_bytes(int block);

// Persistent grid of one ragged pass over ntiles tiles (host queries only).
// wg_cap > 0 limits resident workgroups per CU.
hipError_t ragged_grid(int pass, bool in_f32, bool out_f32, int mask_kind, int block, int wg_cap, int ntiles,
                       int* grid);

// One pass (0: rows forward, 1: columns + mask, 2: rows inverse) over the
// tiles {image, tile} of a ragged batch, one persistent launch of `grid`
// workgroups.  Masks: NONE, GAUSSIAN, BUTTERWORTH.  Enqueues only.
hipError_t launch_ragged_pass(int pass, const void* in, bool in_f32, float2* ws, void* out, bool out_f32,
                              const RaggedImage* imgs, const int2* tiles, int ntiles, int block, int grid,
                              const MaskArgs& mk, const TwTable& tw, bool numpy, hipStream_t st);

// Small images: sides up to 2^kRaggedSmallMaxLog2 can run in one pass from
// LDS (k_ragged_small), ragged_small_ipw(lg) images of side 2^lg per work
// item {first entry of idx, count}; the workgroups have kRaggedSmallBlock
// threads.
constexpr int kRaggedSmallMaxLog2 = 7;
constexpr int kRaggedSmallBlock = 1024;
int ragged_small_ipw(int lg);
hipError_t ragged_small_grid(bool in_f32, bool out_f32, int mask_kind, int nitems, int* grid);
hipError_t launch_ragged_small(const void* in, bool in_f32, void* out, bool out_f32, const RaggedImage* imgs,
                               const int* idx, const int2* items, int nitems, int grid, const MaskArgs& mk,
                               const TwTable& tw, bool numpy, hipStream_t st);

// LDS bytes of one launch configuration (for the host's occupancy checks).
int lds_bytes_rows_rm(int log2L, int tpw);
int lds_bytes_cols(int log2L, int w);
int lds_bytes_rows_blk(int log2L, int nt);
// Most threads a workgroup of transforms of length 2^log2L may have.
int max_block_threads(int log2L);

}  // namespace fftmi
