/*
 * fftmi.h -- C-ABI of libfftmi, an MI355X (gfx950) FFT -> filter -> IFFT library.
 *
 * The operations are those of "Construction of an algorithm in parallel for
 * the Fast Fourier Transform" (Higuera, Sarria, Fonseca, Idarraga):
 *
 *   1D forward   (Section 2, eq. E2):  H[k] = (1/N) sum_j f[j] e^{-2 pi i kj/N}
 *   1D inverse   (Section 3, eq. E3):  f[j] = sum_k c[k] e^{+2 pi i jk/N}   (unscaled)
 *   2D forward   (Section 5, eq. 5):   F[u,v] = (1/N) sum_x sum_y f[x,y] e^{-2 pi i (ux/N + vy/M)}
 *   2D inverse   (Section 5, 2D-IDFT): f[x,y] = (1/M) sum_u sum_v F[u,v] e^{+2 pi i (ux/N + vy/M)}
 *   filter       (Section 6):          g = 2D-IDFT(H . 2D-DFT(f)), H real, scaling the
 *                                      real and the imaginary part of each bin alike.
 *
 * Layout.  Complex data is complex64: interleaved (re, im) float32 pairs.  A 2D
 * image is row-major [N rows][M columns]: x in [0, N) is the row index and y
 * runs along a row; a batch of B images is [B][N][M], contiguous.  A batch of
 * 1D signals is [B][N].  Every length must be a power of two (Section 6 pads
 * images with zeros to the next power of two before transforming).
 *
 * Ownership.  Device buffers (inputs, outputs, workspace, masks) and the HIP
 * stream belong to the caller; all pointers are device pointers unless stated
 * otherwise, and a NULL stream is the default stream.  A plan owns its host
 * metadata; twiddle tables (generated in FP64 on the host and rounded once to
 * float32) are owned by the library, one set per device, and live until the
 * process ends.  A plan is immutable after creation: executing one plan on
 * several streams at once is allowed if each call has its own workspace.  A
 * plan may only be executed on the device that was current at fft_plan time.
 *
 * Errors.  Every call returns FFT_OK or a negative status; nothing aborts or
 * throws across this boundary.  All argument checks happen before any device
 * work is enqueued, so a failed call leaves every buffer untouched.  Kernel
 * launches are asynchronous: FFT_OK means "enqueued"; a fault inside a kernel
 * shows up at the caller's next synchronisation.
 */
#ifndef FFTMI_H
#define FFTMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define FFT_OK 0
#define FFT_ERR_ARG (-1)         /* NULL pointer, bad rank/direction/flag, batch < 0 */
#define FFT_ERR_SIZE (-2)        /* a length is not a power of two or is out of range */
#define FFT_ERR_UNSUPPORTED (-3) /* valid request this library does not implement */
#define FFT_ERR_WORKSPACE (-4)   /* workspace NULL while the plan needs one */
#define FFT_ERR_HIP (-5)         /* a HIP runtime call failed (text via fft_strerror) */
#define FFT_ERR_NOMEM (-6)       /* host or device allocation failed */
#define FFT_ERR_STATE (-7)       /* plan used on another device, or wrong plan kind */
#define FFT_ERR_SCRATCH (-8)     /* fft2d_filter_noalloc: the plan needs more than its static scratch */

/* ------------------------------------------------------------- directions */
#define FFT_FORWARD (-1)     /* eq. E2 (1D) / eq. 5 (2D) */
#define FFT_INVERSE (+1)     /* eq. E3 (1D) / 2D-IDFT (2D) */
#define FFT_ADJ_FORWARD (-2) /* conjugate transpose of FFT_FORWARD */
#define FFT_ADJ_INVERSE (+2) /* conjugate transpose of FFT_INVERSE */

/* ------------------------------------------------------------------ flags */
#define FFT_IN_C64 0x0u       /* input is complex64 (default) */
#define FFT_IN_REAL_F32 0x1u  /* input is real float32; imaginary parts are zero */
#define FFT_OUT_C64 0x0u      /* output is complex64 (default) */
#define FFT_OUT_REAL_F32 0x2u /* output keeps only the real part, float32 */
#define FFT_NORM_PAPER 0x0u   /* the paper's scale factors, listed above (default) */
#define FFT_NORM_NUMPY 0x4u   /* forward unscaled, inverse 1/(number of points) */
/* Rank-2 plans for fft2d_filter on real images with masks even in
 * frequency, H(-u, -v) = H(u, v) with bins taken modulo (N, M) (Gaussian,
 * Butterworth, none, or a disc centred at (N/2, M/2); a disc evaluated on
 * raw bin indices around any other centre is not even and is refused with
 * FFT_ERR_UNSUPPORTED): the 2D spectrum of a real image is
 * Hermitian, so only columns 0 .. M/2 are carried (columns 0 and M/2 packed
 * into one complex column) and the result, which is real, comes from one
 * complex inverse transform per two rows.  Requires FFT_IN_REAL_F32, N >= 32
 * and M >= 4; the output is float32, or complex64 with zero imaginary parts.
 * Other masks, fft_exec, fft2d_filter_save, fft2d_spectrum and the gradients
 * return FFT_ERR_UNSUPPORTED on such a plan. */
#define FFT_REAL_EVEN 0x8u

/* ------------------------------------------------------------------ masks */
#define FFT_MASK_NONE 0        /* H = 1 */
#define FFT_MASK_TENSOR_F32 1  /* H[u][v] = data[u*M + v], a float32 [N][M] device array */
#define FFT_MASK_GAUSSIAN 2    /* H = exp(-r^2 / (2 sigma_f^2)) */
#define FFT_MASK_BUTTERWORTH 3 /* H = 1 / (1 + (r / cutoff)^(2 order)) */
#define FFT_MASK_DISC 4        /* eq. (filtro): H = 0 if sqrt((u-c1)^2+(v-c2)^2) <= b, else 1 */

/* A real frequency-domain filter H over the bins (u, v) of an [N][M] spectrum
 * (Section 6).  For the analytic kinds r is the radius in cycles per pixel on
 * the unshifted frequency grid: f(k) = k/n for k < n/2, (k-n)/n otherwise, and
 * r = sqrt(f(u)^2 + f(v)^2).  The disc works on raw bin indices (u, v); its
 * paper reading puts (c1, c2) at (N/2, M/2). */
typedef struct fft_mask {
  int kind;           /* FFT_MASK_* */
  const float* data;  /* FFT_MASK_TENSOR_F32 only (device pointer) */
  double sigma_f;     /* FFT_MASK_GAUSSIAN */
  double cutoff;      /* FFT_MASK_BUTTERWORTH */
  int order;          /* FFT_MASK_BUTTERWORTH, >= 1 */
  double b, c1, c2;   /* FFT_MASK_DISC */
} fft_mask;

typedef struct fftmi_plan* fft_plan_t;

/* Create a plan for `batch` transforms of rank 1 (dims = {N}) or rank 2
 * (dims = {N, M}) on the current HIP device.  Lengths: powers of two,
 * 1 <= N <= 2^24 for rank 1 and 1 <= N, M <= 2^14 for rank 2.  batch >= 0
 * (0 makes every call a no-op).  flags: FFT_IN_*, FFT_OUT_*, FFT_NORM_*.
 * Errors: FFT_ERR_ARG, FFT_ERR_SIZE, FFT_ERR_NOMEM, FFT_ERR_HIP. */
int fft_plan(fft_plan_t* out, int rank, const int64_t* dims, int64_t batch, uint32_t flags);

/* Bytes of device workspace an exec/filter call on this plan needs (may be 0).
 * The caller allocates it, aligned to at least 16 bytes (a call given a
 * workspace that is not returns FFT_ERR_ARG; hipMalloc and torch give 256),
 * and may reuse it between calls on one stream. */
int fft_workspace_size(fft_plan_t plan, size_t* bytes);

/* One transform of the whole batch: in -> out, out of place (in == out is
 * rejected with FFT_ERR_ARG).  Direction: FFT_FORWARD, FFT_INVERSE,
 * FFT_ADJ_FORWARD or FFT_ADJ_INVERSE (Sections 2, 3 and 5).  Input and output
 * element types follow the plan's flags. */
int fft_exec(fft_plan_t plan, const void* in, void* out, void* workspace, int direction, void* stream);

/* Section 6 on a rank-2 plan: out = 2D-IDFT(H . 2D-DFT(in)) for every image
 * of the batch, one mask shared by the batch.  in may equal out.  The scale
 * of the round trip is 1 under either FFT_NORM_* convention. */
int fft2d_filter(fft_plan_t plan, const void* in, void* out, const fft_mask* mask, void* workspace,
                 void* stream);

/* Plan for images of any size n0 x m0 = dims0[0] x dims0[1] (1 .. 16384
 * each), filtered as Section 6 does: each axis is padded with zeros (rows
 * appended at the bottom, columns at the right) to the next power of two,
 * N x M, the padded image is filtered, and the result is cropped back to the
 * first n0 rows and m0 columns.  fft2d_filter on such a plan takes in
 * [batch][n0][m0] and writes out [batch][n0][m0] (element types from flags);
 * masks are evaluated on the N x M frequency grid (the disc's default centre
 * is (N/2, M/2)).  When n0 and m0 are powers of two this is fft_plan.
 * fft_exec, fft2d_filter_stage, fft2d_filter_save and the mask gradients
 * return FFT_ERR_UNSUPPORTED on a padded plan.  The workspace also holds the
 * padded input and output.  Errors: FFT_ERR_ARG, FFT_ERR_SIZE, as fft_plan. */
int fft_plan_padded(fft_plan_t* out, const int64_t* dims0, int64_t batch, uint32_t flags);

/* Fourier spectrum magnitude |F[u][v]| of every image, F = 2D-DFT of the
 * (zero-padded) image under eq. 5 (or FFT_NORM_NUMPY's unscaled transform):
 * float32 [batch][N][M], unshifted (F[0][0] first), for a rank-2 plan from
 * fft_plan or fft_plan_padded (Section 6 shows this spectrum of its image). */
int fft2d_spectrum(fft_plan_t plan, const void* in, float* magnitude, void* workspace, void* stream);

/* One of the three passes of fft2d_filter, for callers that schedule (or
 * time) the passes themselves; running stages 0, 1, 2 in order on one stream
 * with the same workspace is fft2d_filter.
 *   stage 0: FFT on rows (Section 5), in -> workspace; scale 1/N (eq. 5)
 *   stage 1: FFT on columns, times H, inverse FFT on columns (eq. 5's column
 *            sum, Section 6's product, the 2D-IDFT's column sum), in place in
 *            the workspace; in, out are ignored
 *   stage 2: inverse FFT on rows, workspace -> out; scale 1/M (2D-IDFT)
 * Errors as fft2d_filter, plus FFT_ERR_ARG for another stage number. */
int fft2d_filter_stage(fft_plan_t plan, int stage, const void* in, void* out, const fft_mask* mask,
                       void* workspace, void* stream);

/* fft2d_filter that also stores the forward spectrum X = 2D-DFT(in) of every
 * image (complex64, in the plan's internal blocked layout, fft_spectrum_size
 * bytes) for the mask gradient below.  Differentiable filtering: the mask is
 * a learnable parameter (not in the paper; the transform pair is eq. 5 and
 * the 2D-IDFT). */
int fft2d_filter_save(fft_plan_t plan, const void* in, void* out, const fft_mask* mask, void* spectrum,
                      void* workspace, void* stream);
int fft_spectrum_size(fft_plan_t plan, size_t* bytes);

/* Mask gradient of y = 2D-IDFT(m . X) for a rank-2 plan:
 *   grad_mask[u][v] = sum_b Re( conj(X_b[u,v]) * (2D-IDFT^H g_b)[u,v] )
 * where g_b = grad_y (complex64 [B][N][M] whatever the plan's input type: the
 * gradient of a real loss with respect to y, as conj-Wirtinger
 * "dL/dRe + i dL/dIm") and 2D-IDFT^H is the adjoint transform (eq. 5's sums
 * with the 2D-IDFT's scale, 1/M under FFT_NORM_PAPER).  X is the spectrum
 * saved by fft2d_filter_save with the same plan shape.  The batch sum is taken
 * in float32 over runs of consecutive images, each run in order b0..b1-1, and
 * the runs added in order (deterministic); the result overwrites grad_mask
 * (float32 [N][M], device).  Errors: FFT_ERR_ARG (bad plan, null pointers),
 * FFT_ERR_STATE (not a rank-2 plan, or another device current),
 * FFT_ERR_WORKSPACE, FFT_ERR_HIP. */
int fft2d_filter_mask_grad(fft_plan_t plan, const void* grad_y, const void* spectrum, float* grad_mask,
                           void* workspace, void* stream);

/* Fused forward of the filtered mean-squared error for real images (a plan
 * with FFT_IN_REAL_F32, without padding or FFT_REAL_EVEN):
 *   loss[0] = weight * sum_b sum_{u,v} |y_b[u][v] - c_b[u][v]|^2,
 *   y_b = 2D-IDFT(m . X_b), X_b = 2D-DFT(x_b) (eq. 5 and the 2D-IDFT),
 * evaluated as y - c = 2D-IDFT((m - 1) . X) + (x - c), which holds exactly
 * because the transform pair inverts, so no difference of nearly equal
 * float32 values is formed where m is close to 1.  y is not written; X is
 * stored to `spectrum` (fft2d_filter_save's layout) for the gradient below.
 *   x, c    float32 [B][N][M] (device)
 *   mask    m, float32 [N][M] (device)
 *   weight  e.g. 1 / (B N M) for the mean over all pixels
 *   loss    one float32 on the device
 * The sum is taken in float32 within each tile of rows and in float64 across
 * tiles, in a fixed order.  Errors: FFT_ERR_ARG, FFT_ERR_STATE (not rank 2,
 * other device), FFT_ERR_UNSUPPORTED (other input type, padded or
 * FFT_REAL_EVEN plans, N < 2), FFT_ERR_WORKSPACE, FFT_ERR_HIP. */
int fft2d_filter_mse(fft_plan_t plan, const float* x, const float* c, const float* mask, float weight, void* spectrum,
                     float* loss, void* workspace, void* stream);

/* Mask gradient of (weight/2) sum_b sum |y_b - c_b|^2 for the same y:
 *   dL/dm = weight * sum_b [ Re(conj X_b . 2D-IDFT^H (x_b - c_b))
 *                            + (a_inv / a_fwd) (m - 1) |X_b|^2 ]
 * because 2D-DFT(y_b - c_b) = (m - 1) X_b + 2D-DFT(x_b - c_b); a_fwd and a_inv
 * are the forward and inverse scales (N/M for FFT_NORM_PAPER).  At m = 1 no
 * difference y - c of nearly equal values is formed.
 *   x, c      the images and targets, float32 [B][N][M] for an FFT_IN_REAL_F32
 *             plan (x - c is formed as they are loaded); c == NULL means x is
 *             already the residual x - c (then also complex64 for complex plans)
 *   spectrum  X saved by fft2d_filter_save or fft2d_filter_mse with this plan
 *   mask      m, float32 [N][M] row-major (device, required)
 *   weight    e.g. 2 / (B N M) for the mean over all pixels
 * Batch order and errors as fft2d_filter_mask_grad; FFT_ERR_UNSUPPORTED when
 * c is given for a complex plan. */
int fft2d_filter_mse_grad(fft_plan_t plan, const void* x, const void* c, const void* spectrum, const float* mask,
                          float weight, float* grad_mask, void* workspace, void* stream);

/* The same loss evaluated in the frequency domain, with a forward that also
 * prepares its mask gradient.  The pair of eq. 5 and the 2D-IDFT inverts, so
 * with the unnormalised spectra X = DFT2(x) and R = DFT2(x - c)
 *   y - c = IDFT2((m - 1) X + R) / (N M)   and, by Parseval's relation,
 *   loss[0] = weight * sum_b sum_{u,v} |(m - 1) X_b + R_b|^2 / (N M).
 * No inverse transform is taken and y is never formed.  One complex
 * transform per row of z = x + i (x - c) gives the row spectra of x and of
 * x - c (split by the Hermitian symmetry of real rows); x and c are real, so
 * columns 0 .. M/2 carry every bin (X(N-u, M-v) = conj X(u, v)) and only
 * those are stored and transformed along the columns; the column pass adds
 * the loss terms of each stored bin and of its mirror and stores per run of
 * images the per-bin sums of |X|^2 and Re(conj X . R) in `state`.
 *   x, c    float32 [B][N][M] (device), mask m float32 [N][M] (device)
 *   weight  e.g. 1 / (B N M) for the mean over all pixels
 *   state   fft_spectrum_size(plan) bytes (device, 16-byte aligned): the row
 *           spectra of x - c, then the sums the gradient reads; keep it
 *           unchanged until fft2d_filter_mse_spectral_grad
 *   loss    one float32 on the device
 * The workspace receives the row spectra of x.  The loss terms are summed in
 * float32 per thread over a run of images and in float64 across tiles, the
 * per-bin sums over each run of images in order (deterministic).  Errors as
 * fft2d_filter_mse; FFT_ERR_UNSUPPORTED also for M < 4 and when rows per
 * block times threads per row transform exceeds 1024 (M > 4096 at four rows
 * per block). */
int fft2d_filter_mse_spectral(fft_plan_t plan, const float* x, const float* c, const float* mask, float weight,
                              void* state, float* loss, void* workspace, void* stream);

/* Mask gradient of (weight/2) sum_b sum |y_b - c_b|^2 from the state of
 * fft2d_filter_mse_spectral with the same plan (any mask m, since the sums
 * do not depend on it):
 *   grad_mask = weight * ((m - 1) sum_b |X_b|^2 + sum_b Re(conj X_b . R_b)) / (N M)
 * with the runs added in order; a bin (u, v) with v > M/2 reads the sums of
 * its mirror (N - u, M - v).  No transform is taken.  grad_mask float32
 * [N][M] (device, overwritten).  Errors as fft2d_filter_mse_spectral. */
int fft2d_filter_mse_spectral_grad(fft_plan_t plan, const void* state, const float* mask, float weight,
                                   float* grad_mask, void* stream);

/* Ragged batch: `count` square images of power-of-two sides sizes[i] (host
 * array, copied; 1 <= sizes[i] <= 2048), packed back to back in one buffer:
 * image i starts at element sum_{j<i} sizes[j]^2 and is row-major.  The plan
 * builds the image table and the tile lists of the three passes on the
 * current device (it owns that device memory and a capture stream until
 * fft_plan_destroy).  flags: FFT_IN_*, FFT_OUT_*, FFT_NORM_*.  Errors:
 * FFT_ERR_ARG, FFT_ERR_SIZE (a side that is not a power of two in range),
 * FFT_ERR_NOMEM, FFT_ERR_HIP.  fft_workspace_size gives sum sizes[i]^2 * 8
 * bytes.  If the environment variable FFTMI_TUNE_CACHE names a file holding a
 * schedule recorded by fft_plan_tune for the same device, side list and
 * flags, the plan starts from it. */
int fft_plan_ragged(fft_plan_t* out, int64_t count, const int64_t* sizes, uint32_t flags);

/* fft2d_filter over every image of a ragged plan (Section 6 per image, eq. 5
 * and the 2D-IDFT with each image's own N = M = side): one persistent launch
 * per pass covering all sides, the launches of a call captured in a HIP graph
 * that later calls with the same buffers and mask replay (a call with other
 * buffers captures again).  Images of sides up to the schedule's single-pass
 * limit (128 by default) are filtered whole in LDS by one more persistent
 * launch (read once, written once), which the graph runs as a branch beside
 * the three passes of the larger images.  Masks: FFT_MASK_NONE, GAUSSIAN, BUTTERWORTH (in
 * cycles per pixel, so one mask serves every side); TENSOR and DISC return
 * FFT_ERR_UNSUPPORTED.  Other errors as fft2d_filter. */
int fft2d_filter_ragged(fft_plan_t plan, const void* in_packed, void* out_packed, const fft_mask* mask,
                        void* workspace, void* stream);

/* Autotune a ragged plan's launch schedule on the caller's buffers (which it
 * overwrites), blocking until done: every candidate (threads per workgroup
 * 256 or 512, resident workgroups per CU as many as fit or 2, passes over the
 * whole batch or over runs of images of at most 128 MiB of intermediate, and
 * the largest side filtered in one pass from LDS: none, 64 or 128) is
 * run once to warm up and timed over three calls with HIP events on `stream`;
 * the fastest stays with the plan and, when FFTMI_TUNE_CACHE is set, is
 * appended to that file.  FFT_ERR_UNSUPPORTED for other plan kinds. */
int fft_plan_tune(fft_plan_t plan, const void* in_packed, void* out_packed, const fft_mask* mask, void* workspace,
                  void* stream);

/* The schedule a ragged plan uses (any pointer may be NULL): threads per
 * workgroup, resident workgroups per CU (0: as many as fit), bytes of
 * intermediate per run of images (0: one run), tile order (0: largest images
 * first), and the largest side whose images run in one pass from LDS (0:
 * none; at most 128). */
int fft_plan_schedule(fft_plan_t plan, int* block, int* wg_cap, int64_t* chunk_bytes, int* order, int* small_side);

/* Layout of a rank-2 plan (any pointer may be NULL), for callers that check
 * which kernel path a batch takes: rows per block of the blocked workspace
 * layout, columns per column-pass tile, images per chunk of fft2d_filter (its
 * three passes run chunk by chunk), and the number of runs of consecutive
 * images whose mask-gradient sums are formed separately and then added in run
 * order (images per run = ceil(batch / runs)).  FFT_ERR_STATE for other plan
 * kinds. */
int fft_plan_layout(fft_plan_t plan, int* rows_per_block, int* cols_per_tile, int64_t* chunk_images,
                    int* grad_runs);

/* fft2d_filter for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result as fft2d_filter, but the intermediate lives in a
 * library-owned static device array of FFT_NOALLOC_SCRATCH_BYTES per device
 * (held from library load until the process ends) instead of a caller
 * workspace.  The call allocates no device memory (the plan's twiddle
 * tables were made by fft_plan); its first call on a device also records
 * the array's address and the kernels' occupancy in host-side caches, and
 * later calls allocate nothing at all.  The caller still passes in and out
 * (as fft2d_filter, in may equal out).  A plan whose filter needs more than
 * the array (one chunk's blocked intermediate: up to a 4096 x 4096 image, or
 * a batch chunk of 128 MiB; with a tensor mask and N >= 2048, N * M * 4 bytes
 * more for the mask's transposed copy; a padded plan's whole workspace)
 * returns FFT_ERR_SCRATCH before any device work.  Every call on one device shares
 * that device's array and leaves the last call's contents in it: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  Nothing in the array needs to start at zero.
 * Other errors as fft2d_filter. */
#define FFT_NOALLOC_SCRATCH_BYTES ((size_t)144 << 20)
int fft2d_filter_noalloc(fft_plan_t plan, const void* in, void* out, const fft_mask* mask, void* stream);

/* ------------------------------------------------ the parallel tree (Section 2)
 * Section 2's construction of the FFT by 2^l processes, emulated on one GPU
 * with one workgroup per process.  With N = 2^m data and m1 = m - l:
 *   - process p (0 <= p < 2^l; p = 0 is the master) takes the branch of the
 *     data C(j) with j = p mod 2^l, in the tree's bit-reversed leaf order, and
 *     builds the polynomials of levels 1 .. m1 of that branch alone;
 *   - at level m1 + i (i = 1 .. l) the processes p' = p + 2^(l-i) send their
 *     level-(m1+i-1) vectors to p (a message through device memory: the
 *     sender writes its vector to its level's mailbox and releases a flag, the receiver
 *     acquires it and unpacks the vector next to its own), and each receiver
 *     p < 2^(l-i) merges the two;
 *   - the master's P_0^(m) is the DFT; out = P_0^(m) times eq. (E2)'s 1/N
 *     (FFT_NORM_PAPER) or unscaled (FFT_NORM_NUMPY), complex64.
 * Each process counts the products it generates as Section 4 does (one per
 * coefficient of each polynomial it builds: (m - l) 2^(m-l) for every
 * process in the branch phase, then 2^(m-l+i) at level m1 + i for the
 * receivers), so the master's count is eq. (multi), the critical path of
 * Table 1, and the counts of all processes add up to N log2 N. */
#define FFT_TREE_MAX_LOG2_PROCS 6 /* at most 64 processes, all resident at once */
#define FFT_TREE_MAX_LOG2 20      /* N <= 2^20 */
typedef struct fft_tree_stats {
  int64_t products[1 << FFT_TREE_MAX_LOG2_PROCS];   /* products generated by each process */
  int64_t busy_ticks[1 << FFT_TREE_MAX_LOG2_PROCS]; /* time computing, device wall clock (100 MHz) ticks */
  int64_t wait_ticks[1 << FFT_TREE_MAX_LOG2_PROCS]; /* time waiting for a message, same ticks */
  int64_t sent_to[1 << FFT_TREE_MAX_LOG2_PROCS];    /* receiver of the process's vector; -1 for the master */
  int64_t send_level[1 << FFT_TREE_MAX_LOG2_PROCS]; /* tree level of the vector it sent; -1 for the master */
  int64_t status;                                   /* 0; 1 if a receiver gave up waiting (spin_limit) */
} fft_tree_stats;

/* Plan the tree for N = n data (a power of two, 2^log2_procs <= n <= 2^20)
 * and 2^log2_procs processes (0 .. 6, and no more than the device has
 * compute units).  flags: FFT_NORM_PAPER or FFT_NORM_NUMPY.  The plan holds
 * Table 2's factors Z[j] = e^{-2 pi i j/N} (j < N/2, from the exact integer j
 * in FP64, rounded once to float).  fft_workspace_size gives
 * (1 + log2_procs) * n * 8 + 256 bytes: the tree array [n] (complex64,
 * bit-reversed leaf order), then one mailbox [n] per merge level m1 + i
 * (i = 1 .. log2_procs; each sender's vector at its own position in the tree
 * array, left there after the call), then one flag per process.
 * Errors: FFT_ERR_ARG, FFT_ERR_SIZE, FFT_ERR_UNSUPPORTED (more processes than
 * compute units), FFT_ERR_NOMEM, FFT_ERR_HIP. */
int fft_plan_tree(fft_plan_t* out, int64_t n, int log2_procs, uint32_t flags);

/* Run the emulation on one signal: in, out complex64 [n] (device, distinct);
 * stats a device fft_tree_stats, overwritten; a receiver polls its partner's
 * flag at most spin_limit (>= 1) times, about 0.1 us apart, before it gives up
 * and sets stats->status = 1 (then out is not valid).  Errors: FFT_ERR_ARG,
 * FFT_ERR_STATE (not a tree plan, other device), FFT_ERR_WORKSPACE,
 * FFT_ERR_HIP. */
int fft_tree_exec(fft_plan_t plan, const void* in, void* out, void* workspace, fft_tree_stats* stats,
                  int64_t spin_limit, void* stream);

/* Release a plan (and any graph it instantiated).  NULL is a no-op. */
int fft_plan_destroy(fft_plan_t plan);

/* Static text for a status code; the text of the last HIP failure is
 * appended for FFT_ERR_HIP. */
const char* fft_strerror(int code);

/* Library version, e.g. 0x000100 for 0.1.0. */
int fft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTMI_H */
