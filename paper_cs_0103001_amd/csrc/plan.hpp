// plan.hpp -- the plan object behind the opaque fft_plan_t, and the internal
// helpers shared by the C-ABI translation units of libfftmi.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>

#include "../../include/fftmi.h"

namespace fftmi {

struct DevTables;     // per-device twiddle tables (api.cpp)
struct RaggedState;   // ragged work list, device buffers and graph (ragged.cpp)

constexpr uint32_t kPlanMagic = 0x46465449u;

// A rocTX range around one C-ABI call that enqueues device work: it names the
// call in a profiler's marker trace (rocprofv3 --marker-trace) and costs a
// function call when no profiler listens.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

extern thread_local std::string g_err_text;
int hip_fail(hipError_t e);

int device_tables(int dev, DevTables** out);
const float2* blob_for(const DevTables* t, int log2L);
const float2* lds_blob_for(const DevTables* t, int log2L);
int fourstep_tables(DevTables* t, int log2N, int log2N1, const float2** tab);

}  // namespace fftmi

struct fftmi_plan {
  uint32_t magic = 0;
  int kind = 0;  // 1: rank 1, 2: rank 2, 3: ragged
  int device = -1;
  int64_t n = 1, m = 1, batch = 0;  // rank 1: n; rank 2: n rows, m columns
  uint32_t flags = 0;
  int log_n = 0, log_m = 0;
  fftmi::DevTables* tables = nullptr;
  // rank 2: rows per block of the blocked layout, column tile width, block
  // stride in elements (rb * columns + pad) and elements per image
  int rb = 1, w = 1;
  int64_t bs = 0, img = 0;
  // rank 2: images per chunk of fft2d_filter (passes run chunk by chunk)
  int64_t chunk = 1;
  // rank 2 made by fft_plan_padded: the callers' image size n0 x m0 (zero
  // padded to n x m, the next powers of two), and the workspace offsets of
  // the padded input and the padded (uncropped) output
  bool padded = false;
  // rank 2 with FFT_REAL_EVEN: the workspace holds half spectra
  bool half = false;
  int64_t n0 = 0, m0 = 0;
  size_t pad_in_off = 0, pad_out_off = 0;
  // rank 1 beyond one LDS pass: four-step split N = N1 * N2
  bool fourstep = false;
  int log_n1 = 0, log_n2 = 0, w1 = 1, w2 = 1;
  int fs_rs = 0;  // row stride of the [N2][N1] intermediate (N1 + pad)
  int fs_nt = 0;       // pass two: 1 non-temporal loads, 2 non-temporal stores
  bool fs_nt1 = false;  // pass one with non-temporal loads
  int64_t fs_chunk = 1;  // batch entries per chunk of the two passes
  const float2* tw_fs = nullptr;  // [N2][N1] factors W_N^{k1 n2}
  size_t ws_bytes = 0, spec_bytes = 0;
  // rank 2: image groups of the mask-gradient column pass, and the workspace
  // offsets of their partial sums and of the fused MSE forward's per-tile sums
  int grad_groups = 1;
  size_t part_off = 0, loss_off = 0, loss_mid_off = 0;
  // the frequency-domain MSE: column tile width, stored columns (M/2 + 1
  // rounded up to whole tiles), block stride and image size of its layout,
  // and the offset of its per-bin sums in the caller's state buffer
  int mse_w = 1, mse_mh = 0, mse_groups = 1;
  int64_t mse_bs = 0, mse_img = 0;
  size_t mse_sums_off = 0;
  // rank 2 with columns of 2048 points or more (tiles of one or two columns):
  // workspace offset of a transposed copy of a tensor mask (0: none)
  size_t maskt_off = 0;
  fftmi::RaggedState* ragged = nullptr;
  // fft_plan_tree: log2 of the number of processes, Table 2's factors Z[0 .. N/2)
  int tree_l = 0;
  const float2* tree_z = nullptr;
};

namespace fftmi {

// Live-plan registry: lets every entry point reject freed or foreign handles.
void plan_register(fftmi_plan* p);
bool plan_live(const fftmi_plan* p);
// The kernels store 16-byte vectors into the workspace.
inline bool ws_misaligned(const void* ws) { return (reinterpret_cast<uintptr_t>(ws) & 15) != 0; }
void plan_unregister(fftmi_plan* p);

// Pad (elements) added to a blocked layout's block stride of `stride`
// elements: 32 when the stride is a multiple of 4 KiB, else 0.
int64_t block_pad(int64_t stride);
// Pad (elements) of the four-step intermediate's rows of 2^log_n1 entries.
int fourstep_pad(int log_n1);

// Widest power-of-two column tile (<= wmax, <= cols) that fits one workgroup
// of at most max_threads threads (0: the kernel's usual limit) and the LDS.
int widest_cols_tile(int log2L, int cols, int wmax, int max_threads = 0);

// Column tile width for a rank-2 plan (autotuned value if one is cached).
int tuned_cols_width(const fftmi_plan* p, int cols);

// Images per chunk of the whole filter: the chunk's complex64 intermediate
// stays within half of the memory-side cache (256 MiB on MI355X), so the
// column pass and the inverse row pass read what the row pass just wrote from
// the cache rather than from HBM.
int64_t filter_chunk(int64_t N, int64_t M, int64_t batch);

// Image groups of the mask-gradient column pass: enough (column tile, group)
// work items to fill the chip, each group a run of consecutive images.
int grad_groups(int64_t col_tiles, int64_t batch);
// Runs of images of the frequency-domain MSE's column pass.
int mse_groups(int64_t col_tiles, int64_t batch);

void destroy_ragged_state(fftmi_plan* p);
void destroy_tree_state(fftmi_plan* p);

// fft2d_filter's body: the passes selected by `stages` (bit 0 row pass, bit 1
// column pass, bit 2 inverse row pass), run over the batch in chunks of
// `chunk` images when all three are selected, with `workspace` holding one
// chunk's blocked intermediate.
// maskt: where a tensor mask's transposed copy goes (nullptr: the plan's
// workspace region at maskt_off); used only when the plan has that region.
int filter_run(fftmi_plan* p, const void* in, void* out, const fft_mask* mask, void* spectrum, void* workspace,
               void* stream, int stages, int64_t chunk, float* maskt = nullptr);
// Bytes of the transposed tensor mask (0 when the plan reads masks as given).
size_t maskt_bytes(const fftmi_plan* p);

struct MaskArgs;
// The plan is live and its device is current (FFT_OK, FFT_ERR_ARG, FFT_ERR_STATE, FFT_ERR_HIP).
int plan_check(const fftmi_plan* p, int* dev_out);
// Validate a C-ABI mask and turn it into kernel arguments for the plan's shape.
int mask_args(const fft_mask* mk, const fftmi_plan* p, MaskArgs* out);

}  // namespace fftmi
