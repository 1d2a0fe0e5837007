// api.cpp -- the C-ABI of libfftmi: argument checks, plans, FP64 twiddle
// generation, and the pass sequence of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/fftmi.h"
#include "fft_schedule.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace fftmi;

namespace fftmi {

thread_local std::string g_err_text;

int hip_fail(hipError_t e) {
  g_err_text = std::string("HIP error: ") + hipGetErrorString(e);
  return FFT_ERR_HIP;
}

// exp(-2 pi i t / n) evaluated in double precision from the exact integer
// t mod n, rounded once to float (Table 2's factors Z).
static float2 z_factor(int64_t t, int64_t n) {
  t %= n;
  if (t < 0) t += n;
  const double a = 6.283185307179586476925286766559 * (double)t / (double)n;
  return make_float2((float)std::cos(a), (float)-std::sin(a));
}

struct DevTables {
  float2* blob = nullptr;
  int64_t off[kMaxLog2Row + 1] = {};
  int64_t off_lds[kMaxLog2Row + 1] = {};  // LDS-layout copies, after the global-layout tables
  std::map<int, float2*> fourstep;  // 32 log2 N + log2 N1 -> [N2][N1] factors of that four-step split
};

namespace {

std::mutex g_mu;
std::map<int, DevTables*> g_dev;
std::mutex g_plan_mu;
std::set<const fftmi_plan*> g_plans;

int build_blobs(DevTables* t) {
  std::vector<float2> host;
  for (int lg = 0; lg <= kMaxLog2Row; ++lg) {
    const int L = 1 << lg;
    t->off[lg] = (int64_t)host.size();
    for (int s = 1; s < num_stages(L); ++s) {
      const int ns = stage_ns(L, s), r = stage_radix(L, s);
      for (int k = 0; k < ns; ++k)
        for (int q = 0; q < r; ++q) host.push_back(z_factor((int64_t)q * k, (int64_t)ns * r));
    }
    while (host.size() % 32) host.push_back(make_float2(0.f, 0.f));  // 256-byte aligned starts
  }
  // the same factors in the layout the persistent kernels copy to LDS
  for (int lg = 0; lg <= kMaxLog2Row; ++lg) {
    const int L = 1 << lg;
    t->off_lds[lg] = (int64_t)host.size();
    for (int s = 1; s < num_stages(L); ++s) {
      const int ns = stage_ns(L, s), r = stage_radix(L, s);
      for (int q = 1; q < r; ++q)
        for (int k = 0; k < ns; ++k) host.push_back(z_factor((int64_t)q * k, (int64_t)ns * r));
    }
    while (host.size() % 32) host.push_back(make_float2(0.f, 0.f));
  }
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, host.size() * sizeof(float2));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
  e = hipMemcpy(d, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e);
  }
  t->blob = static_cast<float2*>(d);
  return FFT_OK;
}

}  // namespace

// Tables of the current device (created on first use, kept until exit).
int device_tables(int dev, DevTables** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) {
    *out = it->second;
    return FFT_OK;
  }
  auto* t = new (std::nothrow) DevTables();
  if (!t) return FFT_ERR_NOMEM;
  int rc = build_blobs(t);
  if (rc != FFT_OK) {
    delete t;
    return rc;
  }
  g_dev[dev] = t;
  *out = t;
  return FFT_OK;
}

const float2* blob_for(const DevTables* t, int log2L) { return t->blob + t->off[log2L]; }
const float2* lds_blob_for(const DevTables* t, int log2L) { return t->blob + t->off_lds[log2L]; }

Launch launch_for(hipStream_t st, const DevTables* t, int log2L) {
  return Launch{st, blob_for(t, log2L), lds_blob_for(t, log2L)};
}

void plan_register(fftmi_plan* p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.insert(p);
}
bool plan_live(const fftmi_plan* p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return p && g_plans.count(p) && p->magic == kPlanMagic;
}
void plan_unregister(fftmi_plan* p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.erase(p);
}

// Factors of the four-step split N = N1 N2 (N1 = 2^log2N1), laid out as the
// first pass stores its output: entry n2*N1 + k1 is W_N^{k1 n2}, from the
// exact integer k1 n2 mod N in FP64, rounded once.
int fourstep_tables(DevTables* t, int log2N, int log2N1, const float2** tab) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int key = 32 * log2N + log2N1;
  auto it = t->fourstep.find(key);
  if (it == t->fourstep.end()) {
    const int64_t N = int64_t(1) << log2N, n1 = int64_t(1) << log2N1, n2 = N / n1;
    std::vector<float2> z((size_t)N), host((size_t)N);
    for (int64_t i = 0; i < N; ++i) z[(size_t)i] = z_factor(i, N);
    for (int64_t b = 0; b < n2; ++b)
      for (int64_t k = 0; k < n1; ++k) host[(size_t)(b * n1 + k)] = z[(size_t)((k * b) & (N - 1))];
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, host.size() * sizeof(float2));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
    e = hipMemcpy(d, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return hip_fail(e);
    }
    it = t->fourstep.emplace(key, static_cast<float2*>(d)).first;
  }
  *tab = it->second;
  return FFT_OK;
}

}  // namespace fftmi

// =================================================================== helpers
namespace {

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

int check_plan(fft_plan_t p, int* dev_out) {
  if (!plan_live(p)) return FFT_ERR_ARG;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev != p->device) return FFT_ERR_STATE;
  if (dev_out) *dev_out = dev;
  return FFT_OK;
}

float fwd_scale_1d(const fftmi_plan* p) { return (p->flags & FFT_NORM_NUMPY) ? 1.0f : 1.0f / (float)p->n; }
float inv_scale_1d(const fftmi_plan* p) { return (p->flags & FFT_NORM_NUMPY) ? 1.0f / (float)p->n : 1.0f; }
// 2D: eq. 5 carries 1/N (rows); the 2D-IDFT carries 1/M (columns).
float fwd_scale_2d(const fftmi_plan* p) { return (p->flags & FFT_NORM_NUMPY) ? 1.0f : 1.0f / (float)p->n; }
float inv_scale_2d(const fftmi_plan* p) {
  return (p->flags & FFT_NORM_NUMPY) ? 1.0f / ((float)p->n * (float)p->m) : 1.0f / (float)p->m;
}

int fill_mask(const fft_mask* mk, const fftmi_plan* p, MaskArgs* out) {
  std::memset(out, 0, sizeof(*out));
  out->inv_n = 1.0f / (float)p->n;
  out->inv_m = 1.0f / (float)p->m;
  if (!mk) {
    out->kind = FFT_MASK_NONE;
    return FFT_OK;
  }
  out->kind = mk->kind;
  switch (mk->kind) {
    case FFT_MASK_NONE:
      return FFT_OK;
    case FFT_MASK_TENSOR_F32:
      if (!mk->data) return FFT_ERR_ARG;
      out->data = mk->data;
      return FFT_OK;
    case FFT_MASK_GAUSSIAN:
      if (!(mk->sigma_f > 0.0) || !std::isfinite(mk->sigma_f)) return FFT_ERR_ARG;
      out->gauss_coef = (float)(-1.0 / (2.0 * mk->sigma_f * mk->sigma_f));
      return FFT_OK;
    case FFT_MASK_BUTTERWORTH:
      if (!(mk->cutoff > 0.0) || !std::isfinite(mk->cutoff) || mk->order < 1 || mk->order > 64) return FFT_ERR_ARG;
      out->inv_fc2 = (float)(1.0 / (mk->cutoff * mk->cutoff));
      out->order = mk->order;
      return FFT_OK;
    case FFT_MASK_DISC:
      if (!(mk->b > 0.0) || !std::isfinite(mk->b) || !std::isfinite(mk->c1) || !std::isfinite(mk->c2))
        return FFT_ERR_ARG;
      out->disc_b2 = mk->b * mk->b;
      out->c1 = mk->c1;
      out->c2 = mk->c2;
      return FFT_OK;
    default:
      return FFT_ERR_ARG;
  }
}

}  // namespace

namespace fftmi {
int plan_check(const fftmi_plan* p, int* dev_out) { return check_plan(const_cast<fftmi_plan*>(p), dev_out); }
int mask_args(const fft_mask* mk, const fftmi_plan* p, MaskArgs* out) { return fill_mask(mk, p, out); }
}  // namespace fftmi

// =================================================================== C-ABI
// Pad of the blocked layout's block stride (elements).  A stride that is a
// multiple of 4 KiB puts the row blocks a column tile reads on the same
// memory channels; 32 extra elements (256 bytes) spread them.  FFTMI_BLOCK_PAD
// (a multiple of 32, up to 4096) overrides the pad for tuning.
size_t fftmi::maskt_bytes(const fftmi_plan* p) {
  return p->kind == 2 && !p->half && p->n >= 2048 ? (size_t)p->n * (size_t)p->m * sizeof(float) : 0;
}

int64_t fftmi::block_pad(int64_t stride) {
  if (const char* e = std::getenv("FFTMI_BLOCK_PAD")) {
    const long v = std::atol(e);
    if (v >= 0 && v <= 4096 && v % 32 == 0) return v;
  }
  return (stride * (int64_t)sizeof(float2)) % 4096 == 0 ? 32 : 0;
}

int fftmi::fourstep_pad(int log_n1) {
  if (const char* e = std::getenv("FFTMI_FS_PAD")) {
    const int v = std::atoi(e);
    if (v >= 0 && v <= 4096 && v % 32 == 0) return v;
  }
  return (int)block_pad(int64_t(1) << log_n1);
}

extern "C" {

int fft_version(void) { return 0x000100; }

const char* fft_strerror(int code) {
  switch (code) {
    case FFT_OK:
      return "success";
    case FFT_ERR_ARG:
      return "invalid argument";
    case FFT_ERR_SIZE:
      return "length is not a power of two or is out of range";
    case FFT_ERR_UNSUPPORTED:
      return "unsupported request";
    case FFT_ERR_WORKSPACE:
      return "workspace missing";
    case FFT_ERR_HIP:
      return g_err_text.empty() ? "HIP runtime error" : g_err_text.c_str();
    case FFT_ERR_NOMEM:
      return "out of memory";
    case FFT_ERR_STATE:
      return "plan used on another device or with the wrong entry point";
    case FFT_ERR_SCRATCH:
      return "the plan needs more than the static scratch of fft2d_filter_noalloc";
    default:
      return "unknown status";
  }
}

int fft_plan(fft_plan_t* out, int rank, const int64_t* dims, int64_t batch, uint32_t flags) {
  if (!out) return FFT_ERR_ARG;
  *out = nullptr;
  if ((rank != 1 && rank != 2) || !dims || batch < 0) return FFT_ERR_ARG;
  if (flags & ~(FFT_IN_REAL_F32 | FFT_OUT_REAL_F32 | FFT_NORM_NUMPY | FFT_REAL_EVEN)) return FFT_ERR_ARG;
  const int64_t N = dims[0], M = rank == 2 ? dims[1] : 1;
  if ((flags & FFT_REAL_EVEN) && (rank != 2 || !(flags & FFT_IN_REAL_F32))) return FFT_ERR_ARG;
  if (rank == 1 && (!is_pow2(N) || N > (int64_t(1) << 24))) return FFT_ERR_SIZE;
  if (rank == 2 && (!is_pow2(N) || !is_pow2(M) || N > (1 << kMaxLog2Row) || M > (1 << kMaxLog2Row)))
    return FFT_ERR_SIZE;

  std::unique_ptr<fftmi_plan> p(new (std::nothrow) fftmi_plan());
  if (!p) return FFT_ERR_NOMEM;
  p->magic = kPlanMagic;
  p->kind = rank;
  p->n = N;
  p->m = M;
  p->batch = batch;
  p->flags = flags;
  p->log_n = ilog2c(N);
  p->log_m = ilog2c(M);

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_fail(e);
  DevTables* t = nullptr;
  int rc = device_tables(p->device, &t);
  if (rc != FFT_OK) return rc;
  p->tables = t;

  if (rank == 1) {
    if (p->log_n > kMaxLog2Row) {
      p->fourstep = true;
      // the balanced split, but 2^19 as 2^8 x 2^11 (+3-4% against 2^9 x
      // 2^10; every other uneven split measured slower)
      p->log_n1 = p->log_n == 19 ? 8 : p->log_n / 2;
      // FFTMI_FS_LOG_N1 moves the split N = N1 N2 (both lengths within the
      // four-step kernels' 2^7 .. 2^12), for measurements
      if (const char* e = std::getenv("FFTMI_FS_LOG_N1")) {
        const int v = std::atoi(e);
        if (v >= 7 && v <= 12 && p->log_n - v >= 7 && p->log_n - v <= 12) p->log_n1 = v;
      }
      p->log_n2 = p->log_n - p->log_n1;
      int wmax = 16;
      if (const char* e = std::getenv("FFTMI_FS_W")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 16 && (v & (v - 1)) == 0) wmax = v;
      }
      // threads per tile of each pass (512, or 1024 for twice the columns
      // per tile without the prefetch)
      auto fs_threads = [](const char* name, int dflt) {
        if (const char* e = std::getenv(name)) {
          const int v = std::atoi(e);
          if (v == 512 || v == 1024) return v;
        }
        return dflt;
      };
      // pass one in 512-thread tiles (with the register prefetch) while the
      // input's row stride is at most 8 KiB (2^20 points: +5% against 1024
      // threads), in 1024-thread tiles beyond (2^21, 2^22: 11-15% faster)
      const int threads1 = p->log_n2 <= 10 ? 512 : 1024;
      p->w1 = widest_cols_tile(p->log_n1, 1 << p->log_n2, wmax, fs_threads("FFTMI_FS_THREADS1", threads1));
      p->w2 = widest_cols_tile(p->log_n2, 1 << p->log_n1, wmax, fs_threads("FFTMI_FS_THREADS2", 1024));
      rc = fourstep_tables(t, p->log_n, p->log_n1, &p->tw_fs);
      if (rc != FFT_OK) return rc;
      // the intermediate [N2][N1] rows get a padded stride, so that the
      // second pass's column reads do not all land on the same channels
      p->fs_rs = (1 << p->log_n1) + fourstep_pad(p->log_n1);
      // pass two with non-temporal stores of the result up to 2^20 points
      // (+3-4% at 2^15..2^18 against stores and loads together, which the
      // chunks' cached intermediate does not need; 4-6% slower at 2^21 and
      // 2^22); FFTMI_FS_NT = 0..3 forces (1 loads, 2 stores)
      p->fs_nt = p->log_n <= 20 ? 2 : 0;
      if (const char* e = std::getenv("FFTMI_FS_NT")) p->fs_nt = std::atoi(e) & 3;
      // batch entries per chunk: about FFTMI_FS_CHUNK_MB MiB of intermediate
      // (default 128: 2^15..2^17 +8-12%, 2^19..2^20 +2%, and with pass one's
      // non-temporal loads below, 2^21 and 2^22 +14%; 112 from 2^21, which
      // leaves more of the cache to pass one's 16-32 MiB factor table: 2^21
      // +3%); 0: the whole batch
      {
        int64_t mib = p->log_n >= 21 ? 112 : 128;
        if (const char* e = std::getenv("FFTMI_FS_CHUNK_MB")) mib = std::atoll(e);
        const int64_t per_entry = (int64_t)(1 << p->log_n2) * p->fs_rs * (int64_t)sizeof(float2);
        p->fs_chunk = mib > 0 ? std::max<int64_t>(1, std::min<int64_t>(batch, (mib << 20) / per_entry))
                              : std::max<int64_t>(batch, 1);
        // every chunk reuses the start of the workspace
        p->ws_bytes = (size_t)std::min<int64_t>(batch, p->fs_chunk) * (size_t)per_entry;
        // pass one with non-temporal loads of the input while the chunk's
        // intermediate fits the memory-side cache, so the input read once
        // does not evict what pass two reads next: what makes the chunks pay
        // at 2^21 and 2^22 (1024-thread tiles only; the 512-thread tiles up
        // to 2^20 take no hint); FFTMI_FS_NT1=0/1 forces
        const int64_t inter = p->fs_chunk * per_entry;
        p->fs_nt1 = inter <= (int64_t(128) << 20);
        if (const char* e = std::getenv("FFTMI_FS_NT1")) p->fs_nt1 = std::atoi(e) != 0;
      }
    }
  } else {
    // rows per block of the blocked layout: limited by the column pass's
    // thread split (N/16 % RB); the row passes take whole or half blocks.
    int rb = 4;
    if (const char* e = std::getenv("FFTMI_RB")) {
      const int v = std::atoi(e);
      if (v >= 1 && v <= 16 && (v & (v - 1)) == 0) rb = v;
    }
    while (rb > 1 && threads_per_transform((int)N) % rb) rb /= 2;
    p->rb = rb;
    p->half = (flags & FFT_REAL_EVEN) != 0;
    if (p->half && (N < 32 || M < 4 || rb < 2)) return FFT_ERR_UNSUPPORTED;
    // columns the workspace carries: M, or 0 .. M/2 - 1 of a half spectrum
    const int64_t mc = p->half ? M / 2 : M;
    p->w = tuned_cols_width(p.get(), (int)mc);
    p->bs = rb * mc + fftmi::block_pad(rb * mc);
    p->img = (N / rb) * p->bs;
    p->chunk = filter_chunk(N, mc, batch);
    p->ws_bytes = (size_t)batch * (size_t)p->img * sizeof(float2);
    p->spec_bytes = p->ws_bytes;
    // the mask gradient's per-group partial sums follow the blocked data
    p->grad_groups = grad_groups(M / p->w, batch);
    if (p->grad_groups > 1) {
      p->part_off = (p->ws_bytes + 255) & ~(size_t)255;
      p->ws_bytes = p->part_off + (size_t)p->grad_groups * (size_t)N * (size_t)M * sizeof(float);
    }
    // then the fused MSE forward's per-tile loss sums (at most one per row)
    // and the doubles of their two-level sum
    if (!p->half) {
      p->loss_off = (p->ws_bytes + 255) & ~(size_t)255;
      // (the frequency-domain MSE has one per (run, column tile))
      // the frequency-domain MSE's layout: columns 0 .. M/2 of the row
      // spectra, in column tiles of mse_w, padded to mse_mh columns
      p->mse_w = (int)std::max<int64_t>(1, std::min<int64_t>(p->w, M / 2));
      p->mse_mh = (int)((M / 2) / p->mse_w + 1) * p->mse_w;
      p->mse_bs = rb * p->mse_mh + fftmi::block_pad(rb * p->mse_mh);
      p->mse_img = (N / rb) * p->mse_bs;
      p->mse_groups = fftmi::mse_groups(p->mse_mh / p->mse_w, batch);
      const int64_t nparts =
          std::max<int64_t>({batch * N, (int64_t)p->mse_groups * (p->mse_mh / p->mse_w), (int64_t)1});
      p->loss_mid_off = (p->loss_off + (size_t)nparts * sizeof(float) + 255) & ~(size_t)255;
      p->ws_bytes = p->loss_mid_off + (size_t)sum_partials_scratch(nparts) * sizeof(double);
      // columns of 2048 points or more go in tiles of one or two columns, so
      // a row-major tensor mask would be read one float per row; such plans
      // keep room for a transposed copy, made per call
      if (N >= 2048) {
        p->maskt_off = (p->ws_bytes + 255) & ~(size_t)255;
        p->ws_bytes = p->maskt_off + maskt_bytes(p.get());
      }
      // the frequency-domain MSE's state: the stored row spectra of x - c,
      // then the per-run sums of |X|^2 and Re(conj X . R) per stored bin
      p->mse_sums_off = ((size_t)batch * (size_t)p->mse_img * sizeof(float2) + 255) & ~(size_t)255;
      p->spec_bytes = std::max(p->spec_bytes, p->mse_sums_off + 2 * (size_t)p->mse_groups * (size_t)N *
                                                                    (size_t)p->mse_mh * sizeof(float));
    }
  }
  plan_register(p.get());
  *out = p.release();
  return FFT_OK;
}

int fft_plan_padded(fft_plan_t* out, const int64_t* dims0, int64_t batch, uint32_t flags) {
  if (!out) return FFT_ERR_ARG;
  *out = nullptr;
  if (!dims0 || batch < 0) return FFT_ERR_ARG;
  const int64_t n0 = dims0[0], m0 = dims0[1];
  if (n0 < 1 || m0 < 1 || n0 > (1 << kMaxLog2Row) || m0 > (1 << kMaxLog2Row)) return FFT_ERR_SIZE;
  int64_t N = 1, M = 1;
  while (N < n0) N <<= 1;
  while (M < m0) M <<= 1;
  const int64_t dims[2] = {N, M};
  fft_plan_t p = nullptr;
  int rc = fft_plan(&p, 2, dims, batch, flags);
  if (rc != FFT_OK) return rc;
  if (N != n0 || M != m0) {
    p->padded = true;
    p->n0 = n0;
    p->m0 = m0;
    const size_t plane = (size_t)batch * (size_t)N * (size_t)M;
    const size_t in_bytes = plane * ((flags & FFT_IN_REAL_F32) ? sizeof(float) : sizeof(float2));
    const size_t out_bytes = plane * ((flags & FFT_OUT_REAL_F32) ? sizeof(float) : sizeof(float2));
    p->pad_in_off = (p->ws_bytes + 255) & ~(size_t)255;
    p->pad_out_off = (p->pad_in_off + in_bytes + 255) & ~(size_t)255;
    p->ws_bytes = p->pad_out_off + out_bytes;
  }
  *out = p;
  return FFT_OK;
}

int fft2d_spectrum(fft_plan_t p, const void* in, float* magnitude, void* workspace, void* stream) {
  TraceRange tr("fft2d_spectrum");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (p->half) return FFT_ERR_UNSUPPORTED;
  if (p->batch == 0) return FFT_OK;
  if (!in || !magnitude) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  const bool in_f32 = p->flags & FFT_IN_REAL_F32;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float2* ws = static_cast<float2*>(workspace);
  hipError_t e;
  if (p->padded) {
    char* wsb = static_cast<char*>(workspace);
    e = launch_pad(in, wsb + p->pad_in_off, in_f32, p->batch, (int)p->n0, (int)p->m0, p->log_n, p->log_m, st);
    if (e != hipSuccess) return hip_fail(e);
    in = wsb + p->pad_in_off;
  }
  const int64_t blocks = p->batch * p->n / p->rb;
  const bool pair = in_f32 && p->rb >= 2;
  Launch lr = launch_for(st, p->tables, p->log_m);
  const unsigned bs = (unsigned)p->bs;
  e = launch_rows_to_blk(p->log_m, false, pair, in, in_f32, ws, blocks, p->rb, bs, 1.0f, lr);
  if (e != hipSuccess) return hip_fail(e);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  e = launch_cols_fft(p->log_n, false, ws, p->batch, (int)p->m, p->rb, bs, p->w, lcn);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_unblock_mag(ws, magnitude, p->batch * p->n, (int)p->m, p->rb, bs, fwd_scale_2d(p), st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

int fft_plan_layout(fft_plan_t p, int* rows_per_block, int* cols_per_tile, int64_t* chunk_images,
                    int* grad_runs) {
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (rows_per_block) *rows_per_block = p->rb;
  if (cols_per_tile) *cols_per_tile = p->w;
  if (chunk_images) *chunk_images = p->chunk;
  if (grad_runs) *grad_runs = p->grad_groups;
  return FFT_OK;
}

int fft_workspace_size(fft_plan_t plan, size_t* bytes) {
  if (!plan_live(plan) || !bytes) return FFT_ERR_ARG;
  *bytes = plan->ws_bytes;
  return FFT_OK;
}

int fft_spectrum_size(fft_plan_t plan, size_t* bytes) {
  if (!plan_live(plan) || !bytes) return FFT_ERR_ARG;
  if (plan->kind != 2) return FFT_ERR_STATE;
  *bytes = plan->spec_bytes;
  return FFT_OK;
}

int fft_exec(fft_plan_t p, const void* in, void* out, void* workspace, int direction, void* stream) {
  TraceRange tr("fft_exec");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (direction != FFT_FORWARD && direction != FFT_INVERSE && direction != FFT_ADJ_FORWARD &&
      direction != FFT_ADJ_INVERSE)
    return FFT_ERR_ARG;
  if (p->kind != 1 && p->kind != 2) return FFT_ERR_STATE;
  if (p->padded || p->half) return FFT_ERR_UNSUPPORTED;
  if (p->batch == 0) return FFT_OK;
  if (!in || !out || in == out) return FFT_ERR_ARG;
  if (p->ws_bytes && !workspace) return FFT_ERR_WORKSPACE;
  if (p->ws_bytes && ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;

  const bool inv_tw = (direction == FFT_INVERSE || direction == FFT_ADJ_FORWARD);
  const bool fwd_norm = (direction == FFT_FORWARD || direction == FFT_ADJ_FORWARD);
  const bool in_f32 = p->flags & FFT_IN_REAL_F32, out_f32 = p->flags & FFT_OUT_REAL_F32;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;

  if (p->kind == 1) {
    const float scale = fwd_norm ? fwd_scale_1d(p) : inv_scale_1d(p);
    if (!p->fourstep) {
      Launch lc = launch_for(st, p->tables, p->log_n);
      e = launch_rows_rm(p->log_n, inv_tw, in, in_f32, out, out_f32, p->batch, scale, lc);
      return e == hipSuccess ? FFT_OK : hip_fail(e);
    }
    if (in_f32 || out_f32) return FFT_ERR_UNSUPPORTED;
    // four-step: N = N1 N2; pass 1 column FFTs of length N1 over the [N1][N2]
    // view, twiddle, transposed store; pass 2 column FFTs of length N2 over
    // the [N2][N1] intermediate, natural-order result.
    // The batch goes in chunks whose intermediate stays in the memory-side
    // cache between the two passes; every chunk reuses the start of the
    // workspace.
    const int n1 = 1 << p->log_n1, n2 = 1 << p->log_n2;
    float2* ws = static_cast<float2*>(workspace);
    const int64_t wsb = (int64_t)n2 * p->fs_rs;
    Launch l1 = launch_for(st, p->tables, p->log_n1);
    Launch l2 = launch_for(st, p->tables, p->log_n2);
    for (int64_t b0 = 0; b0 < p->batch; b0 += p->fs_chunk) {
      const int64_t nb = std::min<int64_t>(p->fs_chunk, p->batch - b0);
      e = launch_cols_strided(p->log_n1, inv_tw, true, static_cast<const float2*>(in) + b0 * p->n, ws, nb, n2, p->w1,
                              1.0f, p->tw_fs, p->n, n2, wsb, p->fs_rs, p->fs_nt1 ? 1 : 0, l1);
      if (e != hipSuccess) return hip_fail(e);
      e = launch_cols_strided(p->log_n2, inv_tw, false, ws, static_cast<float2*>(out) + b0 * p->n, nb, n1, p->w2,
                              scale, nullptr, wsb, p->fs_rs, p->n, n1, p->fs_nt, l2);
      if (e != hipSuccess) return hip_fail(e);
    }
    return FFT_OK;
  }

  // rank 2: row pass into the blocked workspace, column pass in place, then
  // the blocks rewritten as rows with the scale
  const float scale = fwd_norm ? fwd_scale_2d(p) : inv_scale_2d(p);
  float2* ws = static_cast<float2*>(workspace);
  const int64_t blocks = p->batch * p->n / p->rb;
  const bool pair = in_f32 && p->rb >= 2;
  Launch lr = launch_for(st, p->tables, p->log_m);
  const unsigned bs = (unsigned)p->bs;
  e = launch_rows_to_blk(p->log_m, inv_tw, pair, in, in_f32, ws, blocks, p->rb, bs, 1.0f, lr);
  if (e != hipSuccess) return hip_fail(e);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  e = launch_cols_fft(p->log_n, inv_tw, ws, p->batch, (int)p->m, p->rb, bs, p->w, lcn);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_unblock(ws, out, out_f32, p->batch * p->n, (int)p->m, p->rb, bs, scale, st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

}  // extern "C"

// stages: bit 0 = row pass, bit 1 = column pass, bit 2 = inverse row pass
int fftmi::filter_run(fftmi_plan* p, const void* in, void* out, const fft_mask* mask, void* spectrum,
                      void* workspace, void* stream, int stages, int64_t chunk_images, float* maskt) {
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  MaskArgs mk;
  int rc = fill_mask(mask, p, &mk);
  if (rc != FFT_OK) return rc;
  if (p->half) {
    // the half-spectrum path needs H(-u, -v) = H(u, v) on the bins modulo
    // (N, M).  The disc is evaluated on raw bin indices, so only a centre at
    // (N/2, M/2) is even: (N - u - N/2)^2 = (u - N/2)^2 for every u, row 0
    // included.  A centre at 0 is not (bin 1 lies inside, bin N - 1 outside).
    const bool even_disc = mk.kind == FFT_MASK_DISC && mk.c1 == 0.5 * (double)p->n && mk.c2 == 0.5 * (double)p->m;
    if (spectrum || (mk.kind != FFT_MASK_NONE && mk.kind != FFT_MASK_GAUSSIAN && mk.kind != FFT_MASK_BUTTERWORTH &&
                     !even_disc))
      return FFT_ERR_UNSUPPORTED;
  }
  if (p->batch == 0) return FFT_OK;
  if (((stages & 1) && !in) || ((stages & 4) && !out)) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  const bool in_f32 = p->flags & FFT_IN_REAL_F32, out_f32 = p->flags & FFT_OUT_REAL_F32;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float2* ws = static_cast<float2*>(workspace);
  const bool pair = in_f32 && p->rb >= 2;
  Launch lr = launch_for(st, p->tables, p->log_m);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  if (mk.kind == FFT_MASK_TENSOR_F32 && p->maskt_off && (stages & 2)) {
    float* mt = maskt ? maskt : reinterpret_cast<float*>(static_cast<char*>(workspace) + p->maskt_off);
    hipError_t e = launch_transpose_f32(mk.data, mt, p->n, p->m, st);
    if (e != hipSuccess) return hip_fail(e);
    mk.data = mt;
    mk.tensor_cm = 1;
  }
  // Section 6's padding: the caller's n0 x m0 images are zero-padded into
  // the workspace, filtered there, and the result cropped back into `out`.
  void* final_out = out;
  if (p->padded) {
    if (stages != 7 || spectrum) return FFT_ERR_UNSUPPORTED;
    char* wsb = static_cast<char*>(workspace);
    hipError_t e = launch_pad(in, wsb + p->pad_in_off, in_f32, p->batch, (int)p->n0, (int)p->m0, p->log_n, p->log_m,
                              st);
    if (e != hipSuccess) return hip_fail(e);
    in = wsb + p->pad_in_off;
    out = wsb + p->pad_out_off;
  }
  // The whole filter runs chunk by chunk: the three passes over one chunk of
  // images before the next, with the chunk's intermediate small enough to
  // stay in the memory-side cache between the passes.  A single stage covers
  // the whole batch.
  const int64_t plane = p->n * p->m;
  const int64_t mc = p->half ? p->m / 2 : p->m;  // workspace columns
  const unsigned bs = (unsigned)p->bs;
  const int64_t chunk = stages == 7 ? std::max<int64_t>(1, chunk_images) : p->batch;
  for (int64_t b0 = 0; b0 < p->batch; b0 += chunk) {
    const int64_t nb = std::min(chunk, p->batch - b0);
    const int64_t blocks = nb * p->n / p->rb;
    const char* cin = static_cast<const char*>(in) + (in ? b0 * plane * (in_f32 ? 4 : 8) : 0);
    char* cout = static_cast<char*>(out) + (out ? b0 * plane * (out_f32 ? 4 : 8) : 0);
    float2* cspec = spectrum ? static_cast<float2*>(spectrum) + b0 * p->img : nullptr;
    hipError_t e = hipSuccess;
    if (stages & 1) {
      e = p->half ? launch_rows_to_blk_half(p->log_m, static_cast<const float*>(static_cast<const void*>(cin)), ws,
                                            blocks, p->rb, bs, fwd_scale_2d(p), lr)
                  : launch_rows_to_blk(p->log_m, false, pair, cin, in_f32, ws, blocks, p->rb, bs, fwd_scale_2d(p), lr);
      if (e != hipSuccess) return hip_fail(e);
    }
    if (stages & 2) {
      e = launch_cols_filter(p->log_n, ws, cspec, nb, (int)mc, p->rb, bs, p->w, p->half, mk, lcn);
      if (e != hipSuccess) return hip_fail(e);
    }
    if (stages & 4) {
      e = p->half ? launch_rows_c2r(p->log_m, ws, cout, out_f32, blocks, p->rb, bs, inv_scale_2d(p), lr)
                  : launch_rows_from_blk(p->log_m, true, ws, cout, out_f32, blocks, p->rb, bs, inv_scale_2d(p), lr);
      if (e != hipSuccess) return hip_fail(e);
    }
  }
  if (p->padded) {
    hipError_t e = launch_crop(out, final_out, out_f32, p->batch, (int)p->n0, (int)p->m0, p->log_n, p->log_m, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  return FFT_OK;
}

extern "C" {

int fft2d_filter(fft_plan_t p, const void* in, void* out, const fft_mask* mask, void* workspace, void* stream) {
  TraceRange tr("fft2d_filter");
  return filter_run(p, in, out, mask, nullptr, workspace, stream, 7, plan_live(p) ? p->chunk : 1);
}

int fft2d_filter_stage(fft_plan_t p, int stage, const void* in, void* out, const fft_mask* mask, void* workspace,
                       void* stream) {
  TraceRange tr("fft2d_filter_stage");
  if (stage < 0 || stage > 2) return FFT_ERR_ARG;
  return filter_run(p, in, out, mask, nullptr, workspace, stream, 1 << stage, 1);
}

int fft2d_filter_save(fft_plan_t p, const void* in, void* out, const fft_mask* mask, void* spectrum,
                      void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_save");
  if (!spectrum) return FFT_ERR_ARG;
  return filter_run(p, in, out, mask, spectrum, workspace, stream, 7, plan_live(p) ? p->chunk : 1);
}

// Mask gradient from a saved spectrum: in_b (the incoming gradient, or the
// residual of the fused MSE form) is forward-transformed in the blocked
// layout, then the column kernel accumulates Re(conj X_b . T(in_b)) over the
// batch in groups of consecutive images.
static int grad_impl(fftmi_plan* p, const void* in, const void* in2, const void* spectrum, const float* mask,
                     float weight, float* grad_mask, void* workspace, void* stream) {
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (p->padded || p->half) return FFT_ERR_UNSUPPORTED;
  if (!grad_mask) return FFT_ERR_ARG;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->batch == 0) {
    int rc = check_plan(p, nullptr);
    if (rc != FFT_OK) return rc;
    hipError_t e = hipMemsetAsync(grad_mask, 0, (size_t)(p->n * p->m) * sizeof(float), st);
    return e == hipSuccess ? FFT_OK : hip_fail(e);
  }
  if (!in || !spectrum) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  float2* ws = static_cast<float2*>(workspace);
  const bool in_f32 = mask && (p->flags & FFT_IN_REAL_F32);
  const bool pair = in_f32 && p->rb % 2 == 0;
  const int64_t blocks = p->batch * p->n / p->rb;
  Launch lr = launch_for(st, p->tables, p->log_m);
  // unscaled forward transform of the rows; the adjoint's scale goes into w_lin
  if (in2 && !pair) return FFT_ERR_UNSUPPORTED;
  const unsigned bs = (unsigned)p->bs;
  hipError_t e = in2 ? launch_rows_to_blk_diff(p->log_m, static_cast<const float*>(in), static_cast<const float*>(in2),
                                               ws, blocks, p->rb, bs, 1.0f, lr)
                     : launch_rows_to_blk(p->log_m, false, pair, in, in_f32, ws, blocks, p->rb, bs, 1.0f, lr);
  if (e != hipSuccess) return hip_fail(e);
  const float b = inv_scale_2d(p), a = fwd_scale_2d(p);
  const float w_lin = weight * b, w_sq = weight * (b / a);
  const int groups = p->grad_groups;
  float* part = grad_mask;
  if (groups > 1) part = reinterpret_cast<float*>(static_cast<char*>(workspace) + p->part_off);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  e = launch_cols_grad(p->log_n, ws, static_cast<const float2*>(spectrum), mask, part, p->batch, groups, (int)p->m,
                       p->rb, bs, p->w, w_lin, w_sq, lcn);
  if (e != hipSuccess) return hip_fail(e);
  if (groups > 1) {
    e = launch_sum_groups(part, grad_mask, p->n * p->m, groups, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  return FFT_OK;
}

int fft2d_filter_mask_grad(fft_plan_t p, const void* grad_y, const void* spectrum, float* grad_mask,
                           void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_mask_grad");
  return grad_impl(p, grad_y, nullptr, spectrum, nullptr, 1.0f, grad_mask, workspace, stream);
}

int fft2d_filter_mse_grad(fft_plan_t p, const void* x, const void* c, const void* spectrum, const float* mask,
                          float weight, float* grad_mask, void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_mse_grad");
  if (!mask && plan_live(p) && p->batch > 0) return FFT_ERR_ARG;
  return grad_impl(p, x, c, spectrum, mask, weight, grad_mask, workspace, stream);
}

int fft2d_filter_mse(fft_plan_t p, const float* x, const float* c, const float* mask, float weight, void* spectrum,
                     float* loss, void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_mse");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (p->padded || p->half || !(p->flags & FFT_IN_REAL_F32) || p->rb < 2) return FFT_ERR_UNSUPPORTED;
  if (!loss) return FFT_ERR_ARG;
  if (p->batch > 0 && (!x || !c || !mask || !spectrum)) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float2* ws = static_cast<float2*>(workspace);
  float* part = reinterpret_cast<float*>(static_cast<char*>(workspace) + p->loss_off);
  MaskArgs mk;
  std::memset(&mk, 0, sizeof(mk));
  mk.kind = FFT_MASK_TENSOR_F32;
  mk.data = mask;
  mk.tensor_bias = -1.0f;
  mk.inv_n = 1.0f / (float)p->n;
  mk.inv_m = 1.0f / (float)p->m;
  Launch lr = launch_for(st, p->tables, p->log_m);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  if (p->maskt_off && p->batch > 0) {
    float* mt = reinterpret_cast<float*>(static_cast<char*>(workspace) + p->maskt_off);
    hipError_t e = launch_transpose_f32(mask, mt, p->n, p->m, st);
    if (e != hipSuccess) return hip_fail(e);
    mk.data = mt;
    mk.tensor_cm = 1;
  }
  const int64_t plane = p->n * p->m;
  int64_t nparts = 0;
  for (int64_t b0 = 0; b0 < p->batch; b0 += p->chunk) {
    const int64_t nb = std::min(p->chunk, p->batch - b0);
    const int64_t blocks = nb * p->n / p->rb;
    const unsigned bs = (unsigned)p->bs;
    hipError_t e = launch_rows_to_blk(p->log_m, false, true, x + b0 * plane, true, ws, blocks, p->rb, bs,
                                      fwd_scale_2d(p), lr);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_cols_filter(p->log_n, ws, static_cast<float2*>(spectrum) + b0 * p->img, nb, (int)p->m, p->rb, bs,
                           p->w, false, mk, lcn);
    if (e != hipSuccess) return hip_fail(e);
    int64_t nt = 0;
    e = launch_rows_loss(p->log_m, ws, x + b0 * plane, c + b0 * plane, part + nparts, blocks, p->rb, bs,
                         inv_scale_2d(p), &nt, lr);
    if (e != hipSuccess) return hip_fail(e);
    nparts += nt;
  }
  double* mid = reinterpret_cast<double*>(static_cast<char*>(workspace) + p->loss_mid_off);
  hipError_t e = launch_sum_partials(part, nparts, weight, loss, mid, st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

// Plans the frequency-domain MSE takes: real rank-2 input without padding
// or half spectra, rows of at least 4 points, and rb rows of one block
// transformed by one workgroup.
static bool mse_spectral_ok(const fftmi_plan* p) {
  return !p->padded && !p->half && (p->flags & FFT_IN_REAL_F32) && p->rb >= 2 && p->rb % 2 == 0 && p->m >= 4 &&
         (int64_t)p->rb * threads_per_transform((int)p->m) <= 1024;
}

int fft2d_filter_mse_spectral(fft_plan_t p, const float* x, const float* c, const float* mask, float weight,
                              void* state, float* loss, void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_mse_spectral");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (!mse_spectral_ok(p)) return FFT_ERR_UNSUPPORTED;
  if (!loss) return FFT_ERR_ARG;
  if (p->batch > 0 && (!x || !c || !mask || !state)) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace) || ws_misaligned(state)) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float* part = reinterpret_cast<float*>(static_cast<char*>(workspace) + p->loss_off);
  double* mid = reinterpret_cast<double*>(static_cast<char*>(workspace) + p->loss_mid_off);
  // sum |y - c|^2 = sum |(m - 1) X + R|^2 / (N M) for the unnormalised spectra
  const float lw = (float)((double)weight / ((double)p->n * (double)p->m));
  if (p->batch == 0) {
    hipError_t e = launch_sum_partials(part, 0, lw, loss, mid, st);
    return e == hipSuccess ? FFT_OK : hip_fail(e);
  }
  float2* wsx = static_cast<float2*>(workspace);
  float2* wsd = static_cast<float2*>(state);
  float* sumx = reinterpret_cast<float*>(static_cast<char*>(state) + p->mse_sums_off);
  float* sumxr = sumx + (size_t)p->mse_groups * (size_t)p->n * (size_t)p->mse_mh;
  const unsigned bs = (unsigned)p->mse_bs;
  Launch lr = launch_for(st, p->tables, p->log_m);
  Launch lcn = launch_for(st, p->tables, p->log_n);
  hipError_t e = launch_rows_xd(p->log_m, x, c, wsx, wsd, p->batch * p->n / p->rb, p->rb, bs, lr);
  if (e != hipSuccess) return hip_fail(e);
  int64_t nparts = 0;
  e = launch_cols_mse(p->log_n, wsx, wsd, mask, sumx, sumxr, part, p->batch, p->mse_groups, (int)p->m, p->mse_mh,
                      p->rb, bs, p->mse_w, &nparts, lcn);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_sum_partials(part, nparts, lw, loss, mid, st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

int fft2d_filter_mse_spectral_grad(fft_plan_t p, const void* state, const float* mask, float weight, float* grad_mask,
                                   void* stream) {
  TraceRange tr("fft2d_filter_mse_spectral_grad");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  if (!mse_spectral_ok(p)) return FFT_ERR_UNSUPPORTED;
  if (!grad_mask || !mask) return FFT_ERR_ARG;
  if (p->batch > 0 && !state) return FFT_ERR_ARG;
  int rc = check_plan(p, nullptr);
  if (rc != FFT_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nm = p->n * p->m;
  if (p->batch == 0) {
    hipError_t e = hipMemsetAsync(grad_mask, 0, (size_t)nm * sizeof(float), st);
    return e == hipSuccess ? FFT_OK : hip_fail(e);
  }
  const float* sumx = reinterpret_cast<const float*>(static_cast<const char*>(state) + p->mse_sums_off);
  const float* sumxr = sumx + (size_t)p->mse_groups * (size_t)p->n * (size_t)p->mse_mh;
  // (weight / 2) d/dm sum |y - c|^2 = weight ((m - 1) sum |X|^2 + sum Re(conj X . R)) / (N M)
  const float gw = (float)((double)weight / ((double)p->n * (double)p->m));
  hipError_t e = launch_mse_grad_sums(sumx, sumxr, mask, grad_mask, (int)p->n, (int)p->m, p->mse_mh, p->mse_groups,
                                      gw, st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

int fft_plan_destroy(fft_plan_t p) {
  if (!p) return FFT_OK;
  if (!plan_live(p)) return FFT_ERR_ARG;
  plan_unregister(p);
  p->magic = 0;
  destroy_ragged_state(p);
  destroy_tree_state(p);
  delete p;
  return FFT_OK;
}

}  // extern "C"
