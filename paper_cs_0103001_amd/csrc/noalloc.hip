// noalloc.hip -- fft2d_filter_noalloc: fft2d_filter with its intermediate in
// a library-owned static device array instead of a caller workspace, for
// callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array, so every device the library runs on
// holds one copy of it, at its own address, from module load until the
// process ends.  Its host-side name is only a stand-in for the symbol: the
// device address of each copy comes from hipGetSymbolAddress, taken once per
// device with that device current, and that address is what the kernels get.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "../../include/fftmi.h"
#include "plan.hpp"

using namespace fftmi;

static __device__ __align__(256) unsigned char scratch[FFT_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> device address of its `scratch`

// Device address of `scratch` on device `dev` (the current device).  The
// first call per device looks it up; later calls read the map.
int scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return FFT_OK;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e);
  if (!p) return FFT_ERR_HIP;
  g_scratch_ptr[dev] = p;
  *out = p;
  return FFT_OK;
}

// Bytes of one chunk's blocked intermediate (the passes run chunk by chunk
// over the same region).
size_t chunk_bytes(const fftmi_plan* p) {
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(p->chunk, 1), std::max<int64_t>(p->batch, 1));
  return (size_t)chunk * (size_t)p->img * sizeof(float2);
}

}  // namespace

extern "C" int fft2d_filter_noalloc(fft_plan_t p, const void* in, void* out, const fft_mask* mask, void* stream) {
  TraceRange tr("fft2d_filter_noalloc");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 2) return FFT_ERR_STATE;
  int dev = -1;
  int rc = plan_check(p, &dev);
  if (rc != FFT_OK) return rc;
  if (p->batch == 0) return FFT_OK;
  // what the filter touches: one chunk's intermediate, then (a tensor mask on
  // a plan with long columns) the mask's transposed copy; a padded plan's
  // whole workspace layout (its transposed mask region included)
  const bool maskt = mask && mask->kind == FFT_MASK_TENSOR_F32 && maskt_bytes(p) > 0;
  const size_t mt_off = (chunk_bytes(p) + 255) & ~(size_t)255;
  const size_t need = p->padded ? p->ws_bytes : (maskt ? mt_off + maskt_bytes(p) : chunk_bytes(p));
  if (need > (size_t)FFT_NOALLOC_SCRATCH_BYTES) return FFT_ERR_SCRATCH;
  void* ws = nullptr;
  rc = scratch_ptr(dev, &ws);
  if (rc != FFT_OK) return rc;
  // Nothing in the scratch needs clearing: the row pass (or the padding
  // kernel) writes every element the later passes read.
  float* mt = maskt && !p->padded ? reinterpret_cast<float*>(static_cast<char*>(ws) + mt_off) : nullptr;
  return filter_run(p, in, out, mask, nullptr, ws, stream, 7, p->chunk, mt);
}
