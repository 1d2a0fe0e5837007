// tree.hip -- Section 2's parallel construction of the FFT emulated on one
// GPU: 2^l processes, one workgroup each, with their coefficient vectors
// passed between them as messages through global memory; the products each
// process generates (Section 4's count) and its busy and waiting times are
// recorded.
//
// The tree (Section 2) works on the data in bit-reversed leaf order; level n
// merges adjacent polynomials of 2^(n-1) coefficients into one of 2^n with
// the factors Z of Table 2.  Process p starts from the leaves C(j) with
// j = p mod 2^l (its branch), which occupy one contiguous region of the
// bit-reversed array, and runs levels 1 .. m1 = m - l on it alone.  Then,
// level by level, the upper half of the processes still working send their
// vectors to the lower half (process q to q - 2^(l-i) at level m1 + i), the
// receivers unpack them next to their own and merge, until process 0 (the
// master) holds P_0^(m): the DFT, to which eq. (E2)'s 1/N is applied.
//
// Messages: the sender writes its region of the tree to the same region of
// the mailbox of its level (one array of N per merge level, so every message
// stays readable after the call), then sets its flag with a device-scope
// release; the receiver
// waits for the flag with a device-scope acquire (polling at most spin_limit
// times, then giving up and recording status 1 so that every workgroup ends),
// copies the mailbox region into its tree array and merges.  Only senders
// write flags and only receivers wait, and the processes are at most 64
// workgroups, resident at once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <new>
#include <vector>

#include "../../include/fftmi.h"
#include "plan.hpp"

using namespace fftmi;

namespace {

constexpr int kTreeThreads = 256;

__device__ __forceinline__ int64_t brev_bits(int64_t v, int bits) {
  return bits > 0 ? (int64_t)(__brevll((unsigned long long)v) >> (64 - bits)) : 0;
}

// Level n of the tree over t[base, base + len): blocks of h = 2^(n-1)
// coefficients merged pairwise, X[k] = A[k] + Z[k N/2h] B[k],
// X[k + h] = A[k] - Z[k N/2h] B[k] (z holds Z[0 .. N/2)).
__device__ void tree_level(float2* t, int64_t base, int64_t len, int n, int m, const float2* __restrict__ z) {
  const int64_t h = int64_t(1) << (n - 1);
  for (int64_t b = threadIdx.x; b < len / 2; b += blockDim.x) {
    const int64_t k = b & (h - 1);
    const int64_t i0 = base + ((b >> (n - 1)) << n) + k, i1 = i0 + h;
    const float2 w = z[k << (m - n)];
    const float2 a = t[i0], c = t[i1];
    const float2 wc = make_float2(c.x * w.x - c.y * w.y, c.x * w.y + c.y * w.x);
    t[i0] = make_float2(a.x + wc.x, a.y + wc.y);
    t[i1] = make_float2(a.x - wc.x, a.y - wc.y);
  }
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_clear(unsigned* flags, fft_tree_stats* st, int nproc) {
  const int i = threadIdx.x;
  if (i < nproc) flags[i] = 0u;
  if (i < (1 << FFT_TREE_MAX_LOG2_PROCS)) {
    st->products[i] = 0;
    st->busy_ticks[i] = 0;
    st->wait_ticks[i] = 0;
    st->sent_to[i] = -1;
    st->send_level[i] = -1;
  }
  if (i == 0) st->status = 0;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_procs(const float2* __restrict__ in, float2* __restrict__ out,
                                                             float2* __restrict__ t, float2* __restrict__ mbox,
                                                             unsigned* flags, const float2* __restrict__ z, int m,
                                                             int l, float scale, int64_t spin_limit,
                                                             fft_tree_stats* st) {
  const int p = blockIdx.x, nproc = 1 << l, m1 = m - l;
  const int64_t S = int64_t(1) << m1;
  __shared__ int give_up;
  int64_t busy = 0, wait = 0, products = 0;
  int64_t t0 = (int64_t)wall_clock64();

  // the branch: leaves C(p + nproc * brev(r)) at r = 0 .. S-1 of region brev(p)
  const int64_t base0 = brev_bits(p, l) * S;
  for (int64_t r = threadIdx.x; r < S; r += blockDim.x) t[base0 + r] = in[p + (brev_bits(r, m1) << l)];
  __syncthreads();
  for (int n = 1; n <= m1; ++n) {
    tree_level(t, base0, S, n, m, z);
    products += S;  // the S coefficients of the branch's polynomials at level n
    __syncthreads();
  }
  busy += (int64_t)wall_clock64() - t0;

  int i = 1;
  for (; i <= l; ++i) {
    const int nsup = nproc >> i;  // processes that work at level m1 + i
    const int64_t len = S << (i - 1);
    if (p >= nsup) {
      // send the level-(m1 + i - 1) vector to p - nsup and stop
      t0 = (int64_t)wall_clock64();
      const int64_t base = brev_bits(p, l - i + 1) * len;
      float2* mb = mbox + (int64_t)(i - 1) * (int64_t(1) << m);  // the mailbox of level m1 + i
      for (int64_t r = threadIdx.x; r < len; r += blockDim.x) mb[base + r] = t[base + r];
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) {
        __hip_atomic_store(&flags[p], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        st->sent_to[p] = p - nsup;
        st->send_level[p] = m1 + i - 1;
      }
      busy += (int64_t)wall_clock64() - t0;
      break;
    }
    // receive the partner's vector, unpack it next to ours, merge
    const int q = p + nsup;
    t0 = (int64_t)wall_clock64();
    if (threadIdx.x == 0) {
      int64_t polls = 0;
      int ok = 1;
      while (__hip_atomic_load(&flags[q], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        if (++polls > spin_limit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      give_up = !ok;
    }
    __syncthreads();
    __threadfence();
    const int64_t t1 = (int64_t)wall_clock64();
    wait += t1 - t0;
    if (give_up) {
      if (threadIdx.x == 0) __hip_atomic_store(&st->status, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    const int64_t qbase = brev_bits(q, l - i + 1) * len;
    const float2* mb = mbox + (int64_t)(i - 1) * (int64_t(1) << m);
    for (int64_t r = threadIdx.x; r < len; r += blockDim.x) t[qbase + r] = mb[qbase + r];
    __syncthreads();
    const int64_t base = brev_bits(p, l - i) * (2 * len);
    tree_level(t, base, 2 * len, m1 + i, m, z);
    products += 2 * len;
    __syncthreads();
    busy += (int64_t)wall_clock64() - t1;
  }

  if (p == 0 && i > l) {
    // the master's P_0^(m), natural order, times eq. (E2)'s 1/N
    t0 = (int64_t)wall_clock64();
    const int64_t N = int64_t(1) << m;
    for (int64_t k = threadIdx.x; k < N; k += blockDim.x) {
      const float2 v = t[k];
      out[k] = make_float2(v.x * scale, v.y * scale);
    }
    __syncthreads();
    busy += (int64_t)wall_clock64() - t0;
  }
  if (threadIdx.x == 0) {
    st->products[p] = products;
    st->busy_ticks[p] = busy;
    st->wait_ticks[p] = wait;
  }
}

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

}  // namespace

void fftmi::destroy_tree_state(fftmi_plan* p) {
  if (p->tree_z) (void)hipFree(const_cast<float2*>(p->tree_z));
  p->tree_z = nullptr;
}

extern "C" {

int fft_plan_tree(fft_plan_t* out, int64_t n, int log2_procs, uint32_t flags) {
  if (!out) return FFT_ERR_ARG;
  *out = nullptr;
  if (flags & ~FFT_NORM_NUMPY) return FFT_ERR_ARG;
  if (log2_procs < 0 || log2_procs > FFT_TREE_MAX_LOG2_PROCS) return FFT_ERR_ARG;
  if (!is_pow2(n) || n > (int64_t(1) << FFT_TREE_MAX_LOG2) || n < (int64_t(1) << log2_procs)) return FFT_ERR_SIZE;
  std::unique_ptr<fftmi_plan> p(new (std::nothrow) fftmi_plan());
  if (!p) return FFT_ERR_NOMEM;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_fail(e);
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) return hip_fail(e);
  if ((1 << log2_procs) > cus) return FFT_ERR_UNSUPPORTED;  // every process must be resident
  p->magic = kPlanMagic;
  p->kind = 4;
  p->n = n;
  p->batch = 1;
  p->flags = flags;
  p->log_n = 0;
  while ((int64_t(1) << p->log_n) < n) ++p->log_n;
  p->tree_l = log2_procs;
  // Table 2's Z[j] = e^{-2 pi i j/N}, j < N/2 (the merges use no others),
  // from the exact integer j in FP64, rounded once
  const int64_t half = std::max<int64_t>(n / 2, 1);
  std::vector<float2> z((size_t)half);
  for (int64_t j = 0; j < half; ++j) {
    const double a = 6.283185307179586476925286766559 * (double)j / (double)n;
    z[(size_t)j] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  void* d = nullptr;
  e = hipMalloc(&d, z.size() * sizeof(float2));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
  e = hipMemcpy(d, z.data(), z.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e);
  }
  p->tree_z = static_cast<float2*>(d);
  // workspace: the tree array, one mailbox per merge level, one flag per process
  p->ws_bytes = (size_t)(1 + log2_procs) * (size_t)n * sizeof(float2) + 256;
  plan_register(p.get());
  *out = p.release();
  return FFT_OK;
}

int fft_tree_exec(fft_plan_t p, const void* in, void* out, void* workspace, fft_tree_stats* stats,
                  int64_t spin_limit, void* stream) {
  TraceRange tr("fft_tree_exec");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 4) return FFT_ERR_STATE;
  if (!in || !out || !stats || in == out || spin_limit < 1) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = plan_check(p, nullptr);
  if (rc != FFT_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float2* t = static_cast<float2*>(workspace);
  float2* mbox = t + p->n;
  unsigned* flags = reinterpret_cast<unsigned*>(mbox + (int64_t)p->tree_l * p->n);
  const int nproc = 1 << p->tree_l;
  const float scale = (p->flags & FFT_NORM_NUMPY) ? 1.0f : 1.0f / (float)p->n;
  hipLaunchKernelGGL(k_tree_clear, dim3(1), dim3(kTreeThreads), 0, st, flags, stats, nproc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  hipLaunchKernelGGL(k_tree_procs, dim3(nproc), dim3(kTreeThreads), 0, st, static_cast<const float2*>(in),
                     static_cast<float2*>(out), t, mbox, flags, p->tree_z, p->log_n, p->tree_l, scale, spin_limit,
                     stats);
  e = hipGetLastError();
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

}  // extern "C"
