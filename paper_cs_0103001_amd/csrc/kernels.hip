// kernels.hip -- gfx950 kernels of the FFT -> filter -> IFFT path and their
// launchers.  Every kernel keeps a transform's data in registers (16 complex
// values per thread), exchanges it through LDS between radix passes, and
// touches HBM exactly once on the way in and once on the way out.
#include <hip/hip_runtime.h>

#include <mutex>
#include <set>
#include <utility>

#include "../../include/fftmi.h"
#include "fft_core.hpp"
#include "launch.hpp"

namespace fftmi {

__device__ __forceinline__ int ilog2_pow2(int x) { return 31 - __clz(x); }

// Make a per-thread pointer opaque to the optimiser so that addresses derived
// from it are recomputed where they are used rather than held in registers
// across a whole transform.
template <typename T>
__device__ __forceinline__ void launder(T*& p) {
  asm volatile("" : "+v"(p));
}

// Workgroup index remap: consecutive indices are dispatched round-robin over
// the 8 XCDs, each with its own L2.  Giving every XCD a contiguous range of
// tiles keeps neighbouring tiles (which share cache lines) on one L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t i, int64_t grid) {
  if ((grid & 7) == 0 && grid >= 16) return (i & 7) * (grid >> 3) + (i >> 3);
  return i;
}

// ----------------------------------------------------------------- masks
__device__ __forceinline__ float freq_of(int k, int n, float inv_n) {
  return (float)(k < ((n + 1) >> 1) ? k : k - n) * inv_n;
}

__device__ __forceinline__ float powi_pos(float x, int n) {
  float r = 1.0f;
  while (n > 0) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

// a[q] *= H(u, v) for the column v owned by this thread, rows u = j + q*TPT.
template <int L>
__device__ __forceinline__ void apply_mask(float2 (&a)[elems_per_thread(L)], int j, int v, int M,
                                           const MaskArgs& mk) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  switch (mk.kind) {
    case FFT_MASK_TENSOR_F32: {
      const float* col = mk.data + v;
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = cscale(a[q], __ldg(col + (int64_t)(j + q * TPT) * M));
      break;
    }
    case FFT_MASK_GAUSSIAN: {
      const float fv = freq_of(v, M, mk.inv_m);
      const float fv2 = fv * fv;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const float fu = freq_of(j + q * TPT, L, mk.inv_n);
        a[q] = cscale(a[q], expf(fmaf(fu, fu, fv2) * mk.gauss_coef));
      }
      break;
    }
    case FFT_MASK_BUTTERWORTH: {
      const float fv = freq_of(v, M, mk.inv_m);
      const float fv2 = fv * fv;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const float fu = freq_of(j + q * TPT, L, mk.inv_n);
        const float qq = fmaf(fu, fu, fv2) * mk.inv_fc2;
        const float p = (mk.order == 4) ? (qq * qq) * (qq * qq) : powi_pos(qq, mk.order);
        a[q] = cscale(a[q], __builtin_amdgcn_rcpf(1.0f + p));
      }
      break;
    }
    case FFT_MASK_DISC: {
      const double dv = (double)v - mk.c2;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const double du = (double)(j + q * TPT) - mk.c1;
        if (du * du + dv * dv <= mk.disc_b2) a[q] = make_float2(0.f, 0.f);
      }
      break;
    }
    default:
      break;
  }
}

// ============================================================== kernel A
// Batched transforms along contiguous rows, row-major in and out.
template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_rows_rm(const void* __restrict__ in, int in_f32, void* __restrict__ out,
                                                  int out_f32, int64_t rows, int tpw, float scale,
                                                  const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int tid = threadIdx.x;
  const int t = tid / TPT, j = tid - t * TPT;
  const int64_t row = (int64_t)blockIdx.x * tpw + t;
  const bool ok = row < rows;
  float2 a[E];
  if (in_f32) {
    const float* src = static_cast<const float*>(in) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = make_float2(ok ? __ldg(src + q * TPT) : 0.f, 0.f);
  } else {
    const float2* src = static_cast<const float2*>(in) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = ok ? __ldg(src + q * TPT) : make_float2(0.f, 0.f);
  }
  fft_reg<L, INV>(a, j, smem + t * lds_size(L), tw);
  if (!ok) return;
  if (out_f32) {
    float* dst = static_cast<float*>(out) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * TPT] = a[q].x * scale;
  } else {
    float2* dst = static_cast<float2*>(out) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * TPT] = cscale(a[q], scale);
  }
}

// ============================================================== kernel B
// Row pass, real input, two rows packed into one complex transform
// z = f[2p] + i f[2p+1]; the two spectra are split with the Hermitian symmetry
// of a real sequence's DFT: A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i.
template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_rows_to_blk_pair(const float* __restrict__ in, float2* __restrict__ ws,
                                                           int rb, float scale, const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E, STR = lds_size(L);
  extern __shared__ float2 smem[];
  const int np = rb >> 1;
  const int tid = threadIdx.x, p = tid / TPT, j = tid - p * TPT;
  const int64_t g = blockIdx.x;
  const float* r0 = in + (g * rb + 2 * p) * (int64_t)L + j;
  const float* r1 = r0 + L;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = make_float2(__ldg(r0 + q * TPT), __ldg(r1 + q * TPT));
  float2* x = smem + p * STR;
  fft_reg<L, INV>(a, j, x, tw);
  __syncthreads();
  scatter_natural<L>(a, j, x);
  __syncthreads();
  const int nt = np * TPT;
  float4* dst = reinterpret_cast<float4*>(ws + g * (int64_t)L * rb);
  const float h = 0.5f * scale;
  for (int v = tid; v < L; v += nt) {
    const int vm = (L - v) & (L - 1);
    for (int pp = 0; pp < np; ++pp) {
      const float2 z = smem[pp * STR + lds_pad(v)];
      const float2 zm = smem[pp * STR + lds_pad(vm)];
      dst[(v * rb + 2 * pp) >> 1] = make_float4(h * (z.x + zm.x), h * (z.y - zm.y), h * (z.y + zm.y), h * (zm.x - z.x));
    }
  }
}

// Row pass into the blocked layout, one transform per row (complex input, or
// real input when rows cannot be paired).  Lanes interleave the RB rows.
template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_rows_to_blk(const void* __restrict__ in, int in_f32, float2* __restrict__ ws,
                                                      int rb, float scale, const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int lrb = ilog2_pow2(rb);
  const int tid = threadIdx.x, s = tid & (rb - 1), j = tid >> lrb;
  const int64_t g = blockIdx.x;
  const int64_t row = g * rb + s;
  float2 a[E];
  if (in_f32) {
    const float* src = static_cast<const float*>(in) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = make_float2(__ldg(src + q * TPT), 0.f);
  } else {
    const float2* src = static_cast<const float2*>(in) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = __ldg(src + q * TPT);
  }
  fft_reg<L, INV>(a, j, smem + s * region_stride(L, rb), tw);
  float2* dst = ws + g * (int64_t)L * rb + j * rb + s;
  const int qs = TPT * rb;
#pragma unroll
  for (int q = 0; q < E; ++q) dst[q * qs] = cscale(a[q], scale);
}

// ============================================================== kernel D
// Row pass out of the blocked layout into row-major output.
template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_rows_from_blk(const float2* __restrict__ ws, void* __restrict__ out,
                                                        int out_f32, int rb, float scale,
                                                        const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int lrb = ilog2_pow2(rb);
  const int tid = threadIdx.x, s = tid & (rb - 1), j = tid >> lrb;
  const int64_t g = blockIdx.x;
  const float2* src = ws + g * (int64_t)L * rb + j * rb + s;
  const int qs = TPT * rb;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = __ldg(src + q * qs);
  fft_reg<L, INV>(a, j, smem + s * region_stride(L, rb), tw);
  const int64_t row = g * rb + s;
  if (out_f32) {
    float* dst = static_cast<float*>(out) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * TPT] = a[q].x * scale;
  } else {
    float2* dst = static_cast<float2*>(out) + row * L + j;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * TPT] = cscale(a[q], scale);
  }
}

// ============================================================== kernel C
// Column tiles of the blocked layout.  Lane order: row-in-block s fastest,
// then column c of the tile, then the rest of the transform index j, so a
// wavefront's load covers runs of W*RB*8 contiguous bytes.
struct ColLanes {
  int s, c, j, jh;
};
__device__ __forceinline__ ColLanes col_lanes(int tid, int rb, int w) {
  const int lrb = ilog2_pow2(rb), lw = ilog2_pow2(w);
  ColLanes r;
  r.s = tid & (rb - 1);
  r.c = (tid >> lrb) & (w - 1);
  r.jh = tid >> (lrb + lw);
  r.j = r.jh * rb + r.s;
  return r;
}

template <int L>
__global__ __launch_bounds__(1024) void k_cols_filter(float2* __restrict__ ws, float2* __restrict__ save, int M,
                                                      int rb, int w, int tiles_per_img, MaskArgs mk,
                                                      const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int64_t i = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t img = i / tiles_per_img;
  const int tile = (int)(i - img * tiles_per_img);
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const int v = tile * w + ln.c;
  const int64_t off = img * (int64_t)L * M + (int64_t)ln.jh * M * rb + (int64_t)v * rb + ln.s;
  const int qs = TPT * M;
  float2* base = ws + off;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = base[q * qs];
  float2* x = smem + ln.c * region_stride(L, w);
  fft_reg<L, false>(a, ln.j, x, tw);
  if (save) {
    float2* sb = save + off;
#pragma unroll
    for (int q = 0; q < E; ++q) sb[q * qs] = a[q];
  }
  apply_mask<L>(a, ln.j, v, M, mk);
  fft_reg<L, true>(a, ln.j, x, tw);
  launder(base);  // recompute the store addresses instead of keeping 16 live
#pragma unroll
  for (int q = 0; q < E; ++q) base[q * qs] = a[q];
}

template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_cols_single(const float2* __restrict__ ws, void* __restrict__ out,
                                                      int out_f32, int M, int rb, int w, int tiles_per_img,
                                                      float scale, const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int64_t i = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t img = i / tiles_per_img;
  const int tile = (int)(i - img * tiles_per_img);
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const int v = tile * w + ln.c;
  const int qs = TPT * M;
  const float2* src = ws + img * (int64_t)L * M + (int64_t)ln.jh * M * rb + (int64_t)v * rb + ln.s;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = __ldg(src + q * qs);
  fft_reg<L, INV>(a, ln.j, smem + ln.c * region_stride(L, w), tw);
  const int64_t o = img * (int64_t)L * M + (int64_t)ln.j * M + v;
  if (out_f32) {
    float* dst = static_cast<float*>(out) + o;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * qs] = a[q].x * scale;
  } else {
    float2* dst = static_cast<float2*>(out) + o;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * qs] = cscale(a[q], scale);
  }
}

template <int L>
__global__ __launch_bounds__(1024) void k_cols_grad(const float2* __restrict__ ws, const float2* __restrict__ save,
                                                    float* __restrict__ grad, int64_t nimg, int M, int rb, int w,
                                                    float scale, const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const int v = tile * w + ln.c;
  const int qs = TPT * M;
  const int64_t off = (int64_t)ln.jh * M * rb + (int64_t)v * rb + ln.s;
  const int64_t plane = (int64_t)L * M;
  float2* x = smem + ln.c * region_stride(L, w);
  float acc[E];
#pragma unroll
  for (int q = 0; q < E; ++q) acc[q] = 0.f;
  for (int64_t b = 0; b < nimg; ++b) {
    const float2* src = ws + b * plane + off;
    float2 a[E];
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = __ldg(src + q * qs);
    fft_reg<L, false>(a, ln.j, x, tw);
    const float2* xs = save + b * plane + off;
    launder(xs);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const float2 X = __ldg(xs + q * qs);
      acc[q] = fmaf(X.x, a[q].x, fmaf(X.y, a[q].y, acc[q]));
    }
  }
  float* dst = grad + (int64_t)ln.j * M + v;
#pragma unroll
  for (int q = 0; q < E; ++q) dst[q * qs] = acc[q] * scale;
}

// ============================================================== kernel E
// Strided column pass over a row-major [L][C] matrix (four-step long 1D).
template <int L, bool INV>
__global__ __launch_bounds__(1024) void k_cols_strided(const float2* __restrict__ in, float2* __restrict__ out,
                                                       int C, int w, int tiles, int twiddle_transpose, float scale,
                                                       const float2* __restrict__ tlo,
                                                       const float2* __restrict__ thi, int h,
                                                       const float2* __restrict__ tw) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  extern __shared__ float2 smem[];
  const int64_t i = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t b = i / tiles;
  const int tile = (int)(i - b * tiles);
  const int c0 = tile * w;
  const int lw = ilog2_pow2(w);
  const int tid = threadIdx.x, c = tid & (w - 1), j = tid >> lw;
  const int64_t N = (int64_t)L * C;
  const int qs = TPT * C;
  const float2* src = in + b * N + (int64_t)j * C + c0 + c;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = __ldg(src + q * qs);
  const int stride = region_stride(L, w);
  float2* x = smem + c * stride;
  fft_reg<L, INV>(a, j, x, tw);
  if (twiddle_transpose) {
    const int n2 = c0 + c;
    const int lomask = (1 << h) - 1;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int t = (j + q * TPT) * n2;  // < N <= 2^24, exact
      const float2 lo = __ldg(tlo + (t & lomask)), hi = __ldg(thi + (t >> h));
      const float2 wv = make_float2(lo.x * hi.x - lo.y * hi.y, lo.x * hi.y + lo.y * hi.x);
      a[q] = cmul_tw<INV>(a[q], wv);
    }
    __syncthreads();
    scatter_natural<L>(a, j, x);
    __syncthreads();
    const int nthr = w * TPT;
    const int lL = ilog2_pow2(L);
    float2* dst = out + b * N + (int64_t)c0 * L;
    for (int idx = tid; idx < w * L; idx += nthr) {
      const int cc = idx >> lL, k = idx & (L - 1);
      dst[idx] = cscale(smem[cc * stride + lds_pad(k)], scale);
    }
  } else {
    float2* dst = out + b * N + (int64_t)j * C + c0 + c;
#pragma unroll
    for (int q = 0; q < E; ++q) dst[q * qs] = cscale(a[q], scale);
  }
}

// ============================================================== launchers
namespace {

std::mutex g_attr_mu;
std::set<std::pair<const void*, int>> g_attr_done;

// Allow up to the full 160 KiB of LDS for a kernel (once per device).
hipError_t allow_lds(const void* fn, int bytes) {
  if (bytes <= 65536) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (g_attr_done.count({fn, dev})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  if (e == hipSuccess) g_attr_done.insert({fn, dev});
  return e;
}

template <typename... Args>
hipError_t go(void (*k)(Args...), dim3 grid, dim3 block, int lds, hipStream_t st, Args... args) {
  if (grid.x == 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, block, lds, st, args...);
  return hipGetLastError();
}

#define FFTMI_LOG2_CASES(F) \
  F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14)

template <int LG>
struct RowsRm {
  static hipError_t run(bool inv, const void* in, bool in_f32, void* out, bool out_f32, int64_t rows, float scale,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    int tpw = TPT >= 256 ? 1 : 256 / TPT;
    if (rows < tpw) tpw = (int)(rows > 0 ? rows : 1);
    const int lds = tpw * lds_size(L) * (int)sizeof(float2);
    const dim3 grid((unsigned)((rows + tpw - 1) / tpw)), block(tpw * TPT);
    if (inv)
      return go(k_rows_rm<L, true>, grid, block, lds, lc.stream, in, (int)in_f32, out, (int)out_f32, rows, tpw,
                scale, lc.tw);
    return go(k_rows_rm<L, false>, grid, block, lds, lc.stream, in, (int)in_f32, out, (int)out_f32, rows, tpw, scale,
              lc.tw);
  }
};

template <int LG>
struct RowsToBlk {
  static hipError_t run(bool inv, bool pair, const void* in, bool in_f32, float2* ws, int64_t blocks, int rb,
                        float scale, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const dim3 grid((unsigned)blocks);
    if (pair) {
      const int np = rb / 2;
      const int lds = np * lds_size(L) * (int)sizeof(float2);
      const float* fin = static_cast<const float*>(in);
      if (inv) return go(k_rows_to_blk_pair<L, true>, grid, dim3(np * TPT), lds, lc.stream, fin, ws, rb, scale, lc.tw);
      return go(k_rows_to_blk_pair<L, false>, grid, dim3(np * TPT), lds, lc.stream, fin, ws, rb, scale, lc.tw);
    }
    const int lds = rb * region_stride(L, rb) * (int)sizeof(float2);
    if (inv)
      return go(k_rows_to_blk<L, true>, grid, dim3(rb * TPT), lds, lc.stream, in, (int)in_f32, ws, rb, scale, lc.tw);
    return go(k_rows_to_blk<L, false>, grid, dim3(rb * TPT), lds, lc.stream, in, (int)in_f32, ws, rb, scale, lc.tw);
  }
};

template <int LG>
struct RowsFromBlk {
  static hipError_t run(bool inv, const float2* ws, void* out, bool out_f32, int64_t blocks, int rb, float scale,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int lds = rb * region_stride(L, rb) * (int)sizeof(float2);
    const dim3 grid((unsigned)blocks), block(rb * TPT);
    if (inv) return go(k_rows_from_blk<L, true>, grid, block, lds, lc.stream, ws, out, (int)out_f32, rb, scale, lc.tw);
    return go(k_rows_from_blk<L, false>, grid, block, lds, lc.stream, ws, out, (int)out_f32, rb, scale, lc.tw);
  }
};

template <int LG>
struct ColsFilter {
  static hipError_t run(float2* ws, float2* save, int64_t nimg, int M, int rb, int w, const MaskArgs& mk,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int tiles = M / w;
    const int lds = w * region_stride(L, w) * (int)sizeof(float2);
    return go(k_cols_filter<L>, dim3((unsigned)(nimg * tiles)), dim3(w * TPT), lds, lc.stream, ws, save, M, rb, w,
              tiles, mk, lc.tw);
  }
};

template <int LG>
struct ColsSingle {
  static hipError_t run(bool inv, const float2* ws, void* out, bool out_f32, int64_t nimg, int M, int rb, int w,
                        float scale, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int tiles = M / w;
    const int lds = w * region_stride(L, w) * (int)sizeof(float2);
    const dim3 grid((unsigned)(nimg * tiles)), block(w * TPT);
    if (inv)
      return go(k_cols_single<L, true>, grid, block, lds, lc.stream, ws, out, (int)out_f32, M, rb, w, tiles, scale,
                lc.tw);
    return go(k_cols_single<L, false>, grid, block, lds, lc.stream, ws, out, (int)out_f32, M, rb, w, tiles, scale,
              lc.tw);
  }
};

template <int LG>
struct ColsGrad {
  static hipError_t run(const float2* ws, const float2* save, float* grad, int64_t nimg, int M, int rb, int w,
                        float scale, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int lds = w * region_stride(L, w) * (int)sizeof(float2);
    return go(k_cols_grad<L>, dim3((unsigned)(M / w)), dim3(w * TPT), lds, lc.stream, ws, save, grad, nimg, M, rb, w,
              scale, lc.tw);
  }
};

template <int LG>
struct ColsStrided {
  static hipError_t run(bool inv, bool twt, const float2* in, float2* out, int64_t batch, int C, int w, float scale,
                        const float2* tlo, const float2* thi, int h, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int tiles = C / w;
    const int lds = w * region_stride(L, w) * (int)sizeof(float2);
    const dim3 grid((unsigned)(batch * tiles)), block(w * TPT);
    if (inv)
      return go(k_cols_strided<L, true>, grid, block, lds, lc.stream, in, out, C, w, tiles, (int)twt, scale, tlo, thi,
                h, lc.tw);
    return go(k_cols_strided<L, false>, grid, block, lds, lc.stream, in, out, C, w, tiles, (int)twt, scale, tlo, thi, h,
              lc.tw);
  }
};

}  // namespace

#define FFTMI_DISPATCH(STRUCT, LOG2, ...)              \
  switch (LOG2) {                                      \
    FFTMI_LOG2_CASES(FFTMI_CASE_##STRUCT)              \
    default:                                           \
      return hipErrorInvalidValue;                     \
  }

#define FFTMI_CASE_RowsRm(K) \
  case K:                    \
    return RowsRm<K>::run(inv, in, in_f32, out, out_f32, rows, scale, lc);
#define FFTMI_CASE_RowsToBlk(K) \
  case K:                       \
    return RowsToBlk<K>::run(inv, pair, in, in_f32, ws, blocks, rb, scale, lc);
#define FFTMI_CASE_RowsFromBlk(K) \
  case K:                         \
    return RowsFromBlk<K>::run(inv, ws, out, out_f32, blocks, rb, scale, lc);
#define FFTMI_CASE_ColsFilter(K) \
  case K:                        \
    return ColsFilter<K>::run(ws, save, nimg, M, rb, w, mask, lc);
#define FFTMI_CASE_ColsSingle(K) \
  case K:                        \
    return ColsSingle<K>::run(inv, ws, out, out_f32, nimg, M, rb, w, scale, lc);
#define FFTMI_CASE_ColsGrad(K) \
  case K:                      \
    return ColsGrad<K>::run(ws, save, grad, nimg, M, rb, w, scale, lc);
#define FFTMI_CASE_ColsStrided(K) \
  case K:                         \
    return ColsStrided<K>::run(inv, twiddle_transpose, in, out, batch, C, w, scale, tw_lo, tw_hi, h, lc);

hipError_t launch_rows_rm(int log2L, bool inv, const void* in, bool in_f32, void* out, bool out_f32, int64_t rows,
                          float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsRm, log2L)
}

hipError_t launch_rows_to_blk(int log2L, bool inv, bool pair, const void* in, bool in_f32, float2* ws,
                              int64_t blocks, int rb, float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsToBlk, log2L)
}

hipError_t launch_rows_from_blk(int log2L, bool inv, const float2* ws, void* out, bool out_f32, int64_t blocks,
                                int rb, float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsFromBlk, log2L)
}

hipError_t launch_cols_filter(int log2L, float2* ws, float2* save, int64_t nimg, int M, int rb, int w,
                              const MaskArgs& mask, const Launch& lc) {
  FFTMI_DISPATCH(ColsFilter, log2L)
}

hipError_t launch_cols_single(int log2L, bool inv, const float2* ws, void* out, bool out_f32, int64_t nimg, int M,
                              int rb, int w, float scale, const Launch& lc) {
  FFTMI_DISPATCH(ColsSingle, log2L)
}

hipError_t launch_cols_grad(int log2L, const float2* ws, const float2* save, float* grad, int64_t nimg, int M,
                            int rb, int w, float scale, const Launch& lc) {
  FFTMI_DISPATCH(ColsGrad, log2L)
}

hipError_t launch_cols_strided(int log2L, bool inv, bool twiddle_transpose, const float2* in, float2* out,
                               int64_t batch, int C, int w, float scale, const float2* tw_lo, const float2* tw_hi,
                               int h, const Launch& lc) {
  FFTMI_DISPATCH(ColsStrided, log2L)
}

int lds_bytes_rows_rm(int log2L, int tpw) { return tpw * lds_size(1 << log2L) * (int)sizeof(float2); }
int lds_bytes_cols(int log2L, int w) { return w * region_stride(1 << log2L, w) * (int)sizeof(float2); }
int lds_bytes_rows_blk(int log2L, int nt) { return nt * region_stride(1 << log2L, nt) * (int)sizeof(float2); }

}  // namespace fftmi
