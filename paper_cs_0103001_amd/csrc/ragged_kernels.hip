// ragged_kernels.hip -- the three passes of the FFT -> filter -> IFFT path over
// a ragged batch of square images with power-of-two sides 1 .. 2048.
//
// Each pass is one persistent kernel over a host-built list of tiles
// {image, tile}.  A workgroup of T threads takes tiles from the list (slot n,
// n + grid, ...) and switches on the tile's image size to the transform of
// that length, so a single launch covers every size.  A tile is always
// T/TPT(s) transforms of 16 points per thread (T*16 points), whatever the
// image side s, which makes tiles of different images cost about the same.
// Twiddles (the FP32 tables of each side, rounded once from FP64): the short
// stage tables (stride <= 16) are copied into the front of LDS whenever a
// workgroup moves to a tile of another side (tiles are sorted by side), the
// long-stride stages' factors are loaded into registers at the start of each
// tile, next to the tile's data.
//
// Image i of side s occupies elements [off, off + s*s) of the packed input
// and output (row-major) and (s / rb) * bs elements from ws_off in the
// workspace, where it is kept in the blocked layout (u / rb) * bs + v * rb +
// u % rb with rb = min(4, TPT(s)) and the padded block stride bs, as in the
// uniform-batch passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/fftmi.h"
#include "fft_core.hpp"
#include "kernel_common.hpp"
#include "launch.hpp"

namespace fftmi {

namespace {

constexpr int kRaggedMaxBlock = 512;
constexpr bool kNtRowsFwd = (FFTMI_NT_RAGGED & 1) != 0, kNtCols = (FFTMI_NT_RAGGED & 2) != 0,
               kNtRowsInv = (FFTMI_NT_RAGGED & 4) != 0;
// LDS bytes reserved for the short stage tables (the largest, 2048 points:
// 15 x 16 entries)
constexpr int kRgTwBytes = 2048;
static_assert(mix_lds_bytes(1 << kRaggedMaxLog2) <= kRgTwBytes, "ragged twiddle area");

// Short stage tables of side 2^lg into the front of LDS when the workgroup's
// current side changes (a uniform branch).  The barrier keeps the copy from
// overwriting factors the previous tile may still read; the transform's first
// exchange orders the copy before the new tile's reads.
template <int L>
__device__ __forceinline__ void rg_tw_lds(const float2* __restrict__ tw) {
  if constexpr (mix_lds_entries(L) > 0) {
    extern __shared__ float4 lds_raw[];
    load_twiddles_lds_mix<L>(reinterpret_cast<float2*>(lds_raw), tw, threadIdx.x, blockDim.x);
  }
}

// Forward row transforms of one tile of complex input: rows u = t*R + r of
// the image, scaled, stored into the blocked workspace.
template <int L>
__device__ __forceinline__ void rg_rows_fwd(const float2* __restrict__ in, float2* __restrict__ ws,
                                            const RaggedImage& im, int t, const float2* __restrict__ tw, char* lds,
                                            float scale) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int R = (int)blockDim.x / TPT;
  const int tid = threadIdx.x, r = tid / TPT, j = tid - r * TPT;
  const int u = t * R + r;
  const bool ok = u < L;
  char* x = lds + r * lds_region_bytes(L, R);
  const float2* src = in + im.off + (int64_t)(ok ? u : 0) * L;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = ok ? ldh<kNtRowsFwd>(src, j + q * TPT) : make_float2(0.f, 0.f);
  float2 twr[reg_tw_count_mix<L>()];
  load_twiddles_reg_mix<L>(twr, j, tw);
  fft_reg<L, false, kTwMix>(a, j, x, twr);
  if (ok) {
    const int rb = im.rb;
    float2* dst = ws + im.ws_off + (int64_t)(u / rb) * im.bs + (u % rb);
#pragma unroll
    for (int q = 0; q < E; ++q) dst[(j + q * TPT) * rb] = cscale(a[q], scale);
  }
}

// The same for real input, two rows per transform: rows u = 2 (t*R + r) and
// u + 1 packed as z = f_u + i f_(u+1).  The two spectra follow from the
// Hermitian symmetry of a real row's DFT, F_u(k) = (Z(k) + conj Z(-k)) / 2
// and F_(u+1)(k) = (Z(k) - conj Z(-k)) / 2i.  Every Z goes through LDS, and
// the stores are remapped so that consecutive lanes take consecutive pairs
// of one column: with rb >= 2 a pair is two neighbouring entries of a block,
// written as one float4.
template <int L>
__device__ __forceinline__ void rg_rows_fwd_pair(const float* __restrict__ in, float2* __restrict__ ws,
                                                 const RaggedImage& im, int t, const float2* __restrict__ tw,
                                                 char* lds, float scale) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int R = (int)blockDim.x / TPT;
  const int rbytes = lds_region_bytes(L, R);
  const int tid = threadIdx.x, r = tid / TPT, j = tid - r * TPT;
  const int u = 2 * (t * R + r);
  char* x = lds + r * rbytes;
  {
    const bool ok = u < L, ok2 = u + 1 < L;
    const float* src = in + im.off + (int64_t)(ok ? u : 0) * L;
    float2 a[E];
#pragma unroll
    for (int q = 0; q < E; ++q)
      a[q] = make_float2(ok ? ldh<kNtRowsFwd>(src, j + q * TPT) : 0.f, ok2 ? ldh<kNtRowsFwd>(src + L, j + q * TPT) : 0.f);
    float2 twr[reg_tw_count_mix<L>()];
    load_twiddles_reg_mix<L>(twr, j, tw);
    fft_reg<L, false, kTwMix>(a, j, x, twr);
    lds_barrier();  // the transform's last readers of x are done
    scatter_natural<L, kBoth>(a, j, x);
    lds_barrier();
  }
  // store lanes: pair pp = tid % R of the tile, columns v = tid / R + i*TPT
  const int pp = tid & (R - 1), v0 = tid / R;
  const int up = 2 * (t * R + pp);
  if (up >= L) return;
  const bool two = up + 1 < L;
  const float2* xs = reinterpret_cast<const float2*>(lds + pp * rbytes);
  const float h = 0.5f * scale;
  const int rb = im.rb;
  float2* d0 = ws + im.ws_off + (int64_t)(up / rb) * im.bs + (up % rb);
  float2* d1 = ws + im.ws_off + (int64_t)((up + 1) / rb) * im.bs + ((up + 1) % rb);
  // one float4 per (pair, column) when the pair shares a block and the
  // image's workspace starts on a 16-byte boundary (uniform per image)
  const bool f4 = rb >= 2 && ((im.ws_off & 1) == 0);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int v = v0 + i * TPT;
    const float2 z = xs[lds_pad(v)];
    const float2 zm = xs[lds_pad((L - v) & (L - 1))];
    const float4 o = make_float4(h * (z.x + zm.x), h * (z.y - zm.y), h * (z.y + zm.y), h * (zm.x - z.x));
    if (f4) {
      *reinterpret_cast<float4*>(d0 + v * rb) = o;
    } else {
      d0[v * rb] = make_float2(o.x, o.y);
      if (two) d1[v * rb] = make_float2(o.z, o.w);
    }
  }
}

// Column tile: w = T/TPT columns v = t*w + c, forward transform, mask,
// inverse transform, in place in the blocked workspace.
template <int L, int MK>
__device__ __forceinline__ void rg_cols(float2* __restrict__ ws, const RaggedImage& im, int t, const MaskArgs& mk0,
                                        const float2* __restrict__ tw, char* lds) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int w = (int)blockDim.x / TPT;
  const int rb = im.rb;
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const int v = t * w + ln.c;
  const bool ok = v < L;
  char* x = lds + ln.c * lds_region_bytes(L, w);
  float2* base = ws + im.ws_off + (int64_t)ln.jh * im.bs + (ok ? v : 0) * rb + ln.s;
  const int64_t qs = (int64_t)(TPT / rb) * im.bs;
  float2 a[E];
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = ok ? ldh<kNtCols>(base + q * qs, 0) : make_float2(0.f, 0.f);
  float2 twr[reg_tw_count_mix<L>()];
  load_twiddles_reg_mix<L>(twr, ln.j, tw);
  fft_reg<L, false, kTwMix>(a, ln.j, x, twr);
  MaskArgs mk = mk0;
  mk.inv_n = mk.inv_m = 1.0f / (float)L;
  const MaskEval<L, MK> me(mk, ln.j, v, L);
  me.apply(a, ln.j, mk);
  fft_reg<L, true, kTwMix>(a, ln.j, x, twr);
  if (ok) {
#pragma unroll
    for (int q = 0; q < E; ++q) base[q * qs] = a[q];
  }
}

// Inverse row transforms of one tile out of the blocked workspace.
template <int L, bool OUT_F32>
__device__ __forceinline__ void rg_rows_inv(const float2* __restrict__ ws, void* __restrict__ out,
                                            const RaggedImage& im, int t, const float2* __restrict__ tw, char* lds,
                                            float scale) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int R = (int)blockDim.x / TPT;
  const int tid = threadIdx.x, r = tid / TPT, j = tid - r * TPT;
  const int u = t * R + r;
  const bool ok = u < L;
  const int rbytes = lds_region_bytes(L, R);
  char* x = lds + r * rbytes;
  const int rb = im.rb;
  float2 a[E];
  if (rb >= 2 && R >= 2 && (im.ws_off & 1) == 0) {
    // rows in pairs (neighbours in a block) as float4s, consecutive lanes
    // on consecutive pairs of one column, handed to the transforms through
    // LDS (R is a power of two)
    const int P = R >> 1;
    const int pp = tid & (P - 1), v0 = tid / P;
    const int up = t * R + 2 * pp;
    lds_barrier();  // the previous tile's readers of the regions are done
    if (up < L) {
      const float4* src = reinterpret_cast<const float4*>(ws + im.ws_off + (int64_t)(up / rb) * im.bs + (up % rb));
      float2* x0 = reinterpret_cast<float2*>(lds + (2 * pp) * rbytes);
      float2* x1 = reinterpret_cast<float2*>(lds + (2 * pp + 1) * rbytes);
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        const int v = v0 + i * 2 * TPT;
        const float4 y = ldh<kNtRowsInv>(src, v * (rb >> 1));
        x0[lds_pad(v)] = make_float2(y.x, y.y);
        x1[lds_pad(v)] = make_float2(y.z, y.w);
      }
    }
    lds_barrier();
    gather_natural<L, kBoth>(a, j, x);
  } else {
    const float2* src = ws + im.ws_off + (int64_t)((ok ? u : 0) / rb) * im.bs + ((ok ? u : 0) % rb);
#pragma unroll
    for (int q = 0; q < E; ++q) a[q] = ok ? ldh<kNtRowsInv>(src, (j + q * TPT) * rb) : make_float2(0.f, 0.f);
  }
  float2 twr[reg_tw_count_mix<L>()];
  load_twiddles_reg_mix<L>(twr, j, tw);
  fft_reg<L, true, kTwMix>(a, j, x, twr);
  if (ok) {
    if constexpr (OUT_F32) {
      float* dst = static_cast<float*>(out) + im.off + (int64_t)u * L;
#pragma unroll
      for (int q = 0; q < E; ++q) dst[j + q * TPT] = a[q].x * scale;
    } else {
      float2* dst = static_cast<float2*>(out) + im.off + (int64_t)u * L;
#pragma unroll
      for (int q = 0; q < E; ++q) dst[j + q * TPT] = cscale(a[q], scale);
    }
  }
}

// Forward scale 1/s (eq. 5) or 1; inverse 1/s (2D-IDFT) or 1/s^2.
__device__ __forceinline__ float rg_scale(int lg, int fwd, int numpy) {
  const float s = (float)(1 << lg);
  if (fwd) return numpy ? 1.0f : 1.0f / s;
  return numpy ? 1.0f / (s * s) : 1.0f / s;
}

#define FFTMI_RG_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

template <bool IN_F32>
__global__ __launch_bounds__(kRaggedMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_ragged_rows_fwd(const void* __restrict__ in, float2* __restrict__ ws,
                                                                     const RaggedImage* __restrict__ imgs,
                                                                     const int2* __restrict__ tiles, int ntiles,
                                                                     TwTable tw, int numpy) {
  char* lds = lds_base() + kRgTwBytes;
  int cur_lg = -1;
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int2 tl = tiles[tile_of(n, ntiles)];
    const RaggedImage im = imgs[tl.x];
    const float sc = rg_scale(im.lg, 1, numpy);
    switch (im.lg) {
#define FFTMI_RG_ROWS_FWD(K)                                              \
  case K:                                                                 \
    if (im.lg != cur_lg) {                                                \
      lds_barrier();                                                      \
      rg_tw_lds<1 << K>(tw.p[K]);                                         \
      cur_lg = im.lg;                                                     \
    }                                                                     \
    if constexpr (IN_F32)                                                 \
      rg_rows_fwd_pair<1 << K>(static_cast<const float*>(in), ws, im, tl.y, tw.p[K], lds, sc); \
    else                                                                  \
      rg_rows_fwd<1 << K>(static_cast<const float2*>(in), ws, im, tl.y, tw.p[K], lds, sc); \
    break;
      FFTMI_RG_CASES(FFTMI_RG_ROWS_FWD)
#undef FFTMI_RG_ROWS_FWD
      default:
        break;
    }
  }
}

template <int MK>
__global__ __launch_bounds__(kRaggedMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_ragged_cols(float2* __restrict__ ws,
                                                                 const RaggedImage* __restrict__ imgs,
                                                                 const int2* __restrict__ tiles, int ntiles,
                                                                 MaskArgs mk, TwTable tw) {
  char* lds = lds_base() + kRgTwBytes;
  int cur_lg = -1;
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int2 tl = tiles[tile_of(n, ntiles)];
    const RaggedImage im = imgs[tl.x];
    switch (im.lg) {
#define FFTMI_RG_COLS(K)                                  \
  case K:                                                 \
    if (im.lg != cur_lg) {                                                \
      lds_barrier();                                                      \
      rg_tw_lds<1 << K>(tw.p[K]);                                         \
      cur_lg = im.lg;                                                     \
    }                                                                     \
    rg_cols<1 << K, MK>(ws, im, tl.y, mk, tw.p[K], lds);  \
    break;
      FFTMI_RG_CASES(FFTMI_RG_COLS)
#undef FFTMI_RG_COLS
      default:
        break;
    }
  }
}

template <bool OUT_F32>
__global__ __launch_bounds__(kRaggedMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_ragged_rows_inv(const float2* __restrict__ ws, void* __restrict__ out,
                                                                     const RaggedImage* __restrict__ imgs,
                                                                     const int2* __restrict__ tiles, int ntiles,
                                                                     TwTable tw, int numpy) {
  char* lds = lds_base() + kRgTwBytes;
  int cur_lg = -1;
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int2 tl = tiles[tile_of(n, ntiles)];
    const RaggedImage im = imgs[tl.x];
    const float sc = rg_scale(im.lg, 0, numpy);
    switch (im.lg) {
#define FFTMI_RG_ROWS_INV(K)                                              \
  case K:                                                                 \
    if (im.lg != cur_lg) {                                                \
      lds_barrier();                                                      \
      rg_tw_lds<1 << K>(tw.p[K]);                                         \
      cur_lg = im.lg;                                                     \
    }                                                                     \
    rg_rows_inv<1 << K, OUT_F32>(ws, out, im, tl.y, tw.p[K], lds, sc);    \
    break;
      FFTMI_RG_CASES(FFTMI_RG_ROWS_INV)
#undef FFTMI_RG_ROWS_INV
      default:
        break;
    }
  }
}

// ------------------------------------------------------------ small images
// Images of side s <= 2^kRaggedSmallMaxLog2 in one pass from LDS: a
// workgroup of kRaggedSmallBlock threads loads IPW(s) whole images of one
// side into LDS (each row in a padded slot), transforms the rows (one
// transform of 16 points per thread per row), writes the row spectra back
// transposed, transforms the columns, applies the mask, transforms back,
// transposes back, transforms the rows back and writes the images out:
// 4 (or 8) bytes read and 8 (or 4) written per pixel instead of the three
// HBM passes.  Each transform uses its own slot as exchange space, since its
// data are in registers while it runs.  Work items are {first entry in the
// index list, count} with the images of one item of one side.
constexpr int small_ipw_c(int lg) {
  return kRaggedSmallBlock / ((1 << lg) * threads_per_transform(1 << lg));
}
// bytes of one row slot: a transform's padded LDS region, spread over the
// banks like the tiles that interleave as many transforms per wavefront
constexpr int small_row_bytes(int lg) {
  return lds_region_bytes(1 << lg, 64 / threads_per_transform(1 << lg) < 32 ? 64 / threads_per_transform(1 << lg) : 32);
}
constexpr int small_lds_c(int lg) { return small_ipw_c(lg) * (1 << lg) * small_row_bytes(lg); }
constexpr int small_lds_max(int lg = 0) {
  return lg > kRaggedSmallMaxLog2 ? 0
                                   : (small_lds_c(lg) > small_lds_max(lg + 1) ? small_lds_c(lg) : small_lds_max(lg + 1));
}
constexpr int kSmallLds = kRgTwBytes + small_lds_max();
static_assert(kSmallLds <= kLdsBytes, "small-image slots exceed LDS");

template <int LG, int MK, bool IN_F32, bool OUT_F32>
__device__ __forceinline__ void rg_small(const void* __restrict__ in, void* __restrict__ out,
                                         const RaggedImage* __restrict__ imgs, const int* __restrict__ idx,
                                         int2 item, const float2* __restrict__ tw, char* lds, const MaskArgs& mk0,
                                         int numpy) {
  constexpr int L = 1 << LG, E = elems_per_thread(L), TPT = L / E, PT = L * TPT;
  constexpr int IPW = small_ipw_c(LG), RS = small_row_bytes(LG);
  static_assert(IPW * PT == kRaggedSmallBlock, "every thread owns one row of one image slot");
  // the thread's indices are laundered per item: otherwise the mask values and
  // LDS addresses, which do not change from item to item, are hoisted out of
  // the item loop and held (spilled) across the transforms
  const int tid = (int)fresh(threadIdx.x), k = tid / PT, tl = tid - k * PT, rr = tl / TPT, j = tl - rr * TPT;
  const bool live = k < item.y;
  char* slot = lds + k * (L * RS);
  char* row = slot + rr * RS;
  auto at = [&](int r, int c) __attribute__((always_inline)) {
    return reinterpret_cast<float2*>(slot + r * RS) + lds_pad(c);
  };
  int64_t off = 0;
  if (live) off = imgs[idx[item.x + k]].off;
  // load the image, coalesced (element e = i * PT + tl), into the row slots
  lds_barrier();  // the previous item's readers of the slots are done
  if (live) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = i * PT + tl;
      float2 v;
      if constexpr (IN_F32)
        v = make_float2(__ldg(static_cast<const float*>(in) + off + e), 0.f);
      else
        v = __ldg(static_cast<const float2*>(in) + off + e);
      *at(e / L, e % L) = v;
    }
  }
  lds_barrier();
  float2 a[E];
  gather_natural<L, kBoth>(a, j, row);
  float2 twr[reg_tw_count_mix<L>()];
  load_twiddles_reg_mix<L>(twr, j, tw);
  // rows forward, eq. 5's 1/s
  fft_reg<L, false, kTwMix>(a, j, row, twr);
  const float fs = rg_scale(LG, 1, numpy), is = rg_scale(LG, 0, numpy);
  // transposed into the slots: slot row v holds column v of the spectrum
  lds_barrier();
#pragma unroll
  for (int q = 0; q < E; ++q) *at(j + q * TPT, rr) = cscale(a[q], fs);
  lds_barrier();
  gather_natural<L, kBoth>(a, j, row);
  // column rr: forward, mask, inverse
  fft_reg<L, false, kTwMix>(a, j, row, twr);
  MaskArgs mk = mk0;
  mk.inv_n = mk.inv_m = 1.0f / (float)L;
  const MaskEval<L, MK> me(mk, j, rr, L);
  me.apply(a, j, mk);
  fft_reg<L, true, kTwMix>(a, j, row, twr);
  // transposed back to rows
  lds_barrier();
#pragma unroll
  for (int q = 0; q < E; ++q) *at(j + q * TPT, rr) = a[q];
  lds_barrier();
  gather_natural<L, kBoth>(a, j, row);
  // rows inverse, the 2D-IDFT's 1/s, out through the slots, coalesced
  fft_reg<L, true, kTwMix>(a, j, row, twr);
  lds_barrier();
  scatter_natural<L, kBoth>(a, j, row);
  lds_barrier();
  if (live) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = i * PT + tl;
      const float2 v = *at(e / L, e % L);
      if constexpr (OUT_F32)
        static_cast<float*>(out)[off + e] = v.x * is;
      else
        static_cast<float2*>(out)[off + e] = cscale(v, is);
    }
  }
}

#define FFTMI_RG_SMALL_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int MK, bool IN_F32, bool OUT_F32>
__global__ __launch_bounds__(kRaggedSmallBlock) void k_ragged_small(const void* __restrict__ in, void* __restrict__ out,
                                                                     const RaggedImage* __restrict__ imgs,
                                                                     const int* __restrict__ idx,
                                                                     const int2* __restrict__ items, int nitems,
                                                                     MaskArgs mk, TwTable tw, int numpy) {
  char* lds = lds_base() + kRgTwBytes;
  int cur_lg = -1;
  for (int n = blockIdx.x; n < nitems; n += gridDim.x) {
    const int2 it = items[n];
    const int lg = imgs[idx[it.x]].lg;
    switch (lg) {
#define FFTMI_RG_SMALL(K)                                                                  \
  case K:                                                                                  \
    if (lg != cur_lg) {                                                                    \
      lds_barrier();                                                                       \
      rg_tw_lds<1 << K>(tw.p[K]);                                                          \
      cur_lg = lg;                                                                         \
    }                                                                                      \
    rg_small<K, MK, IN_F32, OUT_F32>(in, out, imgs, idx, it, tw.p[K], lds, mk, numpy);     \
    break;
      FFTMI_RG_SMALL_CASES(FFTMI_RG_SMALL)
#undef FFTMI_RG_SMALL
      default:
        break;
    }
  }
}

// Persistent grid: resident workgroups (occupancy, optionally capped per
// CU), at most one per tile, a multiple of 8 where possible.
std::mutex g_rg_mu;
std::map<std::tuple<const void*, int, int, int>, int> g_rg_occ;

hipError_t rg_grid(const void* fn, int block, int lds, int cap, int ntiles, int* grid) {
  int dev = 0, per_cu = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(g_rg_mu);
    auto key = std::make_tuple(fn, block, lds, dev);
    auto it = g_rg_occ.find(key);
    if (it == g_rg_occ.end()) {
      if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
      }
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, (size_t)lds);
      if (e != hipSuccess) return e;
      g_rg_occ[key] = per_cu;
    } else {
      per_cu = it->second;
    }
  }
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  if (cap > 0 && per_cu > cap) per_cu = cap;
  int64_t g = persistent_grid(ntiles, (int64_t)per_cu * cus);
  *grid = (int)std::max<int64_t>(g, 1);
  return hipSuccess;
}

}  // namespace

int ragged_lds_bytes(int block) {
  int most = 0;  // transform regions, after the twiddle area
  for (int lg = 0; lg <= kRaggedMaxLog2; ++lg) {
    const int L = 1 << lg, tpt = threads_per_transform(L);
    const int per = block / tpt;  // transforms per tile
    most = std::max(most, per * lds_region_bytes(L, per));
  }
  return kRgTwBytes + most;
}

namespace {
const void* ragged_kernel(int pass, bool in_f32, bool out_f32, int mask_kind) {
  if (pass == 0)
    return in_f32 ? reinterpret_cast<const void*>(k_ragged_rows_fwd<true>)
                  : reinterpret_cast<const void*>(k_ragged_rows_fwd<false>);
  if (pass == 2)
    return out_f32 ? reinterpret_cast<const void*>(k_ragged_rows_inv<true>)
                   : reinterpret_cast<const void*>(k_ragged_rows_inv<false>);
  switch (mask_kind) {
    case FFT_MASK_GAUSSIAN:
      return reinterpret_cast<const void*>(k_ragged_cols<FFT_MASK_GAUSSIAN>);
    case FFT_MASK_BUTTERWORTH:
      return reinterpret_cast<const void*>(k_ragged_cols<FFT_MASK_BUTTERWORTH>);
    case FFT_MASK_NONE:
      return reinterpret_cast<const void*>(k_ragged_cols<FFT_MASK_NONE>);
    default:
      return nullptr;
  }
}
}  // namespace

hipError_t ragged_grid(int pass, bool in_f32, bool out_f32, int mask_kind, int block, int wg_cap, int ntiles,
                       int* grid) {
  *grid = 0;
  if (ntiles <= 0) return hipSuccess;
  if (block < 128 || block > kRaggedMaxBlock || (block & (block - 1))) return hipErrorInvalidValue;
  const void* fn = ragged_kernel(pass, in_f32, out_f32, mask_kind);
  if (!fn) return hipErrorInvalidValue;
  return rg_grid(fn, block, ragged_lds_bytes(block), wg_cap, ntiles, grid);
}

namespace {
template <int MK>
const void* small_kernel_for(bool in_f32, bool out_f32) {
  if (in_f32)
    return out_f32 ? reinterpret_cast<const void*>(k_ragged_small<MK, true, true>)
                   : reinterpret_cast<const void*>(k_ragged_small<MK, true, false>);
  return out_f32 ? reinterpret_cast<const void*>(k_ragged_small<MK, false, true>)
                 : reinterpret_cast<const void*>(k_ragged_small<MK, false, false>);
}
const void* small_kernel(bool in_f32, bool out_f32, int mask_kind) {
  switch (mask_kind) {
    case FFT_MASK_GAUSSIAN:
      return small_kernel_for<FFT_MASK_GAUSSIAN>(in_f32, out_f32);
    case FFT_MASK_BUTTERWORTH:
      return small_kernel_for<FFT_MASK_BUTTERWORTH>(in_f32, out_f32);
    case FFT_MASK_NONE:
      return small_kernel_for<FFT_MASK_NONE>(in_f32, out_f32);
    default:
      return nullptr;
  }
}
template <int MK>
void small_launch(bool in_f32, bool out_f32, int grid, hipStream_t st, const void* in, void* out,
                  const RaggedImage* imgs, const int* idx, const int2* items, int nitems, const MaskArgs& mk,
                  const TwTable& tw, int np) {
  const dim3 g(grid), b(kRaggedSmallBlock);
  if (in_f32 && out_f32)
    hipLaunchKernelGGL((k_ragged_small<MK, true, true>), g, b, (size_t)kSmallLds, st, in, out, imgs, idx, items,
                       nitems, mk, tw, np);
  else if (in_f32)
    hipLaunchKernelGGL((k_ragged_small<MK, true, false>), g, b, (size_t)kSmallLds, st, in, out, imgs, idx, items,
                       nitems, mk, tw, np);
  else if (out_f32)
    hipLaunchKernelGGL((k_ragged_small<MK, false, true>), g, b, (size_t)kSmallLds, st, in, out, imgs, idx, items,
                       nitems, mk, tw, np);
  else
    hipLaunchKernelGGL((k_ragged_small<MK, false, false>), g, b, (size_t)kSmallLds, st, in, out, imgs, idx, items,
                       nitems, mk, tw, np);
}
}  // namespace

int ragged_small_ipw(int lg) { return lg >= 0 && lg <= kRaggedSmallMaxLog2 ? small_ipw_c(lg) : 0; }

hipError_t ragged_small_grid(bool in_f32, bool out_f32, int mask_kind, int nitems, int* grid) {
  *grid = 0;
  if (nitems <= 0) return hipSuccess;
  const void* fn = small_kernel(in_f32, out_f32, mask_kind);
  if (!fn) return hipErrorInvalidValue;
  return rg_grid(fn, kRaggedSmallBlock, kSmallLds, 0, nitems, grid);
}

hipError_t launch_ragged_small(const void* in, bool in_f32, void* out, bool out_f32, const RaggedImage* imgs,
                               const int* idx, const int2* items, int nitems, int grid, const MaskArgs& mk,
                               const TwTable& tw, bool numpy, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (grid <= 0 || !small_kernel(in_f32, out_f32, mk.kind)) return hipErrorInvalidValue;
  const int np = numpy ? 1 : 0;
  if (mk.kind == FFT_MASK_GAUSSIAN)
    small_launch<FFT_MASK_GAUSSIAN>(in_f32, out_f32, grid, st, in, out, imgs, idx, items, nitems, mk, tw, np);
  else if (mk.kind == FFT_MASK_BUTTERWORTH)
    small_launch<FFT_MASK_BUTTERWORTH>(in_f32, out_f32, grid, st, in, out, imgs, idx, items, nitems, mk, tw, np);
  else
    small_launch<FFT_MASK_NONE>(in_f32, out_f32, grid, st, in, out, imgs, idx, items, nitems, mk, tw, np);
  return hipGetLastError();
}

hipError_t launch_ragged_pass(int pass, const void* in, bool in_f32, float2* ws, void* out, bool out_f32,
                              const RaggedImage* imgs, const int2* tiles, int ntiles, int block, int grid,
                              const MaskArgs& mk, const TwTable& tw, bool numpy, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || block < 128 || block > kRaggedMaxBlock || (block & (block - 1))) return hipErrorInvalidValue;
  if (!ragged_kernel(pass, in_f32, out_f32, mk.kind)) return hipErrorInvalidValue;
  const int lds = ragged_lds_bytes(block);
  const int np = numpy ? 1 : 0;
  if (pass == 0) {
    if (in_f32)
      hipLaunchKernelGGL(k_ragged_rows_fwd<true>, dim3(grid), dim3(block), (size_t)lds, st, in, ws, imgs, tiles,
                         ntiles, tw, np);
    else
      hipLaunchKernelGGL(k_ragged_rows_fwd<false>, dim3(grid), dim3(block), (size_t)lds, st, in, ws, imgs, tiles,
                         ntiles, tw, np);
  } else if (pass == 1) {
    if (mk.kind == FFT_MASK_GAUSSIAN)
      hipLaunchKernelGGL(k_ragged_cols<FFT_MASK_GAUSSIAN>, dim3(grid), dim3(block), (size_t)lds, st, ws, imgs, tiles,
                         ntiles, mk, tw);
    else if (mk.kind == FFT_MASK_BUTTERWORTH)
      hipLaunchKernelGGL(k_ragged_cols<FFT_MASK_BUTTERWORTH>, dim3(grid), dim3(block), (size_t)lds, st, ws, imgs,
                         tiles, ntiles, mk, tw);
    else
      hipLaunchKernelGGL(k_ragged_cols<FFT_MASK_NONE>, dim3(grid), dim3(block), (size_t)lds, st, ws, imgs, tiles,
                         ntiles, mk, tw);
  } else {
    if (out_f32)
      hipLaunchKernelGGL(k_ragged_rows_inv<true>, dim3(grid), dim3(block), (size_t)lds, st, ws, out, imgs, tiles,
                         ntiles, tw, np);
    else
      hipLaunchKernelGGL(k_ragged_rows_inv<false>, dim3(grid), dim3(block), (size_t)lds, st, ws, out, imgs, tiles,
                         ntiles, tw, np);
  }
  return hipGetLastError();
}

}  // namespace fftmi
