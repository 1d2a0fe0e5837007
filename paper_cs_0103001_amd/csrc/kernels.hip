// kernels.hip -- gfx950 kernels of the FFT -> filter -> IFFT path and their
// launchers.
//
// Every kernel is persistent and software-pipelined: a workgroup copies the
// twiddle tables of its transform length into LDS once, loads its first tile,
// then loops over tiles, issuing the global loads of the next tile before it
// transforms the current one.  A transform keeps its data in registers (16
// complex values per thread), exchanges it through LDS between radix passes
// and touches HBM once on the way in and once on the way out.  With no global
// loads inside the transform (the twiddles are in LDS), the next tile's loads
// stay in flight for the whole computation.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <utility>

#include "../../include/fftmi.h"
#include "fft_core.hpp"
#include "kernel_common.hpp"
#include "launch.hpp"

namespace fftmi {

// ============================================================== kernel A
// Batched transforms along contiguous rows, row-major in and out.  A tile is
// tpw rows; the last tile may be partial.  The workgroup loops over tiles
// (slot n, n + grid, ...) and prefetches the next tile into registers while
// the current one is transformed.
template <int L, bool INV>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_rm(const void* __restrict__ in, int in_f32, void* __restrict__ out,
                                                  int out_f32, int64_t rows, int tpw, int ntiles, float scale,
                                                  const float2* __restrict__ tws) {
  using S = Shape<L>;
  using C = Rows1DCfg<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const int tid = threadIdx.x, t = tid / TPT, j = tid - t * TPT;
  const Twiddles<L, C::TWM> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = regions<L, C>() + t * C::region(1);
  const unsigned lane = (unsigned)(t * L + j);
  float2 a[E], nx[Prefetch<L, kPassRows1D>::on ? E : 1];
  auto load = [&](float2(&d)[E], int tile) __attribute__((always_inline)) {
    const bool ok = (int64_t)tile * tpw + t < rows;
    if (in_f32) {
      const float* b = static_cast<const float*>(in) + (int64_t)tile * tpw * L;
      {
        const unsigned f_lane = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) d[q] = make_float2(ok ? ldh<(FFTMI_NT_1D & 1) != 0>(b, f_lane + q * TPT) : 0.f, 0.f);
      }
    } else {
      const float2* b = static_cast<const float2*>(in) + (int64_t)tile * tpw * L;
      {
        const unsigned f_lane = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) d[q] = ok ? ldh<(FFTMI_NT_1D & 1) != 0>(b, f_lane + q * TPT) : make_float2(0.f, 0.f);
      }
    }
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassRows1D>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int tile = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassRows1D>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, tile);
    }
    fft_reg<L, INV, C::TWM, C::SPLIT>(a, j, x, tw);
    if ((int64_t)tile * tpw + t < rows) {
      if (out_f32) {
        float* b = static_cast<float*>(out) + (int64_t)tile * tpw * L;
        {
          const unsigned f_lane = fresh(lane);
#pragma unroll
          for (int q = 0; q < E; ++q) sth<(FFTMI_NT_1D & 2) != 0>(b + f_lane + q * TPT, a[q].x * scale);
        }
      } else {
        float2* b = static_cast<float2*>(out) + (int64_t)tile * tpw * L;
        {
          const unsigned f_lane = fresh(lane);
#pragma unroll
          for (int q = 0; q < E; ++q) sth<(FFTMI_NT_1D & 2) != 0>(b + f_lane + q * TPT, cscale(a[q], scale));
        }
      }
    }
    if constexpr (Prefetch<L, kPassRows1D>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// ============================================================== kernel B
// Row pass of real rows into the blocked layout, rows packed in pairs into
// complex transforms z = f[2p] + i f[2p+1]; the two spectra are split with the
// Hermitian symmetry of a real sequence's DFT:
// A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i.
// A tile is npt pairs (a power of two) of one block of rb rows.
//
// HALF: only columns 0 .. L/2-1 are stored (blocks of L/2 columns), the
// half spectrum that a real row determines.  Column 0 carries the two real
// values A[0] and A[L/2] of a row as one complex number (A[0] + i A[L/2]).
//
// DIFF: the rows are in - in2 (the residual x - c of the fused MSE form),
// formed as the two inputs are loaded.
template <int L, bool INV, bool HALF, bool DIFF = false>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_to_blk_pair(const float* __restrict__ in,
                                                                   float2* __restrict__ ws, int rb, unsigned bs,
                                                                   int npt, int ntiles, float scale,
                                                                   const float2* __restrict__ tws,
                                                                   const float* __restrict__ in2 = nullptr) {
  static_assert(!HALF || !kSplitExchange, "half spectrum with whole complex LDS entries");
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT, RBY = lds_region_bytes(L, 1);
  char* reg = regions<L>();
  const int np = rb >> 1;                      // pairs per block
  const int lsub = ilog2_pow2(np / npt);       // tiles per block = np / npt
  const int tid = threadIdx.x, p = tid / TPT, j = tid - p * TPT;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = reg + p * RBY;
  const unsigned lane_in = (unsigned)(2 * p * L + j);
  // epilogue lanes: pair pp of the tile, columns v = v0 + i*TPT; each writes
  // rows 2pp, 2pp+1 as one float4 at float4 index v*np + pair
  const int lnpt = ilog2_pow2(npt);
  const int pp = tid & (npt - 1), v0 = tid >> lnpt;
  const unsigned lane_out = (unsigned)(v0 * np + pp);
  const char* xs = reg + pp * RBY;
  const float h = 0.5f * scale;
  float2 a[E], nx[Prefetch<L, kPassRowsIn>::on ? E : 1];
  auto first_row = [&](int t) __attribute__((always_inline)) {
    return (int64_t)(t >> lsub) * rb + (t & ((1 << lsub) - 1)) * 2 * npt;
  };
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    const float* b = in + first_row(t) * L;
    const unsigned l = fresh(lane_in);
#pragma unroll
    for (int q = 0; q < E; ++q) d[q] = make_float2(ld_nt(b, l + q * TPT), ld_nt(b, l + L + q * TPT));
    if constexpr (DIFF) {
      const float* b2 = in2 + first_row(t) * L;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        d[q].x -= ld_nt(b2, l + q * TPT);
        d[q].y -= ld_nt(b2, l + L + q * TPT);
      }
    }
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassRowsIn>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassRowsIn>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    fft_reg<L, INV, S::TWM>(a, j, x, tw);
    // float4 base of this tile: block start plus the tile's first pair
    float4* dst = reinterpret_cast<float4*>(ws + (int64_t)(t >> lsub) * bs) + (t & ((1 << lsub) - 1)) * npt;
    const unsigned lo = fresh(lane_out);
    if constexpr (kSplitExchange) {
      float ax[E], by[E];
      lds_barrier();
      scatter_natural<L, kRe>(a, j, x);
      lds_barrier();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int v = v0 + i * TPT, vm = (L - v) & (L - 1);
        const float zr = reinterpret_cast<const float*>(xs)[lds_pad(v)];
        const float zmr = reinterpret_cast<const float*>(xs)[lds_pad(vm)];
        ax[i] = h * (zr + zmr);
        by[i] = h * (zmr - zr);
      }
      lds_barrier();
      scatter_natural<L, kIm>(a, j, x);
      lds_barrier();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int v = v0 + i * TPT, vm = (L - v) & (L - 1);
        const float zi = reinterpret_cast<const float*>(xs)[lds_pad(v)];
        const float zmi = reinterpret_cast<const float*>(xs)[lds_pad(vm)];
        sth<DIFF && (FFTMI_NT_DIFF != 0)>(dst + lo + i * TPT * np, make_float4(ax[i], h * (zi - zmi), h * (zi + zmi), by[i]));
      }
    } else {
      lds_barrier();
      scatter_natural<L, kBoth>(a, j, x);
      lds_barrier();
#pragma unroll
      for (int i = 0; i < (HALF ? E / 2 : E); ++i) {
        const int v = v0 + i * TPT, vm = (L - v) & (L - 1);
        const float2 z = reinterpret_cast<const float2*>(xs)[lds_pad(v)];
        const float2 zm = reinterpret_cast<const float2*>(xs)[lds_pad(vm)];
        float4 o = make_float4(h * (z.x + zm.x), h * (z.y - zm.y), h * (z.y + zm.y), h * (zm.x - z.x));
        if (HALF && i == 0 && v0 == 0) {
          // A[0], B[0] are 2h Re Z[0], 2h Im Z[0]; A[L/2], B[L/2] likewise from Z[L/2]
          const float2 zh = reinterpret_cast<const float2*>(xs)[lds_pad(L / 2)];
          o = make_float4(2.f * h * z.x, 2.f * h * zh.x, 2.f * h * z.y, 2.f * h * zh.y);
        }
        sth<DIFF && (FFTMI_NT_DIFF != 0)>(dst + lo + i * TPT * np, o);
      }
    }
    if constexpr (Prefetch<L, kPassRowsIn>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// Inverse row transforms of a half spectrum (last pass of the half-spectrum
// path).  Two rows' half spectra Y1, Y2 (columns 0 .. L/2-1 of the blocked
// layout, column 0 holding Y(0) + i Y(L/2)) give W = Y1 + i Y2 on all L
// columns through Y(L - v) = conj Y(v); the inverse transform of W is
// y1 + i y2 with both rows real.  A tile is npt pairs of one block, loaded as
// float4 (Y1(v), Y2(v)) and staged through LDS.
template <int L, bool F32>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_c2r_pair(const float2* __restrict__ ws, void* __restrict__ out,
                                                                int rb, unsigned bs, int npt, int ntiles, float scale,
                                                                const float2* __restrict__ tws) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT, RBY = lds_region_bytes(L, 1), H = L / 2, EH = E / 2;
  static_assert(L >= 2 && !kSplitExchange, "half spectrum rows");
  char* reg = regions<L>();
  const int np = rb >> 1;
  const int lsub = ilog2_pow2(np / npt);
  const int tid = threadIdx.x, p = tid / TPT, j = tid - p * TPT;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  float2* x = reinterpret_cast<float2*>(reg + p * RBY);
  const unsigned lane = (unsigned)(j * np);
  constexpr bool PF = TPT <= 512;  // 1024-thread transforms have no room for a second tile
  float4 a[EH], nx[PF ? EH : 1];
  auto pair_of = [&](int t) __attribute__((always_inline)) { return (t & ((1 << lsub) - 1)) * npt + p; };
  auto load = [&](float4(&d)[EH], int t) __attribute__((always_inline)) {
    const float4* b = reinterpret_cast<const float4*>(ws + (int64_t)(t >> lsub) * bs) + pair_of(t);
    const unsigned l = fresh(lane);
#pragma unroll
    for (int q = 0; q < EH; ++q) d[q] = ld(b, l + q * TPT * np);
  };
  int n = blockIdx.x;
  if constexpr (PF) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
#pragma unroll
    for (int q = 0; q < EH; ++q) asm volatile("" : "+v"(a[q].x), "+v"(a[q].y), "+v"(a[q].z), "+v"(a[q].w));
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (PF) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    lds_barrier();  // the previous tile's readers of x are done
#pragma unroll
    for (int q = 0; q < EH; ++q) {
      const int v = j + q * TPT;
      x[lds_pad(v)] = make_float2(a[q].x, a[q].y);
      x[lds_pad(H + v)] = make_float2(a[q].z, a[q].w);
    }
    lds_barrier();
    float2 w[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int u = j + q * TPT;
      if (q < EH) {
        const float2 y1 = x[lds_pad(u)], y2 = x[lds_pad(H + u)];
        w[q] = (u == 0) ? make_float2(y1.x, y2.x) : make_float2(y1.x - y2.y, y1.y + y2.x);
      } else {
        const int k = (u == H) ? 0 : L - u;  // u = H reads the packed column 0
        const float2 y1 = x[lds_pad(k)], y2 = x[lds_pad(H + k)];
        w[q] = (u == H) ? make_float2(y1.y, y2.y) : make_float2(y1.x + y2.y, y2.x - y1.y);
      }
    }
    fft_reg<L, true, S::TWM>(w, j, reinterpret_cast<char*>(x), tw);
    const int64_t r0 = (int64_t)(t >> lsub) * rb + 2 * pair_of(t);
    if constexpr (F32) {
      float* o = static_cast<float*>(out) + r0 * L;
      const unsigned l = fresh((unsigned)j);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        st_nt(&o[l + q * TPT], w[q].x * scale);
        st_nt(&o[l + L + q * TPT], w[q].y * scale);
      }
    } else {
      float2* o = static_cast<float2*>(out) + r0 * L;
      const unsigned l = fresh((unsigned)j);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        st_nt(&o[l + q * TPT], make_float2(w[q].x * scale, 0.f));
        st_nt(&o[l + L + q * TPT], make_float2(w[q].y * scale, 0.f));
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < EH; ++q) a[q] = nx[q];
    }
  }
}

// Row pass into the blocked layout, one transform per row (complex input, or
// real input when rows cannot be paired).  A tile is nt rows of one block
// (rows g*rb + sub*nt ...); lanes interleave those nt rows.
template <int L, bool INV>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_to_blk(const void* __restrict__ in, int in_f32, float2* __restrict__ ws,
                                                      int rb, unsigned bs, int nt, int ntiles, float scale,
                                                      const float2* __restrict__ tws) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const int lnt = ilog2_pow2(nt), lsub = ilog2_pow2(rb / nt);
  const int tid = threadIdx.x, sl = tid & (nt - 1), j = tid >> lnt;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = regions<L>() + sl * lds_region_bytes(L, nt);
  const unsigned lane_in = (unsigned)(sl * L + j), lane_out = (unsigned)(j * rb + sl);
  const int qs = TPT * rb;
  // first row of tile t; its block starts at element (t >> lsub) * bs
  auto row0 = [&](int t) __attribute__((always_inline)) {
    return (int64_t)(t >> lsub) * rb + (t & ((1 << lsub) - 1)) * nt;
  };
  float2 a[E], nx[Prefetch<L, kPassRowsIn>::on ? E : 1];
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    if (in_f32) {
      const float* b = static_cast<const float*>(in) + row0(t) * L;
      {
        const unsigned f_lane_in = fresh(lane_in);
#pragma unroll
        for (int q = 0; q < E; ++q) d[q] = make_float2(ld_nt(b, f_lane_in + q * TPT), 0.f);
      }
    } else {
      const float2* b = static_cast<const float2*>(in) + row0(t) * L;
      {
        const unsigned f_lane_in = fresh(lane_in);
#pragma unroll
        for (int q = 0; q < E; ++q) d[q] = ld_nt(b, f_lane_in + q * TPT);
      }
    }
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassRowsIn>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassRowsIn>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    fft_reg<L, INV, S::TWM>(a, j, x, tw);
    float2* b = ws + (int64_t)(t >> lsub) * bs + (t & ((1 << lsub) - 1)) * nt;
    {
      const unsigned f_lane_out = fresh(lane_out);
#pragma unroll
      for (int q = 0; q < E; ++q) b[f_lane_out + q * qs] = cscale(a[q], scale);
    }
    if constexpr (Prefetch<L, kPassRowsIn>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// ============================================================== kernel D
// Row pass out of the blocked layout into row-major output; tiles as above.
template <int L, bool INV, bool F32>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_from_blk(const float2* __restrict__ ws, void* __restrict__ out,
                                                                int rb, unsigned bs, int nt, int ntiles, float scale,
                                                                const float2* __restrict__ tws) {
  using S = Shape<L>;
  using C = RowsOutCfg<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const int lnt = ilog2_pow2(nt), lsub = ilog2_pow2(rb / nt);
  const int tid = threadIdx.x, sl = tid & (nt - 1), j = tid >> lnt;
  const Twiddles<L, C::TWM> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = regions<L, C>() + sl * C::region(nt);
  const unsigned lane_in = (unsigned)(j * rb + sl), lane_out = (unsigned)(sl * L + j);
  const int qs = TPT * rb;
  float2 a[E], nx[Prefetch<L, kPassRowsOut>::on ? E : 1];
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    const float2* b = ws + (int64_t)(t >> lsub) * bs + (t & ((1 << lsub) - 1)) * nt;
    {
      const unsigned f_lane_in = fresh(lane_in);
#pragma unroll
      for (int q = 0; q < E; ++q) d[q] = ld(b, f_lane_in + q * qs);
    }
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassRowsOut>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassRowsOut>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    fft_reg<L, INV, C::TWM, C::SPLIT>(a, j, x, tw);
    const int64_t r0 = (int64_t)(t >> lsub) * rb + (t & ((1 << lsub) - 1)) * nt;
    if constexpr (F32) {
      float* b = static_cast<float*>(out) + r0 * L;
      {
        const unsigned f_lane_out = fresh(lane_out);
#pragma unroll
        for (int q = 0; q < E; ++q) st_nt(&b[f_lane_out + q * TPT], a[q].x * scale);
      }
    } else {
      float2* b = static_cast<float2*>(out) + r0 * L;
      {
        const unsigned f_lane_out = fresh(lane_out);
#pragma unroll
        for (int q = 0; q < E; ++q) st_nt(&b[f_lane_out + q * TPT], cscale(a[q], scale));
      }
    }
    if constexpr (Prefetch<L, kPassRowsOut>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// Last pass of the fused filter + mean-squared-error forward (real images).
// The workspace holds the column-filtered spectrum of (m - 1) X, so the
// inverse row transform gives y - x; with the inputs x and c the tile's
// elements of y - c = (y - x) + (x - c) are squared and summed, and the sum
// goes to part[tile] (a fixed-order tree in LDS).  y is not written.
template <int L>
__global__ __launch_bounds__(Shape<L>::LB) void k_rows_loss(const float2* __restrict__ ws, const float* __restrict__ xin,
                                                            const float* __restrict__ cin, float* __restrict__ part,
                                                            int rb, unsigned bs, int nt, int ntiles, float scale,
                                                            const float2* __restrict__ tws) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const int lnt = ilog2_pow2(nt), lsub = ilog2_pow2(rb / nt);
  const int tid = threadIdx.x, sl = tid & (nt - 1), j = tid >> lnt;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = regions<L>() + sl * lds_region_bytes(L, nt);
  const unsigned lane_in = (unsigned)(j * rb + sl), lane_out = (unsigned)(sl * L + j);
  const int qs = TPT * rb;
  float* red = reinterpret_cast<float*>(regions<L>());
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    float2 a[E];
    {
      const float2* b = ws + (int64_t)(t >> lsub) * bs + (t & ((1 << lsub) - 1)) * nt;
      const unsigned f = fresh(lane_in);
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = ld(b, f + q * qs);
    }
    fft_reg<L, true, S::TWM>(a, j, x, tw);
    const int64_t r0 = (int64_t)(t >> lsub) * rb + (t & ((1 << lsub) - 1)) * nt;
    float acc = 0.f;
    {
      const float* xb = xin + r0 * L;
      const float* cb = cin + r0 * L;
      const unsigned f = fresh(lane_out);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const float re = fmaf(a[q].x, scale, ld_nt(xb, f + q * TPT) - ld_nt(cb, f + q * TPT));
        const float im = a[q].y * scale;
        acc = fmaf(re, re, fmaf(im, im, acc));
      }
    }
    lds_barrier();  // the transform's last LDS reads are done
    red[tid] = acc;
    lds_barrier();
    for (int h = (int)blockDim.x >> 1; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      lds_barrier();
    }
    if (tid == 0) part[t] = red[0];
    lds_barrier();  // red[0] read before the next tile's transform reuses LDS
  }
}

// out[0] = weight * (part[0] + ... + part[n-1]) in double precision, in a
// fixed order, in two launches: workgroup g of the first adds its run of
// kSumRun consecutive partials (thread t takes elements t, t + 256, ... of
// the run, then a fixed tree in LDS) into mid[g]; one workgroup then adds
// mid[0 .. G) the same way.  The order depends only on n.
constexpr int kSumRun = 4096;
__global__ __launch_bounds__(256) void k_sum_runs(const float* __restrict__ part, int64_t n,
                                                  double* __restrict__ mid) {
  __shared__ double red[256];
  const int64_t i0 = (int64_t)blockIdx.x * kSumRun;
  const int64_t i1 = min(n, i0 + kSumRun);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += (double)part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) mid[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_mid(const double* __restrict__ mid, int g, float weight,
                                                 float* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < g; i += 256) s += mid[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] * (double)weight);
}

// ============================================================== kernel C

// Forward column transform, mask, inverse column transform, in place.  A tile
// is w columns of one image (ltiles = log2(M / w) tiles per image); the tile
// base is image * L * M + v0 * rb and the lane offset jh*M*rb + c*rb + s.
// Tensor-mask values are read after the forward transform.
//
// HALF: the workspace holds the half spectrum of real images (M = half of the
// image's columns; frequencies are those of 2M columns).  Column 0 holds the
// sequences c0 = X(., 0) and cn = X(., M) of the full spectrum as c0 + i cn;
// both are transforms of real columns, so after the column transform
// C0(u) = (Z(u) + conj Z(-u)) / 2 and Cn(u) = (Z(u) - conj Z(-u)) / 2i, each
// is multiplied by its own mask column, and Z' = H0 C0 + i Hn Cn is
// transformed back.
template <int L, int MK, bool HALF>
__global__ __launch_bounds__(Shape<L>::LB) void k_cols_filter(float2* __restrict__ ws, float2* __restrict__ save, int M,
                                                      int rb, unsigned bs, int w, int ltiles, int ntiles, MaskArgs mk,
                                                      const float2* __restrict__ tws) {
  using C = std::conditional_t<HALF, DefCfg<L>, ColsCfg<L>>;
  static_assert(!HALF || (!C::SPLIT && MK != FFT_MASK_TENSOR_F32), "half spectrum: analytic masks");
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const Twiddles<L, C::TWM> twd(tws, ln.j);
  const float2* tw = twd.ptr();
  char* x = regions<L, C>() + ln.c * C::region(w);
  // byte offsets: the thread's within a tile (VGPR), element q's and the
  // tile's within the image (SGPR)
  const unsigned qs8 = (unsigned)(TPT / rb) * bs * 8u;
  const unsigned vlane = ((unsigned)ln.jh * bs + (unsigned)(ln.c * rb + ln.s)) * 8u;
  const int64_t img = (int64_t)(L / rb) * bs;
  const int tmask = (1 << ltiles) - 1;
  float2 a[E], nx[Prefetch<L, kPassCols>::on ? E : 1];
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    const BlkBuf b(ws + (int64_t)(t >> ltiles) * img, (uint64_t)img * 8u);
    const unsigned toff = (unsigned)((t & tmask) * w * rb) * 8u;
#pragma unroll
    for (int q = 0; q < E; ++q) d[q] = b.ld(vlane, toff + q * qs8);
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassCols>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassCols>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    const BlkBuf out(ws + (int64_t)(t >> ltiles) * img, (uint64_t)img * 8u);
    const unsigned toff = (unsigned)((t & tmask) * w * rb) * 8u;
    const int v = (t & tmask) * w + ln.c;
    fft_reg<L, false, C::TWM, C::SPLIT>(a, ln.j, x, tw);
    if (save) {
      const BlkBuf sb(save + (int64_t)(t >> ltiles) * img, (uint64_t)img * 8u);
#pragma unroll
      for (int q = 0; q < E; ++q) sb.template st<FFTMI_NT_SAVE != 0>(a[q], vlane, toff + q * qs8);
    }
    const int mfreq = HALF ? 2 * M : M;  // columns of the frequency grid
    if constexpr (HALF) {
      if ((t & tmask) == 0) {
      // the tile with column 0: every thread passes its values through LDS
      // (barriers are workgroup-wide); column 0's threads split c0 and cn
      lds_barrier();
      scatter_natural<L, kBoth>(a, ln.j, x);
      lds_barrier();
      const MaskEval<L, MK> m0(mk, ln.j, 0, mfreq), mn(mk, ln.j, M, mfreq), mv(mk, ln.j, v, mfreq);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int u = ln.j + q * TPT;
        if (ln.c == 0) {
          const float2 z = a[q];
          const float2 zm = reinterpret_cast<const float2*>(x)[lds_pad((L - u) & (L - 1))];
          const float h0 = m0.value(ln.j, q, mk), hn = mn.value(ln.j, q, mk);
          const float c0x = 0.5f * (z.x + zm.x), c0y = 0.5f * (z.y - zm.y);
          const float cnx = 0.5f * (z.y + zm.y), cny = 0.5f * (zm.x - z.x);
          a[q] = make_float2(h0 * c0x - hn * cny, h0 * c0y + hn * cnx);
        } else {
          a[q] = cscale(a[q], mv.value(ln.j, q, mk));
        }
      }
      } else {
        const MaskEval<L, MK> me(mk, ln.j, v, mfreq);
        me.apply(a, ln.j, mk);
      }
    } else {
      const MaskEval<L, MK> me(mk, ln.j, v, mfreq);
      me.apply(a, ln.j, mk);
    }
    fft_reg<L, true, C::TWM, C::SPLIT>(a, ln.j, x, tw);
#pragma unroll
    for (int q = 0; q < E; ++q) out.st(a[q], vlane, toff + q * qs8);
    if constexpr (Prefetch<L, kPassCols>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// One column transform of the blocked layout, in place (unscaled).
template <int L, bool INV>
__global__ __launch_bounds__(Shape<L>::LB) void k_cols_fft(float2* __restrict__ ws, int M, int rb, unsigned bs, int w,
                                                           int ltiles, int ntiles, const float2* __restrict__ tws) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const Twiddles<L> twd(tws, ln.j);
  const float2* tw = twd.ptr();
  char* x = regions<L>() + ln.c * lds_region_bytes(L, w);
  const unsigned qs = (unsigned)(TPT / rb) * bs;
  const unsigned lane = (unsigned)ln.jh * bs + (unsigned)(ln.c * rb + ln.s);
  const int64_t img = (int64_t)(L / rb) * bs;
  const int tmask = (1 << ltiles) - 1;
  float2 a[E], nx[Prefetch<L, kPassCols>::on ? E : 1];
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    const float2* b = ws + (int64_t)(t >> ltiles) * img + (t & tmask) * w * rb;
    const unsigned f_lane = fresh(lane);
#pragma unroll
    for (int q = 0; q < E; ++q) d[q] = b[f_lane + q * qs];
  };
  int n = blockIdx.x;
  if constexpr (Prefetch<L, kPassCols>::on) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (Prefetch<L, kPassCols>::on) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    fft_reg<L, INV, S::TWM>(a, ln.j, x, tw);
    float2* b = ws + (int64_t)(t >> ltiles) * img + (t & tmask) * w * rb;
    {
      const unsigned f_lane = fresh(lane);
#pragma unroll
      for (int q = 0; q < E; ++q) b[f_lane + q * qs] = a[q];
    }
    if constexpr (Prefetch<L, kPassCols>::on) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// Blocked workspace -> row-major output, times scale.  A thread owns column v
// of one block: it reads the block's RB values of that column (RB*8
// contiguous bytes) and writes them to the RB rows, so each of a wavefront's
// stores covers 64 consecutive elements of one row.
template <int RB, bool F32>
__global__ __launch_bounds__(256) void k_unblock(const float2* __restrict__ ws, void* __restrict__ out, int M,
                                                 unsigned bs, int64_t items, float scale) {
  const int lm = ilog2_pow2(M);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i >> lm;
    const int v = (int)(i & (M - 1));
    const float2* src = ws + blk * bs + v * RB;
    float2 a[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) a[s] = __ldg(src + s);
    const int64_t row0 = blk * RB;
    if constexpr (F32) {
      float* dst = static_cast<float*>(out) + row0 * M + v;
#pragma unroll
      for (int s = 0; s < RB; ++s) dst[(int64_t)s * M] = a[s].x * scale;
    } else {
      float2* dst = static_cast<float2*>(out) + row0 * M + v;
#pragma unroll
      for (int s = 0; s < RB; ++s) dst[(int64_t)s * M] = cscale(a[s], scale);
    }
  }
}

// out[v][u] = in[u][v] for a float32 [N][M] array: 64 x 64 tiles through
// LDS (padded rows), each read and written along contiguous 256-byte rows.
__global__ __launch_bounds__(256) void k_transpose_f32(const float* __restrict__ in, float* __restrict__ out,
                                                        int64_t N, int64_t M) {
  __shared__ float t[64][65];
  const int64_t u0 = (int64_t)blockIdx.y * 64, v0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4)
    if (u0 + r < N && v0 + tx < M) t[r][tx] = __ldg(in + (u0 + r) * M + v0 + tx);
  __syncthreads();
  for (int r = ty; r < 64; r += 4)
    if (v0 + r < M && u0 + tx < N) out[(v0 + r) * N + u0 + tx] = t[tx][r];
}

// Section 6 front end: zero padding of [B][n0][m0] images to [B][N][M]
// (appended rows and columns), and cropping back.  Element-wise, coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_pad(const T* __restrict__ in, T* __restrict__ out, int64_t total, int n0,
                                             int m0, int lN, int lM) {
  const int64_t N = int64_t(1) << lN, M = int64_t(1) << lM;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i >> (lN + lM);
    const int u = (int)((i >> lM) & (N - 1)), v = (int)(i & (M - 1));
    out[i] = (u < n0 && v < m0) ? in[(b * n0 + u) * m0 + v] : T{};
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_crop(const T* __restrict__ in, T* __restrict__ out, int64_t total, int n0,
                                              int m0, int lN, int lM) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bu = i / m0;
    const int v = (int)(i - bu * m0);
    const int64_t b = bu / n0;
    const int u = (int)(bu - b * n0);
    out[i] = in[((b << lN) + u) * (int64_t(1) << lM) + v];
  }
}

// |z| * scale of the blocked workspace into row-major float32 (the spectrum
// magnitude), laid out like k_unblock's output.
template <int RB>
__global__ __launch_bounds__(256) void k_unblock_mag(const float2* __restrict__ ws, float* __restrict__ out, int M,
                                                     unsigned bs, int64_t items, float scale) {
  const int lm = ilog2_pow2(M);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i >> lm;
    const int v = (int)(i & (M - 1));
    const float2* src = ws + blk * bs + v * RB;
    float* dst = out + blk * RB * M + v;
#pragma unroll
    for (int s = 0; s < RB; ++s) {
      const float2 z = __ldg(src + s);
      dst[(int64_t)s * M] = sqrtf(fmaf(z.x, z.x, z.y * z.y)) * scale;
    }
  }
}

// Mask gradient.  A tile is (image group g, column tile): loop over the
// group's images in order, forward-transform the blocked rows of the incoming
// gradient (or residual), multiply by conj(saved spectrum X) and accumulate
// the real part.  The group's
// partial sum goes to part[g][u][v]:
//   w_lin * sum_b Re(conj X_b . T_b)  (+ w_sq * (m - 1) * sum_b |X_b|^2  when MT)
// where T_b is the unscaled transform.  Partials of consecutive groups are
// added in group order by k_sum_groups, so the result does not depend on the
// launch shape's timing.
#ifndef FFTMI_GRAD_XFIRST
#define FFTMI_GRAD_XFIRST 0
#endif
#ifndef FFTMI_GRAD_NT
#define FFTMI_GRAD_NT 1
#endif
template <int L, bool MT>
__global__ __launch_bounds__(Shape<L>::LB) void k_cols_grad(const float2* __restrict__ ws, const float2* __restrict__ save,
                                                            const float* __restrict__ mask, float* __restrict__ part,
                                                            int nimg, int per_group, int M, int rb, unsigned bs,
                                                            int w, int ltiles,
                                                            int ntiles, float w_lin, float w_sq,
                                                            const float2* __restrict__ tws) {
  using S = Shape<L>;
  using C = GradCfg<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const Twiddles<L, C::TWM> twd(tws, ln.j);
  const float2* tw = twd.ptr();
  char* x = regions<L, C>() + ln.c * C::region(w);
  const unsigned qs = (unsigned)(TPT / rb) * bs;        // blocked layout, rows j + q*TPT
  const unsigned qs_out = (unsigned)(TPT * M);           // row-major mask and partial sums
  const unsigned lane = (unsigned)ln.jh * bs + (unsigned)(ln.c * rb + ln.s);
  const unsigned lane_out = (unsigned)(ln.j * M + ln.c);
  const int64_t plane = (int64_t)(L / rb) * bs;
  const int tmask = (1 << ltiles) - 1;
  // the residual and the saved spectrum are each read once: non-temporal
  auto gl = [](const float2* base, unsigned off) __attribute__((always_inline)) {
    return ldh<FFTMI_GRAD_NT != 0>(base, off);
  };
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    const int g = t >> ltiles, ct = t & tmask;
    const int b0 = g * per_group, b1 = min(nimg, b0 + per_group);
    float acc[E], acc2[E];
#pragma unroll
    for (int q = 0; q < E; ++q) acc[q] = acc2[q] = 0.f;
    // one image at a time: the residual's loads, its transform, and the
    // saved spectrum's loads and products
    for (int bi = b0; bi < b1; ++bi) {
      float2 a[E], X[E];
      const float2* b = ws + bi * plane + ct * w * rb;
      const float2* xs = save + bi * plane + ct * w * rb;
      {
        const unsigned f_lane = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) a[q] = gl(b, f_lane + q * qs);
        if constexpr (FFTMI_GRAD_XFIRST) {
          // the spectrum's loads in flight during the transform
#pragma unroll
          for (int q = 0; q < E; ++q) X[q] = gl(xs, f_lane + q * qs);
        }
      }
      fft_reg<L, false, C::TWM, C::SPLIT>(a, ln.j, x, tw);
      if constexpr (!FFTMI_GRAD_XFIRST) {
        const unsigned f_lane = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) X[q] = gl(xs, f_lane + q * qs);
      }
#pragma unroll
      for (int q = 0; q < E; ++q) {
        acc[q] = fmaf(X[q].x, a[q].x, fmaf(X[q].y, a[q].y, acc[q]));
        if constexpr (MT) acc2[q] = fmaf(X[q].x, X[q].x, fmaf(X[q].y, X[q].y, acc2[q]));
      }
    }
    const unsigned f_lane_out = fresh(lane_out);
    float* dst = part + (int64_t)g * L * M + ct * w;
    if constexpr (MT) {
      const float* mrow = mask + ct * w;
#pragma unroll
      for (int q = 0; q < E; ++q)
        dst[f_lane_out + q * qs_out] = fmaf(w_sq * (ld(mrow, f_lane_out + q * qs_out) - 1.0f), acc2[q], w_lin * acc[q]);
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) dst[f_lane_out + q * qs_out] = w_lin * acc[q];
    }
  }
}

// ------------------------------------------------ MSE in the frequency domain
// The filtered MSE and its mask gradient from the two spectra X = DFT2(x) and
// R = DFT2(x - c), unnormalised.  The transform pair inverts, so
//   y - c = IDFT2((m - 1) X + R) / (N M),
// and Parseval's relation for the unnormalised DFT turns the spatial sum into
//   sum |y - c|^2 = sum_{u,v} |(m - 1) X + R|^2 / (N M)
// with mask gradient (2 / (N M)) [(m - 1) |X|^2 + Re(conj X . R)] per bin.
// x and c are real, so X(N-u, M-v) = conj X(u, v) and likewise R: columns
// v = 0 .. M/2 of the spectra carry every bin, and a bin (u, v) with
// 0 < v < M/2 stands for itself and for its mirror (N-u, M-v), which has the
// same |X|^2, Re(conj X . R) and |.|^2 of a loss term (with its own mask
// value).
// Pass 1 (k_rows_xd): one complex transform per row of z = x + i (x - c),
// split by Hermitian symmetry into the row spectra of x and of x - c;
// columns 0 .. M/2 of both are stored in a blocked layout of mh columns.
// Pass 2 (k_cols_mse): the column transforms of both, the loss terms, and
// per run of images the sums of |X|^2 and Re(conj X . R) per stored bin.

// A tile is one block of rows (rb rows, rb * TPT threads); bs is the block
// stride of the mh-column layout.
template <int L>
__global__ __launch_bounds__(1024) void k_rows_xd(const float* __restrict__ xin, const float* __restrict__ cin,
                                                  float2* __restrict__ wsx, float2* __restrict__ wsd, int rb,
                                                  unsigned bs, int ntiles, const float2* __restrict__ tws) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT, RBY = lds_region_bytes(L, 1);
  static_assert(!kSplitExchange, "whole complex LDS entries");
  char* reg = regions<L>();
  const int tid = threadIdx.x, p = tid / TPT, j = tid - p * TPT;
  const int nthr = rb * TPT;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  char* x = reg + p * RBY;
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);  // block index over the batch
    float2 a[E];
    {
      const int64_t row = (int64_t)t * rb + p;
      const float* xb = xin + row * L;
      const float* cb = cin + row * L;
      const unsigned f = fresh((unsigned)j);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const float xv = ld_nt(xb, f + q * TPT);
        a[q] = make_float2(xv, xv - ld_nt(cb, f + q * TPT));
      }
    }
    fft_reg<L, false, S::TWM>(a, j, x, tw);
    lds_barrier();  // the transform's last LDS reads are done
    scatter_natural<L, kBoth>(a, j, x);
    lds_barrier();
    // column v = 0 .. L/2 of the block: rows 0 .. rb-1 of both spectra, two
    // rows per float4
    float4* ox = reinterpret_cast<float4*>(wsx + (int64_t)t * bs);
    float4* od = reinterpret_cast<float4*>(wsd + (int64_t)t * bs);
    const int v0 = (int)fresh((unsigned)tid);
    for (int v = v0; v <= L / 2; v += nthr) {
      const int vm = (L - v) & (L - 1);
      for (int s = 0; s < rb; s += 2) {
        const float2 z0 = reinterpret_cast<const float2*>(reg + s * RBY)[lds_pad(v)];
        const float2 m0 = reinterpret_cast<const float2*>(reg + s * RBY)[lds_pad(vm)];
        const float2 z1 = reinterpret_cast<const float2*>(reg + (s + 1) * RBY)[lds_pad(v)];
        const float2 m1 = reinterpret_cast<const float2*>(reg + (s + 1) * RBY)[lds_pad(vm)];
        // X = (Z + conj Z(-v)) / 2, D = (Z - conj Z(-v)) / 2i
        ox[(v * rb + s) >> 1] = make_float4(0.5f * (z0.x + m0.x), 0.5f * (z0.y - m0.y), 0.5f * (z1.x + m1.x),
                                            0.5f * (z1.y - m1.y));
        od[(v * rb + s) >> 1] = make_float4(0.5f * (z0.y + m0.y), 0.5f * (m0.x - z0.x), 0.5f * (z1.y + m1.y),
                                            0.5f * (m1.x - z1.x));
      }
    }
    lds_barrier();  // the regions are read before the next tile's transform reuses them
  }
}

// A tile is (run g of images, column tile ct of `tiles` per run): both
// column transforms per image for the stored columns v = ct*w + c <= M/2,
// the loss terms of the bin and of its mirror summed per thread, and per bin
// the run's sums of |X|^2 and Re(conj X . R), stored to sumx[g] and
// sumxr[g] ([N][mh]); the tile's loss sum goes to part[tile].  Columns of
// the last tile beyond M/2 are not read and add nothing.
template <int L>
__global__ __launch_bounds__(Shape<L>::LB) void k_cols_mse(const float2* __restrict__ wsx,
                                                           const float2* __restrict__ wsd,
                                                           const float* __restrict__ mask, float* __restrict__ sumx,
                                                           float* __restrict__ sumxr, float* __restrict__ part,
                                                           int nimg, int per_group, int M, int mh, int rb, unsigned bs,
                                                           int w, int tiles, int ntiles,
                                                           const float2* __restrict__ tws) {
  using S = Shape<L>;
  using C = GradCfg<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const ColLanes ln = col_lanes(threadIdx.x, rb, w);
  const Twiddles<L, C::TWM> twd(tws, ln.j);
  const float2* tw = twd.ptr();
  char* x = regions<L, C>() + ln.c * C::region(w);
  const unsigned qs = (unsigned)(TPT / rb) * bs;
  const unsigned lane = (unsigned)ln.jh * bs + (unsigned)(ln.c * rb + ln.s);
  const int64_t plane = (int64_t)(L / rb) * bs;
  double* red = reinterpret_cast<double*>(regions<L, C>());
  for (int n = blockIdx.x; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    const int g = t / tiles, ct = t - g * tiles;
    const int b0 = g * per_group, b1 = min(nimg, b0 + per_group);
    const int v = ct * w + ln.c;
    const bool ok = v <= M / 2;                // a stored column
    const bool mir = ok && v > 0 && v < M / 2;  // it also stands for column M - v
    // mask values minus one at the bin (u, v) and at its mirror (N - u, M - v)
    float m1[E], m2[E], ax[E], axr[E];
    {
      const int jf = (int)fresh((unsigned)ln.j);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int u = jf + q * TPT;
        m1[q] = ok ? ld(mask, (unsigned)(u * M + v)) - 1.0f : 0.f;
        m2[q] = mir ? ld(mask, (unsigned)(((L - u) & (L - 1)) * M + (M - v))) - 1.0f : 0.f;
        ax[q] = axr[q] = 0.f;
      }
    }
    double lacc = 0.0;  // the loss terms of the tile, in double
    for (int bi = b0; bi < b1; ++bi) {
      float2 X[E], R[E];
      {
        const float2* b = wsx + bi * plane + ct * w * rb;
        const unsigned f = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) X[q] = ok ? ld_nt(b, f + q * qs) : make_float2(0.f, 0.f);
      }
      fft_reg<L, false, C::TWM, C::SPLIT>(X, ln.j, x, tw);
      {
        const float2* b = wsd + bi * plane + ct * w * rb;
        const unsigned f = fresh(lane);
#pragma unroll
        for (int q = 0; q < E; ++q) R[q] = ok ? ld_nt(b, f + q * qs) : make_float2(0.f, 0.f);
      }
      fft_reg<L, false, C::TWM, C::SPLIT>(R, ln.j, x, tw);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        ax[q] = fmaf(X[q].x, X[q].x, fmaf(X[q].y, X[q].y, ax[q]));
        axr[q] = fmaf(X[q].x, R[q].x, fmaf(X[q].y, R[q].y, axr[q]));
        const float ex = fmaf(m1[q], X[q].x, R[q].x), ey = fmaf(m1[q], X[q].y, R[q].y);
        const float fx = fmaf(m2[q], X[q].x, R[q].x), fy = fmaf(m2[q], X[q].y, R[q].y);
        lacc += (double)fmaf(ex, ex, ey * ey);
        if (mir) lacc += (double)fmaf(fx, fx, fy * fy);
      }
    }
    if (ok) {
      const unsigned f = (unsigned)(fresh((unsigned)ln.j) * mh + v);
      const unsigned qo = (unsigned)(TPT * mh);
      float* dx = sumx + (int64_t)g * L * mh;
      float* dxr = sumxr + (int64_t)g * L * mh;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        dx[f + q * qo] = ax[q];
        dxr[f + q * qo] = axr[q];
      }
    }
    // the tile's loss sum: an LDS tree over the workgroup, in a fixed order,
    // in double
    const int tid = threadIdx.x;
    lds_barrier();  // the last transform's LDS reads are done
    red[tid] = lacc;
    lds_barrier();
    for (int h = (int)blockDim.x >> 1; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      lds_barrier();
    }
    if (tid == 0) part[t] = (float)red[0];
    lds_barrier();  // red read before the next tile's transform reuses LDS
  }
}

// grad[u][v] = w * ((m - 1) * sum_g sumx[g] + sum_g sumxr[g]) at the stored
// bin (u, v), or at (N - u, M - v) for v > M/2; the runs added in order.
__global__ __launch_bounds__(256) void k_mse_grad_sums(const float* __restrict__ sumx, const float* __restrict__ sumxr,
                                                       const float* __restrict__ mask, float* __restrict__ grad, int N,
                                                       int M, int mh, int groups, float w) {
  const int64_t n = (int64_t)N * M, plane = (int64_t)N * mh;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(i / M), v = (int)(i - (int64_t)u * M);
    const int64_t k = v <= M / 2 ? (int64_t)u * mh + v : (int64_t)((N - u) & (N - 1)) * mh + (M - v);
    float sx = sumx[k], sxr = sumxr[k];
    for (int g = 1; g < groups; ++g) {
      sx += sumx[g * plane + k];
      sxr += sumxr[g * plane + k];
    }
    grad[i] = w * fmaf(mask[i] - 1.0f, sx, sxr);
  }
}

// grad[i] = part[0][i] + part[1][i] + ... + part[G-1][i], in that order.
__global__ __launch_bounds__(256) void k_sum_groups(const float4* __restrict__ part, float4* __restrict__ grad,
                                                    int64_t n4, int groups) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    float4 s = part[i];
    for (int g = 1; g < groups; ++g) {
      const float4 v = part[g * n4 + i];
      s.x += v.x;
      s.y += v.y;
      s.z += v.z;
      s.w += v.w;
    }
    grad[i] = s;
  }
}

// ============================================================== kernel E
// Strided column pass over an [L][C] matrix per batch entry (the four-step
// long 1D transform): row r of entry b starts at b*ib + r*irs.
// TT: pass one (store transposed, column c as the row of L
// entries at b*ob + c*ors, each entry times W_N^{k1 n2} = tfs[n2*L + k1],
// read in the same order as the stores); otherwise pass two (store [L][C]
// with row stride ors).
// WIDE: tiles of up to 1024 threads (twice the columns of the 512-thread
// tiles, so twice the contiguous bytes per row), with no prefetch, as the
// 128 VGPRs a thread then has leave no room for a second tile.
// nt: bit 1 non-temporal loads (pass one: of the input, in 1024-thread
// tiles only; pass two: of the intermediate), bit 2 (pass two) non-temporal
// stores of the result.
template <int L, bool INV, bool WIDE, bool TT>
__global__ __launch_bounds__(WIDE ? 1024 : Shape<L>::LB) void k_cols_strided(
    const float2* __restrict__ in, float2* __restrict__ out, int C, int w, int ltiles, int ntiles, float scale,
    const float2* __restrict__ tfs, const float2* __restrict__ tws, int64_t ib, int irs, int64_t ob, int ors,
    int nt) {
  using S = Shape<L>;
  constexpr int E = S::E, TPT = S::TPT;
  const int lw = ilog2_pow2(w);
  const int tid = threadIdx.x, c = tid & (w - 1), j = tid >> lw;
  const Twiddles<L> twd(tws, j);
  const float2* tw = twd.ptr();
  const int rbytes = lds_region_bytes(L, w);
  char* reg = regions<L>();
  char* x = reg + c * rbytes;
  const unsigned qs = (unsigned)(TPT * irs);
  const unsigned lane = (unsigned)(j * irs + c);
  const int tmask = (1 << ltiles) - 1;
  constexpr bool PF = TPT <= 512 && !WIDE;  // 1024-thread workgroups have no room for a second tile
  // pass one takes the hint in 1024-thread tiles only: with the register
  // prefetch of the smaller tiles, a second load path costs VGPRs and a wave
  // per SIMD
  constexpr bool kHintsTT = TT && WIDE;
  float2 a[E], nx[PF ? E : 1];
  // tile t -> (batch entry, column tile).  Pass one takes the batch entries
  // of one column tile in a row (t = column tile * entries + entry), so that
  // the workgroups on one XCD read the tile's factors W_N^{k1 n2} from its L2
  // after the first entry, instead of once per entry from memory.
  const int nent = ntiles >> ltiles;
  auto entry_of = [&](int t) __attribute__((always_inline)) { return TT ? t % nent : t >> ltiles; };
  auto ctile_of = [&](int t) __attribute__((always_inline)) { return TT ? t / nent : t & tmask; };
  auto load = [&](float2(&d)[E], int t) __attribute__((always_inline)) {
    const float2* b = in + (int64_t)entry_of(t) * ib + ctile_of(t) * w;
    const unsigned f_lane = fresh(lane);
    if ((!TT || kHintsTT) && (nt & 1) != 0) {
#pragma unroll
      for (int q = 0; q < E; ++q) d[q] = ld_nt(b, f_lane + q * qs);
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) d[q] = ld(b, f_lane + q * qs);
    }
  };
  int n = blockIdx.x;
  if constexpr (PF) {
    if (n < ntiles) load(a, (int)tile_of(n, ntiles));
    settle(a);
  }
  for (; n < ntiles; n += gridDim.x) {
    const int t = (int)tile_of(n, ntiles);
    if constexpr (PF) {
      if (n + (int)gridDim.x < ntiles) load(nx, (int)tile_of(n + gridDim.x, ntiles));
    } else {
      load(a, t);
    }
    const int64_t bo = (int64_t)entry_of(t) * ob;
    const int c0 = ctile_of(t) * w;
    fft_reg<L, INV, S::TWM>(a, j, x, tw);
    if constexpr (TT) {
      // transposed store through LDS: out[n2][k1], contiguous along k1
      const int nthr = w * TPT;
      const int lL = ilog2_pow2(L);
      float2 o[E];
      if constexpr (kSplitExchange) {
        lds_barrier();
        scatter_natural<L, kRe>(a, j, x);
        lds_barrier();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int idx = tid + e * nthr, cc = idx >> lL, k = idx & (L - 1);
          o[e].x = reinterpret_cast<const float*>(reg + cc * rbytes)[lds_pad(k)];
        }
        lds_barrier();
        scatter_natural<L, kIm>(a, j, x);
        lds_barrier();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int idx = tid + e * nthr, cc = idx >> lL, k = idx & (L - 1);
          o[e].y = reinterpret_cast<const float*>(reg + cc * rbytes)[lds_pad(k)];
        }
      } else {
        lds_barrier();
        scatter_natural<L, kBoth>(a, j, x);
        lds_barrier();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int idx = tid + e * nthr, cc = idx >> lL, k = idx & (L - 1);
          o[e] = reinterpret_cast<const float2*>(reg + cc * rbytes)[lds_pad(k)];
        }
      }
      float2* b = out + bo + (int64_t)c0 * ors;
      const float2* tf = tfs + (int64_t)c0 * L;  // rows n2 = c0 .. c0 + w - 1
      // the store indices come from an opaque thread index: otherwise their
      // addresses are computed once, before the tile loop, and held in
      // registers across the transform (pass one then needs 150-240 VGPRs
      // instead of 100-150)
      const int t0 = (int)fresh((unsigned)tid);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = t0 + e * nthr;
        const float2 wv = tf[(unsigned)idx];  // W_N^{k1 n2}, k1 = idx % L, n2 = c0 + idx / L
        b[(unsigned)((idx >> lL) * ors + (idx & (L - 1)))] = cscale(cmul_tw<INV>(o[e], wv), scale);
      }
    } else {
      float2* b = out + bo + c0;
      {
        const unsigned f_lane = fresh((unsigned)(j * ors + c));
        const unsigned oqs = (unsigned)(TPT * ors);
        if (nt & 2) {
#pragma unroll
          for (int q = 0; q < E; ++q) st_nt(b + f_lane + q * oqs, cscale(a[q], scale));
        } else {
#pragma unroll
          for (int q = 0; q < E; ++q) b[f_lane + q * oqs] = cscale(a[q], scale);
        }
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < E; ++q) a[q] = nx[q];
    }
  }
}

// ============================================================== launchers
namespace {

std::mutex g_mu;
std::set<std::pair<const void*, int>> g_attr_done;
std::map<std::tuple<const void*, int, int, int>, int> g_occ;
std::map<int, int> g_cus;

// Allow up to the full 160 KiB of LDS for a kernel (once per device).
hipError_t allow_lds(const void* fn, int bytes, int dev) {
  if (bytes <= 65536) return hipSuccess;
  if (g_attr_done.count({fn, dev})) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  if (e == hipSuccess) g_attr_done.insert({fn, dev});
  return e;
}

// Persistent grid: as many workgroups as fit on the device at once (a
// multiple of 8 when possible, for the XCD tile order), never more than the
// number of tiles.

// Optional cap on resident workgroups per CU (FFTMI_WG_PER_CU), for tuning.
inline int wg_cap() {
  const char* e = std::getenv("FFTMI_WG_PER_CU");
  return e ? std::atoi(e) : 0;
}

template <typename... Args>
hipError_t go(void (*k)(Args...), int64_t ntiles, int block, int lds, hipStream_t st, Args... args) {
  if (ntiles <= 0) return hipSuccess;
  const void* fn = reinterpret_cast<const void*>(k);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int per_cu = 0, cus = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    e = allow_lds(fn, lds, dev);
    if (e != hipSuccess) return e;
    auto key = std::make_tuple(fn, block, lds, dev);
    auto it = g_occ.find(key);
    if (it == g_occ.end()) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, (size_t)lds);
      if (e != hipSuccess) return e;
      g_occ[key] = per_cu;
    } else {
      per_cu = it->second;
    }
    auto ic = g_cus.find(dev);
    if (ic == g_cus.end()) {
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      g_cus[dev] = cus;
    } else {
      cus = ic->second;
    }
  }
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int cap = wg_cap();
  if (cap > 0 && per_cu > cap) per_cu = cap;
  const int64_t grid = persistent_grid(ntiles, (int64_t)per_cu * cus);
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(block), (size_t)lds, st, args...);
  return hipGetLastError();
}

template <int L>
constexpr int tw_bytes() {
  return Shape<L>::TWB;
}

template <int L>
constexpr int max_block() {
  return Shape<L>::LB;
}

template <int L, class C = DefCfg<L>>
const float2* twiddle_src(const Launch& lc) {
  return C::TWM == kTwLds ? lc.tw_lds : lc.tw;
}

#define FFTMI_LOG2_CASES(F) \
  F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14)

template <int LG>
struct RowsRm {
  static hipError_t run(bool inv, const void* in, bool in_f32, void* out, bool out_f32, int64_t rows, float scale,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    int tpw = TPT >= 256 ? 1 : 256 / TPT;
    static_assert(TPT <= max_block<L>(), "block");
    if (rows < tpw) tpw = (int)(rows > 0 ? rows : 1);
    using C = Rows1DCfg<L>;
    const int lds = C::TWB + tpw * C::region(1);
    const int ntiles = (int)((rows + tpw - 1) / tpw);
    const float2* tw = twiddle_src<L, C>(lc);
    if (inv)
      return go(k_rows_rm<L, true>, ntiles, tpw * TPT, lds, lc.stream, in, (int)in_f32, out, (int)out_f32, rows, tpw,
                ntiles, scale, tw);
    return go(k_rows_rm<L, false>, ntiles, tpw * TPT, lds, lc.stream, in, (int)in_f32, out, (int)out_f32, rows, tpw,
              ntiles, scale, tw);
  }
};

// Real-row pairs per tile of the packed row pass: one whole block of rb rows
// (rb / 2 pairs) while that fits the workgroup and LDS limits.
template <int L>
int pair_per_tile(int rb) {
  constexpr int TPT = threads_per_transform(L);
  int npt = rb / 2;
  if (const char* e = std::getenv("FFTMI_PAIR_NPT")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= npt && (v & (v - 1)) == 0) npt = v;
  }
  while (npt > 1 && (npt * TPT > max_block<L>() || tw_bytes<L>() + npt * lds_region_bytes(L, 1) > kLdsBytes))
    npt /= 2;
  return npt;
}

// Rows per tile of the blocked row passes.  The pass that writes the blocked
// layout takes as many rows of a block as a workgroup holds (up to `target`
// threads), so that more of each block's interleaved segments are written by
// one workgroup; the pass that reads it aims at 256-thread workgroups,
// several of which share a CU.
template <int L, class C = DefCfg<L>>
int rows_per_tile(int rb, int target) {
  int nt = rb;
  while (nt > 1 && nt * threads_per_transform(L) > target) nt /= 2;
  if (const char* e = std::getenv("FFTMI_ROWS_NT")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= rb && (v & (v - 1)) == 0) nt = v;
  }
  while (nt > 1 && (C::TWB + nt * C::region(nt) > kLdsBytes ||
                    nt * threads_per_transform(L) > max_block<L>()))
    nt /= 2;
  return nt;
}

template <int LG>
struct RowsToBlk {
  static hipError_t run(bool inv, bool pair, bool half, const void* in, const void* in2, bool in_f32, float2* ws,
                        int64_t blocks, int rb, unsigned bs, float scale, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const float2* tw = twiddle_src<L>(lc);
    if (pair && rb >= 2) {
      // pairs per tile: aim at 256-thread workgroups, within LDS and block limits
      int npt = pair_per_tile<L>(rb);
      if (tw_bytes<L>() + npt * lds_region_bytes(L, 1) <= kLdsBytes && npt * TPT <= max_block<L>()) {
        const int lds = tw_bytes<L>() + npt * lds_region_bytes(L, 1);
        const float* fin = static_cast<const float*>(in);
        const int64_t ntiles = blocks * (rb / 2 / npt);
        if (in2)
          return go(k_rows_to_blk_pair<L, false, false, true>, ntiles, npt * TPT, lds, lc.stream, fin, ws, rb, bs,
                    npt, (int)ntiles, scale, tw, static_cast<const float*>(in2));
        if constexpr (L >= 2) {
          if (half)
            return go(inv ? k_rows_to_blk_pair<L, true, true> : k_rows_to_blk_pair<L, false, true>, ntiles,
                      npt * TPT, lds, lc.stream, fin, ws, rb, bs, npt, (int)ntiles, scale, tw,
                      static_cast<const float*>(nullptr));
        }
        return go(inv ? k_rows_to_blk_pair<L, true, false> : k_rows_to_blk_pair<L, false, false>, ntiles, npt * TPT,
                  lds, lc.stream, fin, ws, rb, bs, npt, (int)ntiles, scale, tw, static_cast<const float*>(nullptr));
      }
    }
    if (half || in2) return hipErrorInvalidValue;
    const int nt = rows_per_tile<L>(rb, 512);
    const int lds = tw_bytes<L>() + nt * lds_region_bytes(L, nt);
    const int64_t ntiles = blocks * (rb / nt);
    if (inv)
      return go(k_rows_to_blk<L, true>, ntiles, nt * TPT, lds, lc.stream, in, (int)in_f32, ws, rb, bs, nt,
                (int)ntiles, scale, tw);
    return go(k_rows_to_blk<L, false>, ntiles, nt * TPT, lds, lc.stream, in, (int)in_f32, ws, rb, bs, nt,
              (int)ntiles, scale, tw);
  }
};

template <int LG>
struct RowsFromBlk {
  static hipError_t run(bool inv, const float2* ws, void* out, bool out_f32, int64_t blocks, int rb, unsigned bs,
                        float scale, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    using C = RowsOutCfg<L>;
    const float2* tw = twiddle_src<L, C>(lc);
    const int nt = rows_per_tile<L, C>(rb, 256);
    const int lds = C::TWB + nt * C::region(nt);
    const int64_t ntiles = blocks * (rb / nt);
    auto k = inv ? (out_f32 ? k_rows_from_blk<L, true, true> : k_rows_from_blk<L, true, false>)
                 : (out_f32 ? k_rows_from_blk<L, false, true> : k_rows_from_blk<L, false, false>);
    return go(k, ntiles, nt * TPT, lds, lc.stream, ws, out, rb, bs, nt, (int)ntiles, scale, tw);
  }
};

template <int LG>
struct RowsLoss {
  static hipError_t run(const float2* ws, const float* x, const float* c, float* part, int64_t blocks, int rb,
                        unsigned bs, float scale, int64_t* ntiles_out, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int nt = rows_per_tile<L>(rb, 256);
    const int lds = tw_bytes<L>() + std::max(nt * lds_region_bytes(L, nt), (int)(nt * TPT * sizeof(float)));
    const int64_t ntiles = blocks * (rb / nt);
    *ntiles_out = ntiles;
    return go(k_rows_loss<L>, ntiles, nt * TPT, lds, lc.stream, ws, x, c, part, rb, bs, nt, (int)ntiles, scale,
              twiddle_src<L>(lc));
  }
};

template <int LG>
struct RowsC2R {
  static hipError_t run(const float2* ws, void* out, bool out_f32, int64_t blocks, int rb, unsigned bs, float scale,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    if constexpr (L < 2) {
      return hipErrorInvalidValue;
    } else {
      if (rb < 2) return hipErrorInvalidValue;
      const int npt = pair_per_tile<L>(rb);
      const int lds = tw_bytes<L>() + npt * lds_region_bytes(L, 1);
      if (lds > kLdsBytes || npt * TPT > max_block<L>()) return hipErrorInvalidValue;
      const int64_t ntiles = blocks * (rb / 2 / npt);
      return go(out_f32 ? k_rows_c2r_pair<L, true> : k_rows_c2r_pair<L, false>, ntiles, npt * TPT, lds, lc.stream, ws,
                out, rb, bs, npt, (int)ntiles, scale, twiddle_src<L>(lc));
    }
  }
};

template <int LG>
struct ColsFilter {
  template <bool HALF>
  static hipError_t launch(float2* ws, float2* save, int64_t nimg, int M, int rb, unsigned bs, int w,
                           const MaskArgs& mk, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    using C = std::conditional_t<HALF, DefCfg<L>, ColsCfg<L>>;
    const int tiles = M / w;
    const int lds = C::TWB + w * C::region(w);
    const int64_t ntiles = nimg * tiles;
    const float2* tw = twiddle_src<L, C>(lc);
    const int lt = ilog2c(tiles);
    switch (mk.kind) {
      case FFT_MASK_TENSOR_F32:
        if constexpr (HALF) return hipErrorInvalidValue;
        return go(k_cols_filter<L, FFT_MASK_TENSOR_F32, false>, ntiles, w * TPT, lds, lc.stream, ws, save, M, rb, bs, w, lt,
                  (int)ntiles, mk, tw);
      case FFT_MASK_GAUSSIAN:
        return go(k_cols_filter<L, FFT_MASK_GAUSSIAN, HALF>, ntiles, w * TPT, lds, lc.stream, ws, save, M, rb, bs, w, lt,
                  (int)ntiles, mk, tw);
      case FFT_MASK_BUTTERWORTH:
        return go(k_cols_filter<L, FFT_MASK_BUTTERWORTH, HALF>, ntiles, w * TPT, lds, lc.stream, ws, save, M, rb, bs, w,
                  lt, (int)ntiles, mk, tw);
      case FFT_MASK_DISC:
        return go(k_cols_filter<L, FFT_MASK_DISC, HALF>, ntiles, w * TPT, lds, lc.stream, ws, save, M, rb, bs, w, lt,
                  (int)ntiles, mk, tw);
      default:
        return go(k_cols_filter<L, FFT_MASK_NONE, HALF>, ntiles, w * TPT, lds, lc.stream, ws, save, M, rb, bs, w, lt,
                  (int)ntiles, mk, tw);
    }
  }
  static hipError_t run(float2* ws, float2* save, int64_t nimg, int M, int rb, unsigned bs, int w, bool half,
                        const MaskArgs& mk, const Launch& lc) {
    return half ? launch<true>(ws, save, nimg, M, rb, bs, w, mk, lc)
                : launch<false>(ws, save, nimg, M, rb, bs, w, mk, lc);
  }
};

template <int LG>
struct ColsFft {
  static hipError_t run(bool inv, float2* ws, int64_t nimg, int M, int rb, unsigned bs, int w, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    const int tiles = M / w;
    const int lds = tw_bytes<L>() + w * lds_region_bytes(L, w);
    const float2* tw = twiddle_src<L>(lc);
    const int64_t ntiles = nimg * tiles;
    const int lt = ilog2c(tiles);
    auto k = inv ? k_cols_fft<L, true> : k_cols_fft<L, false>;
    return go(k, ntiles, w * TPT, lds, lc.stream, ws, M, rb, bs, w, lt, (int)ntiles, tw);
  }
};

template <int LG>
struct ColsGrad {
  static hipError_t run(const float2* ws, const float2* save, const float* mask, float* part, int64_t nimg,
                        int groups, int M, int rb, unsigned bs, int w, float w_lin, float w_sq, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    using C = GradCfg<L>;
    const int lds = C::TWB + w * C::region(w);
    const int ctiles = M / w;
    const int per_group = (int)((nimg + groups - 1) / groups);
    const int64_t ntiles = (int64_t)groups * ctiles;
    const int lt = ilog2c(ctiles);
    if (mask)
      return go(k_cols_grad<L, true>, ntiles, w * TPT, lds, lc.stream, ws, save, mask, part, (int)nimg, per_group,
                M, rb, bs, w, lt, (int)ntiles, w_lin, w_sq, twiddle_src<L, C>(lc));
    return go(k_cols_grad<L, false>, ntiles, w * TPT, lds, lc.stream, ws, save, mask, part, (int)nimg, per_group, M,
              rb, bs, w, lt, (int)ntiles, w_lin, w_sq, twiddle_src<L, C>(lc));
  }
};

template <int LG>
struct RowsXd {
  static hipError_t run(const float* x, const float* c, float2* wsx, float2* wsd, int64_t blocks, int rb, unsigned bs,
                        const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    if constexpr (L < 2) {
      return hipErrorInvalidValue;
    } else {
      if (rb < 2 || rb % 2 || rb * TPT > 1024) return hipErrorInvalidValue;
      const int lds = tw_bytes<L>() + rb * lds_region_bytes(L, 1);
      if (lds > kLdsBytes) return hipErrorInvalidValue;
      return go(k_rows_xd<L>, blocks, rb * TPT, lds, lc.stream, x, c, wsx, wsd, rb, bs, (int)blocks,
                twiddle_src<L>(lc));
    }
  }
};

template <int LG>
struct ColsMse {
  static hipError_t run(const float2* wsx, const float2* wsd, const float* mask, float* sumx, float* sumxr,
                        float* part, int64_t nimg, int groups, int M, int mh, int rb, unsigned bs, int w,
                        int64_t* ntiles_out, const Launch& lc) {
    constexpr int L = 1 << LG, TPT = threads_per_transform(L);
    using C = GradCfg<L>;
    if (mh % w || mh < M / 2 + 1) return hipErrorInvalidValue;
    const int lds = std::max(C::TWB + w * C::region(w), (int)(w * TPT * sizeof(double)));
    const int tiles = mh / w;
    const int per_group = (int)((nimg + groups - 1) / groups);
    const int64_t ntiles = (int64_t)groups * tiles;
    *ntiles_out = ntiles;
    return go(k_cols_mse<L>, ntiles, w * TPT, lds, lc.stream, wsx, wsd, mask, sumx, sumxr, part, (int)nimg, per_group,
              M, mh, rb, bs, w, tiles, (int)ntiles, twiddle_src<L, C>(lc));
  }
};

template <int LG>
struct ColsStrided {
  template <bool INV, bool WIDE, bool TT>
  static hipError_t go_one(const float2* in, float2* out, int64_t ntiles, int w, int lds, int C, int lt, float scale,
                           const float2* tfs, const float2* tw, int64_t ib, int irs, int64_t ob, int ors, int nt,
                           const Launch& lc) {
    constexpr int TPT = threads_per_transform(1 << LG);
    return go(k_cols_strided<1 << LG, INV, WIDE, TT>, ntiles, w * TPT, lds, lc.stream, in, out, C, w, lt,
              (int)ntiles, scale, tfs, tw, ib, irs, ob, ors, nt);
  }
  template <bool INV, bool WIDE>
  static hipError_t go_tt(bool twt, const float2* in, float2* out, int64_t ntiles, int w, int lds, int C, int lt,
                          float scale, const float2* tfs, const float2* tw, int64_t ib, int irs, int64_t ob, int ors,
                          int nt, const Launch& lc) {
    return twt ? go_one<INV, WIDE, true>(in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc)
               : go_one<INV, WIDE, false>(in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc);
  }
  static hipError_t run(bool inv, bool twt, const float2* in, float2* out, int64_t batch, int C, int w, float scale,
                        const float2* tfs, int64_t ib, int irs, int64_t ob, int ors, int nt, const Launch& lc) {
    // the four-step splits use column lengths 2^7 .. 2^12 only
    if constexpr (LG < 7 || LG > 12) {
      return hipErrorInvalidValue;
    } else {
      constexpr int L = 1 << LG, TPT = threads_per_transform(L);
      const int tiles = C / w;
      const int lds = tw_bytes<L>() + w * lds_region_bytes(L, w);
      const float2* tw = twiddle_src<L>(lc);
      const int64_t ntiles = batch * tiles;
      const int lt = ilog2c(tiles);
      if (w * TPT > 1024) return hipErrorInvalidValue;
      const bool wide = w * TPT > max_block<L>();
      if (inv)
        return wide ? go_tt<true, true>(twt, in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc)
                    : go_tt<true, false>(twt, in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc);
      return wide ? go_tt<false, true>(twt, in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc)
                  : go_tt<false, false>(twt, in, out, ntiles, w, lds, C, lt, scale, tfs, tw, ib, irs, ob, ors, nt, lc);
    }
  }
};

}  // namespace

#define FFTMI_DISPATCH(STRUCT, LOG2, ...) \
  switch (LOG2) {                         \
    FFTMI_LOG2_CASES(FFTMI_CASE_##STRUCT) \
    default:                              \
      return hipErrorInvalidValue;        \
  }

#define FFTMI_CASE_RowsRm(K) \
  case K:                    \
    return RowsRm<K>::run(inv, in, in_f32, out, out_f32, rows, scale, lc);
#define FFTMI_CASE_RowsToBlk(K) \
  case K:                       \
    return RowsToBlk<K>::run(inv, pair, half, in, in2, in_f32, ws, blocks, rb, bs, scale, lc);
#define FFTMI_CASE_RowsLoss(K) \
  case K:                      \
    return RowsLoss<K>::run(ws, x, c, part, blocks, rb, bs, scale, ntiles, lc);
#define FFTMI_CASE_RowsC2R(K) \
  case K:                     \
    return RowsC2R<K>::run(ws, out, out_f32, blocks, rb, bs, scale, lc);
#define FFTMI_CASE_RowsFromBlk(K) \
  case K:                         \
    return RowsFromBlk<K>::run(inv, ws, out, out_f32, blocks, rb, bs, scale, lc);
#define FFTMI_CASE_ColsFilter(K) \
  case K:                        \
    return ColsFilter<K>::run(ws, save, nimg, M, rb, bs, w, half, mask, lc);
#define FFTMI_CASE_ColsFft(K) \
  case K:                     \
    return ColsFft<K>::run(inv, ws, nimg, M, rb, bs, w, lc);
#define FFTMI_CASE_ColsGrad(K) \
  case K:                      \
    return ColsGrad<K>::run(ws, save, mask, part, nimg, groups, M, rb, bs, w, w_lin, w_sq, lc);
#define FFTMI_CASE_RowsXd(K) \
  case K:                    \
    return RowsXd<K>::run(x, c, wsx, wsd, blocks, rb, bs, lc);
#define FFTMI_CASE_ColsMse(K) \
  case K:                     \
    return ColsMse<K>::run(wsx, wsd, mask, sumx, sumxr, part, nimg, groups, M, mh, rb, bs, w, ntiles, lc);
#define FFTMI_CASE_ColsStrided(K) \
  case K:                         \
    return ColsStrided<K>::run(inv, twiddle_transpose, in, out, batch, C, w, scale, tw_fs, in_bstride, in_rstride, \
                               out_bstride, out_rstride, nt, lc);

hipError_t launch_rows_rm(int log2L, bool inv, const void* in, bool in_f32, void* out, bool out_f32, int64_t rows,
                          float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsRm, log2L)
}

hipError_t launch_rows_to_blk(int log2L, bool inv, bool pair, const void* in, bool in_f32, float2* ws,
                              int64_t blocks, int rb, unsigned bs, float scale, const Launch& lc) {
  const bool half = false;
  const void* in2 = nullptr;
  FFTMI_DISPATCH(RowsToBlk, log2L)
}

hipError_t launch_rows_to_blk_diff(int log2L, const float* in, const float* in2, float2* ws, int64_t blocks, int rb,
                                   unsigned bs, float scale, const Launch& lc) {
  if (rb < 2) return hipErrorInvalidValue;
  const bool inv = false, pair = true, half = false, in_f32 = true;
  FFTMI_DISPATCH(RowsToBlk, log2L)
}

hipError_t launch_rows_to_blk_half(int log2L, const float* in, float2* ws, int64_t blocks, int rb, unsigned bs,
                                   float scale, const Launch& lc) {
  const bool inv = false, pair = true, half = true, in_f32 = true;
  const void* in2 = nullptr;
  FFTMI_DISPATCH(RowsToBlk, log2L)
}

hipError_t launch_rows_loss(int log2L, const float2* ws, const float* x, const float* c, float* part, int64_t blocks,
                            int rb, unsigned bs, float scale, int64_t* ntiles, const Launch& lc) {
  FFTMI_DISPATCH(RowsLoss, log2L)
}

int64_t sum_partials_scratch(int64_t n) { return std::max<int64_t>(1, (n + kSumRun - 1) / kSumRun); }

hipError_t launch_sum_partials(const float* part, int64_t n, float weight, float* out, double* mid, hipStream_t st) {
  const int64_t g = sum_partials_scratch(n);
  if (n > 0) hipLaunchKernelGGL(k_sum_runs, dim3((unsigned)g), dim3(256), 0, st, part, n, mid);
  hipLaunchKernelGGL(k_sum_mid, dim3(1), dim3(256), 0, st, mid, n > 0 ? (int)g : 0, weight, out);
  return hipGetLastError();
}

hipError_t launch_rows_c2r(int log2L, const float2* ws, void* out, bool out_f32, int64_t blocks, int rb, unsigned bs,
                           float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsC2R, log2L)
}

hipError_t launch_rows_from_blk(int log2L, bool inv, const float2* ws, void* out, bool out_f32, int64_t blocks,
                                int rb, unsigned bs, float scale, const Launch& lc) {
  FFTMI_DISPATCH(RowsFromBlk, log2L)
}

hipError_t launch_cols_filter(int log2L, float2* ws, float2* save, int64_t nimg, int M, int rb, unsigned bs, int w,
                              bool half, const MaskArgs& mask, const Launch& lc) {
  FFTMI_DISPATCH(ColsFilter, log2L)
}

hipError_t launch_cols_fft(int log2L, bool inv, float2* ws, int64_t nimg, int M, int rb, unsigned bs, int w,
                           const Launch& lc) {
  FFTMI_DISPATCH(ColsFft, log2L)
}

namespace {
dim3 elementwise_grid(int64_t n) { return dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)); }
}  // namespace

hipError_t launch_pad(const void* in, void* out, bool f32, int64_t nimg, int n0, int m0, int log2N, int log2M,
                      hipStream_t st) {
  const int64_t total = nimg << (log2N + log2M);
  if (total == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_pad<float>, elementwise_grid(total), dim3(256), 0, st, static_cast<const float*>(in),
                       static_cast<float*>(out), total, n0, m0, log2N, log2M);
  else
    hipLaunchKernelGGL(k_pad<float2>, elementwise_grid(total), dim3(256), 0, st, static_cast<const float2*>(in),
                       static_cast<float2*>(out), total, n0, m0, log2N, log2M);
  return hipGetLastError();
}

hipError_t launch_crop(const void* in, void* out, bool f32, int64_t nimg, int n0, int m0, int log2N, int log2M,
                       hipStream_t st) {
  const int64_t total = nimg * n0 * m0;
  if (total == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_crop<float>, elementwise_grid(total), dim3(256), 0, st, static_cast<const float*>(in),
                       static_cast<float*>(out), total, n0, m0, log2N, log2M);
  else
    hipLaunchKernelGGL(k_crop<float2>, elementwise_grid(total), dim3(256), 0, st, static_cast<const float2*>(in),
                       static_cast<float2*>(out), total, n0, m0, log2N, log2M);
  return hipGetLastError();
}

hipError_t launch_transpose_f32(const float* in, float* out, int64_t N, int64_t M, hipStream_t st) {
  if (N <= 0 || M <= 0) return hipSuccess;
  const dim3 g((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL(k_transpose_f32, g, dim3(256), 0, st, in, out, N, M);
  return hipGetLastError();
}

hipError_t launch_unblock_mag(const float2* ws, float* out, int64_t rows, int M, int rb, unsigned bs, float scale,
                              hipStream_t st) {
  if (rows % rb || (M & (M - 1))) return hipErrorInvalidValue;
  const int64_t items = rows / rb * M;
  if (items == 0) return hipSuccess;
  const dim3 g = elementwise_grid(items), b(256);
  switch (rb) {
    case 1:
      hipLaunchKernelGGL(k_unblock_mag<1>, g, b, 0, st, ws, out, M, bs, items, scale);
      break;
    case 2:
      hipLaunchKernelGGL(k_unblock_mag<2>, g, b, 0, st, ws, out, M, bs, items, scale);
      break;
    case 4:
      hipLaunchKernelGGL(k_unblock_mag<4>, g, b, 0, st, ws, out, M, bs, items, scale);
      break;
    case 8:
      hipLaunchKernelGGL(k_unblock_mag<8>, g, b, 0, st, ws, out, M, bs, items, scale);
      break;
    case 16:
      hipLaunchKernelGGL(k_unblock_mag<16>, g, b, 0, st, ws, out, M, bs, items, scale);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unblock(const float2* ws, void* out, bool out_f32, int64_t rows, int M, int rb, unsigned bs,
                          float scale, hipStream_t st) {
  if (rows % rb || (M & (M - 1))) return hipErrorInvalidValue;
  const int64_t items = rows / rb * M;
  if (items == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((items + 255) / 256, 65536);
  const dim3 g((unsigned)blocks), b(256);
#define FFTMI_UNBLOCK(R)                                                                                   \
  if (rb == R) {                                                                                           \
    if (out_f32)                                                                                           \
      hipLaunchKernelGGL((k_unblock<R, true>), g, b, 0, st, ws, out, M, bs, items, scale);                     \
    else                                                                                                   \
      hipLaunchKernelGGL((k_unblock<R, false>), g, b, 0, st, ws, out, M, bs, items, scale);                    \
    return hipGetLastError();                                                                              \
  }
  FFTMI_UNBLOCK(1)
  FFTMI_UNBLOCK(2)
  FFTMI_UNBLOCK(4)
  FFTMI_UNBLOCK(8)
  FFTMI_UNBLOCK(16)
#undef FFTMI_UNBLOCK
  return hipErrorInvalidValue;
}

hipError_t launch_cols_grad(int log2L, const float2* ws, const float2* save, const float* mask, float* part,
                            int64_t nimg, int groups, int M, int rb, unsigned bs, int w, float w_lin, float w_sq,
                            const Launch& lc) {
  FFTMI_DISPATCH(ColsGrad, log2L)
}

hipError_t launch_rows_xd(int log2L, const float* x, const float* c, float2* wsx, float2* wsd, int64_t blocks, int rb,
                          unsigned bs, const Launch& lc) {
  FFTMI_DISPATCH(RowsXd, log2L)
}

hipError_t launch_cols_mse(int log2L, const float2* wsx, const float2* wsd, const float* mask, float* sumx,
                           float* sumxr, float* part, int64_t nimg, int groups, int M, int mh, int rb, unsigned bs,
                           int w, int64_t* ntiles, const Launch& lc) {
  FFTMI_DISPATCH(ColsMse, log2L)
}

hipError_t launch_mse_grad_sums(const float* sumx, const float* sumxr, const float* mask, float* grad, int N, int M,
                                int mh, int groups, float w, hipStream_t stream) {
  const int64_t n = (int64_t)N * M;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mse_grad_sums, dim3((unsigned)blocks), dim3(256), 0, stream, sumx, sumxr, mask, grad, N, M, mh,
                     groups, w);
  return hipGetLastError();
}

hipError_t launch_sum_groups(const float* part, float* grad, int64_t n, int groups, hipStream_t stream) {
  if (n % 4) return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  if (n4 == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)blocks), dim3(256), 0, stream,
                     reinterpret_cast<const float4*>(part), reinterpret_cast<float4*>(grad), n4, groups);
  return hipGetLastError();
}

hipError_t launch_cols_strided(int log2L, bool inv, bool twiddle_transpose, const float2* in, float2* out,
                               int64_t batch, int C, int w, float scale, const float2* tw_fs, int64_t in_bstride,
                               int in_rstride, int64_t out_bstride, int out_rstride, int nt, const Launch& lc) {
  FFTMI_DISPATCH(ColsStrided, log2L)
}

static int tw_lds_bytes_rt(int L) { return L <= (1 << kLdsTwMaxLog2) ? lds_tw_bytes(L) : 0; }
int lds_bytes_rows_rm(int log2L, int tpw) { return tw_lds_bytes_rt(1 << log2L) + tpw * lds_region_bytes(1 << log2L, 1); }
int lds_bytes_cols(int log2L, int w) {
  const int L = 1 << log2L;
  const int cols = tw_lds_bytes_for(L, twm_for(L, FFTMI_TWM_COLS)) + w * lds_region_bytes(L, w, FFTMI_SPLIT_COLS != 0);
  return std::max(cols, tw_lds_bytes_rt(L) + w * lds_region_bytes(L, w));
}
int max_block_threads(int log2L) { return threads_per_transform(1 << log2L) > 512 ? 1024 : 512; }
int lds_bytes_rows_blk(int log2L, int nt) {
  return tw_lds_bytes_rt(1 << log2L) + nt * lds_region_bytes(1 << log2L, nt);
}

}  // namespace fftmi
