// fft_core.hpp -- device-side building blocks: complex helpers, radix-2/4/8/16
// butterflies held in registers, and the LDS-staged Stockham pass sequence.
//
// Conventions: a forward pass uses the factors e^{-2 pi i t/n} (eq. E2 and
// Table 2's Z), an inverse pass their conjugates e^{+2 pi i t/n} (eq. E3).
// Nothing here scales; callers fold 1/N (or 1/M) into a load or a store.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_schedule.hpp"

#ifndef FFTMI_TW_PREFETCH
#define FFTMI_TW_PREFETCH 0
#endif


namespace fftmi {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * w (forward) or a * conj(w) (inverse)
template <bool INV>
__device__ __forceinline__ float2 cmul_tw(float2 a, float2 w) {
  if constexpr (!INV)
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
  else
    return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

// a * (-i) (forward) or a * (+i) (inverse): the quarter-turn factor W_4^1.
template <bool INV>
__device__ __forceinline__ float2 mul_quarter(float2 a) {
  if constexpr (!INV)
    return make_float2(a.y, -a.x);
  else
    return make_float2(-a.y, a.x);
}

// Constants cos(pi/8), sin(pi/8), sqrt(1/2), rounded once to float.
constexpr float kC8 = 0.923879532511286756128f;
constexpr float kS8 = 0.382683432365089771728f;
constexpr float kH2 = 0.707106781186547524401f;

// a * W_16^m (forward: e^{-i pi m/8}) for the m that occur inside a 4x4 split.
template <bool INV, int m>
__device__ __forceinline__ float2 mul_w16(float2 a) {
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return mul_quarter<INV>(a);
  } else if constexpr (m == 2) {  // (1 - i)/sqrt2
    return INV ? make_float2((a.x - a.y) * kH2, (a.x + a.y) * kH2)
               : make_float2((a.x + a.y) * kH2, (a.y - a.x) * kH2);
  } else if constexpr (m == 6) {  // (-1 - i)/sqrt2
    return INV ? make_float2(-(a.x + a.y) * kH2, (a.x - a.y) * kH2)
               : make_float2((a.y - a.x) * kH2, -(a.x + a.y) * kH2);
  } else if constexpr (m == 1) {
    return cmul_tw<INV>(a, make_float2(kC8, -kS8));
  } else if constexpr (m == 3) {
    return cmul_tw<INV>(a, make_float2(kS8, -kC8));
  } else if constexpr (m == 9) {
    return cmul_tw<INV>(a, make_float2(-kC8, kS8));
  } else {
    static_assert(m == 0, "unused W16 power");
    return a;
  }
}

// In-register DFTs of length R on v[0..R-1] (stride 1), natural order out.
template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 t0 = cadd(v0, v2), t1 = csub(v0, v2);
  float2 t2 = cadd(v1, v3), t3 = mul_quarter<INV>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v1 = cadd(t1, t3);
  v2 = csub(t0, t2);
  v3 = csub(t1, t3);
}

// Radix 8 as 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2.
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  // twiddles W_8^{k1} on the n2 = 1 branch (k1 = 0..3 at v[1], v[3], v[5], v[7])
  v[3] = mul_w16<INV, 2>(v[3]);
  v[5] = mul_w16<INV, 4>(v[5]);
  v[7] = mul_w16<INV, 6>(v[7]);
  float2 o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
    o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// Radix 16 as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
  // column DFT4s over n1 for each n2; results Y[n2][k1] stay at v[4 k1 + n2]
  dft4<INV>(v[0], v[4], v[8], v[12]);
  dft4<INV>(v[1], v[5], v[9], v[13]);
  dft4<INV>(v[2], v[6], v[10], v[14]);
  dft4<INV>(v[3], v[7], v[11], v[15]);
  // twiddles W_16^{n2 k1}
  v[5] = mul_w16<INV, 1>(v[5]);
  v[9] = mul_w16<INV, 2>(v[9]);
  v[13] = mul_w16<INV, 3>(v[13]);
  v[6] = mul_w16<INV, 2>(v[6]);
  v[10] = mul_w16<INV, 4>(v[10]);
  v[14] = mul_w16<INV, 6>(v[14]);
  v[7] = mul_w16<INV, 3>(v[7]);
  v[11] = mul_w16<INV, 6>(v[11]);
  v[15] = mul_w16<INV, 9>(v[15]);
  // row DFT4s over n2 for each k1; X[k1 + 4 k2]
  dft4<INV>(v[0], v[1], v[2], v[3]);
  dft4<INV>(v[4], v[5], v[6], v[7]);
  dft4<INV>(v[8], v[9], v[10], v[11]);
  dft4<INV>(v[12], v[13], v[14], v[15]);
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<INV>(v);
  } else {
    static_assert(R == 16, "radix");
    dft16<INV>(v);
  }
}

// ---------------------------------------------------------------------------
// One Stockham pass.  Butterfly b = j + s*TPT (s < E/R) reads the positions
// b + r*(L/R), i.e. register slots q = s + r*(E/R); stage outputs go to
// (b / NS) * NS * R + (b % NS) + r * NS.
// ---------------------------------------------------------------------------
template <int L, int S>
struct StageInfo {
  static constexpr int E = elems_per_thread(L);
  static constexpr int TPT = L / E;
  static constexpr int R = stage_radix(L, S);
  static constexpr int NS = stage_ns(L, S);
  static constexpr int BPT = E / R;
  static constexpr int NTW = (NS > 1) ? BPT * (R - 1) : 0;  // twiddles per thread
};

// Twiddles of stage S for thread j, fetched ahead of the LDS exchange.
template <int L, int S>
__device__ __forceinline__ void stage_twiddles(float2* tw_reg, int j, const float2* __restrict__ blob) {
  using I = StageInfo<L, S>;
  if constexpr (I::NS > 1) {
    const float2* base = blob + tw_stage_offset(L, S);
#pragma unroll
    for (int s = 0; s < I::BPT; ++s) {
      const int k = (j + s * I::TPT) & (I::NS - 1);
      const float2* t = base + k * I::R;
#pragma unroll
      for (int r = 1; r < I::R; ++r) tw_reg[s * (I::R - 1) + r - 1] = __ldg(t + r);
    }
  }
}

// The same from the LDS copy of the tables (layout of lds_tw_offset).
template <int L, int S>
__device__ __forceinline__ void stage_twiddles_lds(float2* tw_reg, int j, const float2* twl) {
  using I = StageInfo<L, S>;
  if constexpr (I::NS > 1) {
    const float2* base = twl + lds_tw_offset(L, S);
#pragma unroll
    for (int s = 0; s < I::BPT; ++s) {
      const int k = (j + s * I::TPT) & (I::NS - 1);
#pragma unroll
      for (int r = 1; r < I::R; ++r) tw_reg[s * (I::R - 1) + r - 1] = base[(r - 1) * I::NS + k];
    }
  }
}

// Copy the LDS-layout twiddles of length L into LDS (all threads of the
// workgroup; the first exchange's barriers order it before any use).
template <int L>
__device__ __forceinline__ void load_twiddles_lds(float2* twl, const float2* __restrict__ src, int tid, int nthr) {
  for (int i = tid; i < lds_tw_entries(L); i += nthr) twl[i] = __ldg(src + i);
}

template <int L, int S, bool INV>
__device__ __forceinline__ void stage_compute(float2 (&a)[elems_per_thread(L)], const float2* tw_reg) {
  using I = StageInfo<L, S>;
#pragma unroll
  for (int s = 0; s < I::BPT; ++s) {
    float2 v[I::R];
#pragma unroll
    for (int r = 0; r < I::R; ++r) v[r] = a[s + r * I::BPT];
    if constexpr (I::NS > 1) {
#pragma unroll
      for (int r = 1; r < I::R; ++r) v[r] = cmul_tw<INV>(v[r], tw_reg[s * (I::R - 1) + r - 1]);
    }
    dft<I::R, INV>(v);
#pragma unroll
    for (int r = 0; r < I::R; ++r) a[s + r * I::BPT] = v[r];
  }
}

// Workgroup barrier for LDS exchanges.  __syncthreads() also waits for every
// outstanding global load and store of the wave (a workgroup fence), which
// would stall on the next tile's prefetch; the exchanges only need LDS
// accesses ordered: wait for this wave's LDS operations, then meet at the
// barrier.  The memory clobber keeps the compiler from moving LDS accesses
// across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// LDS parts: the real and the imaginary halves of a complex value go through
// LDS separately when FFTMI_SPLIT_X is set (4-byte entries, half the LDS per
// transform, twice the barriers); otherwise whole complex values (8 bytes).
enum { kRe = 0, kIm = 1, kBoth = 2 };

template <int PART>
__device__ __forceinline__ void lds_put(void* x, int i, float2 v) {
  if constexpr (PART == kBoth)
    static_cast<float2*>(x)[i] = v;
  else
    static_cast<float*>(x)[i] = PART == kRe ? v.x : v.y;
}

template <int PART>
__device__ __forceinline__ void lds_get(const void* x, int i, float2& v) {
  if constexpr (PART == kBoth)
    v = static_cast<const float2*>(x)[i];
  else if constexpr (PART == kRe)
    v.x = static_cast<const float*>(x)[i];
  else
    v.y = static_cast<const float*>(x)[i];
}

// Padded LDS positions are written as pad(base) + pad(offset) with a
// compile-time offset, which the hardware takes as an instruction immediate.
// This is exact when the offset is a multiple of 16, or when base is a
// multiple of 16 and the offset is below 16, or (natural positions
// j + q*TPT, j < TPT, TPT a power of two) when base % 16 + offset % 16 < 16.
template <int L, int S, int PART>
__device__ __forceinline__ void stage_store(const float2 (&a)[elems_per_thread(L)], int j, void* x) {
  using I = StageInfo<L, S>;
  static_assert(I::NS % 16 == 0 || (I::NS == 1 && I::R == 16), "padded offsets must split exactly");
#pragma unroll
  for (int s = 0; s < I::BPT; ++s) {
    const int b = j + s * I::TPT;
    const int pb = lds_pad((b & ~(I::NS - 1)) * I::R + (b & (I::NS - 1)));
#pragma unroll
    for (int r = 0; r < I::R; ++r) lds_put<PART>(x, pb + lds_pad(r * I::NS), a[s + r * I::BPT]);
  }
}

template <int L, int PART>
__device__ __forceinline__ void gather_natural(float2 (&a)[elems_per_thread(L)], int j, const void* x) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int pj = lds_pad(j);
#pragma unroll
  for (int q = 0; q < E; ++q) lds_get<PART>(x, pj + lds_pad(q * TPT), a[q]);
}

template <int L, int PART>
__device__ __forceinline__ void scatter_natural(const float2 (&a)[elems_per_thread(L)], int j, void* x) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  const int pj = lds_pad(j);
#pragma unroll
  for (int q = 0; q < E; ++q) lds_put<PART>(x, pj + lds_pad(q * TPT), a[q]);
}

// Stage S-1 outputs -> LDS -> stage S inputs (natural positions j + q*TPT).
template <int L, int S, bool SPLIT = kSplitExchange>
__device__ __forceinline__ void exchange(float2 (&a)[elems_per_thread(L)], int j, void* x) {
  if constexpr (SPLIT) {
    lds_barrier();  // earlier readers of x are done
    stage_store<L, S - 1, kRe>(a, j, x);
    lds_barrier();
    gather_natural<L, kRe>(a, j, x);
    lds_barrier();
    stage_store<L, S - 1, kIm>(a, j, x);
    lds_barrier();
    gather_natural<L, kIm>(a, j, x);
  } else {
    lds_barrier();
    stage_store<L, S - 1, kBoth>(a, j, x);
    lds_barrier();
    gather_natural<L, kBoth>(a, j, x);
  }
}

// Where a transform's twiddle factors come from.
enum TwMode {
  kTwGlobal = 0,  // loaded from the global tables at every stage
  kTwLds = 1,     // loaded from an LDS copy of the tables
  kTwReg = 2,     // held in registers for the kernel's whole run
  kTwMix = 3,     // small stage tables (NS <= 16) in LDS, the rest in registers
};

// kTwMix: stage s >= 1 reads its factors from LDS when its table is small
// (stride NS <= 16: at most 15 x 16 entries, 1920 bytes), so that the
// registers hold only the factors of the long-stride stages.  NS grows with
// s, so the LDS stages are a prefix 1 .. mix_lds_end(L) - 1.
FFTMI_HD constexpr bool mix_in_lds(int L, int s) { return stage_ns(L, s) <= 16; }
FFTMI_HD constexpr int mix_lds_end(int L) {
  int s = 1;
  while (s < num_stages(L) && mix_in_lds(L, s)) ++s;
  return s;
}
// LDS entries of the small tables (LDS layout of lds_tw_offset).
FFTMI_HD constexpr int mix_lds_entries(int L) { return lds_tw_offset(L, mix_lds_end(L)); }
FFTMI_HD constexpr int mix_lds_bytes(int L) { return mix_lds_entries(L) > 0 ? ((mix_lds_entries(L) * 8 + 255) / 256) * 256 : 0; }

// Register-held twiddles: all stages s >= 1 of one thread, in stage order.
template <int L>
__host__ __device__ constexpr int reg_tw_offset(int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) {
    const int ns = stage_ns(L, i), r = stage_radix(L, i);
    off += ns > 1 ? (elems_per_thread(L) / r) * (r - 1) : 0;
  }
  return off;
}
template <int L>
__host__ __device__ constexpr int reg_tw_count() {
  return reg_tw_offset<L>(num_stages(L)) > 0 ? reg_tw_offset<L>(num_stages(L)) : 1;
}

// Load thread j's twiddles of every stage from the global tables once.
template <int L, int S = 1>
__device__ __forceinline__ void load_twiddles_reg(float2 (&twr)[reg_tw_count<L>()], int j,
                                                  const float2* __restrict__ blob) {
  if constexpr (S < num_stages(L)) {
    stage_twiddles<L, S>(twr + reg_tw_offset<L>(S), j, blob);
    load_twiddles_reg<L, S + 1>(twr, j, blob);
  }
}

// kTwMix: register offsets count only the stages kept in registers.
template <int L>
__host__ __device__ constexpr int reg_tw_offset_mix(int s) {
  int off = 0;
  for (int i = mix_lds_end(L); i < s; ++i) off += (elems_per_thread(L) / stage_radix(L, i)) * (stage_radix(L, i) - 1);
  return off;
}
template <int L>
__host__ __device__ constexpr int reg_tw_count_mix() {
  return reg_tw_offset_mix<L>(num_stages(L)) > 0 ? reg_tw_offset_mix<L>(num_stages(L)) : 1;
}

// kTwMix set-up: thread j's register factors of the long-stride stages, and
// the workgroup's LDS copy of the small tables, rearranged from the global
// layout [k][r] to the LDS layout [r-1][k] (entries (r-1)*NS + k).  The
// first exchange's barriers order the copy before any read.
template <int L, int S = mix_lds_end(L)>
__device__ __forceinline__ void load_twiddles_reg_mix(float2 (&twr)[reg_tw_count_mix<L>()], int j,
                                                      const float2* __restrict__ blob) {
  if constexpr (S < num_stages(L)) {
    stage_twiddles<L, S>(twr + reg_tw_offset_mix<L>(S), j, blob);
    load_twiddles_reg_mix<L, S + 1>(twr, j, blob);
  }
}
template <int L, int S = 1>
__device__ __forceinline__ void load_twiddles_lds_mix(float2* twl, const float2* __restrict__ blob, int tid, int nthr) {
  if constexpr (S < mix_lds_end(L)) {
    constexpr int NS = stage_ns(L, S), R = stage_radix(L, S), n = NS * (R - 1);
    const float2* src = blob + tw_stage_offset(L, S);
    float2* dst = twl + lds_tw_offset(L, S);
    for (int i = tid; i < n; i += nthr) dst[i] = __ldg(src + (i % NS) * R + i / NS + 1);
    load_twiddles_lds_mix<L, S + 1>(twl, blob, tid, nthr);
  }
}

template <int L, int S, bool INV, int TWM, bool SPLIT = kSplitExchange>
struct StageChain {
  __device__ __forceinline__ static void run(float2 (&a)[elems_per_thread(L)], int j, void* x,
                                             const float2* __restrict__ tws) {
    if constexpr (S < num_stages(L)) {
      if constexpr (TWM == kTwReg) {
        exchange<L, S, SPLIT>(a, j, x);
        stage_compute<L, S, INV>(a, tws + reg_tw_offset<L>(S));
      } else if constexpr (TWM == kTwMix && !mix_in_lds(L, S)) {
        exchange<L, S, SPLIT>(a, j, x);
        stage_compute<L, S, INV>(a, tws + reg_tw_offset_mix<L>(S));
      } else if constexpr (TWM == kTwMix) {
        // the small tables sit at the start of the workgroup's dynamic LDS
        extern __shared__ float4 lds_raw[];
        float2 tw[StageInfo<L, S>::NTW > 0 ? StageInfo<L, S>::NTW : 1];
        exchange<L, S, SPLIT>(a, j, x);
        stage_twiddles_lds<L, S>(tw, j, reinterpret_cast<const float2*>(lds_raw));
        stage_compute<L, S, INV>(a, tw);
      } else {
        float2 tw[StageInfo<L, S>::NTW > 0 ? StageInfo<L, S>::NTW : 1];
        if constexpr (TWM == kTwLds) {
          exchange<L, S, SPLIT>(a, j, x);
          stage_twiddles_lds<L, S>(tw, j, tws);
        } else {
          if constexpr (FFTMI_TW_PREFETCH) stage_twiddles<L, S>(tw, j, tws);
          exchange<L, S, SPLIT>(a, j, x);
          if constexpr (!FFTMI_TW_PREFETCH) stage_twiddles<L, S>(tw, j, tws);
        }
        stage_compute<L, S, INV>(a, tw);
      }
      StageChain<L, S + 1, INV, TWM, SPLIT>::run(a, j, x, tws);
    }
  }
};

// Whole transform of length L.  On entry a[q] = x_in[j + q*TPT]; on exit
// a[q] = X[j + q*TPT] (unscaled).  x is this transform's LDS region
// (lds_region_bytes(L, .) bytes).  Every thread of the workgroup must call
// this the same number of times (it contains workgroup barriers when L > 16).
// tws: the global tables (kTwGlobal), the LDS copy (kTwLds) or this thread's
// register array from load_twiddles_reg (kTwReg).
template <int L, bool INV, int TWM = kTwGlobal, bool SPLIT = kSplitExchange>
__device__ __forceinline__ void fft_reg(float2 (&a)[elems_per_thread(L)], int j, void* x,
                                        const float2* __restrict__ tws) {
  if constexpr (num_stages(L) > 0) {
    // Hide the table address and the thread index from the optimiser: with
    // two transforms in one kernel, twiddles and LDS addresses are then
    // recomputed per transform instead of being held live from the first
    // transform to the second.  (LDS and register tables are left alone:
    // laundering an LDS pointer would turn its reads into flat loads.)
    const float2* tw = tws;
    if constexpr (TWM == kTwGlobal) asm volatile("" : "+s"(tw));
    asm volatile("" : "+v"(j));
    stage_compute<L, 0, INV>(a, nullptr);
    StageChain<L, 1, INV, TWM, SPLIT>::run(a, j, x, tw);
  }
}

}  // namespace fftmi
