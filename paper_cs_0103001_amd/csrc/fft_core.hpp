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

template <int L, int S>
__device__ __forceinline__ void stage_store(const float2 (&a)[elems_per_thread(L)], int j, float2* x) {
  using I = StageInfo<L, S>;
#pragma unroll
  for (int s = 0; s < I::BPT; ++s) {
    const int b = j + s * I::TPT;
    const int base = (b & ~(I::NS - 1)) * I::R + (b & (I::NS - 1));
#pragma unroll
    for (int r = 0; r < I::R; ++r) x[lds_pad(base + r * I::NS)] = a[s + r * I::BPT];
  }
}

template <int L>
__device__ __forceinline__ void gather_natural(float2 (&a)[elems_per_thread(L)], int j, const float2* x) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) a[q] = x[lds_pad(j + q * TPT)];
}

template <int L>
__device__ __forceinline__ void scatter_natural(const float2 (&a)[elems_per_thread(L)], int j, float2* x) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) x[lds_pad(j + q * TPT)] = a[q];
}

template <int L, int S, bool INV>
struct StageChain {
  __device__ __forceinline__ static void run(float2 (&a)[elems_per_thread(L)], int j, float2* x,
                                             const float2* __restrict__ blob) {
    if constexpr (S < num_stages(L)) {
      float2 tw[StageInfo<L, S>::NTW > 0 ? StageInfo<L, S>::NTW : 1];
#if FFTMI_TW_PREFETCH
      stage_twiddles<L, S>(tw, j, blob);
#endif
      __syncthreads();  // earlier readers of x are done
      stage_store<L, S - 1>(a, j, x);
      __syncthreads();
      gather_natural<L>(a, j, x);
#if !FFTMI_TW_PREFETCH
      stage_twiddles<L, S>(tw, j, blob);
#endif
      stage_compute<L, S, INV>(a, tw);
      StageChain<L, S + 1, INV>::run(a, j, x, blob);
    }
  }
};

// Whole transform of length L.  On entry a[q] = x_in[j + q*TPT]; on exit
// a[q] = X[j + q*TPT] (unscaled).  x is this transform's LDS region
// (lds_size(L) entries).  Every thread of the workgroup must call this the
// same number of times (it contains workgroup barriers when L > 16).
template <int L, bool INV>
__device__ __forceinline__ void fft_reg(float2 (&a)[elems_per_thread(L)], int j, float2* x,
                                        const float2* __restrict__ blob) {
  if constexpr (num_stages(L) > 0) {
    // Hide the table address from the optimiser: the twiddles of two
    // transforms in one kernel are then loaded per transform, instead of
    // being kept live in registers from the first one to the second.
    const float2* tw = blob;
    asm volatile("" : "+s"(tw));
    stage_compute<L, 0, INV>(a, nullptr);
    StageChain<L, 1, INV>::run(a, j, x, tw);
  }
}

}  // namespace fftmi
