// kernel_common.hpp -- device helpers shared by the kernels of libfftmi: the
// per-length launch shape, twiddle sources, LDS regions, tile order, global
// addressing helpers and the mask evaluators.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fftmi.h"
#include "fft_core.hpp"
#include "launch.hpp"

namespace fftmi {

__device__ __forceinline__ int ilog2_pow2(int x) { return 31 - __clz(x); }

// Dynamic LDS of the workgroup: [twiddle tables][per-transform regions].
__device__ __forceinline__ char* lds_base() {
  extern __shared__ float4 lds_raw[];
  return reinterpret_cast<char*>(lds_raw);
}

// Twiddle source of the single-pass kernels (lengths up to 2^12): small
// stage tables in LDS, the long-stride stages' factors in registers.
#ifndef FFTMI_TWM
#define FFTMI_TWM 3
#endif

// Software prefetch of the next tile into registers (persistent kernels of
// the 2D path), per pass: the row pass into the blocked layout, the column
// pass, the row pass out of it.  Without it a kernel uses fewer registers and
// relies on more resident workgroups per CU to overlap memory and arithmetic:
// at 4096 points the column pass and the last row pass fit four workgroups
// per CU (the LDS limit) without it, three or fewer with it, and run faster
// so; the first row pass (two transforms per workgroup) is faster with it.
#ifndef FFTMI_PF_ROWS_IN
#define FFTMI_PF_ROWS_IN 1
#endif
#ifndef FFTMI_PF_COLS
#define FFTMI_PF_COLS 0
#endif
#ifndef FFTMI_PF_ROWS_OUT
#define FFTMI_PF_ROWS_OUT 0
#endif
#ifndef FFTMI_PF_ROWS_1D
#define FFTMI_PF_ROWS_1D 0
#endif
enum { kPassRowsIn = 0, kPassCols = 1, kPassRowsOut = 2, kPassRows1D = 3 };
// Non-temporal accesses per kernel family, as bit masks, measured per
// family.  One-pass 1D rows: 1 loads, 2 stores (stores only: 2^10..2^14 at
// 6.4-6.6 / 5.7 / 4.7 TB/s against 5.0 / 4.3 / 3.9 without; loads too: less).
// Ragged passes: 1 the first row pass's loads, 2 the column pass's loads, 4
// the last row pass's loads (none: each was slower).  The four-step passes
// choose at plan creation.
#ifndef FFTMI_NT_1D
#define FFTMI_NT_1D 2
#endif
#ifndef FFTMI_NT_RAGGED
#define FFTMI_NT_RAGGED 0
#endif
// Stores with the non-temporal hint: the saved spectrum of the fused MSE
// forward (FFTMI_NT_SAVE: read back only by the backward pass, after the
// whole batch), the residual spectrum rows of the mask gradient
// (FFTMI_NT_DIFF: slower).
#ifndef FFTMI_NT_SAVE
#define FFTMI_NT_SAVE 1
#endif
#ifndef FFTMI_NT_DIFF
#define FFTMI_NT_DIFF 0
#endif
// Transforms of 2^14 points take 1024-thread workgroups, whose threads have
// at most 128 VGPRs: too few for a second tile, so they never prefetch.
template <int L, int PASS>
struct Prefetch {
  static constexpr bool on = L > 0 && threads_per_transform(L) <= 512 && (PASS == kPassRowsIn ? FFTMI_PF_ROWS_IN != 0
                                       : PASS == kPassCols ? FFTMI_PF_COLS != 0
                                       : PASS == kPassRowsOut ? FFTMI_PF_ROWS_OUT != 0
                                                              : FFTMI_PF_ROWS_1D != 0);
};

// Mixed twiddles need little LDS at any length; the register share grows
// with the stages beyond the first, so they are used up to 2^FFTMI_MIX_MAX_LOG2.
#ifndef FFTMI_MIX_MAX_LOG2
#define FFTMI_MIX_MAX_LOG2 12
#endif
FFTMI_HD constexpr int twm_for(int L, int req, int mix_max_log2 = FFTMI_MIX_MAX_LOG2) {
  return req == kTwMix ? (L <= (1 << mix_max_log2) ? kTwMix : kTwGlobal)
                       : (L <= (1 << kLdsTwMaxLog2) ? req : kTwGlobal);
}

template <int L>
struct Shape {
  static constexpr int E = elems_per_thread(L);
  static constexpr int TPT = L / E;
  // Workgroups hold at most 512 threads (one 2^14-point transform needs
  // 1024): a thread may then use up to 256 VGPRs, enough for the current
  // tile, the prefetched one and its twiddle factors.
  static constexpr int LB = TPT > 512 ? 1024 : 512;
  // Twiddles: in registers up to 2^12 points (30 complex values per thread),
  // from the global tables beyond.
  static constexpr int TWM = twm_for(L, FFTMI_TWM);
  static constexpr int TWB = TWM == kTwLds ? lds_tw_bytes(L) : (TWM == kTwMix ? mix_lds_bytes(L) : 0);  // LDS bytes
};

// A kernel's twiddle factors for thread index j: a register array loaded
// once (kTwReg), an LDS copy made by the whole workgroup (kTwLds), both
// (kTwMix: small tables in LDS, the long-stride stages in registers), or the
// global tables (kTwGlobal).  The host passes the matching table layout
// (the global layout for kTwMix).
template <int L, int M = Shape<L>::TWM>
struct Twiddles {
  const float2* p;
  __device__ __forceinline__ Twiddles(const float2* __restrict__ src, int) : p(src) {}
  __device__ __forceinline__ const float2* ptr() const { return p; }
};
template <int L>
struct Twiddles<L, kTwLds> {
  const float2* p;
  __device__ __forceinline__ Twiddles(const float2* __restrict__ src, int) {
    extern __shared__ float4 lds_raw[];
    float2* t = reinterpret_cast<float2*>(lds_raw);
    load_twiddles_lds<L>(t, src, threadIdx.x, blockDim.x);
    p = t;
  }
  __device__ __forceinline__ const float2* ptr() const { return p; }
};
template <int L>
struct Twiddles<L, kTwReg> {
  float2 r[reg_tw_count<L>()];
  __device__ __forceinline__ Twiddles(const float2* __restrict__ src, int j) { load_twiddles_reg<L>(r, j, src); }
  __device__ __forceinline__ const float2* ptr() const { return r; }
};

template <int L>
struct Twiddles<L, kTwMix> {
  float2 r[reg_tw_count_mix<L>()];
  __device__ __forceinline__ Twiddles(const float2* __restrict__ src, int j) {
    extern __shared__ float4 lds_raw[];
    load_twiddles_lds_mix<L>(reinterpret_cast<float2*>(lds_raw), src, threadIdx.x, blockDim.x);
    load_twiddles_reg_mix<L>(r, j, src);
  }
  __device__ __forceinline__ const float2* ptr() const { return r; }
};

// Transform configuration of one kernel: where its twiddle factors come from
// and whether its LDS exchanges carry real and imaginary parts separately
// (4-byte entries: half the LDS per transform, twice the barriers).  The
// column pass and the row pass out of the blocked layout have their own.
#ifndef FFTMI_TWM_COLS
#define FFTMI_TWM_COLS FFTMI_TWM
#endif
#ifndef FFTMI_SPLIT_COLS
#define FFTMI_SPLIT_COLS FFTMI_SPLIT_X
#endif
#ifndef FFTMI_TWM_ROWS_OUT
#define FFTMI_TWM_ROWS_OUT FFTMI_TWM
#endif
#ifndef FFTMI_SPLIT_ROWS_OUT
#define FFTMI_SPLIT_ROWS_OUT FFTMI_SPLIT_X
#endif
FFTMI_HD constexpr int tw_lds_bytes_for(int L, int mode) {
  return mode == kTwLds ? lds_tw_bytes(L) : (mode == kTwMix ? mix_lds_bytes(L) : 0);
}
template <int L, int TWM_REQ, bool SPLIT_REQ, int MIX_MAX_LOG2 = FFTMI_MIX_MAX_LOG2>
struct XCfg {
  static constexpr int TWM = twm_for(L, TWM_REQ, MIX_MAX_LOG2);
  static constexpr bool SPLIT = SPLIT_REQ;
  static constexpr int TWB = tw_lds_bytes_for(L, TWM);
  static constexpr int region(int inter) { return lds_region_bytes(L, inter, SPLIT); }
};
template <int L>
using DefCfg = XCfg<L, FFTMI_TWM, kSplitExchange>;
template <int L>
using ColsCfg = XCfg<L, FFTMI_TWM_COLS, FFTMI_SPLIT_COLS != 0>;
template <int L>
using RowsOutCfg = XCfg<L, FFTMI_TWM_ROWS_OUT, FFTMI_SPLIT_ROWS_OUT != 0>;
// The mask-gradient column pass (see k_cols_grad).
#ifndef FFTMI_TWM_GRAD
#define FFTMI_TWM_GRAD FFTMI_TWM
#endif
#ifndef FFTMI_SPLIT_GRAD
#define FFTMI_SPLIT_GRAD FFTMI_SPLIT_X
#endif
template <int L>
using GradCfg = XCfg<L, FFTMI_TWM_GRAD, FFTMI_SPLIT_GRAD != 0>;
// 1D transforms in one pass (up to 2^14 points): mixed twiddles at every
// length, since these kernels run without a prefetch buffer (2^13 points:
// 4.1 TB/s against 3.1 with the global tables and a prefetch).
template <int L>
using Rows1DCfg = XCfg<L, FFTMI_TWM, kSplitExchange, kMaxLog2Row>;

// The workgroup's transform regions follow its LDS twiddle tables.
template <int L, class C = DefCfg<L>>
__device__ __forceinline__ char* regions() {
  return lds_base() + C::TWB;
}

// Make a per-thread pointer opaque to the optimiser so that addresses derived
// from it are recomputed where they are used rather than held in registers
// across a whole transform.
template <typename T>
__device__ __forceinline__ void launder(T*& p) {
  asm volatile("" : "+v"(p));
}

// Tile order: workgroup slots are dispatched round-robin over the 8 XCDs
// (each with its own L2).  Mapping slot n to tile (n % 8) * (T / 8) + n / 8
// gives every XCD a contiguous range of tiles, so neighbouring tiles that
// share cache lines are processed on one L2 at the same time.
__device__ __forceinline__ int64_t tile_of(int64_t n, int64_t ntiles) {
  if ((ntiles & 7) == 0 && ntiles >= 16) return (n & 7) * (ntiles >> 3) + (n >> 3);
  return n;
}

// Global addressing: every access is (uniform tile base) + (32-bit lane
// offset), which the hardware takes as an SGPR base plus one VGPR, instead of
// a 64-bit address per element.
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ base, unsigned off) {
  return __ldg(base + off);
}

// Streaming accesses: data read or written exactly once by the whole path
// (the input image, the final output) carry the non-temporal hint, so they
// displace less of the intermediate that the next pass reads from the caches
// (the memory-side cache holds a 4096^2 complex64 image between passes).
typedef float fftmi_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float ld_nt(const float* __restrict__ base, unsigned off) {
  return __builtin_nontemporal_load(base + off);
}
__device__ __forceinline__ float2 ld_nt(const float2* __restrict__ base, unsigned off) {
  const fftmi_f2v v = __builtin_nontemporal_load(reinterpret_cast<const fftmi_f2v*>(base + off));
  return make_float2(v.x, v.y);
}
typedef float fftmi_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4* __restrict__ base, unsigned off) {
  const fftmi_f4v v = __builtin_nontemporal_load(reinterpret_cast<const fftmi_f4v*>(base + off));
  return make_float4(v.x, v.y, v.z, v.w);
}
// A load with the non-temporal hint when NT: for data that a pass reads once
// and that is larger than the memory-side cache (a batch's intermediate, the
// saved spectrum), so it does not evict what is still to be read or written.
template <bool NT, typename T>
__device__ __forceinline__ T ldh(const T* __restrict__ base, unsigned off) {
  if constexpr (NT) {
    return ld_nt(base, off);
  } else {
    return __ldg(base + off);
  }
}
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  fftmi_f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<fftmi_f2v*>(p));
}
__device__ __forceinline__ void st_nt(float4* p, float4 v) {
  fftmi_f4v w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  __builtin_nontemporal_store(w, reinterpret_cast<fftmi_f4v*>(p));
}
// A store with the non-temporal hint when NT.
template <bool NT, typename T>
__device__ __forceinline__ void sth(T* p, T v) {
  if constexpr (NT) {
    st_nt(p, v);
  } else {
    *p = v;
  }
}

// Buffer-resource access to one image of the blocked workspace.  The image's
// base and byte size sit in a resource descriptor (SGPRs), the thread's fixed
// byte offset in one VGPR, and the per-tile and per-element byte offsets in
// an SGPR, so an access needs no vector-ALU address arithmetic.  The hardware
// checks the offsets against the size: an access outside the image reads
// zero and writes nothing instead of faulting.  Sizes must be below 4 GiB
// (an image of at most 2^14 x 2^14 complex64 values is 2 GiB plus padding).
typedef int fftmi_i2v __attribute__((ext_vector_type(2)));
struct BlkBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ BlkBuf(const float2* base, uint64_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), (short)0, (int)(uint32_t)bytes,
                                            0x00020000)) {}
  __device__ __forceinline__ float2 ld(unsigned voff, unsigned soff) const {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  // NT: the non-temporal cache policy (bit 1 of the instruction's cache
  // policy operand on this architecture)
  template <bool NT = false>
  __device__ __forceinline__ void st(float2 v, unsigned voff, unsigned soff) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(fftmi_i2v, v), r, voff, soff, NT ? 2 : 0);
  }
};

// A lane offset made opaque where it is used: the per-element offsets
// lane + q*stride are then computed next to the access instead of being
// hoisted out of the tile loop and held in registers for its whole length.
__device__ __forceinline__ unsigned fresh(unsigned v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Wait for a tile's loads before the tile loop.  The loop issues the next
// tile's loads ahead of the current transform; if the first tile's loads were
// still in flight at the loop head, the compiler's wait counting (merged over
// the loop entry and its back edge) would make every iteration wait for its
// own prefetch before transforming.  Passing the registers through an empty
// asm statement completes those loads once, before the loop.
template <int E>
__device__ __forceinline__ void settle(float2 (&a)[E]) {
#pragma unroll
  for (int q = 0; q < E; ++q) asm volatile("" : "+v"(a[q].x), "+v"(a[q].y));
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

// Mask evaluators, one per kind (a template parameter of the column kernel so
// that each kernel carries only its own state).  For the column v owned by a
// thread, H is applied to rows u = j + q*TPT, q = 0..E-1.  With E = 16 and
// j < TPT, u < N/2 exactly when q < 8, so the fftfreq value of row u is
// j/N + (q/16 - [q >= 8]), an exact float sum.
template <int L>
__device__ __forceinline__ float row_freq(float fj, int q) {
  constexpr int E = elems_per_thread(L), TPT = L / E;
  if constexpr (E == 16) {
    return fj + ((float)q * (1.0f / 16.0f) - (q >= 8 ? 1.0f : 0.0f));
  } else {  // short columns: the general fftfreq rule
    (void)TPT;
    const int u = (int)(fj * (float)L + 0.5f) + q * TPT;
    return (float)(u < ((L + 1) >> 1) ? u : u - L) * (1.0f / (float)L);
  }
}

template <int L, int MK>
struct MaskEval;

// value(j, q, mk) is H at row j + q*TPT of the evaluator's column.
template <int L>
struct MaskEval<L, FFT_MASK_NONE> {
  __device__ __forceinline__ MaskEval(const MaskArgs&, int, int, int) {}
  __device__ __forceinline__ void apply(float2 (&)[elems_per_thread(L)], int, const MaskArgs&) const {}
  __device__ __forceinline__ float value(int, int, const MaskArgs&) const { return 1.0f; }
};

template <int L>
struct MaskEval<L, FFT_MASK_BUTTERWORTH> {
  float fj, fv2;
  __device__ __forceinline__ MaskEval(const MaskArgs& mk, int j, int v, int M)
      : fj((float)j * (1.0f / (float)L)) {
    const float fv = freq_of(v, M, mk.inv_m);
    fv2 = fv * fv;
  }
  __device__ __forceinline__ void apply(float2 (&a)[elems_per_thread(L)], int, const MaskArgs& mk) const {
    // the order is uniform: one branch around straight-line code for the
    // usual order 4 (exponent 8), the general power otherwise
    if (mk.order == 4) {
#pragma unroll
      for (int q = 0; q < elems_per_thread(L); ++q) {
        const float fu = row_freq<L>(fj, q);
        const float qq = fmaf(fu, fu, fv2) * mk.inv_fc2;
        const float q2 = qq * qq;
        a[q] = cscale(a[q], __builtin_amdgcn_rcpf(fmaf(q2, q2, 1.0f)));
      }
    } else {
#pragma unroll
      for (int q = 0; q < elems_per_thread(L); ++q) {
        const float fu = row_freq<L>(fj, q);
        const float qq = fmaf(fu, fu, fv2) * mk.inv_fc2;
        a[q] = cscale(a[q], __builtin_amdgcn_rcpf(1.0f + powi_pos(qq, mk.order)));
      }
    }
  }
  __device__ __forceinline__ float value(int, int q, const MaskArgs& mk) const {
    const float fu = row_freq<L>(fj, q);
    const float qq = fmaf(fu, fu, fv2) * mk.inv_fc2;
    const float p = (mk.order == 4) ? (qq * qq) * (qq * qq) : powi_pos(qq, mk.order);
    return __builtin_amdgcn_rcpf(1.0f + p);
  }
};

template <int L>
struct MaskEval<L, FFT_MASK_GAUSSIAN> {
  float fj, fv2;
  __device__ __forceinline__ MaskEval(const MaskArgs& mk, int j, int v, int M)
      : fj((float)j * (1.0f / (float)L)) {
    const float fv = freq_of(v, M, mk.inv_m);
    fv2 = fv * fv;
  }
  // exp(-r^2 / (2 sigma^2)) = 2^(r^2 * gauss_coef * log2(e))
  __device__ __forceinline__ void apply(float2 (&a)[elems_per_thread(L)], int, const MaskArgs& mk) const {
    const float c = mk.gauss_coef * 1.44269504088896340736f;
#pragma unroll
    for (int q = 0; q < elems_per_thread(L); ++q) {
      const float fu = row_freq<L>(fj, q);
      a[q] = cscale(a[q], __builtin_amdgcn_exp2f(fmaf(fu, fu, fv2) * c));
    }
  }
  __device__ __forceinline__ float value(int, int q, const MaskArgs& mk) const {
    const float fu = row_freq<L>(fj, q);
    return __builtin_amdgcn_exp2f(fmaf(fu, fu, fv2) * (mk.gauss_coef * 1.44269504088896340736f));
  }
};

template <int L>
struct MaskEval<L, FFT_MASK_DISC> {
  double dv2;
  __device__ __forceinline__ MaskEval(const MaskArgs& mk, int, int v, int) {
    const double dv = (double)v - mk.c2;
    dv2 = dv * dv;
  }
  __device__ __forceinline__ void apply(float2 (&a)[elems_per_thread(L)], int j, const MaskArgs& mk) const {
    constexpr int TPT = L / elems_per_thread(L);
#pragma unroll
    for (int q = 0; q < elems_per_thread(L); ++q) {
      const double du = (double)(j + q * TPT) - mk.c1;
      if (fma(du, du, dv2) <= mk.disc_b2) a[q] = make_float2(0.f, 0.f);
    }
  }
  __device__ __forceinline__ float value(int j, int q, const MaskArgs& mk) const {
    constexpr int TPT = L / elems_per_thread(L);
    const double du = (double)(j + q * TPT) - mk.c1;
    return fma(du, du, dv2) <= mk.disc_b2 ? 0.0f : 1.0f;
  }
};

// Tensor masks: H[u][v] = data[u*M + v], read for the thread's column after
// the forward transform (base: column v of the tile, stride M per row); or,
// with tensor_cm, from the transposed copy data[v*L + u], whose column is
// contiguous (a wavefront's reads of one element index cover consecutive
// rows of one column instead of one float per row).
template <int L>
struct MaskEval<L, FFT_MASK_TENSOR_F32> {
  const float* col;
  unsigned lane, qs;
  __device__ __forceinline__ MaskEval(const MaskArgs& mk, int j, int v, int M)
      : col(mk.tensor_cm ? mk.data + (int64_t)v * L : mk.data + v),
        lane(mk.tensor_cm ? (unsigned)j : (unsigned)(j * M)),
        qs(mk.tensor_cm ? (unsigned)(L / elems_per_thread(L)) : (unsigned)((L / elems_per_thread(L)) * M)) {}
  __device__ __forceinline__ void apply(float2 (&a)[elems_per_thread(L)], int, const MaskArgs& mk) const {
    const unsigned l = fresh(lane);
#pragma unroll
    for (int q = 0; q < elems_per_thread(L); ++q) a[q] = cscale(a[q], __ldg(col + l + q * qs) + mk.tensor_bias);
  }
};

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

}  // namespace fftmi
