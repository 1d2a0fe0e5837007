// fft_schedule.hpp -- compile-time radix schedule shared by host and device code.
//
// A length-L transform (L = 2^m) is split over L/E threads with E = min(16, L)
// complex elements each; thread j holds the elements at positions j + q*(L/E),
// q = 0..E-1, on entry and on exit (natural order both ends: self-sorting
// Stockham).  The stages are as many radix-16 passes as fit, then one radix-2,
// -4 or -8 pass for the remaining factor.  This replaces the paper's level-by-
// level radix-2 tree (Section 2): four tree levels are merged into one radix-16
// pass held in registers, so data crosses LDS once per four levels.
//
// Stage s has stride NS(s) = product of the radices before it.  For s >= 1 the
// twiddle factors exp(-2 pi i r k / (NS R)) (k < NS, r < R) live in a table
// T_s[k*R + r]; all stage tables of one L are concatenated into one "blob".
#pragma once
#include <stdint.h>

namespace fftmi {

#if defined(__HIPCC__)
#define FFTMI_HD __host__ __device__
#else
#define FFTMI_HD
#endif

FFTMI_HD constexpr int ilog2c(int64_t L) {
  int m = 0;
  while ((int64_t(1) << m) < L) ++m;
  return m;
}
FFTMI_HD constexpr int elems_per_thread(int L) { return L >= 16 ? 16 : L; }
FFTMI_HD constexpr int threads_per_transform(int L) { return L / elems_per_thread(L); }
FFTMI_HD constexpr int num_stages(int L) {
  return L <= 1 ? 0 : (L < 16 ? 1 : ilog2c(L) / 4 + ((ilog2c(L) % 4) ? 1 : 0));
}
FFTMI_HD constexpr int stage_radix(int L, int s) {
  return L < 16 ? L : (s < ilog2c(L) / 4 ? 16 : (1 << (ilog2c(L) % 4)));
}
FFTMI_HD constexpr int stage_ns(int L, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= stage_radix(L, i);
  return ns;
}
// Offset (in complex entries) of stage s's table inside the blob of length L.
FFTMI_HD constexpr int tw_stage_offset(int L, int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += stage_ns(L, i) * stage_radix(L, i);
  return off;
}
FFTMI_HD constexpr int tw_blob_size(int L) { return tw_stage_offset(L, num_stages(L)); }

// The same factors in the layout kept in LDS by the persistent kernels:
// stage s >= 1 occupies (R-1)*NS entries, entry (r-1)*NS + k = e^{-2 pi i r k/(NS R)},
// so that lanes with consecutive k read consecutive entries.
FFTMI_HD constexpr int lds_tw_offset(int L, int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += stage_ns(L, i) * (stage_radix(L, i) - 1);
  return off;
}
FFTMI_HD constexpr int lds_tw_entries(int L) { return lds_tw_offset(L, num_stages(L)); }
// LDS twiddles are used up to this length (2^12: 32640 bytes).
constexpr int kLdsTwMaxLog2 = 12;
FFTMI_HD constexpr int lds_tw_bytes(int L) {
  return L <= (1 << kLdsTwMaxLog2) ? ((lds_tw_entries(L) * 8 + 255) / 256) * 256 : 0;
}

// LDS footprint of one transform: one padding slot per 2^FFTMI_PAD_SHIFT
// entries so that the strided writes of a radix-16 pass and the natural-order
// reads fall into distinct banks.  For shifts 4 and 5 the split
// pad(base + off) = pad(base) + pad(off) used for immediate offsets is exact
// for every stage of every length up to 2^14 (checked exhaustively).
#ifndef FFTMI_PAD_SHIFT
#define FFTMI_PAD_SHIFT 4
#endif
static_assert(FFTMI_PAD_SHIFT == 4 || FFTMI_PAD_SHIFT == 5, "padding shift");
FFTMI_HD constexpr int lds_pad(int i) { return i + (i >> FFTMI_PAD_SHIFT); }
FFTMI_HD constexpr int lds_size(int L) { return L >= 16 ? L + L / 16 : L; }

#ifndef FFTMI_SPLIT_X
#define FFTMI_SPLIT_X 0
#endif
// Exchange real and imaginary parts through LDS one after the other.
constexpr bool kSplitExchange = FFTMI_SPLIT_X != 0;
constexpr int kLdsEntryBytes = kSplitExchange ? 4 : 8;

// Bytes of one transform's LDS region when `inter` transforms are interleaved
// lane by lane inside a wavefront: offsetting consecutive regions by a share
// of the 64 four-byte banks puts their lanes in disjoint bank groups.
#ifndef FFTMI_BANK_SPAN
#define FFTMI_BANK_SPAN 128
#endif
// `split`: the kernel exchanges real and imaginary parts separately (4-byte
// entries, half the LDS per transform).
FFTMI_HD constexpr int lds_region_bytes(int L, int inter, bool split = kSplitExchange) {
  return (split ? 4 : 8) * (lds_size(L) + (inter > 1 && inter <= 32 ? (FFTMI_BANK_SPAN / (split ? 4 : 8)) / inter : 0));
}

constexpr int kMaxLog2Row = 14;      // longest single-pass transform, 2^14
constexpr int kLdsBytes = 160 * 1024; // gfx950 LDS per workgroup

}  // namespace fftmi
