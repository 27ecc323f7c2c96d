// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/lbmfvm.h"

// set the thread-local error message and return st
lf_status lf_fail(lf_status st, const char* fmt, ...);

#define LF_HIP_TRY(expr)                                                   \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return lf_fail(LF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

static inline size_t lf_align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Rows per wave of the Mode H step for a grid (or live set) that yields
// `row_waves` waves at one row per wave: single rows (the step kernel's
// 5-wave form) up to three waves per wave slot of the chip (256 CUs x 4
// SIMDs x 8 slots), else bands of 4 rows (measured on MI355X: 1024^2 runs
// best in single rows, 1536^2 and up in bands of 4).
static inline int lf_rows_per_wave(long long row_waves) {
  return row_waves <= 24576 ? 1 : 4;
}

// Elements between successive planes of a cavity's populations (row pitch
// = nx rounded up to 64): the plane plus 2112 elements (33 x 256 B in FP32).
// The usual 2^k-sized cavities otherwise have planes a power of two apart,
// which puts a node's nine populations on the same DRAM address bits; the
// pad moves them off it (a stride can still land on a power of two for a
// rare shape, e.g. 64 x 223 in FP32).  Measured 1.6-2.1 % faster on the
// 256-cavity sweep and 0.5-1.8 % on 2048^2 and 4096^2 (the pad's size
// mattered little: 320 to 4160 elements).
static inline long long lf_plane_elems(long long pitch, int ny) {
  return pitch * ny + 2112;
}

// A buffer set of nine planes must be addressable by the step kernels: 32-bit
// element indices and buffer descriptors with a 32-bit byte range.
static inline bool lf_planes_fit(long long plane, size_t es) {
  return 9 * plane < (1LL << 31) && 9 * plane * (long long)es < (1LL << 32);
}

// lattice parameters from Ra, Pr, U_char (0 = default rule), T_ref (NaN = 0)
lf_status lf_derive_params(const lf_physics* ph, int ny, int split, double out[8]);

#include "lf_stop.h"

// band heights chosen per cavity-height class by the autotuner (0 = none)
struct lf_tuning {
  int valid;
  int ny_class[16];
  int band[16];
  int nclass;
};

struct lf_ctx {
  int device;
  hipStream_t stream;
  int band;  // rows per wave for single cavities; 0: automatic
  lf_tuning tune;
};
