// Launch shapes of the FFT-convolution kernels, shared by the per-length
// kernel translation units and the host-side dispatch.
#pragma once

#include "fft.hpp"

namespace cisor {

// Transform lengths with compiled kernels (one translation unit per length).
#define CISOR_FFT_SIZES X(64) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Column-kernel variants the autotuner chooses from (FP32 compute only; the
// FP64 residual kernels always use variant 0):
//   bit 0: radix plan (0: Plan<P>, 1: PlanAlt<P>)
//   bit 1: tile (0: 16 points per thread for powers of two, 24 otherwise,
//          blocks of up to 512 threads; 1: 8 points per thread and 256-thread
//          blocks for powers of two, 48 points per thread otherwise)
constexpr int COL_VARIANTS = 4;

constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }

// Column-stage tiling: V points per thread, COLS columns per block, block of
// COLS * P/V threads; LDS holds COLS columns of P points (at most 64 KiB).
template <typename Rc, int P, int CV> struct ColCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr bool F32 = sizeof(Rc) == 4;
  static constexpr int PV = F32 ? (CV & 1) : 0;
  static constexpr bool ALT_TILE = F32 && (CV & 2) != 0;
  static constexpr int V = POW2 ? (F32 ? (ALT_TILE ? 8 : 16) : 16) : (ALT_TILE ? 48 : 24);
  static constexpr int NT = P / V;
  static constexpr int TARGET = F32 ? ((ALT_TILE && POW2) ? 256 : 512) : 256;
  static constexpr int BY_THREADS = TARGET / NT > 0 ? TARGET / NT : 1;
  static constexpr int BY_LDS = 65536 / (P * 2 * (int)sizeof(Rc));
  static constexpr int COLS_RAW = pow2_floor(BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS);
  static constexpr int COLS = COLS_RAW > P ? P : (COLS_RAW < 1 ? 1 : COLS_RAW);
  static constexpr int THREADS = COLS * NT;
  static constexpr int LS = COLS;   // LDS row stride (complex elements)
  using plan = typename PlanSel<P, PV>::type;
  static_assert(P % COLS == 0, "column tile must divide P");
  static_assert(THREADS <= 1024, "block too large");
};

// Rows per block of the row kernels: up to 256 threads, and at most 4096
// complex points of LDS (64 KiB in FP64) so that the FP64 residual kernels
// share the same blocking.
template <int P> struct RowCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int NT = POW2 ? P / 8 : Plan<P>::NT_ROW;
  static constexpr int BY_THREADS = 256 / NT > 0 ? 256 / NT : 1;
  static constexpr int BY_LDS = 4096 / P > 0 ? 4096 / P : 1;
  static constexpr int ROWS = BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS;
  static constexpr int THREADS = ROWS * NT;
};

}  // namespace cisor
