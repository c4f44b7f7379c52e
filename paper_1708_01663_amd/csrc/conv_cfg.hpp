// Launch shapes of the FFT-convolution kernels, shared by the per-length
// kernel translation units and the host-side dispatch.
#pragma once

#include "fft.hpp"

namespace cisor {

// Transform lengths with compiled kernels (one translation unit per length).
#define CISOR_FFT_SIZES X(64) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Column-kernel variants the autotuner chooses from (FP32 compute only; the
// FP64 residual kernels always use variant 0):
//   0..3: block-wide transforms (a column's threads spread over the block,
//         LDS exchanges behind block barriers); bit 0: radix plan (Plan<P> or
//         PlanAlt<P>); bit 1: tile (16 points per thread for powers of two,
//         24 otherwise, blocks of up to 512 threads; or 8 points per thread
//         and 256-thread blocks for powers of two, 48 otherwise)
//   4, 5: wave-private transforms (each column transformed inside one wave,
//         exchanges with wave-level ordering only; global loads and stores
//         coalesced through an LDS transpose); radix plan Plan<P> or PlanAlt<P>
//   6, 7: the tile of variant 0 with scalar-offset buffer access and per-pass
//         twiddle tables in LDS (k_colb); radix plan Plan<P> or PlanAlt<P>
//   8, 9: k_colb's transforms with 8 points per thread (power-of-two P;
//         otherwise variant 6): 8 columns per block, tiles sharing a 128-byte
//         line dispatched to one XCD (k_colbn), or 16 columns per block
//         (k_colbw); radix plan Plan<P>
constexpr int COL_VARIANTS = 10;

constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }

// Column-stage tiling: V points per thread, COLS columns per block, block of
// COLS * P/V threads; LDS holds COLS columns of P points (at most 64 KiB).
template <typename Rc, int P, int CV> struct ColCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr bool F32 = sizeof(Rc) == 4;
  static constexpr int PV = F32 ? (CV & 1) : 0;
  static constexpr bool ALT_TILE = F32 && (CV & 2) != 0;
  // FP64 (residual checks, complex128 contexts): 8 points per thread in blocks of
  // up to 512 threads for powers of two, so the block's registers allow 4 waves
  // per SIMD where 16 points held it at 2
  static constexpr int V = POW2 ? (F32 ? (ALT_TILE ? 8 : 16) : 8) : (ALT_TILE ? 48 : 24);
  static constexpr int NT = P / V;
  static constexpr int TARGET = F32 ? ((ALT_TILE && POW2) ? 256 : 512) : (POW2 ? 512 : 256);
  static constexpr int BY_THREADS = TARGET / NT > 0 ? TARGET / NT : 1;
  static constexpr int BY_LDS = 65536 / (P * 2 * (int)sizeof(Rc));
  static constexpr int COLS_RAW = pow2_floor(BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS);
  static constexpr int COLS = COLS_RAW > P ? P : (COLS_RAW < 1 ? 1 : COLS_RAW);
  static constexpr int THREADS = COLS * NT;
  static constexpr int LS = COLS;   // LDS row stride (complex elements)
  static constexpr int PAD = 0;     // LDS padding mode of the transforms (lds_index)
  static constexpr int LROWS = P;   // LDS rows of the tile
  using plan = typename PlanSel<P, PV>::type;
  static_assert(P % COLS == 0, "column tile must divide P");
  static_assert(THREADS <= 1024, "block too large");
};

// Wave-private column tiling: V points per thread, NT = P / V threads per
// column (at most one wave, so 64 / NT columns per wave), COLS columns per
// block so that a row segment of the tile is 128 bytes where LDS allows
// (tile COLS x (P + PAD) complex values, at most 72 KiB so that two blocks
// share a CU).
template <typename Rc, int P, int PV> struct ColWCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int V = POW2 ? (P / 64 > 8 ? P / 64 : 8) : 24;
  static constexpr int NT = P / V;
  static constexpr int CPW = 64 / NT;
  static constexpr int PAD = 4;
  static constexpr int LS = P + PAD;   // offset between the columns of the tile
  static constexpr int SEG = 128 / (2 * (int)sizeof(Rc));      // columns per 128-byte row segment
  static constexpr int BY_LDS = 73728 / (LS * 2 * (int)sizeof(Rc));
  static constexpr int COLS_RAW = SEG < BY_LDS ? SEG : BY_LDS;
  static constexpr int COLS = COLS_RAW < CPW ? CPW : pow2_floor(COLS_RAW) / CPW * CPW;
  static constexpr int THREADS = COLS / CPW * 64;
  using plan = typename PlanSel<P, PV>::type;
  static_assert(NT <= 64 && 64 % NT == 0, "a column's threads must fit in one wave");
  static_assert(P % COLS == 0 && COLS % CPW == 0, "column tile");
  static_assert(THREADS <= 1024, "block too large");
};

// Rows per block of the row kernels: up to 256 threads, and at most 4096
// complex points of LDS (64 KiB in FP64, padded rows of lds_span(P)) so that
// the FP64 residual kernels share the same blocking.
template <int P> struct RowCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int NT = POW2 ? P / 8 : Plan<P>::NT_ROW;
  static constexpr int SPAN = lds_span(P);
  static constexpr int BY_THREADS = 256 / NT > 0 ? 256 / NT : 1;
  static constexpr int BY_LDS = 4096 / SPAN > 0 ? 4096 / SPAN : 1;
  static constexpr int ROWS = BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS;
  static constexpr int THREADS = ROWS * NT;
};

}  // namespace cisor
