// Kernels of the FFT-convolution operator (included by the per-length
// translation units only; see conv.hip for the operator and its stages).
#pragma once

#include <cmath>
#include <type_traits>

#include "conv_cfg.hpp"
#include "internal.hpp"

namespace cisor {

template <typename C> __device__ __forceinline__ C czero() { return mk<C>(0, 0); }

// ---------------------------------------------------------------- stage 1
// LDS elements of a row kernel: the rows' transforms, and with PM (plane-major
// layout of the intermediates, 3D plane path) the transposition of the block's
// P x ROWS outputs or inputs, row stride ROWS + 1.
template <int P, bool PM> constexpr int row_lds() {
  return PM && P * (RowCfg<P>::ROWS + 1) > RowCfg<P>::ROWS * RowCfg<P>::SPAN ? P * (RowCfg<P>::ROWS + 1)
                                                                             : RowCfg<P>::ROWS * RowCfg<P>::SPAN;
}

// PM: X1 is written plane-major, X1[t][k][row] (3D: the n^2 rows of one kz
// together) instead of X1[t][row][k].  EXACT (2D, power-of-two P = 2n, rows a
// multiple of the block's): every row is valid and column j + r P/R0 < n
// exactly when r < R0/2, so the element checks are decided at compile time.
template <typename Rs, typename Rc, int P, int PRO, bool MULF, bool PM = false, bool EXACT = false>
__global__ void __launch_bounds__(256) k_row_fwd(ConvArgs<Rs, Rc> a) {
  using Cs = cplx_t<Rs>;
  using Cc = cplx_t<Rc>;
  using PL = Plan<P>;
  constexpr int NT = RowCfg<P>::NT, ROWS = RowCfg<P>::ROWS, V = P / NT;
  constexpr int R0 = FirstRadix<typename PL::fwd>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, typename PL::fwd>::LAST;
  const int t = blockIdx.y;
  if (a.st && !(a.st[t].flags & a.flag)) return;
  if (a.fmask && !a.fmask[t]) return;
  const Rs *fr = a.frow ? a.frow[t] : a.f;
  constexpr int SPAN = RowCfg<P>::SPAN;
  __shared__ Cc lds[row_lds<P, PM>()];
  const int lr = threadIdx.x / NT, tid = threadIdx.x % NT;
  TwSet<Cc, P, NT, -1, typename PL::fwd> twf;
  twf.load(tid, a.tw);
  const int row = blockIdx.x * ROWS + lr;
  const bool vr = EXACT || row < a.rows;
  const size_t rowoff = (size_t)t * a.N + (size_t)row * a.n;
  static_assert(!EXACT || R0 % 2 == 0, "EXACT needs an even first radix");
  // BiCGSTAB prologues: the residual of the previous iteration is
  // r = s - omega t unless a true-residual step stored it (r_fresh)
  Cc al = czero<Cc>(), be = czero<Cc>(), om = czero<Cc>();
  int fresh = 0, pend = 0;
  bool bz = false;   // beta = 0 (first iteration, restart): p = r, p and v not read
  if constexpr (PRO == PRO_PUPD || PRO == PRO_SUPD) {
    al = ccast<Cc>(a.st[t].alpha);
    om = ccast<Cc>(a.st[t].omega);
    fresh = a.st[t].r_fresh;
  }
  if constexpr (PRO == PRO_PUPD) {
    be = ccast<Cc>(a.st[t].beta);
    pend = a.st[t].x_pending;
    bz = a.st[t].beta.x == 0.0 && a.st[t].beta.y == 0.0;
  }
  Cc v[V];
#pragma unroll
  for (int b = 0; b < V / R0; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int col = j + r * (P / R0);
      Cc val = czero<Cc>();
      if (EXACT ? (r < R0 / 2) : (vr && col < a.n)) {
        const size_t e = rowoff + col;
        if constexpr (PRO == PRO_X) {
          val = ccast<Cc>(a.x[e]);
        } else if constexpr (PRO == PRO_PUPD) {
          // x += alpha p + omega s (last iteration); p = r + beta (p - omega v),
          // which is p = r when beta = 0: p and v are then not read, so a
          // solve's first iteration needs no initial p and v
          Cc pp = czero<Cc>();
          if (pend || !bz) pp = ccast<Cc>(a.p[e]);
          Cc rr;
          if (fresh) {
            rr = ccast<Cc>(a.r[e]);
          } else {
            const Cc ss = ccast<Cc>(a.s[e]);
            rr = csub(ss, cmul(om, ccast<Cc>(a.tt[e])));
            if (pend) a.xw[e] = ccast<Cs>(cadd(ccast<Cc>(a.xw[e]), cadd(cmul(al, pp), cmul(om, ss))));
          }
          val = bz ? rr : cadd(rr, cmul(be, csub(pp, cmul(om, ccast<Cc>(a.v[e])))));
          a.p[e] = ccast<Cs>(val);
        } else {
          // s = r - alpha v (alpha of this iteration, omega of the last)
          const Cc rr = fresh ? ccast<Cc>(a.r[e]) : csub(ccast<Cc>(a.s[e]), cmul(om, ccast<Cc>(a.tt[e])));
          val = csub(rr, cmul(al, ccast<Cc>(a.v[e])));
          a.s[e] = ccast<Cs>(val);
        }
        if constexpr (MULF) val = cscale(val, static_cast<Rc>(fr[(size_t)row * a.n + col]));
      }
      v[b * R0 + r] = val;
    }
  }
  // the row is zero from column n <= P/2 on: the first pass is pruned
  fft_regs<Cc, P, NT, -1, typename PL::fwd, decltype(twf), BlockSync, true, true, false>(v, tid, lds + lr * SPAN, 1,
                                                                                       twf);
  if constexpr (PM) {
    // every thread has passed the transform's last barrier, so the LDS is
    // free: the block's outputs go through it so that the rows of one k are
    // stored together
    constexpr int TS = ROWS + 1;
#pragma unroll
    for (int b = 0; b < V / RL; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < RL; ++r) lds[(j + r * (P / RL)) * TS + lr] = v[b * RL + r];
    }
    __syncthreads();
    const int row0 = blockIdx.x * ROWS;
    for (int idx = threadIdx.x; idx < P * ROWS; idx += RowCfg<P>::THREADS) {
      const int k = idx / ROWS, l2 = idx % ROWS;
      if (row0 + l2 < a.rows) a.X1[((size_t)t * P + k) * a.rows + row0 + l2] = lds[k * TS + l2];
    }
  } else if (vr) {
    Cc *out = a.X1 + ((size_t)t * a.rows + row) * P;
#pragma unroll
    for (int b = 0; b < V / RL; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < RL; ++r) out[j + r * (P / RL)] = v[b * RL + r];
    }
  }
}

// ---------------------------------------------------------------- column stages
// Transforms along the strided axis of [batch][rows][width] arrays, one
// column per COLS lane group.  MODE: COL_CONV = forward FFT of in_rows
// non-zero rows, x Ghat[k][col] (or its conjugate), inverse FFT, keep
// out_rows rows (2D stage 2; 3D x-axis stage with width P^2); COL_FWD =
// forward FFT only, all P outputs kept (3D y-axis); COL_INV = inverse FFT of
// P rows, out_rows kept (3D inverse y-axis).
enum : int { COL_CONV = 0, COL_FWD = 1, COL_INV = 2 };

template <typename Rs, typename Rc, int P, int MODE, bool CONJ, bool MASK, int CV>
__global__ void __launch_bounds__((ColCfg<Rc, P, CV>::THREADS)) k_col(ConvArgs<Rs, Rc> a) {
  using Cc = cplx_t<Rc>;
  using CF = ColCfg<Rc, P, CV>;
  using PL = typename CF::plan;
  constexpr int NT = CF::NT, COLS = CF::COLS, V = CF::V;
  constexpr int R0 = FirstRadix<typename PL::fwd>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, typename PL::fwd>::LAST;
  constexpr int R0I = FirstRadix<typename PL::inv>::value;
  constexpr int RLI = Stockham<Cc, P, NT, +1, 1, typename PL::inv>::LAST;
  static_assert(R0I == RL, "inverse must start with the forward's last radix");
  const int bt = blockIdx.y;
  if constexpr (MASK) {
    if (!(a.st[bt / a.ydiv].flags & a.flag)) return;
  }
  if (a.fmask && !a.fmask[bt / a.ydiv]) return;
  __shared__ Cc lds[P * CF::LS];
  const int lc = threadIdx.x % COLS, tid = threadIdx.x / COLS;
  // LDS copy of the twiddle table; the first LDS exchange's barrier (after
  // the first pass, which needs no twiddles) publishes it
  __shared__ Cc stw[P];
  for (int i = threadIdx.x; i < P; i += CF::THREADS) stw[i] = a.tw[i];
  const TwTable<Cc, P, NT, -1, typename PL::fwd> twf{stw, tid};
  const TwTable<Cc, P, NT, +1, typename PL::inv> twi{stw, tid};
  const int col = blockIdx.x * COLS + lc;
  const Cc *in = a.cin + (size_t)bt * a.in_rows * a.width + col;
  Cc v[V];
  constexpr int RIN = (MODE == COL_INV) ? R0I : R0;
#pragma unroll
  for (int b = 0; b < V / RIN; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < RIN; ++r) {
      const int row = j + r * (P / RIN);
      v[b * RIN + r] = row < a.in_rows ? in[(size_t)row * a.width] : czero<Cc>();
    }
  }
  // in_rows <= P/2 for the forward modes, out_rows <= P/2 for the inverse ones
  if constexpr (MODE != COL_INV)
    fft_regs<Cc, P, NT, -1, typename PL::fwd, decltype(twf), BlockSync, false, true, false>(v, tid, lds + lc, CF::LS,
                                                                                          twf);
  if constexpr (MODE == COL_CONV) {
#pragma unroll
    for (int b = 0; b < V / RL; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = j + r * (P / RL);
        Cc g = a.Ghat[(size_t)k * a.width + col];
        if constexpr (CONJ) g.y = -g.y;
        v[b * RL + r] = cmul(v[b * RL + r], g);
      }
    }
  }
  if constexpr (MODE != COL_FWD)
    fft_regs<Cc, P, NT, +1, typename PL::inv, decltype(twi), BlockSync, false, false, true>(v, tid, lds + lc, CF::LS,
                                                                                          twi);
  Cc *out = a.cout + (size_t)bt * a.out_rows * a.width + col;
  constexpr int ROUT = (MODE == COL_FWD) ? RL : RLI;
#pragma unroll
  for (int b = 0; b < V / ROUT; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < ROUT; ++r) {
      const int row = j + r * (P / ROUT);
      if (row < a.out_rows) out[(size_t)row * a.width] = v[b * ROUT + r];
    }
  }
}

// 2D column stage (COL_CONV, FP32 compute) with scalar-offset buffer access
// and per-pass twiddle tables.  The tile and the transforms are those of
// k_col's block-wide variants (CV 0 / 1 give the radix plan); what differs is
// the instruction count of the surrounding work:
//  * global accesses go through buffer descriptors whose base is the block's
//    first column; a thread's lane offset is computed once and every row
//    offset is a compile-time constant passed as the scalar offset, so an
//    access needs no vector address arithmetic;
//  * the twiddles of every pass are read from LDS tables laid out [k][r]
//    (TwPass), so no twiddle product is formed and one address serves a
//    butterfly's R - 1 reads;
//  * EXACT (n = P/2, every grid whose transform length is twice its side)
//    drops the row bounds checks: the loaded rows are then exactly the
//    non-zero ones and the stored rows exactly the kept ones.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
// Two dword loads, which the compiler pairs into one dwordx2 load (the 64-bit
// load builtin was seen to fetch only the first dword with this compiler).
__device__ __forceinline__ cf buf_load_cf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  cf c;
  c.x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  c.y = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4u, soff, 0));
  return c;
}
__device__ __forceinline__ void buf_store_cf(__amdgpu_buffer_rsrc_t r, cf v, unsigned voff, unsigned soff) {
  using U2 = unsigned int __attribute__((ext_vector_type(2)));
  U2 q;
  q[0] = __builtin_bit_cast(unsigned, v.x);
  q[1] = __builtin_bit_cast(unsigned, v.y);
  __builtin_amdgcn_raw_buffer_store_b64(q, r, voff, soff, 0);
}

template <typename CF, typename Rs, int P, bool CONJ, bool MASK, bool EXACT, int PV>
__device__ __forceinline__ void colb_body(const ConvArgs<Rs, float> &a, const int tile) {
  using Cc = cf;
  using PL = typename PlanSel<P, PV>::type;
  using FL = typename PL::fwd;
  using IL = typename PL::inv;
  constexpr int NT = CF::NT, COLS = CF::COLS, V = CF::V;
  constexpr int R0 = FirstRadix<FL>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, FL>::LAST;
  constexpr int RLI = Stockham<Cc, P, NT, +1, 1, IL>::LAST;
  static_assert(FirstRadix<IL>::value == RL, "inverse must start with the forward's last radix");
  constexpr bool SAME = std::is_same<FL, IL>::value;
  constexpr int TF = TwPassLayout<1, FL>::SIZE, TI = SAME ? 0 : TwPassLayout<1, IL>::SIZE;
  const int t = blockIdx.y;
  if constexpr (MASK) {
    if (!(a.st[t].flags & a.flag)) return;
  }
  __shared__ Cc lds[CF::LROWS * CF::LS];
  __shared__ Cc stab[TF + TI];
  // pass tables; the first exchange's barrier (after the first pass, which
  // has no twiddles) publishes them
  tw_pass_build<Cc, P, FL>(stab, a.tw, threadIdx.x, CF::THREADS);
  if constexpr (!SAME) tw_pass_build<Cc, P, IL>(stab + TF, a.tw, threadIdx.x, CF::THREADS);
  const int lc = threadIdx.x % COLS, tid = threadIdx.x / COLS;
  const TwPass<Cc, P, NT, -1, 1, FL> twf{stab, tid};
  const TwPass<Cc, P, NT, +1, 1, IL> twi{stab + (SAME ? 0 : TF), tid};
  const int col0 = tile * COLS;
  constexpr unsigned RB = P * 8u;   // bytes per row (width == P)
  const unsigned voff = (unsigned)tid * RB + (unsigned)lc * 8u;
  // the kernel spectrum's tile is requested first: it arrives during the forward transform
  const auto rg = buf_rsrc(a.Ghat + col0, (unsigned)(P * RB - col0 * 8u));
  Cc gv[V];
#pragma unroll
  for (int b = 0; b < V / RL; ++b) {
#pragma unroll
    for (int r = 0; r < RL; ++r) gv[b * RL + r] = buf_load_cf(rg, voff, (unsigned)(b * NT + r * (P / RL)) * RB);
  }
  const auto rin = buf_rsrc(a.cin + (size_t)t * a.in_rows * P + col0, (unsigned)(a.in_rows * RB - col0 * 8u));
  Cc v[V];
#pragma unroll
  for (int b = 0; b < V / R0; ++b) {
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int row = tid + b * NT + r * (P / R0);
      v[b * R0 + r] = czero<Cc>();
      // an even first radix is pruned: its inputs r >= R0/2 (rows >= P/2) are zero
      if (R0 % 2 == 0 && r >= R0 / 2) continue;
      if (EXACT || row < a.in_rows) v[b * R0 + r] = buf_load_cf(rin, voff, (unsigned)(b * NT + r * (P / R0)) * RB);
    }
  }
  fft_regs<Cc, P, NT, -1, FL, decltype(twf), BlockSync, CF::PAD, true, false>(v, tid, lds + lc, CF::LS, twf);
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = CONJ ? cmulc(gv[i], v[i]) : cmul(v[i], gv[i]);
  fft_regs<Cc, P, NT, +1, IL, decltype(twi), BlockSync, CF::PAD, false, true>(v, tid, lds + lc, CF::LS, twi);
  const auto rout = buf_rsrc(a.cout + (size_t)t * a.out_rows * P + col0, (unsigned)(a.out_rows * RB - col0 * 8u));
#pragma unroll
  for (int b = 0; b < V / RLI; ++b) {
#pragma unroll
    for (int r = 0; r < RLI; ++r) {
      const int row = tid + b * NT + r * (P / RLI);
      // an even last radix is pruned: only its outputs r < RLI/2 (rows < P/2) are formed
      if (RLI % 2 == 0 && r >= RLI / 2) continue;
      if (EXACT || row < a.out_rows) buf_store_cf(rout, v[b * RLI + r], voff, (unsigned)(b * NT + r * (P / RLI)) * RB);
    }
  }
}

template <typename Rs, int P, bool CONJ, bool MASK, bool EXACT, int PV>
__global__ void __launch_bounds__((ColCfg<float, P, 0>::THREADS)) k_colb(ConvArgs<Rs, float> a) {
  colb_body<ColCfg<float, P, 0>, Rs, P, CONJ, MASK, EXACT, PV>(a, blockIdx.x);
}

// The narrow tile of the same kernel: 8 points per thread and 8 columns per
// block (power-of-two P), so a block needs half the registers and half the
// LDS of k_colb's 16 x 16 tile and twice as many waves fit on a CU.  A row
// segment of 8 columns is half a 128-byte line; the tile order is remapped so
// that the two tiles sharing each line are dispatched together on the same
// XCD (workgroups go round-robin over the eight XCDs), where the second read
// of the line is served by that XCD's L2.
template <int P, int C = 8> struct ColNarrowCfg {
  static constexpr int V = 8;
  static constexpr int NT = P / V;
  static constexpr int COLS = C;
  // LDS stride between the points of a column (columns interleaved).  With
  // 8 columns per row the first exchanges' stores of a wave would fall on 16
  // banks; one padding row per 16 rows (PAD 2) spreads them over all banks
  // for 1/16 more LDS (at 256^2 x 60: 32.3 instead of 34.2 us per launch),
  // where padding every row would raise the block's LDS above a quarter of
  // the CU's.  The 16-column tile keeps the plain layout (measured 2.6 %
  // slower padded)
  static constexpr int LS = C;
  static constexpr int PAD = C == 8 ? 2 : 0;
  static constexpr int LROWS = PAD == 2 ? P + P / 16 : P;
  static constexpr int THREADS = COLS * NT;
  static_assert((P & (P - 1)) == 0 && THREADS <= 1024, "narrow column tile");
};
// Tile of block x of a row of G tiles: tiles 2m and 2m + 1 go to blocks eight
// apart in the same residue mod 8 (G a multiple of 16; otherwise identity).
__device__ __forceinline__ int paired_tile(int x, int G) {
  if (G % 16) return x;
  const int xcd = x % 8, slot = x / 8;
  return 16 * (slot / 2) + 2 * xcd + (slot % 2);
}
template <typename Rs, int P, bool CONJ, bool MASK, bool EXACT>
__global__ void __launch_bounds__((ColNarrowCfg<P>::THREADS)) k_colbn(ConvArgs<Rs, float> a) {
  colb_body<ColNarrowCfg<P>, Rs, P, CONJ, MASK, EXACT, 0>(a, paired_tile(blockIdx.x, gridDim.x));
}
// The same 8 points per thread with 16 columns per block (whole 128-byte row
// segments, twice the block and its LDS; where that exceeds 1024 threads the
// 8-column tile runs).
template <int P> using ColNarrow16 = ColNarrowCfg<P, (P / 8) * 16 <= 1024 ? 16 : 8>;
template <typename Rs, int P, bool CONJ, bool MASK, bool EXACT>
__global__ void __launch_bounds__((ColNarrow16<P>::THREADS)) k_colbw(ConvArgs<Rs, float> a) {
  colb_body<ColNarrow16<P>, Rs, P, CONJ, MASK, EXACT, 0>(a, ColNarrow16<P>::COLS == 8 ? paired_tile(blockIdx.x, gridDim.x)
                                                                                        : (int)blockIdx.x);
}

// 2D column stage with wave-private transforms (COL_CONV only).  Phase 1:
// the block reads its COLS columns of the n non-zero rows with column-fastest
// (coalesced) loads into an LDS tile stored column-major.  Phase 2: each
// column is transformed by the NT threads of one wave (forward FFT, kernel
// spectrum, inverse FFT) with its exchanges inside that column's LDS slice,
// ordered by wave-level fences only.  Phase 3: the kept rows go back through
// the tile with coalesced stores.  Two block barriers in all.  The kernel
// spectrum is read as Ghat[col][k]: the embedded kernel is radial and has the
// same embedding on both axes, so its spectrum is symmetric, and along k a
// wave's reads are contiguous.
template <typename Rs, typename Rc, int P, bool CONJ, bool MASK, int PV>
__global__ void __launch_bounds__((ColWCfg<Rc, P, PV>::THREADS)) k_colw(ConvArgs<Rs, Rc> a) {
  using Cc = cplx_t<Rc>;
  using CF = ColWCfg<Rc, P, PV>;
  using PL = typename CF::plan;
  constexpr int NT = CF::NT, V = CF::V, CPW = CF::CPW, COLS = CF::COLS, LS = CF::LS;
  constexpr int R0 = FirstRadix<typename PL::fwd>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, typename PL::fwd>::LAST;
  constexpr int RLI = Stockham<Cc, P, NT, +1, 1, typename PL::inv>::LAST;
  static_assert(FirstRadix<typename PL::inv>::value == RL, "inverse must start with the forward's last radix");
  const int bt = blockIdx.y;
  if constexpr (MASK) {
    if (!(a.st[bt].flags & a.flag)) return;
  }
  __shared__ Cc tile[COLS * LS];
  __shared__ Cc stw[P];
  for (int i = threadIdx.x; i < P; i += CF::THREADS) stw[i] = a.tw[i];
  const int col0 = blockIdx.x * COLS;
  // phase 1: coalesced loads of the n non-zero rows into the column-major tile
  {
    constexpr int RSTEP = CF::THREADS / COLS;
    const int lc = threadIdx.x % COLS, rr = threadIdx.x / COLS;
    const Cc *in = a.cin + (size_t)bt * a.in_rows * a.width + col0 + lc;
    for (int row = rr; row < a.in_rows; row += RSTEP) tile[lc * LS + row] = in[(size_t)row * a.width];
  }
  __syncthreads();
  // phase 2: one column per NT lanes of a wave
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = wave * CPW + lane / NT, tid = lane % NT;
  Cc *cb = tile + c * LS;
  const TwTable<Cc, P, NT, -1, typename PL::fwd> twf{stw, tid};
  const TwTable<Cc, P, NT, +1, typename PL::inv> twi{stw, tid};
  Cc v[V];
#pragma unroll
  for (int b = 0; b < V / R0; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int row = j + r * (P / R0);
      v[b * R0 + r] = row < a.in_rows ? cb[row] : czero<Cc>();
    }
  }
  WaveSync::sync();
  fft_regs<Cc, P, NT, -1, typename PL::fwd, decltype(twf), WaveSync, false, true, false>(v, tid, cb, 1, twf);
  const Cc *gk = a.Ghat + (size_t)(col0 + c) * P;
#pragma unroll
  for (int b = 0; b < V / RL; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      Cc g = gk[j + r * (P / RL)];
      if constexpr (CONJ) g.y = -g.y;
      v[b * RL + r] = cmul(v[b * RL + r], g);
    }
  }
  fft_regs<Cc, P, NT, +1, typename PL::inv, decltype(twi), WaveSync, false, false, true>(v, tid, cb, 1, twi);
  WaveSync::sync();
#pragma unroll
  for (int b = 0; b < V / RLI; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < RLI; ++r) {
      const int row = j + r * (P / RLI);
      if (row < a.out_rows) cb[row] = v[b * RLI + r];
    }
  }
  __syncthreads();
  // phase 3: coalesced stores of the kept rows
  {
    constexpr int RSTEP = CF::THREADS / COLS;
    const int lc = threadIdx.x % COLS, rr = threadIdx.x / COLS;
    Cc *out = a.cout + (size_t)bt * a.out_rows * a.width + col0 + lc;
    for (int row = rr; row < a.out_rows; row += RSTEP) out[(size_t)row * a.width] = tile[lc * LS + row];
  }
}

// ---------------------------------------------------------------- stage 3
// PM: X2 is read plane-major, X2[t][k][row].  EXACT: as for k_row_fwd (every
// row valid, column j + r P/RL < n exactly when r < RL/2).
template <typename Rs, typename Rc, int P, int EPI, bool MULF, bool PM = false, bool EXACT = false>
__global__ void __launch_bounds__(256) k_row_inv(ConvArgs<Rs, Rc> a) {
  using Cs = cplx_t<Rs>;
  using Cc = cplx_t<Rc>;
  using PL = Plan<P>;
  constexpr int NT = RowCfg<P>::NT, ROWS = RowCfg<P>::ROWS, V = P / NT;
  constexpr int R0 = FirstRadix<typename PL::inv>::value;
  constexpr int RL = Stockham<Cc, P, NT, +1, 1, typename PL::inv>::LAST;
  constexpr bool DOTS = (EPI == EPI_V || EPI == EPI_T || EPI == EPI_TR);
  constexpr int NA = (EPI == EPI_T) ? 8 : (EPI == EPI_TR) ? 4 : 2;   // partial sums this epilogue produces
  const int t = blockIdx.y;
  if (a.st && !(a.st[t].flags & a.flag)) return;
  if (a.fmask && !a.fmask[t]) return;
  const Rs *fr = a.frow ? a.frow[t] : a.f;
  constexpr int SPAN = RowCfg<P>::SPAN;
  __shared__ Cc lds[row_lds<P, PM>()];
  __shared__ double scratch[16 * NA];
  const int lr = threadIdx.x / NT, tid = threadIdx.x % NT;
  TwSet<Cc, P, NT, +1, typename PL::inv> twi;
  twi.load(tid, a.tw);
  const int row = blockIdx.x * ROWS + lr;
  const bool vr = EXACT || row < a.rows;
  static_assert(!EXACT || RL % 2 == 0, "EXACT needs an even last radix");
  const size_t rowoff = (size_t)t * a.N + (size_t)row * a.n;
  Cc v[V];
  if constexpr (PM) {
    // the rows of one k are read together and transposed through the LDS
    constexpr int TS = ROWS + 1;
    const int row0 = blockIdx.x * ROWS;
    for (int idx = threadIdx.x; idx < P * ROWS; idx += RowCfg<P>::THREADS) {
      const int k = idx / ROWS, l2 = idx % ROWS;
      lds[k * TS + l2] = row0 + l2 < a.rows ? a.X2[((size_t)t * P + k) * a.rows + row0 + l2] : czero<Cc>();
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < V / R0; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = lds[(j + r * (P / R0)) * TS + lr];
    }
    __syncthreads();   // the transform's first exchange reuses the LDS
  } else {
    const Cc *in = a.X2 + ((size_t)t * a.rows + (vr ? row : 0)) * P;
#pragma unroll
    for (int b = 0; b < V / R0; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = vr ? in[j + r * (P / R0)] : czero<Cc>();
    }
  }
  // only columns below n <= P/2 are kept: the last pass is pruned
  fft_regs<Cc, P, NT, +1, typename PL::inv, decltype(twi), BlockSync, true, false, true>(v, tid, lds + lr * SPAN, 1,
                                                                                       twi);
  const Rc scale = static_cast<Rc>(a.scale);
  int restart = 0;
  if constexpr (EPI == EPI_TR) restart = a.st ? a.st[t].restart : 1;
  double acc[NA] = {};
#pragma unroll
  for (int b = 0; b < V / RL; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int col = j + r * (P / RL);
      if (EXACT ? (r >= RL / 2) : !(vr && col < a.n)) continue;
      const size_t e = rowoff + col;
      Cc cv = cscale(v[b * RL + r], scale);
      if constexpr (MULF) cv = cscale(cv, static_cast<Rc>(fr[(size_t)row * a.n + col]));
      if constexpr (EPI == EPI_AX) {
        a.y[e] = ccast<Cs>(csub(ccast<Cc>(a.x[e]), cv));
      } else if constexpr (EPI == EPI_G || EPI == EPI_GF) {
        a.y[e] = ccast<Cs>(cv);
      } else if constexpr (EPI == EPI_V) {
        const Cs vv = ccast<Cs>(csub(ccast<Cc>(a.p[e]), cv));
        a.y[e] = vv;
        const cd h = ccast<cd>(a.rhat[e]);
        const cd w = ccast<cd>(vv);
        acc[0] += h.x * w.x + h.y * w.y;
        acc[1] += h.x * w.y - h.y * w.x;
      } else if constexpr (EPI == EPI_T) {
        // t = A s; <t,s>, <t,t>, <s,s>, <rhat,s>, <rhat,t> (the residual
        // r = s - omega t is never formed: its dot products follow from these)
        const Cs tt = ccast<Cs>(csub(ccast<Cc>(a.s[e]), cv));
        a.y[e] = tt;
        const cd tv = ccast<cd>(tt);
        const cd sv = ccast<cd>(a.s[e]);
        const cd h = ccast<cd>(a.rhat[e]);
        acc[0] += tv.x * sv.x + tv.y * sv.y;
        acc[1] += tv.x * sv.y - tv.y * sv.x;
        acc[2] += tv.x * tv.x + tv.y * tv.y;
        acc[3] += sv.x * sv.x + sv.y * sv.y;
        acc[4] += h.x * sv.x + h.y * sv.y;
        acc[5] += h.x * sv.y - h.y * sv.x;
        acc[6] += h.x * tv.x + h.y * tv.y;
        acc[7] += h.x * tv.y - h.y * tv.x;
      } else if constexpr (EPI == EPI_TR) {
        // r = b - A x = b - x + conv, evaluated in the compute precision
        const Cc bb = ccast<Cc>(a.b[e]);
        const Cc rr = cadd(csub(bb, ccast<Cc>(a.x[e])), cv);
        const Cs rs = ccast<Cs>(rr);
        a.y[e] = rs;
        const cd rd = ccast<cd>(rr);
        acc[0] += rd.x * rd.x + rd.y * rd.y;
        const cd r2 = ccast<cd>(rs);
        cd h;
        if (restart) {
          a.rhat[e] = rs;
          h = r2;
        } else {
          h = ccast<cd>(a.rhat[e]);
        }
        acc[1] += h.x * r2.x + h.y * r2.y;
        acc[2] += h.x * r2.y - h.y * r2.x;
        const cd bd = ccast<cd>(bb);
        acc[3] += bd.x * bd.x + bd.y * bd.y;
      } else {  // EPI_GRAD: Re{conj(u) (q + G^H v)}
        const Cc uu = ccast<Cc>(a.u[e]);
        const Cc s = cadd(ccast<Cc>(a.q[e]), cv);
        a.gpart[e] = static_cast<Rs>(uu.x * s.x + uu.y * s.y);
      }
    }
  }
  if constexpr (DOTS) {
    block_sum<NA>(acc, scratch);
    if (threadIdx.x == 0) {
      double *dst = a.part + ((size_t)t * gridDim.x + blockIdx.x) * NPART;
#pragma unroll
      for (int i = 0; i < NPART; ++i) dst[i] = i < NA ? acc[i] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- 3D planes
// The y-, x- and inverse y-passes of the 3D convolution fused per kz plane.
// With the plane-major row stages, field t's samples of one kz, X1[t][kz][x][y],
// are contiguous; one block takes one (field, kz) plane:
//  1. y-forward of the lines x (n -> P points, first pass pruned) into an LDS
//     plane B[x][ky] (one line's threads inside one wave, exchanges in its own
//     row of B);
//  2. for the lines ky, in batches of L: x-forward of B[.][ky] (n -> P), times
//     the kernel spectrum at (kx, ky, kz), x-inverse keeping the rows x < n
//     (last pass pruned), back into B[.][ky];
//  3. y-inverse of the lines x keeping y < n, into X2[t][kz][x][y].
// The intermediates never leave the CU: the three passes' n P^2 x 2 x 3 HBM
// streams per field become one read and one write of n^2 P.  The spectrum is
// read from its kz-major copy, so a batch's reads are contiguous in ky.
template <typename Rc, int P> struct PlaneCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int V = 8;                       // points per thread and line
  static constexpr int NT = P / V;                  // threads per line
  static constexpr int THREADS = (sizeof(Rc) == 4 && P == 128) ? 1024 : 256;
  static constexpr int LINES = THREADS / NT;        // lines per round (y) and per batch (x)
  static constexpr int NROW = P / 2;                // rows of B: n <= P/2
  static constexpr int SPAN = lds_span(P);
  static constexpr int BATCHES = P / LINES;        // batches of x-lines
  static constexpr size_t LDS_BYTES = ((size_t)NROW * SPAN + (size_t)P * LINES + P) * 2 * sizeof(Rc);
  static constexpr bool OK = POW2 && P >= 64 && P <= 128 && NT <= 64 && 64 % NT == 0 && LINES >= NROW &&
                             P % LINES == 0 && BATCHES <= 2 && LDS_BYTES <= 160 * 1024;
};

template <typename Rs, typename Rc, int P, bool CONJ, bool MASK>
__global__ void __launch_bounds__((PlaneCfg<Rc, P>::THREADS)) k_plane(ConvArgs<Rs, Rc> a) {
  using Cc = cplx_t<Rc>;
  using CF = PlaneCfg<Rc, P>;
  using PL = Plan<P>;
  using FL = typename PL::fwd;
  using IL = typename PL::inv;
  constexpr int NT = CF::NT, V = CF::V, SPAN = CF::SPAN, L = CF::LINES;
  constexpr int R0 = FirstRadix<FL>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, FL>::LAST;
  constexpr int R0I = FirstRadix<IL>::value;
  constexpr int RLI = Stockham<Cc, P, NT, +1, 1, IL>::LAST;
  static_assert(CF::OK, "plane kernel configuration");
  static_assert(R0I == RL, "inverse must start with the forward's last radix");
  static_assert(R0 % 2 == 0 && RLI % 2 == 0, "the first and last radix are pruned");
  const int kz = blockIdx.x, t = blockIdx.y;
  if constexpr (MASK) {
    if (!(a.st[t].flags & a.flag)) return;
  }
  if (a.fmask && !a.fmask[t]) return;
  __shared__ Cc B[CF::NROW * SPAN];
  __shared__ Cc E[P * L];
  __shared__ Cc stw[P];
  for (int i = threadIdx.x; i < P; i += CF::THREADS) stw[i] = a.tw[i];
  __syncthreads();
  const int n = a.n;
  const size_t plane = ((size_t)t * P + kz) * (size_t)n * n;
  const Cc *in = a.cin + plane;
  Cc *out = a.cout + plane;
  // the spectrum values of every batch of step 2, requested first so that
  // they arrive during step 1: thread (lc, tk) of batch q needs (kx, ky) with
  // ky = q L + lc and kx in the forward transform's output layout
  constexpr int NB = CF::BATCHES;
  Cc g[NB][V];
  {
    const int lc = threadIdx.x % L, tk = threadIdx.x / L;
    const Cc *G = a.Gpm + (size_t)kz * P * P;   // [kx][ky]
#pragma unroll
    for (int q = 0; q < NB; ++q) {
#pragma unroll
      for (int b = 0; b < V / RL; ++b) {
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          Cc gg = G[(size_t)(tk + b * NT + r * (P / RL)) * P + q * L + lc];
          if constexpr (CONJ) gg.y = -gg.y;
          g[q][b * RL + r] = gg;
        }
      }
    }
  }
  // 1. y-forward; line x = threadIdx.x / NT (rows x >= n transform zeros)
  {
    const int x = threadIdx.x / NT, tid = threadIdx.x % NT;
    const TwTable<Cc, P, NT, -1, FL> twf{stw, tid};
    Cc v[V];
#pragma unroll
    for (int b = 0; b < V / R0; ++b) {
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int y = tid + b * NT + r * (P / R0);
        v[b * R0 + r] = (x < n && r < R0 / 2 && y < n) ? in[(size_t)x * n + y] : czero<Cc>();
      }
    }
    if (x < CF::NROW) {
      fft_regs<Cc, P, NT, -1, FL, decltype(twf), WaveSync, true, true, false>(v, tid, B + x * SPAN, 1, twf);
#pragma unroll
      for (int b = 0; b < V / RL; ++b) {
#pragma unroll
        for (int r = 0; r < RL; ++r) B[x * SPAN + lds_index<true>(tid + b * NT + r * (P / RL))] = v[b * RL + r];
      }
    }
  }
  __syncthreads();
  // 2. x-forward, spectrum, x-inverse of the lines ky
  {
    const int lc = threadIdx.x % L, tk = threadIdx.x / L;
    const TwTable<Cc, P, NT, -1, FL> twf{stw, tk};
    const TwTable<Cc, P, NT, +1, IL> twi{stw, tk};
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int ky = q * L + lc;
      Cc v[V];
#pragma unroll
      for (int b = 0; b < V / R0; ++b) {
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int x = tk + b * NT + r * (P / R0);
          v[b * R0 + r] = (r < R0 / 2 && x < n) ? B[x * SPAN + lds_index<true>(ky)] : czero<Cc>();
        }
      }
      fft_regs<Cc, P, NT, -1, FL, decltype(twf), BlockSync, false, true, false>(v, tk, E + lc, L, twf);
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = cmul(v[i], g[q][i]);
      fft_regs<Cc, P, NT, +1, IL, decltype(twi), BlockSync, false, false, true>(v, tk, E + lc, L, twi);
#pragma unroll
      for (int b = 0; b < V / RLI; ++b) {
#pragma unroll
        for (int r = 0; r < RLI / 2; ++r) {
          const int x = tk + b * NT + r * (P / RLI);
          if (x < n) B[x * SPAN + lds_index<true>(ky)] = v[b * RLI + r];
        }
      }
    }
  }
  __syncthreads();
  // 3. y-inverse, keeping y < n
  {
    const int x = threadIdx.x / NT, tid = threadIdx.x % NT;
    const TwTable<Cc, P, NT, +1, IL> twi{stw, tid};
    if (x < CF::NROW) {
      Cc v[V];
#pragma unroll
      for (int b = 0; b < V / R0I; ++b) {
#pragma unroll
        for (int r = 0; r < R0I; ++r) v[b * R0I + r] = B[x * SPAN + lds_index<true>(tid + b * NT + r * (P / R0I))];
      }
      fft_regs<Cc, P, NT, +1, IL, decltype(twi), WaveSync, true, false, true>(v, tid, B + x * SPAN, 1, twi);
      if (x < n) {
#pragma unroll
        for (int b = 0; b < V / RLI; ++b) {
#pragma unroll
          for (int r = 0; r < RLI / 2; ++r) {
            const int y = tid + b * NT + r * (P / RLI);
            if (y < n) out[(size_t)x * n + y] = v[b * RLI + r];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- launch
// The kz-major spectrum in the compute precision Rc (null where the context
// has none: 2D).
// Row kernels with compile-time element checks: power-of-two P (even first
// and last radices), n = P/2 and whole row blocks (rows n in 2D, n^2 in 3D).
template <int P> constexpr bool row_exact_ok() { return (P & (P - 1)) == 0; }
template <int P> static bool row_exact(const Ctx &c, int rows) {
  return row_exact_ok<P>() && 2 * c.n == P && rows % RowCfg<P>::ROWS == 0;
}
template <typename Rc> static const cplx_t<Rc> *plane_table(const Ctx &c) {
  if constexpr (sizeof(Rc) == 8) return c.precision == 1 ? (const cd *)c.Gpm : c.Gpm_d;
  else return c.precision == 0 ? (const cf *)c.Gpm : nullptr;
}

// 2D column stage (X1 -> X2) with the context's column-kernel variant.
template <typename Rs, typename Rc, int P, bool MASKED, int CV>
static void launch_col2d_v(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  using CF = ColCfg<Rc, P, CV>;
  a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
  const dim3 g(P / CF::COLS, c.T);
  if (adjoint)
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, true, MASKED, CV>), g, dim3(CF::THREADS), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, false, MASKED, CV>), g, dim3(CF::THREADS), 0, c.stream, a);
}
template <typename Rs, typename Rc, int P, bool MASKED, int PV>
static void launch_col2d_w(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  using CF = ColWCfg<Rc, P, PV>;
  a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
  const dim3 g(P / CF::COLS, c.T);
  if (adjoint)
    hipLaunchKernelGGL((k_colw<Rs, Rc, P, true, MASKED, PV>), g, dim3(CF::THREADS), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_colw<Rs, Rc, P, false, MASKED, PV>), g, dim3(CF::THREADS), 0, c.stream, a);
}
template <typename Rs, typename Rc, int P, bool MASKED, bool EXACT, int PV>
static void launch_col2d_b(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  using CF = ColCfg<Rc, P, 0>;
  a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
  const dim3 g(P / CF::COLS, c.T);
  if (adjoint)
    hipLaunchKernelGGL((k_colb<Rs, P, true, MASKED, EXACT, PV>), g, dim3(CF::THREADS), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_colb<Rs, P, false, MASKED, EXACT, PV>), g, dim3(CF::THREADS), 0, c.stream, a);
}
// k_colb, with the row checks dropped when n = P/2
template <typename Rs, typename Rc, int P, bool MASKED, int PV>
static void launch_col2d_bx(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  if (2 * c.n == P)
    launch_col2d_b<Rs, Rc, P, MASKED, true, PV>(c, a, adjoint);
  else
    launch_col2d_b<Rs, Rc, P, MASKED, false, PV>(c, a, adjoint);
}
// k_colbn / k_colbw (the narrow tiles, 8 or 16 columns; power-of-two P only,
// else variant 6)
template <typename Rs, typename Rc, int P, bool MASKED, bool EXACT, bool WIDE>
static void launch_col2d_n(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  using CF = std::conditional_t<WIDE, ColNarrow16<P>, ColNarrowCfg<P>>;
  a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
  const dim3 g(P / CF::COLS, c.T);
  if constexpr (WIDE) {
    if (adjoint)
      hipLaunchKernelGGL((k_colbw<Rs, P, true, MASKED, EXACT>), g, dim3(CF::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_colbw<Rs, P, false, MASKED, EXACT>), g, dim3(CF::THREADS), 0, c.stream, a);
  } else {
    if (adjoint)
      hipLaunchKernelGGL((k_colbn<Rs, P, true, MASKED, EXACT>), g, dim3(CF::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_colbn<Rs, P, false, MASKED, EXACT>), g, dim3(CF::THREADS), 0, c.stream, a);
  }
}
template <typename Rs, typename Rc, int P, bool MASKED, bool WIDE>
static void launch_col2d_nx(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  if constexpr ((P & (P - 1)) == 0) {
    if (2 * c.n == P)
      launch_col2d_n<Rs, Rc, P, MASKED, true, WIDE>(c, a, adjoint);
    else
      launch_col2d_n<Rs, Rc, P, MASKED, false, WIDE>(c, a, adjoint);
  } else {
    launch_col2d_bx<Rs, Rc, P, MASKED, 0>(c, a, adjoint);
  }
}
template <typename Rs, typename Rc, int P, bool MASKED>
static void launch_col2d(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  if constexpr (sizeof(Rc) == 4) {
    switch (c.col_variant) {
      case 1: return launch_col2d_v<Rs, Rc, P, MASKED, 1>(c, a, adjoint);
      case 2: return launch_col2d_v<Rs, Rc, P, MASKED, 2>(c, a, adjoint);
      case 3: return launch_col2d_v<Rs, Rc, P, MASKED, 3>(c, a, adjoint);
      case 4: return launch_col2d_w<Rs, Rc, P, MASKED, 0>(c, a, adjoint);
      case 5: return launch_col2d_w<Rs, Rc, P, MASKED, 1>(c, a, adjoint);
      case 6: return launch_col2d_bx<Rs, Rc, P, MASKED, 0>(c, a, adjoint);
      case 7: return launch_col2d_bx<Rs, Rc, P, MASKED, 1>(c, a, adjoint);
      case 8: return launch_col2d_nx<Rs, Rc, P, MASKED, false>(c, a, adjoint);
      case 9: return launch_col2d_nx<Rs, Rc, P, MASKED, true>(c, a, adjoint);
      default: break;
    }
  }
  launch_col2d_v<Rs, Rc, P, MASKED, 0>(c, a, adjoint);
}

template <typename Rs, typename Rc, int P, int PRO, int EPI>
int launch_conv_p(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  const bool pure_g = (EPI == EPI_G || EPI == EPI_GRAD || EPI == EPI_GF);
  const bool mulf_in = (!adjoint && !pure_g) || EPI == EPI_GF;
  const bool mulf_out = adjoint && !pure_g;
  // solver stages skip transmitters that are paused or done
  constexpr bool MASKED = (EPI == EPI_V || EPI == EPI_T || EPI == EPI_TR);
  a.rows = c.rows;
  a.scale = 1.0 / std::pow((double)P, c.dim);
  a.frow = (const Rs *const *)c.frow;
  using CF = ColCfg<Rc, P, 0>;
  constexpr int CT = CF::THREADS, CC = CF::COLS;
  dim3 grow((a.rows + RowCfg<P>::ROWS - 1) / RowCfg<P>::ROWS, c.T);
  // grids with n = P/2 and whole row blocks take the row kernels whose
  // element checks are decided at compile time (EXACT)
  const bool exact = row_exact<P>(c, a.rows);
  auto row_fwd = [&](auto pm, auto ex) {
    constexpr bool PMV = decltype(pm)::value, EX = decltype(ex)::value;
    if (mulf_in)
      hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO, true, PMV, EX>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO, false, PMV, EX>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  };
  auto row_inv = [&](auto pm, auto ex) {
    constexpr bool PMV = decltype(pm)::value, EX = decltype(ex)::value;
    if (mulf_out)
      hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI, true, PMV, EX>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI, false, PMV, EX>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  };
  auto rows = [&](auto pm, bool inverse) {
    if constexpr (row_exact_ok<P>()) {
      if (exact) {
        if (inverse) row_inv(pm, std::true_type{});
        else row_fwd(pm, std::true_type{});
        return;
      }
    }
    if (inverse) row_inv(pm, std::false_type{});
    else row_fwd(pm, std::false_type{});
  };
  if constexpr (PlaneCfg<Rc, P>::OK) {
    // 3D: plane-major row stages around the fused per-plane kernel
    a.Gpm = plane_table<Rc>(c);
    if (c.dim == 3 && a.Gpm) {
      rows(std::true_type{}, false);
      a.cin = a.X1, a.cout = a.X2;
      const dim3 gp(P, c.T), bp(PlaneCfg<Rc, P>::THREADS);
      if (adjoint)
        hipLaunchKernelGGL((k_plane<Rs, Rc, P, true, MASKED>), gp, bp, 0, c.stream, a);
      else
        hipLaunchKernelGGL((k_plane<Rs, Rc, P, false, MASKED>), gp, bp, 0, c.stream, a);
      rows(std::true_type{}, true);
      return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
    }
  }
  rows(std::false_type{}, false);
  if (c.dim == 2) {
    // X1 [T][n][P] -> X2 [T][n][P]: column FFT, kernel spectrum, inverse
    launch_col2d<Rs, Rc, P, MASKED>(c, a, adjoint);
  } else {
    // X1 [T][n x][n y][P kz] -> X2 [T][n x][P ky][P kz]: forward along y
    a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = P, a.ydiv = c.n;
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_FWD, false, MASKED, 0>), dim3(P / CC, c.T * c.n), dim3(CT), 0, c.stream,
                       a);
    // X2 [T][n x][P*P] -> X1 [T][n x][P*P]: forward along x, kernel spectrum, inverse
    a.cin = a.X2, a.cout = a.X1, a.width = P * P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
    if (adjoint)
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, true, MASKED, 0>), dim3(P * P / CC, c.T), dim3(CT), 0,
                         c.stream, a);
    else
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, false, MASKED, 0>), dim3(P * P / CC, c.T), dim3(CT), 0,
                         c.stream, a);
    // X1 [T][n x][P ky][P kz] -> X2 [T][n x][n y][P kz]: inverse along y
    a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = P, a.out_rows = c.n, a.ydiv = c.n;
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_INV, false, MASKED, 0>), dim3(P / CC, c.T * c.n), dim3(CT), 0, c.stream,
                       a);
  }
  rows(std::false_type{}, true);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

// One stage of the unmasked 2D operator y = A x (or A^H x): stage 1 writes
// X1, stage 2 maps X1 to X2 (with the context's column variant), stage 3
// reads X2 and writes y.
template <typename Rs, typename Rc, int P>
int launch_stage_p(Ctx &c, ConvArgs<Rs, Rc> &a, int stage, bool adjoint) {
  if (c.dim != 2) return CISOR_E_UNSUPPORTED;
  a.rows = c.rows;
  a.scale = 1.0 / ((double)P * P);
  a.frow = (const Rs *const *)c.frow;
  dim3 grow((c.n + RowCfg<P>::ROWS - 1) / RowCfg<P>::ROWS, c.T);
  const bool exact = row_exact<P>(c, a.rows);
  auto rows = [&](auto ex) {
    constexpr bool EX = decltype(ex)::value;
    if (stage == 1) {
      if (!adjoint)
        hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO_X, true, false, EX>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream,
                           a);
      else
        hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO_X, false, false, EX>), grow, dim3(RowCfg<P>::THREADS), 0,
                           c.stream, a);
    } else {
      if (adjoint)
        hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI_AX, true, false, EX>), grow, dim3(RowCfg<P>::THREADS), 0,
                           c.stream, a);
      else
        hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI_AX, false, false, EX>), grow, dim3(RowCfg<P>::THREADS), 0,
                           c.stream, a);
    }
  };
  if (stage == 2) {
    launch_col2d<Rs, Rc, P, false>(c, a, adjoint);
  } else if constexpr (row_exact_ok<P>()) {
    if (exact) rows(std::true_type{});
    else rows(std::false_type{});
  } else {
    rows(std::false_type{});
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

}  // namespace cisor
