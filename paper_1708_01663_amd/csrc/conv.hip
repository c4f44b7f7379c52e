// FFT-convolution operator of the discretised Lippmann-Schwinger equation.
//
// A x = x - G (f x) and A^H x = x - f (G^H x) (eq. A_def; G applied by FFT as
// the paper does), with G the convolution by the Green's kernel embedded on the
// (2n)^2 circulant grid.  Since that kernel is even per axis, G^H x is the
// convolution with conj(Ghat).  The 2D transform of the zero-padded n x n
// input is split into three launches that each stream HBM once:
//
//   stage 1  (row kernel)    prologue (contrast, BiCGSTAB vector update)
//                            + forward row FFTs of the n non-zero rows, half
//                            of every row being zero padding      -> X1 [n][P]
//   stage 2  (column kernel) forward column FFTs of the n non-zero rows,
//                            pointwise Ghat (or conj(Ghat)), inverse column
//                            FFTs, keep the first n rows          -> X2 [n][P]
//   stage 3  (row kernel)    inverse row FFTs, keep n columns, scale 1/P^2,
//                            epilogue (x - conv, BiCGSTAB fused dot products,
//                            FP64 residual, gradient term)
//
// Every launch covers all transmitters; blocks of transmitters whose solve
// is paused or finished exit at once.
#include <cmath>

#include "fft.hpp"
#include "internal.hpp"

namespace cisor {

// Column-stage tiling: V points per thread, COLS columns per block, block of
// COLS * P/V threads; LDS holds COLS columns of P points, rows padded by PAD.
#ifndef CISOR_COL_V32
#define CISOR_COL_V32 16
#endif
#ifndef CISOR_COL_THREADS32
#define CISOR_COL_THREADS32 512
#endif
#ifndef CISOR_COL_PAD
#define CISOR_COL_PAD 0
#endif
constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }
template <typename Rc, int P> struct ColCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int V = POW2 ? (sizeof(Rc) == 4 ? CISOR_COL_V32 : 16) : 24;
  static constexpr int NT = P / V;
  static constexpr int BY_THREADS = (sizeof(Rc) == 4 ? CISOR_COL_THREADS32 : 256) / NT;
  static constexpr int BY_LDS = 65536 / (P * 2 * (int)sizeof(Rc));   // at most 64 KiB of LDS
  static constexpr int COLS_RAW = pow2_floor(BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS);
  static constexpr int COLS = COLS_RAW > P ? P : (COLS_RAW < 1 ? 1 : COLS_RAW);
  static constexpr int THREADS = COLS * NT;
  static constexpr int LS = COLS + CISOR_COL_PAD;   // LDS row stride (complex elements)
  static_assert(P % COLS == 0, "column tile must divide P");
};

// Rows per block: up to 256 threads, and at most 4096 complex points of LDS
// (64 KiB in FP64) so that the FP64 residual kernels share the same blocking.
#ifndef CISOR_ROW_V
#define CISOR_ROW_V 8
#endif
template <int P> struct RowCfg {
  static constexpr bool POW2 = (P & (P - 1)) == 0;
  static constexpr int NT = POW2 ? P / CISOR_ROW_V : Plan<P>::NT_ROW;
  static constexpr int BY_THREADS = 256 / NT > 0 ? 256 / NT : 1;
  static constexpr int BY_LDS = 4096 / P > 0 ? 4096 / P : 1;
  static constexpr int ROWS = BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS;
  static constexpr int THREADS = ROWS * NT;
};

template <typename C> __device__ __forceinline__ C czero() { return mk<C>(0, 0); }

// ---------------------------------------------------------------- stage 1
template <typename Rs, typename Rc, int P, int PRO, bool MULF>
__global__ void __launch_bounds__(256) k_row_fwd(ConvArgs<Rs, Rc> a) {
  using Cs = cplx_t<Rs>;
  using Cc = cplx_t<Rc>;
  using PL = Plan<P>;
  constexpr int NT = RowCfg<P>::NT, ROWS = RowCfg<P>::ROWS, V = P / NT;
  constexpr int R0 = FirstRadix<typename PL::fwd>::value;
  constexpr int RL = Stockham<Cc, P, NT, -1, 1, typename PL::fwd>::LAST;
  const int t = blockIdx.y;
  if (a.st && !(a.st[t].flags & a.flag)) return;
  __shared__ Cc lds[ROWS * P];
  const int lr = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int row = blockIdx.x * ROWS + lr;
  const bool vr = row < a.rows;
  const size_t rowoff = (size_t)t * a.N + (size_t)row * a.n;
  Cc al = czero<Cc>(), be = czero<Cc>(), om = czero<Cc>();
  if constexpr (PRO == PRO_PUPD) {
    be = ccast<Cc>(a.st[t].beta);
    om = ccast<Cc>(a.st[t].omega);
  }
  if constexpr (PRO == PRO_SUPD) al = ccast<Cc>(a.st[t].alpha);
  Cc v[V];
#pragma unroll
  for (int b = 0; b < V / R0; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int col = j + r * (P / R0);
      Cc val = czero<Cc>();
      if (vr && col < a.n) {
        const size_t e = rowoff + col;
        if constexpr (PRO == PRO_X) {
          val = ccast<Cc>(a.x[e]);
        } else if constexpr (PRO == PRO_PUPD) {
          const Cc pp = ccast<Cc>(a.p[e]);
          const Cc vv = ccast<Cc>(a.v[e]);
          val = cadd(ccast<Cc>(a.r[e]), cmul(be, csub(pp, cmul(om, vv))));
          a.p[e] = ccast<Cs>(val);
        } else {
          val = csub(ccast<Cc>(a.r[e]), cmul(al, ccast<Cc>(a.v[e])));
          a.s[e] = ccast<Cs>(val);
        }
        if constexpr (MULF) val = cscale(val, static_cast<Rc>(a.f[(size_t)row * a.n + col]));
      }
      v[b * R0 + r] = val;
    }
  }
  fft_regs<Cc, P, NT, -1, typename PL::fwd>(v, tid, lds + lr * P, 1, a.tw);
  if (vr) {
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

template <typename Rs, typename Rc, int P, int MODE, bool CONJ, bool MASK>
__global__ void __launch_bounds__((ColCfg<Rc, P>::THREADS)) k_col(ConvArgs<Rs, Rc> a) {
  using Cc = cplx_t<Rc>;
  using PL = Plan<P>;
  using CF = ColCfg<Rc, P>;
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
  __shared__ Cc lds[P * CF::LS];
  const int lc = threadIdx.x % COLS, tid = threadIdx.x / COLS;
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
  if constexpr (MODE != COL_INV) fft_regs<Cc, P, NT, -1, typename PL::fwd>(v, tid, lds + lc, CF::LS, a.tw);
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
  if constexpr (MODE != COL_FWD) fft_regs<Cc, P, NT, +1, typename PL::inv>(v, tid, lds + lc, CF::LS, a.tw);
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

// ---------------------------------------------------------------- stage 3
template <typename Rs, typename Rc, int P, int EPI, bool MULF>
__global__ void __launch_bounds__(256) k_row_inv(ConvArgs<Rs, Rc> a) {
  using Cs = cplx_t<Rs>;
  using Cc = cplx_t<Rc>;
  using PL = Plan<P>;
  constexpr int NT = RowCfg<P>::NT, ROWS = RowCfg<P>::ROWS, V = P / NT;
  constexpr int R0 = FirstRadix<typename PL::inv>::value;
  constexpr int RL = Stockham<Cc, P, NT, +1, 1, typename PL::inv>::LAST;
  constexpr bool DOTS = (EPI == EPI_V || EPI == EPI_T || EPI == EPI_TR);
  const int t = blockIdx.y;
  if (a.st && !(a.st[t].flags & a.flag)) return;
  __shared__ Cc lds[ROWS * P];
  __shared__ double scratch[16 * NPART];
  const int lr = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int row = blockIdx.x * ROWS + lr;
  const bool vr = row < a.rows;
  const size_t rowoff = (size_t)t * a.N + (size_t)row * a.n;
  Cc v[V];
  {
    const Cc *in = a.X2 + ((size_t)t * a.rows + (vr ? row : 0)) * P;
#pragma unroll
    for (int b = 0; b < V / R0; ++b) {
      const int j = tid + b * NT;
#pragma unroll
      for (int r = 0; r < R0; ++r) v[b * R0 + r] = vr ? in[j + r * (P / R0)] : czero<Cc>();
    }
  }
  fft_regs<Cc, P, NT, +1, typename PL::inv>(v, tid, lds + lr * P, 1, a.tw);
  const Rc scale = static_cast<Rc>(a.scale);
  int restart = 0;
  if constexpr (EPI == EPI_TR) restart = a.st ? a.st[t].restart : 1;
  double acc[NPART] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < V / RL; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int col = j + r * (P / RL);
      if (!(vr && col < a.n)) continue;
      const size_t e = rowoff + col;
      Cc cv = cscale(v[b * RL + r], scale);
      if constexpr (MULF) cv = cscale(cv, static_cast<Rc>(a.f[(size_t)row * a.n + col]));
      if constexpr (EPI == EPI_AX) {
        a.y[e] = ccast<Cs>(csub(ccast<Cc>(a.x[e]), cv));
      } else if constexpr (EPI == EPI_G) {
        a.y[e] = ccast<Cs>(cv);
      } else if constexpr (EPI == EPI_V) {
        const Cs vv = ccast<Cs>(csub(ccast<Cc>(a.p[e]), cv));
        a.y[e] = vv;
        const cd h = ccast<cd>(a.rhat[e]);
        const cd w = ccast<cd>(vv);
        acc[0] += h.x * w.x + h.y * w.y;
        acc[1] += h.x * w.y - h.y * w.x;
      } else if constexpr (EPI == EPI_T) {
        const Cs tt = ccast<Cs>(csub(ccast<Cc>(a.s[e]), cv));
        a.y[e] = tt;
        const cd tv = ccast<cd>(tt);
        const cd sv = ccast<cd>(a.s[e]);
        acc[0] += tv.x * sv.x + tv.y * sv.y;
        acc[1] += tv.x * sv.y - tv.y * sv.x;
        acc[2] += tv.x * tv.x + tv.y * tv.y;
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
    block_sum<NPART>(acc, scratch);
    if (threadIdx.x == 0) {
      double *dst = a.part + ((size_t)t * gridDim.x + blockIdx.x) * NPART;
#pragma unroll
      for (int i = 0; i < NPART; ++i) dst[i] = acc[i];
    }
  }
}

// ---------------------------------------------------------------- launch
template <typename Rs, typename Rc, int P, int PRO, int EPI>
static int launch_conv_p(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  const bool pure_g = (EPI == EPI_G || EPI == EPI_GRAD);
  const bool mulf_in = !adjoint && !pure_g;
  const bool mulf_out = adjoint && !pure_g;
  // solver stages skip transmitters that are paused or done
  constexpr bool MASKED = (EPI == EPI_V || EPI == EPI_T || EPI == EPI_TR);
  a.rows = c.rows;
  a.scale = 1.0 / std::pow((double)P, c.dim);
  constexpr int CT = ColCfg<Rc, P>::THREADS, CC = ColCfg<Rc, P>::COLS;
  dim3 grow((a.rows + RowCfg<P>::ROWS - 1) / RowCfg<P>::ROWS, c.T);
  if (mulf_in)
    hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO, true>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO, false>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  if (c.dim == 2) {
    // X1 [T][n][P] -> X2 [T][n][P]: column FFT, kernel spectrum, inverse
    a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
    dim3 g(P / CC, c.T);
    if (adjoint)
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, true, MASKED>), g, dim3(CT), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, false, MASKED>), g, dim3(CT), 0, c.stream, a);
  } else {
    // X1 [T][n x][n y][P kz] -> X2 [T][n x][P ky][P kz]: forward along y
    a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = P, a.ydiv = c.n;
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_FWD, false, MASKED>), dim3(P / CC, c.T * c.n), dim3(CT), 0, c.stream, a);
    // X2 [T][n x][P*P] -> X1 [T][n x][P*P]: forward along x, kernel spectrum, inverse
    a.cin = a.X2, a.cout = a.X1, a.width = P * P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
    if (adjoint)
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, true, MASKED>), dim3(P * P / CC, c.T), dim3(CT), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, false, MASKED>), dim3(P * P / CC, c.T), dim3(CT), 0, c.stream,
                         a);
    // X1 [T][n x][P ky][P kz] -> X2 [T][n x][n y][P kz]: inverse along y
    a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = P, a.out_rows = c.n, a.ydiv = c.n;
    hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_INV, false, MASKED>), dim3(P / CC, c.T * c.n), dim3(CT), 0, c.stream, a);
  }
  if (mulf_out)
    hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI, true>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI, false>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

#ifndef CISOR_FFT_SIZES
#define CISOR_FFT_SIZES X(64) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#endif

int row_blocks(int P, int n) {
  switch (P) {
#define X(p) \
  case p:    \
    return (n + RowCfg<p>::ROWS - 1) / RowCfg<p>::ROWS;
    CISOR_FFT_SIZES
#undef X
    default:
      return 0;
  }
}

// Smallest compiled transform length P >= 2n (0 if none): a circulant of
// length P >= 2n - 1 reproduces the linear convolution on the n samples.
int fft_length_for(int n) {
  int best = 0;
#define X(p) \
  if (p >= 2 * n && (best == 0 || p < best)) best = p;
  CISOR_FFT_SIZES
#undef X
  return best;
}

bool fft_length_supported(int P) {
  switch (P) {
#define X(p) \
  case p:    \
    return true;
    CISOR_FFT_SIZES
#undef X
    default:
      return false;
  }
}

template <typename Rs, typename Rc, int PRO, int EPI>
int launch_conv(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint) {
  a.n = c.n;
  a.N = c.N;
  a.T = c.T;
  switch (c.P) {
#define X(p) \
  case p:    \
    return launch_conv_p<Rs, Rc, p, PRO, EPI>(c, a, adjoint);
    CISOR_FFT_SIZES
#undef X
    default:
      return CISOR_E_UNSUPPORTED;
  }
}

template <typename R>
void fill_tables(Ctx &c, const cplx_t<R> *&G, const cplx_t<R> *&tw, cplx_t<R> *&X1, cplx_t<R> *&X2) {
  if constexpr (std::is_same<R, double>::value) {
    if (c.precision == 1) {
      G = (const cd *)c.Ghat;
      tw = (const cd *)c.tw;
      X1 = (cd *)c.X1;
      X2 = (cd *)c.X2;
    } else {
      G = c.Ghat_d;
      tw = c.tw_d;
      X1 = c.X1d;
      X2 = c.X2d;
    }
  } else {
    G = (const cf *)c.Ghat;
    tw = (const cf *)c.tw;
    X1 = (cf *)c.X1;
    X2 = (cf *)c.X2;
  }
}

template <typename R>
int launch_apply_A(Ctx &c, const R *f, const cplx_t<R> *x, cplx_t<R> *y, bool adjoint) {
  ConvArgs<R, R> a{};
  a.f = f;
  a.x = x;
  a.y = y;
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  return launch_conv<R, R, PRO_X, EPI_AX>(c, a, adjoint);
}

// One stage of the unmasked operator y = A x (or A^H x): stage 1 writes the
// context's X1, stage 2 maps X1 to X2, stage 3 reads X2 and writes y.
template <typename Rs, typename Rc, int P>
static int launch_stage_p(Ctx &c, ConvArgs<Rs, Rc> &a, int stage, bool adjoint) {
  if (c.dim != 2) return CISOR_E_UNSUPPORTED;
  a.rows = c.rows;
  a.scale = 1.0 / ((double)P * P);
  a.cin = a.X1, a.cout = a.X2, a.width = P, a.in_rows = c.n, a.out_rows = c.n, a.ydiv = 1;
  dim3 grow((c.n + RowCfg<P>::ROWS - 1) / RowCfg<P>::ROWS, c.T);
  dim3 gcol(P / ColCfg<Rc, P>::COLS, c.T);
  if (stage == 1) {
    if (!adjoint)
      hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO_X, true>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_row_fwd<Rs, Rc, P, PRO_X, false>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  } else if (stage == 2) {
    if (adjoint)
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, true, false>), gcol, dim3(ColCfg<Rc, P>::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_col<Rs, Rc, P, COL_CONV, false, false>), gcol, dim3(ColCfg<Rc, P>::THREADS), 0, c.stream, a);
  } else {
    if (adjoint)
      hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI_AX, true>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
    else
      hipLaunchKernelGGL((k_row_inv<Rs, Rc, P, EPI_AX, false>), grow, dim3(RowCfg<P>::THREADS), 0, c.stream, a);
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template <typename R>
int launch_conv_stage(Ctx &c, const R *f, const cplx_t<R> *x, cplx_t<R> *y, int stage, bool adjoint) {
  ConvArgs<R, R> a{};
  a.n = c.n;
  a.N = c.N;
  a.T = c.T;
  a.f = f;
  a.x = x;
  a.y = y;
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  switch (c.P) {
#define X(p) \
  case p:    \
    return launch_stage_p<R, R, p>(c, a, stage, adjoint);
    CISOR_FFT_SIZES
#undef X
    default:
      return CISOR_E_UNSUPPORTED;
  }
}
template int launch_conv_stage<float>(Ctx &, const float *, const cf *, cf *, int, bool);
template int launch_conv_stage<double>(Ctx &, const double *, const cd *, cd *, int, bool);

template <typename R>
int launch_apply_G(Ctx &c, const cplx_t<R> *x, cplx_t<R> *y, bool conj) {
  ConvArgs<R, R> a{};
  a.x = x;
  a.y = y;
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  return launch_conv<R, R, PRO_X, EPI_G>(c, a, conj);
}

// explicit instantiations
template void fill_tables<float>(Ctx &, const cf *&, const cf *&, cf *&, cf *&);
template void fill_tables<double>(Ctx &, const cd *&, const cd *&, cd *&, cd *&);
template int launch_apply_A<float>(Ctx &, const float *, const cf *, cf *, bool);
template int launch_apply_A<double>(Ctx &, const double *, const cd *, cd *, bool);
template int launch_apply_G<float>(Ctx &, const cf *, cf *, bool);
template int launch_apply_G<double>(Ctx &, const cd *, cd *, bool);

#define CISOR_INST(Rs, Rc)                                                             \
  template int launch_conv<Rs, Rc, PRO_X, EPI_AX>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv<Rs, Rc, PRO_X, EPI_TR>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv<Rs, Rc, PRO_X, EPI_G>(Ctx &, ConvArgs<Rs, Rc> &, bool);    \
  template int launch_conv<Rs, Rc, PRO_X, EPI_GRAD>(Ctx &, ConvArgs<Rs, Rc> &, bool); \
  template int launch_conv<Rs, Rc, PRO_PUPD, EPI_V>(Ctx &, ConvArgs<Rs, Rc> &, bool); \
  template int launch_conv<Rs, Rc, PRO_SUPD, EPI_T>(Ctx &, ConvArgs<Rs, Rc> &, bool);
CISOR_INST(float, float)
CISOR_INST(double, double)
template int launch_conv<float, double, PRO_X, EPI_TR>(Ctx &, ConvArgs<float, double> &, bool);

}  // namespace cisor
