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

#include "conv_cfg.hpp"
#include "internal.hpp"

namespace cisor {

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
int launch_apply_G(Ctx &c, const cplx_t<R> *x, cplx_t<R> *y, bool conj, const int *fmask) {
  ConvArgs<R, R> a{};
  a.x = x;
  a.y = y;
  a.fmask = fmask;
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  return launch_conv<R, R, PRO_X, EPI_G>(c, a, conj);
}

template <typename R> int launch_born_field(Ctx &c, const R *f, cplx_t<R> *y) {
  ConvArgs<R, R> a{};
  a.f = f;
  a.x = (const cplx_t<R> *)c.uin;
  a.y = y;
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  return launch_conv<R, R, PRO_X, EPI_GF>(c, a, false);
}
template int launch_born_field<float>(Ctx &, const float *, cf *);
template int launch_born_field<double>(Ctx &, const double *, cd *);

// Autotuner of the 2D column stage: every column variant (radix plan x tile
// shape) is timed on the context's own buffers and the fastest is kept.
int autotune_columns(Ctx &c, int reps, float *times_ms) {
  if (c.dim != 2 || reps < 1) return CISOR_E_ARG;
  if (times_ms)
    for (int v = 0; v < COL_VARIANTS; ++v) times_ms[v] = -1.0f;
  if (c.precision != 0) {  // FP64 compute has one variant
    c.col_variant = 0;
    return CISOR_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return CISOR_E_DEVICE;
  }
  launch_fill<cf>(c.stream, (cf *)c.X1, (size_t)c.T * c.n * c.P, mk<cf>(0.0f, 0.0f));
  float best = 0.0f;
  int best_v = 0, rc = CISOR_OK;
  for (int v = 0; v < COL_VARIANTS && rc == CISOR_OK; ++v) {
    c.col_variant = v;
    rc = launch_conv_stage<float>(c, nullptr, nullptr, nullptr, 2, false);   // warm-up
    if (rc) break;
    if (hipEventRecord(e0, c.stream) != hipSuccess) rc = CISOR_E_DEVICE;
    for (int r = 0; r < reps && rc == CISOR_OK; ++r) rc = launch_conv_stage<float>(c, nullptr, nullptr, nullptr, 2, false);
    if (rc == CISOR_OK && (hipEventRecord(e1, c.stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      rc = CISOR_E_DEVICE;
    float ms = 0.0f;
    if (rc == CISOR_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CISOR_E_DEVICE;
    ms /= reps;
    if (times_ms) times_ms[v] = ms;
    if (v == 0 || ms < best) {
      best = ms;
      best_v = v;
    }
  }
  c.col_variant = rc == CISOR_OK ? best_v : 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// explicit instantiations
template void fill_tables<float>(Ctx &, const cf *&, const cf *&, cf *&, cf *&);
template void fill_tables<double>(Ctx &, const cd *&, const cd *&, cd *&, cd *&);
template int launch_apply_A<float>(Ctx &, const float *, const cf *, cf *, bool);
template int launch_apply_A<double>(Ctx &, const double *, const cd *, cd *, bool);
template int launch_apply_G<float>(Ctx &, const cf *, cf *, bool, const int *);
template int launch_apply_G<double>(Ctx &, const cd *, cd *, bool, const int *);

#define CISOR_INST(Rs, Rc)                                                             \
  template int launch_conv<Rs, Rc, PRO_X, EPI_AX>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv<Rs, Rc, PRO_X, EPI_TR>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv<Rs, Rc, PRO_X, EPI_G>(Ctx &, ConvArgs<Rs, Rc> &, bool);    \
  template int launch_conv<Rs, Rc, PRO_X, EPI_GF>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv<Rs, Rc, PRO_X, EPI_GRAD>(Ctx &, ConvArgs<Rs, Rc> &, bool); \
  template int launch_conv<Rs, Rc, PRO_PUPD, EPI_V>(Ctx &, ConvArgs<Rs, Rc> &, bool); \
  template int launch_conv<Rs, Rc, PRO_SUPD, EPI_T>(Ctx &, ConvArgs<Rs, Rc> &, bool);
CISOR_INST(float, float)
CISOR_INST(double, double)
template int launch_conv<float, double, PRO_X, EPI_TR>(Ctx &, ConvArgs<float, double> &, bool);

}  // namespace cisor
