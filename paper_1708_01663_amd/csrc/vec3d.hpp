// Internal declarations of the 3D vectorial (electromagnetic) model: the
// three-component fields of the appendix on 3D imaging, complex128 throughout.
//
// Fields are stored [T][3][N]: transmitter t, component E^(c) (c = x, y, z),
// cell (i n + j) n + l.  That is [3T][N] scalar fields, so the scalar 3D
// convolution of a context created with 3T transmitters applies G0 to all of
// them in one pass.  With G the scalar kernel (k^2 times the cell-integrated
// Green's function G0):
//
//   A E   = E - (I + D / k^2) G (f E)         (eq. 3DA_def)
//   A^H V = V - f G^H (V + D V / k^2)         (D real symmetric)
//
// where D is the grad-div finite-difference operator with the three-point
// second difference on the diagonal and the four-corner cross difference over
// 4 delta^2 off it (fields zero outside the grid).
#pragma once

#include "internal.hpp"

namespace cisor {
namespace vec {

enum : int { V_ITER = 0, V_TR = 1, V_DONE = 2, V_CAP = 3, V_NONFINITE = 4 };

// Per-system BiCGSTAB state of one 3N-unknown system, kept on the device.
struct VState {
  cd rho, rho_old, rho_next, alpha, omega, beta;
  double bnorm2, rnorm2, rel, pad_;
  int status;   // V_*
  int iters;    // BiCGSTAB iterations done
  int sbreak;   // the iteration ends after s (x += alpha p, r = s)
  int restart;  // the next restart kernel resets rhat, p, v (and zeroes x if zero_b)
  int zero_b;   // right-hand side is zero: the solution is x = 0
  int pad2_[3];
};

constexpr int VB = 256;        // threads per block of the field kernels
constexpr int VMAXB = 128;     // blocks per system of the field kernels
constexpr int VNP = 4;         // doubles per partial-sum slot

struct VecCtx {
  cisor_ctx *sub = nullptr;    // scalar 3D context with 3T transmitters (the convolution)
  Ctx *sc = nullptr;
  int n = 0, N = 0, T = 0, M = 0, nbv = 0;
  double h = 0, k = 0;
  hipStream_t stream = nullptr;
  cd *Ein = nullptr;           // [T][3N] incident fields
  cd *H = nullptr;             // [M][3N] third dyadic row times delta^3
  cd *ws[8] = {};              // r, rhat, p, v, s, t, pre (convolution input), Y (convolution output)
  cd *E = nullptr, *Vv = nullptr, *Q = nullptr, *B = nullptr, *Wr = nullptr;  // gradient buffers
  double *part = nullptr;      // [T][nbv][VNP]
  VState *st = nullptr;        // [T]
  VState *h_st = nullptr;      // pinned host copy
  int *fmask = nullptr;        // [3T] per component field: 1 where its system takes part in the convolution
  float *rx_mask = nullptr;    // [T][M] 1 = receiver active for the transmitter (null: all)
  double *f3 = nullptr;        // [3N] contrast repeated per component (projection operand)
  void *gemm_part = nullptr;   // split-K partials of the projection
  double *dpart = nullptr;     // block partials of D
  double *gbuf = nullptr, *zb = nullptr, *fk = nullptr;  // [N] each: gradient, gradient step, prox output
};

// y = A x or A^H x for every transmitter.
int launch_apply(VecCtx &v, const double *f, const cd *x, cd *y, bool adjoint);
// Solve A x = b (or A^H x = b) for every transmitter; x holds the start on
// entry when start == 3.  iters: host [T] or null; max_rel: largest final
// true relative residual.  Returns the worst status.
int launch_solve(VecCtx &v, const double *f, const cd *b, cd *x, bool adjoint, const cisor_ls_opts &o, int *iters,
                 double *max_rel);
// y = Ht (I_3 x diag f) E; with y_meas, w = y - y_meas and D = 0.5 ||w||^2.
int launch_project(VecCtx &v, const double *f, const cd *E, const cd *y_meas, cd *y, cd *w, double *D);
// q = Ht^H w and rhs = (I_3 x diag f) q.
int launch_backproject(VecCtx &v, const double *f, const cd *w, cd *q, cd *rhs);
// grad = Re sum_t sum_c conj(E) (q + G^H (V + D V / k^2)) (eq. 3Dg_def, eq. 3Dgradient).
int launch_gradient(VecCtx &v, const cd *E, const cd *q, const cd *V, double *grad);
// Relaxed-FISTA tail on the 3D volume (eqs. algo1-algo3): f_k = prox(s - gamma
// grad) with the 3D TV prox, then the momentum update of f_prev, f, s, t, k.
int launch_fista_tail(VecCtx &v, cisor_fista_state *s, const double *grad, double gamma, double tau, double alpha,
                      double lo, double hi, int inner);

}  // namespace vec
}  // namespace cisor
