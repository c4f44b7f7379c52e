// Internal declarations of the CISOR library: context, solver state, launchers.
#pragma once

#include "../../include/cisor.h"
#include "common.hpp"

namespace cisor {

// Per-transmitter BiCGSTAB state, kept on the device.
enum : int { ST_ITER = 0, ST_PAUSED = 1, ST_DONE = 2, ST_FAILED = 3 };
enum : int { FLAG_ITER = 1, FLAG_TR = 2 };

struct TxState {
  cd rho, rho_prev, alpha, omega, beta;   // complex BiCGSTAB scalars
  double bnorm2, rnorm2, true_rel, pad0_;
  int status;    // ST_*
  int flags;     // FLAG_ITER: run the next iteration; FLAG_TR: evaluate the true residual
  int iters;     // BiCGSTAB iterations done
  int last_tr;   // value of iters at the last true-residual evaluation
  int restart;   // next true-residual step restarts the recurrence (rhat = r, beta = 0)
  int zero_x;    // right-hand side was zero: the solution is x = 0
  int pad_[2];
};

// Prologue of the forward row-FFT stage.
enum : int { PRO_X = 0, PRO_PUPD = 1, PRO_SUPD = 2 };
// Epilogue of the inverse row-FFT stage.
enum : int { EPI_AX = 0, EPI_V = 1, EPI_T = 2, EPI_TR = 3, EPI_G = 4, EPI_GRAD = 5 };

constexpr int NPART = 4;          // doubles per partial-sum slot
constexpr int UPD_EPT = 4;        // elements per thread of the update kernel
constexpr int UPD_THREADS = 256;

// Arguments of the three FFT-convolution stages (typed by storage real Rs and
// compute real Rc).  Unused pointers are null.
template <typename Rs, typename Rc> struct ConvArgs {
  using Cs = cplx_t<Rs>;
  using Cc = cplx_t<Rc>;
  int n, N, T;
  int rows;               // rows of n samples per transmitter (n^(dim-1)) for the row stages
  double scale;           // 1 / P^dim
  // column stages: input/output arrays, column count, non-zero input rows,
  // kept output rows, and the divisor from the batch index to the transmitter
  const Cc *cin;
  Cc *cout;
  int width, in_rows, out_rows, ydiv;
  const Rs *f;            // contrast [N]
  // stage 1 inputs
  const Cs *x;            // PRO_X input / EPI_AX, EPI_TR minuend field
  const Cs *r;            // PRO_PUPD, PRO_SUPD
  Cs *p;                  // PRO_PUPD in/out; EPI_V reads it
  const Cs *v;            // PRO_PUPD, PRO_SUPD
  Cs *s;                  // PRO_SUPD out; EPI_T reads it
  // stage 3
  Cs *y;                  // output field (EPI_AX -> y, EPI_V -> v, EPI_T -> t, EPI_TR -> r, EPI_G -> y)
  Cs *rhat;               // EPI_V / EPI_TR (written on restart)
  const Cs *b;            // EPI_TR right-hand side
  const Cs *u;            // EPI_GRAD
  const Cs *q;            // EPI_GRAD
  Rs *gpart;              // EPI_GRAD per-transmitter contribution [T][N]
  double *part;           // partial sums [T][nblk][NPART]
  TxState *st;            // per-transmitter state or null (all active)
  int flag;               // FLAG_ITER or FLAG_TR
  // intermediates and tables
  Cc *X1, *X2;            // [T][n][P]
  const Cc *Ghat;         // [P][P]
  const Cc *tw;           // [P]
};

// Identity of a captured chunk of solver iterations: the kernels' pointer and
// scalar arguments are baked into the graph.
struct GraphKey {
  const void *f, *b;
  void *x;
  bool adjoint;
  int chunk;
  double tol;
  int replace_every, maxit;
  bool operator==(const GraphKey &o) const {
    return f == o.f && b == o.b && x == o.x && adjoint == o.adjoint && chunk == o.chunk && tol == o.tol &&
           replace_every == o.replace_every && maxit == o.maxit;
  }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

struct Ctx {
  int dim = 2, n = 0, N = 0, P = 0, T = 0, M = 0, precision = 0;
  // hipGraph replay of solver iteration chunks (captured on a private stream,
  // launched on the caller's stream)
  int use_graphs = 1;
  hipStream_t cap_stream = nullptr;
  GraphEntry graphs[8] = {};
  int n_graphs = 0, next_graph = 0;
  double h = 0, k = 0, kb = 0, eps_b = 1;
  hipStream_t stream = nullptr;
  int rows = 0;       // rows of n samples per field: n^(dim-1)
  int nrb = 0;        // row blocks per transmitter of the row-FFT stages
  int nub = 0;        // blocks per transmitter of the update kernel
  int nblk = 0;       // partial-sum slots per transmitter
  // device data (typed by precision; the *_d tables are FP64 copies used by
  // the FP64 true-residual operator)
  void *Ghat = nullptr, *tw = nullptr, *H = nullptr, *uin = nullptr;
  cd *Ghat_d = nullptr, *tw_d = nullptr;
  void *ws[6] = {};                 // r, rhat, p, v, s, t  ([T][N] complex each)
  void *X1 = nullptr, *X2 = nullptr;
  cd *X1d = nullptr, *X2d = nullptr;
  double *part = nullptr;
  TxState *st = nullptr;
  int *d_count = nullptr;
  int *h_pinned = nullptr;
  double *rel_tmp = nullptr;        // [T] true residuals of the caller's guesses (start mode 3)
  int *start_choice = nullptr;      // [T] 1 where start mode 3 fell back to the first-Born guess
  // gradient / FISTA buffers
  void *U = nullptr, *V = nullptr, *Q = nullptr, *Bv = nullptr, *W = nullptr, *gpart = nullptr;
  void *zbuf = nullptr;             // [N] real
  void *tvbuf = nullptr;            // TV duals: 4 arrays of 2N reals (p, r ping-pong)
  bool fields_valid = false;        // U/V hold fields of a previous FISTA iteration
  // projection GEMM
  void *gemm_part = nullptr;        // split-K partials
  int gemm_kchunks = 0;
  double *dpart = nullptr;          // FP64 block partials of D
};

// ---- launchers (all enqueue on ctx.stream; return a cisor status) ----

// y = A x or A^H x over all transmitters (plain operator, precision of ctx).
template <typename R>
int launch_apply_A(Ctx &c, const R *f, const cplx_t<R> *x, cplx_t<R> *y, bool adjoint);
// One stage (1, 2 or 3) of the unmasked operator A or A^H.
template <typename R>
int launch_conv_stage(Ctx &c, const R *f, const cplx_t<R> *x, cplx_t<R> *y, int stage, bool adjoint);
// y = G x or G^H x (no identity, no contrast).
template <typename R>
int launch_apply_G(Ctx &c, const cplx_t<R> *x, cplx_t<R> *y, bool conj);
// Generic three-stage convolution with the given prologue/epilogue.
template <typename Rs, typename Rc, int PRO, int EPI>
int launch_conv(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint);

template <typename R>
int solve_batch(Ctx &c, const R *f, const cplx_t<R> *b, cplx_t<R> *x, bool adjoint,
                const cisor_ls_opts &o, int *iters_host, double *max_rel);

template <typename R>
int launch_project(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *y_meas,
                   cplx_t<R> *y, double *D_host);
template <typename R>
int launch_backproject(Ctx &c, const cplx_t<R> *w, cplx_t<R> *q, const R *f, cplx_t<R> *b);

template <typename R>
int launch_tv_prox(Ctx &c, const R *z, R *x, double lam, double lo, double hi, int iters);

template <typename R>
int launch_grad(Ctx &c, const R *f, const cplx_t<R> *y_meas, R *grad, double *D,
                cplx_t<R> *u, cplx_t<R> *v, const cisor_ls_opts &o, int *iters, double *max_rel,
                int *worst_status);

template <typename R>
int launch_vjp(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *w, R *grad, cplx_t<R> *v,
               const cisor_ls_opts &o, int *iters, double *max_rel, int *status);

template <typename R>
int launch_fista_tail(Ctx &c, cisor_fista_state *s, const R *grad, double gamma, double tau,
                      double alpha, double lo, double hi, int inner);

template <typename R>
int launch_born_lipschitz(Ctx &c, int iters, double *L);

// Host-side setup: FP64 geometry, kernels, spectrum, receiver matrix.
int build_geometry(Ctx &c, const cisor_geometry &g);

bool fft_length_supported(int P);
int row_blocks(int P, int n);
int fft_length_for(int n);

}  // namespace cisor
