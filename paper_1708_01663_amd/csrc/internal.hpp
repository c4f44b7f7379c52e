// Internal declarations of the CISOR library: context, solver state, launchers.
#pragma once

#include <vector>

#include "../../include/cisor.h"
#include "common.hpp"

namespace cisor {

// Per-transmitter BiCGSTAB state, kept on the device.
enum : int { ST_ITER = 0, ST_PAUSED = 1, ST_DONE = 2, ST_FAILED = 3 };
enum : int { FLAG_ITER = 1, FLAG_TR = 2 };

struct TxState {
  cd rho, rho_prev, alpha, omega, beta;   // complex BiCGSTAB scalars
  double bnorm2, rnorm2, true_rel;
  double rmax2;  // largest recurrence residual^2 since the last true-residual evaluation
  int status;    // ST_*
  int flags;     // FLAG_ITER: run the next iteration; FLAG_TR: evaluate the true residual
  int iters;     // BiCGSTAB iterations done
  int last_tr;   // value of iters at the last true-residual evaluation
  int restart;   // next true-residual step restarts the recurrence (rhat = r, beta = 0)
  int zero_x;    // right-hand side was zero: the solution is x = 0
  int r_fresh;   // the residual buffer holds r (after a true-residual step); else r = s - omega t
  int x_pending; // x still lacks alpha p + omega s of the last completed iteration
};

// Prologue of the forward row-FFT stage.
enum : int { PRO_X = 0, PRO_PUPD = 1, PRO_SUPD = 2 };
// Epilogue of the inverse row-FFT stage.
// EPI_GF: y = G (f x), the convolution of the contrast-weighted input (the
// first-Born scattered field when x = u_in).
enum : int { EPI_AX = 0, EPI_V = 1, EPI_T = 2, EPI_TR = 3, EPI_G = 4, EPI_GRAD = 5, EPI_GF = 6 };

constexpr int NPART = 8;          // doubles per partial-sum slot
constexpr int PROJ_KCHUNK = 512;  // pixels per split-K chunk of the receiver projection
constexpr int PROJ_REDUCE_OUT = 32;  // projection outputs per block of the split-K sum
// Doubles of the projection's D scratch for M*T outputs: one partial per
// split-K-sum block, plus the slot that receives D.
inline size_t proj_dpart_slots(size_t MT) { return (MT + PROJ_REDUCE_OUT - 1) / PROJ_REDUCE_OUT + 1; }
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
  const Rs *const *frow;  // per-field contrast pointers [T] (replace f when set)
  // stage 1 inputs
  const Cs *x;            // PRO_X input / EPI_AX, EPI_TR minuend field
  const Cs *r;            // PRO_PUPD, PRO_SUPD (read where the state says r is stored)
  Cs *p;                  // PRO_PUPD in/out; EPI_V reads it
  const Cs *v;            // PRO_PUPD, PRO_SUPD
  Cs *s;                  // PRO_PUPD reads it; PRO_SUPD in/out; EPI_T reads it
  const Cs *tt;           // PRO_PUPD, PRO_SUPD: t of the previous iteration
  Cs *xw;                 // PRO_PUPD: the iterate x (pending update applied)
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
  // per field, or null: the row stages and the generic column kernel skip the
  // fields whose entry is zero (their outputs are left as they were); the
  // other column kernels transform every field
  const int *fmask;
  // intermediates and tables
  Cc *X1, *X2;            // [T][n][P]
  const Cc *Ghat;         // [P][P]
  const Cc *tw;           // [P]
  const Cc *Gpm;          // 3D plane path: the kernel spectrum kz-major, [kz][kx][ky]
};

// Identity of a captured launch sequence: the kernels' pointer and scalar
// arguments are baked into the graph, so every one of them is part of the key.
struct GraphKey {
  std::vector<const void *> ptrs;
  std::vector<double> vals;
  bool operator==(const GraphKey &o) const { return ptrs == o.ptrs && vals == o.vals; }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
};

// Graph cache and host-visible counters shared by the systems solved
// together (one context, or every group of a batch).  Captures run on a
// private stream; replays go to the caller's stream.
constexpr int GRAPH_SLOTS = 32;
struct SolveShared {
  int use_graphs = 1;
  hipStream_t cap_stream = nullptr;
  GraphEntry graphs[GRAPH_SLOTS];
  int n_graphs = 0, next_graph = 0;
  int max_jobs = 0;
  int *d_count = nullptr;          // device [max_jobs] open systems per job
  int *h_pinned = nullptr;         // pinned host copy of d_count
  hipEvent_t ev_fork = nullptr;    // fork / join events of multi-stream launches
  std::vector<hipEvent_t> ev_join;
};

struct Ctx {
  int dim = 2, n = 0, N = 0, P = 0, T = 0, M = 0, precision = 0;
  int col_variant = 0;              // 2D column-kernel variant (autotuned, FP32 compute)
  // most BiCGSTAB iterations any system needed in the context's last forward
  // and adjoint solve (0: none yet); the next solve's first chunk is cut to it
  int ls_hint[2] = {0, 0};
  const void *const *frow = nullptr;  // device [T] per-field contrast pointers (grouped problems)
  SolveShared sh;                   // solver graph cache and counters of a single context
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
  // 3D: the kernel spectrum kz-major, Gpm[kz][kx][ky] = Ghat[kx][ky][kz] (the
  // plane kernel's copy; context precision and FP64)
  void *Gpm = nullptr;
  cd *Gpm_d = nullptr;
  void *ws[6] = {};                 // r, rhat, p, v, s, t  ([T][N] complex each)
  void *X1 = nullptr, *X2 = nullptr;
  cd *X1d = nullptr, *X2d = nullptr;
  double *part = nullptr;
  TxState *st = nullptr;
  double *rel_tmp = nullptr;        // [T] true residuals of the caller's guesses (start mode 3)
  int *start_choice = nullptr;      // [T] 1 where start mode 3 fell back to the first-Born guess
  // gradient / FISTA buffers
  void *U = nullptr, *V = nullptr, *Q = nullptr, *Bv = nullptr, *W = nullptr, *gpart = nullptr;
  float *rx_mask = nullptr;         // [T][M] 1 = receiver active for the transmitter (null: all)
  void *zbuf = nullptr;             // [N] real
  void *tvbuf = nullptr;            // TV duals: 4 arrays of 2N reals (p, r ping-pong)
  bool fields_valid = false;        // U/V hold fields of a previous FISTA iteration
  // extrapolated starts (FISTA start mode 4), allocated on first use: the
  // fields and evaluation points of the two previous iterations
  void *U2 = nullptr, *V2 = nullptr;  // [T][N] complex: fields at s_{k-2}
  void *S1 = nullptr, *S2 = nullptr;  // [N] real: s_{k-1}, s_{k-2}
  double *xpart = nullptr;          // block partials and theta of the extrapolation
  int hist_depth = 0;               // evaluation points recorded (0, 1 or 2)
  // monotone APG steps, allocated on first use: the estimates' fields and
  // five N-vectors (y, gradient, gradient step, z and v estimates)
  void *apg_A1 = nullptr, *apg_A2 = nullptr, *apg_buf = nullptr;
  int apg_fields = 0;               // 1 / 2: apg_A1 / apg_A2 holds the forward fields of x_k
  // projection GEMM
  void *gemm_part = nullptr;        // split-K partials
  int gemm_kchunks = 0;
  double *dpart = nullptr;          // FP64 block partials of D
  // deferred read-back of one gradient evaluation: pinned host copies of the
  // final solver states (forward then adjoint, [2T]) and of D
  TxState *h_states = nullptr;
  double *d_D = nullptr, *h_D = nullptr;
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
int launch_apply_G(Ctx &c, const cplx_t<R> *x, cplx_t<R> *y, bool conj, const int *fmask = nullptr);
// y_t = G (f u_in,t) for all transmitters (first-Born scattered fields).
template <typename R>
int launch_born_field(Ctx &c, const R *f, cplx_t<R> *y);
// Kernel spectrum, twiddles and FFT intermediates in compute precision R.
template <typename R>
void fill_tables(Ctx &c, const cplx_t<R> *&G, const cplx_t<R> *&tw, cplx_t<R> *&X1, cplx_t<R> *&X2);
// Generic three-stage convolution with the given prologue/epilogue.
template <typename Rs, typename Rc, int PRO, int EPI>
int launch_conv(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint);
// The same for one compiled transform length (defined per length in conv_p.hip).
template <typename Rs, typename Rc, int P, int PRO, int EPI>
int launch_conv_p(Ctx &c, ConvArgs<Rs, Rc> &a, bool adjoint);
template <typename Rs, typename Rc, int P>
int launch_stage_p(Ctx &c, ConvArgs<Rs, Rc> &a, int stage, bool adjoint);

template <typename R>
int solve_batch(Ctx &c, const R *f, const cplx_t<R> *b, cplx_t<R> *x, bool adjoint,
                const cisor_ls_opts &o, int *iters_host, double *max_rel);

// One group of systems solved together with others: the context supplies the
// operator, workspaces and per-system states (its stream is the group's
// stream); f may be null when the context has per-field contrast pointers.
struct SolveJob {
  Ctx *c = nullptr;
  const void *f = nullptr, *b = nullptr;
  void *x = nullptr;
  int *iters = nullptr;   // host [c->T] or null (output)
  double max_rel = 0.0;   // output: largest final true relative residual
  int status = CISOR_OK;  // output: worst status of the group
  // pinned host [c->T]: the final states are copied there without waiting;
  // the caller synchronises the stream and calls solve_collect
  TxState *host_states = nullptr;
  int dir = 0;            // set by solve_multi: 0 forward, 1 adjoint
};
// Iteration counts, status and largest true residual of a job from its
// final states (after the copy into host memory has completed).
int solve_collect(SolveJob &j, const TxState *hs);
// Solve every job's systems; jobs whose stream differs from `main` run on
// their own streams between a fork and a join on `main`.  Returns the worst
// status (negative: error).
template <typename R>
int solve_multi(SolveJob *jobs, int njobs, SolveShared &sh, hipStream_t main, bool adjoint,
                const cisor_ls_opts &o);
// Create the counters and events of a SolveShared for up to max_jobs jobs.
int solve_shared_init(SolveShared &sh, int max_jobs);
void solve_shared_free(SolveShared &sh);
// Replay the launch sequence captured under `key` on `main`, capturing it on
// first use: launch(m) must enqueue on m, or on streams forked from m with
// events and joined back.  Contexts in `ctxs` whose stream is `main` are
// pointed at the capture stream while capturing.  Returns 0 when the sequence
// ran as a graph, 1 when graphs are off or capture failed (nothing ran: the
// caller launches directly), or a negative status.
template <typename Fn>
int graph_run(SolveShared &sh, const GraphKey &key, hipStream_t main, const std::vector<Ctx *> &ctxs, Fn &&launch) {
  if (!sh.use_graphs) return 1;
  hipGraphExec_t exec = nullptr;
  for (int i = 0; i < sh.n_graphs; ++i)
    if (sh.graphs[i].key == key) exec = sh.graphs[i].exec;
  if (!exec) {
    if (!sh.cap_stream && hipStreamCreateWithFlags(&sh.cap_stream, hipStreamNonBlocking) != hipSuccess) {
      sh.use_graphs = 0;
      return 1;
    }
    std::vector<Ctx *> swapped;
    for (Ctx *c : ctxs)
      if (c->stream == main) {
        c->stream = sh.cap_stream;
        swapped.push_back(c);
      }
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(sh.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const int rc = launch(sh.cap_stream);
      ok = (hipStreamEndCapture(sh.cap_stream, &graph) == hipSuccess) && rc == CISOR_OK && graph;
    }
    for (Ctx *c : swapped) c->stream = main;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
      sh.use_graphs = 0;
      return 1;
    }
    GraphEntry &slot = sh.graphs[sh.next_graph];
    if (sh.next_graph < sh.n_graphs && slot.exec) (void)hipGraphExecDestroy(slot.exec);
    slot.key = key;
    slot.exec = exec;
    sh.next_graph = (sh.next_graph + 1) % GRAPH_SLOTS;
    sh.n_graphs = sh.n_graphs + 1 < GRAPH_SLOTS ? sh.n_graphs + 1 : GRAPH_SLOTS;
  }
  return hipGraphLaunch(exec, main) == hipSuccess ? 0 : CISOR_E_DEVICE;
}

// Run body(j) for j = 0..n-1, body(j) enqueueing on stream_of(j): streams
// other than `main` start after the work already on `main` and `main` waits
// for all of them afterwards.
template <typename StreamOf, typename Body>
int fork_join(SolveShared &sh, hipStream_t main, int n, StreamOf &&stream_of, Body &&body) {
  bool fork = false;
  for (int j = 0; j < n; ++j) fork |= (stream_of(j) != main);
  if (!fork) {
    for (int j = 0; j < n; ++j)
      if (int rc = body(j)) return rc;
    return CISOR_OK;
  }
  if ((int)sh.ev_join.size() < n || !sh.ev_fork) return CISOR_E_ARG;
  if (hipEventRecord(sh.ev_fork, main) != hipSuccess) return CISOR_E_DEVICE;
  int rc = CISOR_OK;
  for (int j = 0; j < n; ++j) {
    hipStream_t s = stream_of(j);
    if (s != main && hipStreamWaitEvent(s, sh.ev_fork, 0) != hipSuccess) return CISOR_E_DEVICE;
    if (!rc) rc = body(j);
    if (s != main && hipEventRecord(sh.ev_join[j], s) != hipSuccess) return CISOR_E_DEVICE;
  }
  for (int j = 0; j < n; ++j)
    if (stream_of(j) != main && hipStreamWaitEvent(main, sh.ev_join[j], 0) != hipSuccess) return CISOR_E_DEVICE;
  return rc;
}

// D_host: synchronous host result; D_dev: device slot written without a sync.
template <typename R>
int launch_project(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *y_meas,
                   cplx_t<R> *y, double *D_host, double *D_dev = nullptr);
template <typename R>
int launch_backproject(Ctx &c, const cplx_t<R> *w, cplx_t<R> *q, const R *f, cplx_t<R> *b);

template <typename R>
int launch_tv_prox(Ctx &c, const R *z, R *x, double lam, double lo, double hi, int iters);
// Isotropic TV of x (2D, FP64 sum; synchronises the context stream).
template <typename R> int launch_tv_value(Ctx &c, const R *x, double *tv);

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

// Relaxed-FISTA tail with the scalar t_k kept on the device (graph-safe):
// z = s - gamma grad; f_k = prox(z); t_{k+1}, s_{k+1}, f_prev, f updated and
// *t_dev advanced.
template <typename R>
int launch_fista_tail_dev(Ctx &c, R *f, R *f_prev, R *s, const R *grad, double *t_dev, double gamma, double tau,
                          double alpha, double lo, double hi, int inner);
// grad[q] = sum over rows [0, rows) of gpart[row][q] (FP64 accumulation).
// Transmitter description of a geometry is usable (directions or sources).
bool transmitters_ok(const cisor_geometry &g);
// The scalar context behind a C handle.
Ctx *ctx_of(cisor_ctx *h);
// Starting guesses of the next FISTA gradient at s from the last two (depth 2),
// the last (depth 1) or no (depth 0) recorded evaluations; records s.
template <typename R> int launch_extrapolate(Ctx &c, const R *s, int depth);
template <typename R>
int launch_sum_rows(Ctx &c, const R *gpart, R *grad, int rows);
// Copy / fill kernels (graph-safe replacements of memcpy / memset).
template <typename C> void launch_copy(hipStream_t s, C *dst, const C *src, size_t n);
template <typename C> void launch_fill(hipStream_t s, C *dst, size_t n, C v);

// Time `reps` launches of the 2D column stage for every column variant and
// keep the fastest in c.col_variant; times_ms (host [COL_VARIANTS] or null)
// receives the mean per launch.
int autotune_columns(Ctx &c, int reps, float *times_ms);

// Host-side setup: FP64 geometry, kernels, spectrum, receiver matrix.  With
// spectrum = false the kernel spectrum and twiddles are left as they are
// (problems that share a grid share one spectrum).
int build_geometry(Ctx &c, const cisor_geometry &g, bool spectrum = true);

bool fft_length_supported(int P);
int row_blocks(int P, int n);
int fft_length_for(int n);

}  // namespace cisor
