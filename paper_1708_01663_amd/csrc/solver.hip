// Batched BiCGSTAB for the Lippmann-Schwinger systems A u_t = u_in,t and
// A^H v_t = b_t (eq. u_and_v), all transmitters at once.
//
// The paper names conjugate gradients for these solves; A = I - G diag(f) is
// complex non-Hermitian, so BiCGSTAB (van der Vorst 1992) is used instead.
// All vector work is fused into the FFT-convolution stages, and the residual
// r = s - omega t of an iteration is never stored:
//   it.  stage A: r <- s - omega t ; x <- x + alpha p + omega s (last
//                 iteration's scalars) ; p <- r + beta (p - omega v) ;
//                 v <- A p ; <rhat, v>
//        alpha = rho / <rhat, v>
//        stage B: s <- (s - omega t) - alpha v ; t <- A s ;
//                 <t, s>, <t, t>, <s, s>, <rhat, s>, <rhat, t>
//        omega = <t, s> / <t, t> ; rho_new = <rhat, s> - omega <rhat, t> ;
//        ||r||^2 = <s, s> - |<t, s>|^2 / <t, t> ;
//        beta = (rho_new / rho) (alpha / omega)
// so one iteration is two operator applications and two scalar steps.  The
// update of x left pending by the last iteration is applied before every
// true-residual evaluation; a true-residual step stores r, which the next
// iteration reads instead of s - omega t.  Scalars live on the device (one
// TxState per transmitter); every inner product is accumulated in FP64 with a
// fixed reduction order.
//
// Stop test: the true relative residual ||b - A x|| / ||b|| computed with an
// FP64 operator (FP64 FFTs and kernel spectrum).  A system whose recurrence
// residual reaches tol pauses until the next check point, where its true
// residual decides between "converged" and "replace r by the true residual
// and continue".  The recurrence residual of a running system is replaced by
// the true one every replace_every iterations, and also once its square has
// fallen below REPLACE_DROP2 times the largest squared recurrence residual seen
// since the last replacement (the "reliable updates" idea of van der Vorst and Ye,
// 2000): both keep the FP32 recurrence from drifting away from the true
// residual, the second where the drift grows, in the steep parts of the
// convergence.  A breakdown
// (<rhat, v> = 0, omega = 0, rho = 0 or a non-finite scalar) restarts the
// recurrence from the current x with rhat = r.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace cisor {

// STG_TR: FP64 true residual (the stop test); STG_TR0: provisional starting
// residual in the field precision, which never finishes a system with x != 0.
enum : int { STG_ALPHA = 0, STG_OMEGA = 1, STG_TR = 3, STG_TR0 = 4 };

// Residual replacement when the recurrence residual^2 has fallen below this
// fraction of its largest value since the last replacement (a drop by ~31.6x
// in norm).  Measured on the 256^2 x 60 true-phantom solves: the slowest of 60
// systems needed 443-467 iterations instead of 508-933 (the FP32 tail varies
// with rounding; the FP64 solver needs 375), at about 1 % more time per solve
// where the solves are short.
constexpr double REPLACE_DROP2 = 1e-3;

__device__ __forceinline__ cd cd_div(cd a, cd b) {
  const double den = b.x * b.x + b.y * b.y;
  return mk<cd>((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ __forceinline__ cd cd_mul(cd a, cd b) { return mk<cd>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ bool cd_ok(cd a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ bool cd_zero(cd a) { return a.x == 0.0 && a.y == 0.0; }

__global__ void k_init_state(TxState *st, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  TxState s{};
  s.status = ST_PAUSED;
  s.flags = FLAG_TR;
  s.restart = 1;
  s.rho = s.rho_prev = s.alpha = s.omega = mk<cd>(1.0, 0.0);
  s.beta = mk<cd>(0.0, 0.0);
  st[t] = s;
}

// One block of 64 threads per transmitter: sum the partial slots in a fixed
// order, then lane 0 advances the scalar recurrence.
__global__ void __launch_bounds__(64) k_scalar(TxState *st, const double *part, int nslots, int stage,
                                               double tol, int replace_every, int maxit) {
  const int t = blockIdx.x;
  // the partial sums are loaded before the state so that the two reads
  // overlap (a masked system's slots are read and ignored)
  double acc[NPART] = {};
  const double *p = part + (size_t)t * nslots * NPART;
  for (int i = threadIdx.x; i < nslots; i += 64) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) acc[k] += p[i * NPART + k];
  }
  TxState s = st[t];
  const int need = (stage == STG_TR || stage == STG_TR0) ? FLAG_TR : FLAG_ITER;
  if (!(s.flags & need)) return;
#pragma unroll
  for (int k = 0; k < NPART; ++k) acc[k] = wave_sum(acc[k]);
  if (threadIdx.x != 0) return;
  const double tol2 = tol * tol;
  if (stage == STG_ALPHA) {
    const cd rhv = mk<cd>(acc[0], acc[1]);
    s.x_pending = 0;   // stage A has applied the last iteration's x update
    if (cd_zero(rhv) || !cd_ok(rhv)) {
      s.status = ST_PAUSED;
      s.flags = FLAG_TR;
      s.restart = 1;
    } else {
      s.alpha = cd_div(s.rho, rhv);
    }
  } else if (stage == STG_OMEGA) {
    const cd ts = mk<cd>(acc[0], acc[1]);
    const double tt = acc[2], ss = acc[3];
    const cd rs = mk<cd>(acc[4], acc[5]), rt = mk<cd>(acc[6], acc[7]);
    double rr;
    if (tt == 0.0 || !std::isfinite(tt) || !cd_ok(ts)) {
      s.omega = mk<cd>(0.0, 0.0);
      rr = ss;
    } else {
      s.omega = mk<cd>(ts.x / tt, ts.y / tt);
      rr = fmax(ss - (ts.x * ts.x + ts.y * ts.y) / tt, 0.0);   // ||s - omega t||^2
    }
    const cd wrt = cd_mul(s.omega, rt);
    const cd rho_new = mk<cd>(rs.x - wrt.x, rs.y - wrt.y);       // <rhat, s - omega t>
    s.r_fresh = 0;
    s.x_pending = 1;
    s.iters += 1;
    s.rnorm2 = rr;
    s.rmax2 = fmax(s.rmax2, rr);
    const bool conv = rr <= tol2 * s.bnorm2;
    const bool brk = cd_zero(s.omega) || cd_zero(rho_new) || !cd_ok(rho_new) || !std::isfinite(rr);
    if (!brk) {
      s.beta = cd_mul(cd_div(rho_new, s.rho), cd_div(s.alpha, s.omega));
      s.rho_prev = s.rho;
      s.rho = rho_new;
    }
    if (conv) {
      s.status = ST_PAUSED;
      s.flags = FLAG_TR;
      s.restart = brk ? 1 : 0;
    } else if (brk) {
      s.status = ST_PAUSED;
      s.flags = FLAG_TR;
      s.restart = 1;
    } else if (s.iters - s.last_tr >= replace_every || s.iters >= maxit || rr < REPLACE_DROP2 * s.rmax2) {
      s.flags = FLAG_ITER | FLAG_TR;
    }
  } else {  // STG_TR: r = b - A x has just been computed in FP64 (x up to date)
    const double rr = acc[0];
    const cd rhr = mk<cd>(acc[1], acc[2]);
    if (s.restart) s.bnorm2 = acc[3];
    s.last_tr = s.iters;
    s.rmax2 = rr;
    s.rnorm2 = rr;
    s.x_pending = 0;
    s.r_fresh = 1;
    if (s.bnorm2 == 0.0) {
      s.true_rel = 0.0;
      s.status = ST_DONE;
      s.flags = 0;
      s.zero_x = 1;
    } else if (!std::isfinite(rr)) {
      s.true_rel = rr;
      s.status = ST_FAILED;
      s.flags = 0;
    } else {
      s.true_rel = sqrt(rr / s.bnorm2);
      if (rr <= tol2 * s.bnorm2 && stage == STG_TR0) {
        s.status = ST_PAUSED;   // looks converged: confirm with the FP64 residual
        s.flags = FLAG_TR;
      } else if (rr <= tol2 * s.bnorm2) {
        s.status = ST_DONE;
        s.flags = 0;
      } else if (s.restart) {
        s.rho = rhr;
        s.rho_prev = mk<cd>(1.0, 0.0);
        s.alpha = s.omega = mk<cd>(1.0, 0.0);
        s.beta = mk<cd>(0.0, 0.0);
        s.restart = 0;
        s.status = ST_ITER;
        s.flags = FLAG_ITER;
      } else {
        // residual replacement: keep the search directions, rebase rho
        if (cd_zero(rhr) || !cd_ok(rhr)) {
          s.restart = 1;
          s.status = ST_PAUSED;
          s.flags = FLAG_TR;
        } else {
          s.beta = cd_mul(cd_div(rhr, s.rho_prev), cd_div(s.alpha, s.omega));
          s.rho = rhr;
          s.status = ST_ITER;
          s.flags = FLAG_ITER;
        }
      }
    }
  }
  st[t] = s;
}

// x <- x + alpha p + omega s for the systems about to get a true residual
// whose last iteration's update of x is still pending.
template <typename R>
__global__ void __launch_bounds__(UPD_THREADS) k_apply_pending(const TxState *st, cplx_t<R> *x, const cplx_t<R> *p,
                                                               const cplx_t<R> *s, int N) {
  using C = cplx_t<R>;
  const int t = blockIdx.y;
  if (!(st[t].flags & FLAG_TR) || !st[t].x_pending) return;
  const C al = ccast<C>(st[t].alpha), om = ccast<C>(st[t].omega);
  const size_t base = (size_t)t * N;
  const int i0 = blockIdx.x * UPD_THREADS * UPD_EPT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < UPD_EPT; ++k) {
    const int i = i0 + k * UPD_THREADS;
    if (i < N) {
      const size_t e = base + i;
      x[e] = cadd(x[e], cadd(cmul(al, p[e]), cmul(om, s[e])));
    }
  }
}

template <typename C> __global__ void k_fill(C *x, size_t n, C v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}
template <typename C> __global__ void k_copy(C *dst, const C *src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_save_rel(const TxState *st, double *rel, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) rel[t] = st[t].true_rel;
}

// Keep the caller's guess where its true residual is the smaller one, else
// take the first-Born guess x = b; choice[t] = 1 records the fallback.
template <typename C>
__global__ void k_pick_start(const TxState *st_born, const double *rel_guess, C *x, const C *b, int *choice, int N) {
  const int t = blockIdx.y;
  const bool born = st_born[t].true_rel < rel_guess[t] || !isfinite(rel_guess[t]);
  if (blockIdx.x == 0 && threadIdx.x == 0) choice[t] = born ? 1 : 0;
  if (!born) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    x[(size_t)t * N + i] = b[(size_t)t * N + i];
}

// Start mode 5: where the caller's guess starts further from the solution
// than the zero guess (||b - A x0|| > ||b||, or a non-finite residual), that
// system restarts from x = 0 with r = rhat = b.  The zero guess's residual is
// the right-hand side, so the comparison costs no operator application.
// k_zero_fallback rewrites the vectors and must run before
// k_zero_fallback_state, which rewrites the recurrence and records the choice.
__device__ __forceinline__ bool zero_fallback(const TxState &s) { return s.bnorm2 > 0.0 && !(s.rnorm2 <= s.bnorm2); }
template <typename C>
__global__ void k_zero_fallback(const TxState *st, C *x, C *r, C *rhat, const C *b, int N) {
  const int t = blockIdx.y;
  if (!zero_fallback(st[t])) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const size_t e = (size_t)t * N + i;
    const C bv = b[e];
    x[e] = mk<C>(0, 0);
    r[e] = bv;
    rhat[e] = bv;
  }
}
__global__ void k_zero_fallback_state(TxState *st, int *choice, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  TxState s = st[t];
  const bool fb = zero_fallback(s);
  choice[t] = fb ? 1 : 0;
  if (!fb) return;
  s.rnorm2 = s.rmax2 = s.bnorm2;
  s.true_rel = 1.0;
  s.rho = mk<cd>(s.bnorm2, 0.0);   // <rhat, r> = ||b||^2
  s.rho_prev = s.alpha = s.omega = mk<cd>(1.0, 0.0);
  s.beta = mk<cd>(0.0, 0.0);
  s.restart = 0;
  s.r_fresh = 1;
  s.x_pending = 0;
  s.zero_x = 0;
  s.status = ST_ITER;
  s.flags = FLAG_ITER;
  st[t] = s;
}

template <typename C> __global__ void k_zero_solved(const TxState *st, C *x, int N) {
  const int t = blockIdx.y;
  if (!st[t].zero_x) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    x[(size_t)t * N + i] = mk<C>(0, 0);
}

// Flag every unfinished system for a final true-residual evaluation.
__global__ void k_mark_unfinished(TxState *st, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  if (st[t].status == ST_ITER || st[t].status == ST_PAUSED) st[t].flags = FLAG_TR;
}

// Number of open (iterating or paused) systems: one wave, strided count then
// a wave reduction.
__global__ void __launch_bounds__(64) k_count_open(const TxState *st, int T, int *count) {
  double c = 0.0;
  for (int t = threadIdx.x; t < T; t += 64) c += (st[t].status == ST_ITER || st[t].status == ST_PAUSED) ? 1.0 : 0.0;
  c = wave_sum(c);
  if (threadIdx.x == 0) *count = (int)c;
}

template <typename C> void launch_fill(hipStream_t s, C *x, size_t n, C v) {
  hipLaunchKernelGGL(k_fill<C>, dim3(std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0, s, x, n, v);
}
template <typename C> void launch_copy(hipStream_t s, C *d, const C *src, size_t n) {
  hipLaunchKernelGGL(k_copy<C>, dim3(std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0, s, d, src, n);
}
template void launch_fill<cf>(hipStream_t, cf *, size_t, cf);
template void launch_fill<cd>(hipStream_t, cd *, size_t, cd);
template void launch_fill<float>(hipStream_t, float *, size_t, float);
template void launch_fill<double>(hipStream_t, double *, size_t, double);
template void launch_copy<cf>(hipStream_t, cf *, const cf *, size_t);
template void launch_copy<cd>(hipStream_t, cd *, const cd *, size_t);
template void launch_copy<float>(hipStream_t, float *, const float *, size_t);
template void launch_copy<double>(hipStream_t, double *, const double *, size_t);

template <typename R> void fill_tables(Ctx &c, const cplx_t<R> *&G, const cplx_t<R> *&tw, cplx_t<R> *&X1, cplx_t<R> *&X2);

int solve_shared_init(SolveShared &sh, int max_jobs) {
  sh.max_jobs = max_jobs;
  if (hipMalloc((void **)&sh.d_count, sizeof(int) * max_jobs) != hipSuccess) return CISOR_E_NOMEM;
  if (hipHostMalloc((void **)&sh.h_pinned, sizeof(int) * max_jobs) != hipSuccess) return CISOR_E_NOMEM;
  if (max_jobs > 1) {
    if (hipEventCreateWithFlags(&sh.ev_fork, hipEventDisableTiming) != hipSuccess) return CISOR_E_DEVICE;
    sh.ev_join.assign(max_jobs, nullptr);
    for (auto &e : sh.ev_join)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CISOR_E_DEVICE;
  }
  return CISOR_OK;
}

void solve_shared_free(SolveShared &sh) {
  for (int i = 0; i < sh.n_graphs; ++i)
    if (sh.graphs[i].exec) (void)hipGraphExecDestroy(sh.graphs[i].exec);
  sh.n_graphs = 0;
  if (sh.cap_stream) (void)hipStreamDestroy(sh.cap_stream);
  if (sh.d_count) (void)hipFree(sh.d_count);
  if (sh.h_pinned) (void)hipHostFree(sh.h_pinned);
  if (sh.ev_fork) (void)hipEventDestroy(sh.ev_fork);
  for (auto e : sh.ev_join)
    if (e) (void)hipEventDestroy(e);
  sh = SolveShared{};
}

// True residual r = b - A x (storage in the field precision) computed in
// precision Rc: FP64 for every stop test; the field precision for the
// provisional residual that starts a solve from a caller's or first-Born guess.
template <typename R, typename Rc = double>
static int true_residual(Ctx &c, const R *f, const cplx_t<R> *b, const cplx_t<R> *x, cplx_t<R> *r,
                         cplx_t<R> *rhat, bool adjoint) {
  ConvArgs<R, Rc> a{};
  a.f = f;
  a.x = x;
  a.b = b;
  a.y = r;
  a.rhat = rhat;
  a.part = c.part;
  a.st = c.st;
  a.flag = FLAG_TR;
  fill_tables<Rc>(c, a.Ghat, a.tw, a.X1, a.X2);
  return launch_conv<R, Rc, PRO_X, EPI_TR>(c, a, adjoint);
}

// Start of one job: starting guess, fresh states, first true residual.
template <typename R>
static int job_start(SolveJob &j, bool adjoint, const cisor_ls_opts &o, int replace_every) {
  using C = cplx_t<R>;
  Ctx &c = *j.c;
  const R *f = (const R *)j.f;
  const C *b = (const C *)j.b;
  C *x = (C *)j.x;
  const size_t TN = (size_t)c.T * c.N;
  C *r = (C *)c.ws[0], *rhat = (C *)c.ws[1], *p = (C *)c.ws[2], *v = (C *)c.ws[3], *s = (C *)c.ws[4];
  int e;
  if (o.start == 0) {
    launch_fill<C>(c.stream, x, TN, mk<C>(0, 0));
  } else if (o.start == 1) {
    launch_copy<C>(c.stream, x, b, TN);
  } else if (o.start == 3) {
    // per system: the caller's guess or the first-Born guess, whichever has
    // the smaller FP64 true residual
    hipLaunchKernelGGL(k_init_state, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.T);
    if ((e = true_residual<R>(c, f, b, x, r, rhat, adjoint))) return e;
    hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_TR, o.tol,
                       replace_every, o.maxit);
    hipLaunchKernelGGL(k_save_rel, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.rel_tmp, c.T);
    launch_copy<C>(c.stream, s, b, TN);
    hipLaunchKernelGGL(k_init_state, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.T);
    if ((e = true_residual<R>(c, f, b, s, r, rhat, adjoint))) return e;
    hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_TR, o.tol,
                       replace_every, o.maxit);
    hipLaunchKernelGGL(k_pick_start<C>, dim3((c.N + 255) / 256, c.T), dim3(256), 0, c.stream, c.st, c.rel_tmp, x, b,
                       c.start_choice, c.N);
  }
  // p and v need no initial values: the first iteration (beta = 0) forms
  // p = r without reading them
  hipLaunchKernelGGL(k_init_state, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.T);
  // the starting residual only seeds the recurrence: computed in the field
  // precision, and a system it shows as converged waits for the FP64 check
  if ((e = true_residual<R, R>(c, f, b, x, r, rhat, adjoint))) return e;
  hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_TR0, o.tol,
                     replace_every, o.maxit);
  if (o.start == 5) {
    hipLaunchKernelGGL(k_zero_fallback<C>, dim3((c.N + 255) / 256, c.T), dim3(256), 0, c.stream, c.st, x, r, rhat, b,
                       c.N);
    hipLaunchKernelGGL(k_zero_fallback_state, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.start_choice,
                       c.T);
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

// `count` BiCGSTAB iterations of one job, then (check) the FP64 true residual
// of the systems that asked for it and the count of open systems into
// *d_count.  Which systems work is decided on the device, so the launch
// sequence is static and can be captured.
template <typename R>
static int job_chunk(SolveJob &j, bool adjoint, const cisor_ls_opts &o, int replace_every, int count, bool last,
                     int *d_count) {
  using C = cplx_t<R>;
  Ctx &c = *j.c;
  const R *f = (const R *)j.f;
  const C *b = (const C *)j.b;
  C *x = (C *)j.x;
  C *r = (C *)c.ws[0], *rhat = (C *)c.ws[1], *p = (C *)c.ws[2], *v = (C *)c.ws[3], *s = (C *)c.ws[4],
    *tv = (C *)c.ws[5];
  ConvArgs<R, R> aA{}, aB{};
  fill_tables<R>(c, aA.Ghat, aA.tw, aA.X1, aA.X2);
  aA.f = f;
  aA.r = r;
  aA.p = p;
  aA.v = v;
  aA.s = s;
  aA.tt = tv;
  aA.xw = x;
  aA.y = v;
  aA.rhat = rhat;
  aA.part = c.part;
  aA.st = c.st;
  aA.flag = FLAG_ITER;
  aB = aA;
  aB.xw = nullptr;
  aB.y = tv;
  const dim3 gupd(c.nub, c.T);
  int e;
  for (int i = 0; i < count; ++i) {
    if ((e = launch_conv<R, R, PRO_PUPD, EPI_V>(c, aA, adjoint))) return e;
    hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_ALPHA, o.tol,
                       replace_every, o.maxit);
    if ((e = launch_conv<R, R, PRO_SUPD, EPI_T>(c, aB, adjoint))) return e;
    hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_OMEGA, o.tol,
                       replace_every, o.maxit);
  }
  if (last) hipLaunchKernelGGL(k_mark_unfinished, dim3((c.T + 63) / 64), dim3(64), 0, c.stream, c.st, c.T);
  hipLaunchKernelGGL(k_apply_pending<R>, gupd, dim3(UPD_THREADS), 0, c.stream, c.st, x, (const cplx_t<R> *)p,
                     (const cplx_t<R> *)s, c.N);
  if ((e = true_residual<R>(c, f, b, x, r, rhat, adjoint))) return e;
  hipLaunchKernelGGL(k_scalar, dim3(c.T), dim3(64), 0, c.stream, c.st, c.part, c.nrb, (int)STG_TR, o.tol,
                     replace_every, o.maxit);
  hipLaunchKernelGGL(k_count_open, dim3(1), dim3(64), 0, c.stream, c.st, c.T, d_count);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template <typename R>
int solve_multi(SolveJob *jobs, int nj, SolveShared &sh, hipStream_t main, bool adjoint, const cisor_ls_opts &o) {
  using C = cplx_t<R>;
  if (nj < 1 || nj > sh.max_jobs) return CISOR_E_ARG;
  const int replace_every = o.replace_every > 0 ? o.replace_every : 50;
  const int check_every = o.check_every > 0 ? o.check_every : 10;
  auto stream_of = [&](int k) { return jobs[k].c->stream; };
  // Jobs on streams other than `main` (grouped problems) count their open
  // systems after the start and the host reads the counts before the first
  // chunk, so no capture begins while a forked stream still holds work from
  // outside it.  A single-stream solve starts its first chunk at once.
  bool forked = false;
  for (int k = 0; k < nj; ++k) {
    forked |= (stream_of(k) != main);
    jobs[k].dir = adjoint ? 1 : 0;
  }
  int rc = fork_join(sh, main, nj, stream_of, [&](int k) -> int {
    const int e = job_start<R>(jobs[k], adjoint, o, replace_every);
    if (e || !forked) return e;
    Ctx &c = *jobs[k].c;
    hipLaunchKernelGGL(k_count_open, dim3(1), dim3(64), 0, c.stream, c.st, c.T, sh.d_count + k);
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  });
  if (rc) return rc;
  int it = 0, past_hint = 0;
  for (bool first = !forked;; first = false) {
    // a single-stream first chunk runs without asking the device (a job with
    // nothing open only launches masked kernels); after that the open counts
    // written at the end of each chunk decide
    std::vector<int> act;
    if (first) {
      for (int k = 0; k < nj; ++k) act.push_back(k);
    } else {
      CISOR_HIP_CHECK(hipMemcpyAsync(sh.h_pinned, sh.d_count, sizeof(int) * nj, hipMemcpyDeviceToHost, main));
      CISOR_HIP_CHECK(hipStreamSynchronize(main));
      for (int k = 0; k < nj; ++k)
        if (sh.h_pinned[k] > 0) act.push_back(k);
    }
    if (act.empty() || it >= o.maxit) break;
    // Solves along a FISTA path need similar counts, so the first chunk is cut
    // to one iteration more than the last solve of the same kind needed, and a
    // solve that runs past that count usually needs only an iteration or two
    // more (typically after its FP64 check fails): its further chunks grow as
    // 2, 4, 8 iterations up to check_every, so that few iterations of a chunk
    // run masked once every system has finished.  Without a count to go by,
    // chunks have check_every iterations.
    int hint = 0;
    for (int k : act) hint = std::max(hint, jobs[k].c->ls_hint[adjoint ? 1 : 0]);
    int want = check_every;
    if (hint > 0 && it <= hint) want = std::max(2, std::min(check_every, hint + 1 - it));
    else if (hint > 0) want = std::min(check_every, 2 << std::min(past_hint++, 3));
    const int chunk = std::min(want, o.maxit - it);
    const bool last = it + chunk >= o.maxit;
    const int na = (int)act.size();
    auto run = [&](hipStream_t m) {
      // the graph only knows the active jobs, so their streams are read here
      std::vector<hipStream_t> str(na);
      for (int a = 0; a < na; ++a) str[a] = (jobs[act[a]].c->stream == main) ? m : jobs[act[a]].c->stream;
      return fork_join(sh, m, na, [&](int a) { return str[a]; }, [&](int a) -> int {
        const int k = act[a];
        Ctx &c = *jobs[k].c;
        hipStream_t saved = c.stream;
        c.stream = str[a];
        const int e = job_chunk<R>(jobs[k], adjoint, o, replace_every, chunk, last, sh.d_count + k);
        c.stream = saved;
        return e;
      });
    };
    int g = 1;
    if (!last) {
      GraphKey key;
      for (int k : act) {
        key.ptrs.push_back(jobs[k].c);
        key.ptrs.push_back(jobs[k].f);
        key.ptrs.push_back(jobs[k].b);
        key.ptrs.push_back(jobs[k].x);
        key.ptrs.push_back(jobs[k].c->frow);
        key.ptrs.push_back(jobs[k].c->stream);
        key.vals.push_back((double)jobs[k].c->col_variant);
      }
      key.ptrs.push_back(sh.d_count);
      key.vals.insert(key.vals.end(), {adjoint ? 1.0 : 0.0, (double)chunk, o.tol, (double)replace_every,
                                       (double)o.maxit});
      std::vector<Ctx *> ctxs;
      for (int k : act) ctxs.push_back(jobs[k].c);
      g = graph_run(sh, key, main, ctxs, run);
      if (g < 0) return g;
    }
    if (g == 1 && (rc = run(main))) return rc;
    it += chunk;
  }
  // zero solutions of zero right-hand sides; read the states back
  std::vector<std::vector<TxState>> hs(nj);
  rc = fork_join(sh, main, nj, stream_of, [&](int k) -> int {
    Ctx &c = *jobs[k].c;
    hipLaunchKernelGGL(k_zero_solved<C>, dim3((c.N + 255) / 256, c.T), dim3(256), 0, c.stream, c.st,
                       (C *)jobs[k].x, c.N);
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  });
  if (rc) return rc;
  // final states: into the callers' pinned buffers without waiting (the
  // caller synchronises and calls solve_collect), or read back here
  bool defer = true;
  for (int k = 0; k < nj; ++k) defer = defer && jobs[k].host_states;
  for (int k = 0; k < nj; ++k) {
    TxState *dst = jobs[k].host_states;
    if (!dst) {
      hs[k].resize(jobs[k].c->T);
      dst = hs[k].data();
    }
    CISOR_HIP_CHECK(hipMemcpyAsync(dst, jobs[k].c->st, sizeof(TxState) * jobs[k].c->T, hipMemcpyDeviceToHost, main));
  }
  if (defer) return CISOR_OK;
  CISOR_HIP_CHECK(hipStreamSynchronize(main));
  int worst = CISOR_OK;
  for (int k = 0; k < nj; ++k) {
    const int status = solve_collect(jobs[k], jobs[k].host_states ? jobs[k].host_states : hs[k].data());
    if (status < 0 && worst >= 0) worst = status;
    else if (status == CISOR_NOT_CONVERGED && worst == CISOR_OK) worst = status;
  }
  return worst;
}

int solve_collect(SolveJob &j, const TxState *hs) {
  int status = CISOR_OK;
  double mr = 0.0;
  int most = 0;
  for (int t = 0; t < j.c->T; ++t) {
    const TxState &st = hs[t];
    if (j.iters) j.iters[t] = st.iters;
    most = std::max(most, st.iters);
    if (st.status == ST_FAILED) status = CISOR_E_NONFINITE;
    else if (st.status != ST_DONE && status == CISOR_OK) status = CISOR_NOT_CONVERGED;
    if (std::isfinite(st.true_rel)) mr = std::max(mr, st.true_rel);
  }
  j.status = status;
  j.max_rel = mr;
  j.c->ls_hint[j.dir] = most;
  return status;
}

template <typename R>
int solve_batch(Ctx &c, const R *f, const cplx_t<R> *b, cplx_t<R> *x, bool adjoint, const cisor_ls_opts &o,
                int *iters_host, double *max_rel) {
  SolveJob j;
  j.c = &c;
  j.f = f;
  j.b = b;
  j.x = x;
  j.iters = iters_host;
  const int rc = solve_multi<R>(&j, 1, c.sh, c.stream, adjoint, o);
  if (max_rel) *max_rel = j.max_rel;
  return rc;
}

template int solve_batch<float>(Ctx &, const float *, const cf *, cf *, bool, const cisor_ls_opts &, int *, double *);
template int solve_batch<double>(Ctx &, const double *, const cd *, cd *, bool, const cisor_ls_opts &, int *,
                                 double *);
template int solve_multi<float>(SolveJob *, int, SolveShared &, hipStream_t, bool, const cisor_ls_opts &);
template int solve_multi<double>(SolveJob *, int, SolveShared &, hipStream_t, bool, const cisor_ls_opts &);

}  // namespace cisor
