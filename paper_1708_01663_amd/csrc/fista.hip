// Prop. 1 gradient orchestration and the relaxed-FISTA step (eqs. algo1-algo3).
//
// grad D(f) = sum_t Re{ conj(u_t) (H^H w_t + G^H v_t) } with A u_t = u_in,t and
// A^H v_t = diag(f) H^H w_t (eqs. gradient, u_and_v).  The G^H v_t
// convolution reuses the FFT stages; its epilogue forms the per-transmitter
// term Re{conj(u_t)(q_t + G^H v_t)}, and a last kernel sums the transmitters
// in FP64.
#include <cmath>
#include <random>
#include <vector>

#include "internal.hpp"

namespace cisor {

template <typename R> void fill_tables(Ctx &c, const cplx_t<R> *&G, const cplx_t<R> *&tw, cplx_t<R> *&X1, cplx_t<R> *&X2);

// grad[q] = sum_t gpart[t][q]  (FP64 accumulation, fixed order)
template <typename R> __global__ void k_sum_over_tx(const R *gpart, R *grad, int N, int T) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  // eight rows are requested together so that their loads overlap; the sum
  // keeps the row order
  double s = 0.0;
  int t = 0;
  for (; t + 8 <= T; t += 8) {
    R g[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = gpart[(size_t)(t + i) * N + q];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += (double)g[i];
  }
  for (; t < T; ++t) s += (double)gpart[(size_t)t * N + q];
  grad[q] = (R)s;
}

// out[q] = sum_t Re{conj(u_t[q]) q_t[q]} (FP64 accumulation)
template <typename R>
__global__ void k_re_conj_sum(const cplx_t<R> *u, const cplx_t<R> *qv, double *out, int N, int T) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  double s = 0.0;
  for (int t = 0; t < T; ++t) {
    const cplx_t<R> a = u[(size_t)t * N + q], b = qv[(size_t)t * N + q];
    s += (double)a.x * b.x + (double)a.y * b.y;
  }
  out[q] = s;
}

// z = s - gamma g
template <typename R> __global__ void k_grad_step(const R *s, const R *g, R *z, int N, R gamma) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < N) z[q] = s[q] - gamma * g[q];
}

// s = fk + w (fk - f); f_prev = f; f = fk
template <typename R> __global__ void k_momentum(const R *fk, R *f, R *f_prev, R *s, int N, R w) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const R a = fk[q], b = f[q];
  s[q] = a + w * (a - b);
  f_prev[q] = b;
  f[q] = a;
}

// Momentum with the FISTA scalar on the device: t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,
// s = fk + alpha (t_k - 1)/t_{k+1} (fk - f); f_prev = f; f = fk.  t is
// advanced by k_advance_t after every block has read it.
template <typename R>
__global__ void k_momentum_dev(const R *fk, R *f, R *f_prev, R *s, int N, const double *t_dev, double alpha) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const double tk = t_dev[0];
  const double tn = (1.0 + sqrt(1.0 + 4.0 * tk * tk)) / 2.0;
  const R w = (R)(alpha * (tk - 1.0) / tn);
  const R a = fk[q], b = f[q];
  s[q] = a + w * (a - b);
  f_prev[q] = b;
  f[q] = a;
}
__global__ void k_advance_t(double *t_dev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double tk = t_dev[0];
    t_dev[0] = (1.0 + sqrt(1.0 + 4.0 * tk * tk)) / 2.0;
  }
}

// Vector-Jacobian product of the data map f -> y_t = H diag(u_t) f, u_t = A^{-1} u_in,t
// (the proof of Prop. 1 with w := the data-space cotangent):
//   q_t = H^H w_t ; A^H v_t = f q_t ; out = sum_t Re{conj(u_t) (q_t + G^H v_t)}.
// The adjoint half of the gradient.  With `deferred`, the adjoint solve's final
// states go to pinned host memory without a synchronisation and the caller
// collects them (status and max_rel are then left untouched).
template <typename R>
static int vjp_impl(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *w, R *grad, cplx_t<R> *v,
                    const cisor_ls_opts &o, int *iters, double *max_rel, int *status, SolveJob *deferred) {
  using C = cplx_t<R>;
  int rc;
  C *Q = (C *)c.Q, *Bv = (C *)c.Bv;
  if ((rc = launch_backproject<R>(c, w, Q, f, Bv))) return rc;
  int st = CISOR_OK;
  if (deferred) {
    deferred->c = &c;
    deferred->f = f;
    deferred->b = Bv;
    deferred->x = v;
    deferred->iters = iters;
    deferred->host_states = c.h_states + c.T;
    if ((st = solve_multi<R>(deferred, 1, c.sh, c.stream, true, o)) < 0) return st;
  } else {
    st = solve_batch<R>(c, f, Bv, v, true, o, iters, max_rel);
    if (st < 0) return st;
  }
  ConvArgs<R, R> a{};
  fill_tables<R>(c, a.Ghat, a.tw, a.X1, a.X2);
  a.x = v;
  a.u = u;
  a.q = Q;
  a.gpart = (R *)c.gpart;
  if ((rc = launch_conv<R, R, PRO_X, EPI_GRAD>(c, a, true))) return rc;
  hipLaunchKernelGGL(k_sum_over_tx<R>, dim3((c.N + 255) / 256), dim3(256), 0, c.stream, (const R *)c.gpart, grad,
                     c.N, c.T);
  if (status && !deferred) *status = st;
  CISOR_HIP_CHECK(hipGetLastError());
  return CISOR_OK;
}

template <typename R>
int launch_vjp(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *w, R *grad, cplx_t<R> *v,
               const cisor_ls_opts &o, int *iters, double *max_rel, int *status) {
  return vjp_impl<R>(c, f, u, w, grad, v, o, iters, max_rel, status, nullptr);
}

template <typename R>
int launch_grad(Ctx &c, const R *f, const cplx_t<R> *y_meas, R *grad, double *D, cplx_t<R> *u, cplx_t<R> *v,
                const cisor_ls_opts &o, int *iters, double *max_rel, int *worst_status) {
  using C = cplx_t<R>;
  int rc;
  // forward solves  A u_t = u_in,t (final states read back at the end)
  SolveJob jf, ja;
  jf.c = &c;
  jf.f = f;
  jf.b = c.uin;
  jf.x = u;
  jf.iters = iters;
  jf.host_states = c.h_states;
  if ((rc = solve_multi<R>(&jf, 1, c.sh, c.stream, false, o)) < 0) return rc;
  // w = H diag(u) f - y_meas, D (device slot, copied back at the end)
  C *W = (C *)c.W;
  if ((rc = launch_project<R>(c, f, u, y_meas, W, nullptr, c.d_D))) return rc;
  CISOR_HIP_CHECK(hipMemcpyAsync(c.h_D, c.d_D, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  // adjoint solves and the gradient terms
  if ((rc = vjp_impl<R>(c, f, u, W, grad, v, o, iters ? iters + c.T : nullptr, nullptr, nullptr, &ja))) return rc;
  // the one synchronisation of the gradient evaluation
  CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  const int st_f = solve_collect(jf, c.h_states);
  const int st_a = solve_collect(ja, c.h_states + c.T);
  if (D) *D = *c.h_D;
  if (max_rel) *max_rel = std::max(jf.max_rel, ja.max_rel);
  if (worst_status) *worst_status = (st_f < 0) ? st_f : (st_a < 0 ? st_a : (st_f != CISOR_OK ? st_f : st_a));
  return CISOR_OK;
}

template <typename R>
int launch_fista_tail(Ctx &c, cisor_fista_state *s, const R *grad, double gamma, double tau, double alpha, double lo,
                      double hi, int inner) {
  const int N = c.N;
  R *z = (R *)c.zbuf;
  R *fk = z + N;
  const dim3 g((N + 255) / 256), b(256);
  hipLaunchKernelGGL(k_grad_step<R>, g, b, 0, c.stream, (const R *)s->s, grad, z, N, (R)gamma);
  int rc = launch_tv_prox<R>(c, z, fk, gamma * tau, lo, hi, inner);
  if (rc) return rc;
  const double tk = s->t;
  const double tn = (std::sqrt(4.0 * tk * tk + 1.0) + 1.0) / 2.0;
  const double w = alpha * (tk - 1.0) / tn;
  hipLaunchKernelGGL(k_momentum<R>, g, b, 0, c.stream, (const R *)fk, (R *)s->f, (R *)s->f_prev, (R *)s->s, N, (R)w);
  s->t = tn;
  s->k += 1;
  CISOR_HIP_CHECK(hipGetLastError());
  return CISOR_OK;
}

template <typename R>
int launch_fista_tail_dev(Ctx &c, R *f, R *f_prev, R *s, const R *grad, double *t_dev, double gamma, double tau,
                          double alpha, double lo, double hi, int inner) {
  const int N = c.N;
  R *z = (R *)c.zbuf;
  R *fk = z + N;
  const dim3 g((N + 255) / 256), b(256);
  hipLaunchKernelGGL(k_grad_step<R>, g, b, 0, c.stream, (const R *)s, grad, z, N, (R)gamma);
  int rc = launch_tv_prox<R>(c, z, fk, gamma * tau, lo, hi, inner);
  if (rc) return rc;
  hipLaunchKernelGGL(k_momentum_dev<R>, g, b, 0, c.stream, (const R *)fk, f, f_prev, s, N, (const double *)t_dev,
                     alpha);
  hipLaunchKernelGGL(k_advance_t, dim3(1), dim3(64), 0, c.stream, t_dev);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

// ---- extrapolated starting guesses along the FISTA path ----
// The solves at s_k start from u(s_{k-1}) + theta (u(s_{k-1}) - u(s_{k-2}))
// (likewise the adjoint fields), theta = <s_k - s_{k-1}, s_{k-1} - s_{k-2}> /
// ||s_{k-1} - s_{k-2}||^2: the secant through the last two evaluation points,
// evaluated where the projection of the new step onto the last one lands.
// Any start gives the same solution (the stop test is on the true residual);
// this one only shortens the solves.
constexpr int EXTRAP_BLOCKS = 128;
constexpr double EXTRAP_THETA_MAX = 2.0;

// FP64 partial sums of <s - s1, s1 - s2> and ||s1 - s2||^2 per block.
template <typename R>
__global__ void __launch_bounds__(256) k_extrap_part(const R *s, const R *s1, const R *s2, int N, double *part) {
  __shared__ double scratch[2 * 16];
  double v[2] = {0.0, 0.0};
  for (int q = blockIdx.x * 256 + threadIdx.x; q < N; q += EXTRAP_BLOCKS * 256) {
    const double a = (double)s1[q];
    const double d0 = (double)s[q] - a, d1 = a - (double)s2[q];
    v[0] += d0 * d1;
    v[1] += d1 * d1;
  }
  block_sum<2>(v, scratch);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

// theta from the partials, clamped to [0, EXTRAP_THETA_MAX] (0 when the last
// step was empty or a sum is not finite).
__global__ void __launch_bounds__(64) k_extrap_theta(const double *part, double *theta) {
  double num = 0.0, den = 0.0;
  for (int b = threadIdx.x; b < EXTRAP_BLOCKS; b += 64) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (threadIdx.x == 0) {
    double th = den > 0.0 ? num / den : 0.0;
    if (!std::isfinite(th)) th = 0.0;
    *theta = fmin(fmax(th, 0.0), EXTRAP_THETA_MAX);
  }
}

// x <- x + theta (x - x2), x2 <- old x, for the forward and the adjoint fields
// (blockIdx.y selects which); with theta == nullptr x2 <- x only (x2 may hold
// anything then, even non-finite values, and is not read).
// The first N threads of the forward half also shift the evaluation points:
// s2 <- s1, s1 <- s.
template <typename R>
__global__ void __launch_bounds__(256) k_extrap_fields(cplx_t<R> *u, cplx_t<R> *u2, cplx_t<R> *v, cplx_t<R> *v2,
                                                       const R *s, R *s1, R *s2, size_t TN, int N,
                                                       const double *theta) {
  using C = cplx_t<R>;
  const R th = theta ? (R)*theta : (R)0;
  C *x = blockIdx.y ? v : u;
  C *x2 = blockIdx.y ? v2 : u2;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < TN; i += stride) {
    const C a = x[i];
    if (theta) {
      const C b = x2[i];
      x[i] = mk<C>(a.x + th * (a.x - b.x), a.y + th * (a.y - b.y));
    }
    x2[i] = a;
    if (blockIdx.y == 0 && i < (size_t)N) {
      s2[i] = s1[i];
      s1[i] = s[i];
    }
  }
}

template <typename R> int launch_extrapolate(Ctx &c, const R *s, int depth) {
  using C = cplx_t<R>;
  const int N = c.N;
  R *s1 = (R *)c.S1, *s2 = (R *)c.S2;
  if (depth <= 0) {   // nothing recorded yet: remember the evaluation point only
    launch_copy<R>(c.stream, s1, s, N);
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  }
  double *theta = nullptr;
  if (depth >= 2) {
    hipLaunchKernelGGL(k_extrap_part<R>, dim3(EXTRAP_BLOCKS), dim3(256), 0, c.stream, s, (const R *)s1,
                       (const R *)s2, N, c.xpart);
    theta = c.xpart + 2 * EXTRAP_BLOCKS;
    hipLaunchKernelGGL(k_extrap_theta, dim3(1), dim3(64), 0, c.stream, (const double *)c.xpart, theta);
  }
  const size_t TN = (size_t)c.T * N;
  const unsigned gx = (unsigned)std::min<size_t>((TN + 255) / 256, 2048);
  hipLaunchKernelGGL(k_extrap_fields<R>, dim3(gx, 2), dim3(256), 0, c.stream, (C *)c.U, (C *)c.U2, (C *)c.V,
                     (C *)c.V2, s, s1, s2, TN, N, (const double *)theta);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template <typename R> int launch_sum_rows(Ctx &c, const R *gpart, R *grad, int rows) {
  hipLaunchKernelGGL(k_sum_over_tx<R>, dim3((c.N + 255) / 256), dim3(256), 0, c.stream, gpart, grad, c.N, rows);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template <typename R> int launch_born_lipschitz(Ctx &c, int iters, double *L) {
  using C = cplx_t<R>;
  const int N = c.N;
  std::mt19937_64 gen(0);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> hv(N), hw(N);
  double nrm = 0;
  for (int q = 0; q < N; ++q) {
    hv[q] = nd(gen);
    nrm += hv[q] * hv[q];
  }
  nrm = std::sqrt(nrm);
  for (auto &x : hv) x /= nrm;
  R *vdev = (R *)c.zbuf;
  double *wdev = (double *)c.gpart;  // N doubles fit in the [T][N] real buffer
  std::vector<R> hr(N);
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    for (int q = 0; q < N; ++q) hr[q] = (R)hv[q];
    CISOR_HIP_CHECK(hipMemcpyAsync(vdev, hr.data(), sizeof(R) * N, hipMemcpyHostToDevice, c.stream));
    int rc = launch_project<R>(c, vdev, (const C *)c.uin, nullptr, (C *)c.W, nullptr);
    if (rc) return rc;
    if ((rc = launch_backproject<R>(c, (const C *)c.W, (C *)c.Q, nullptr, nullptr))) return rc;
    hipLaunchKernelGGL(k_re_conj_sum<R>, dim3((N + 255) / 256), dim3(256), 0, c.stream, (const C *)c.uin,
                       (const C *)c.Q, wdev, N, c.T);
    CISOR_HIP_CHECK(hipMemcpyAsync(hw.data(), wdev, sizeof(double) * N, hipMemcpyDeviceToHost, c.stream));
    CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
    double vw = 0, ww = 0;
    for (int q = 0; q < N; ++q) {
      vw += hv[q] * hw[q];
      ww += hw[q] * hw[q];
    }
    lam = vw;
    if (ww == 0.0) break;
    const double inv = 1.0 / std::sqrt(ww);
    for (int q = 0; q < N; ++q) hv[q] = hw[q] * inv;
  }
  *L = lam;
  return CISOR_OK;
}

template int launch_extrapolate<float>(Ctx &, const float *, int);
template int launch_extrapolate<double>(Ctx &, const double *, int);
template int launch_grad<float>(Ctx &, const float *, const cf *, float *, double *, cf *, cf *,
                                const cisor_ls_opts &, int *, double *, int *);
template int launch_grad<double>(Ctx &, const double *, const cd *, double *, double *, cd *, cd *,
                                 const cisor_ls_opts &, int *, double *, int *);
template int launch_vjp<float>(Ctx &, const float *, const cf *, const cf *, float *, cf *, const cisor_ls_opts &,
                               int *, double *, int *);
template int launch_vjp<double>(Ctx &, const double *, const cd *, const cd *, double *, cd *,
                                const cisor_ls_opts &, int *, double *, int *);
template int launch_fista_tail<float>(Ctx &, cisor_fista_state *, const float *, double, double, double, double,
                                      double, int);
template int launch_fista_tail<double>(Ctx &, cisor_fista_state *, const double *, double, double, double, double,
                                       double, int);
template int launch_fista_tail_dev<float>(Ctx &, float *, float *, float *, const float *, double *, double, double,
                                          double, double, double, int);
template int launch_fista_tail_dev<double>(Ctx &, double *, double *, double *, const double *, double *, double,
                                           double, double, double, double, int);
template int launch_sum_rows<float>(Ctx &, const float *, float *, int);
template int launch_sum_rows<double>(Ctx &, const double *, double *, int);
template int launch_born_lipschitz<float>(Ctx &, int, double *);
template int launch_born_lipschitz<double>(Ctx &, int, double *);

}  // namespace cisor
