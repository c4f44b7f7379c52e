// Monotone accelerated proximal gradient (Li and Lin, NIPS 2015): the
// comparison method of the paper's "Proposed Method" section, built from the
// same kernels as the relaxed-FISTA step so the two can be compared in
// forward solves and time.
//
// One iteration (t_0 = 0, t_1 = 1, x_0 = x_1 = z_1):
//   y_k     = x_k + (t_{k-1}/t_k)(z_k - x_k) + ((t_{k-1} - 1)/t_k)(x_k - x_{k-1})
//   z_{k+1} = prox_{a_y R}(y_k - a_y grad D(y_k))           (accelerated estimate)
//   v_{k+1} = prox_{a_x R}(x_k - a_x grad D(x_k))           (proximal-gradient estimate)
//   x_{k+1} = z_{k+1} if F(z_{k+1}) <= F(v_{k+1}) else v_{k+1},   F = D + tau TV
// so each iteration needs two gradients (forward and adjoint solves at y_k
// and x_k) and the objective at two points (forward solves at z_{k+1} and
// v_{k+1}).  Every solve starts from the closest fields at hand: the gradient
// at x_k from the fields of the objective evaluation that selected x_k.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace cisor {

namespace {

template <typename R>
__global__ void __launch_bounds__(256) k_apg_extrap(const R *x, const R *z, const R *xp, R *y, int N, double a,
                                                    double b) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const double xv = (double)x[q];
  y[q] = (R)(xv + a * ((double)z[q] - xv) + b * (xv - (double)xp[q]));
}

template <typename R>
__global__ void __launch_bounds__(256) k_apg_step(const R *x, const R *g, R *w, int N, double gamma) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  w[q] = (R)((double)x[q] - gamma * (double)g[q]);
}

int dalloc_bytes(void *&p, size_t bytes) {
  if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
    p = nullptr;
    return CISOR_E_NOMEM;
  }
  return CISOR_OK;
}

struct SolveTally {
  int fwd = 0, adj = 0;
  long long fwd_iters = 0, adj_iters = 0;
  double max_rel = 0.0;
  int worst = CISOR_OK;
  void add(int st) {
    if (st < 0 && worst >= 0) worst = st;
    else if (st == CISOR_NOT_CONVERGED && worst == CISOR_OK) worst = st;
  }
};

// F(x) = D(x) + tau TV(x) with the forward fields solved into u (u holds the
// starting guess on entry).
template <typename R>
int objective(Ctx &c, const R *x, const cplx_t<R> *y_meas, cplx_t<R> *u, double tau, const cisor_ls_opts &o,
              SolveTally &tally, double *F) {
  std::vector<int> its(c.T, 0);
  double mr = 0.0;
  const int st = solve_batch<R>(c, x, (const cplx_t<R> *)c.uin, u, false, o, its.data(), &mr);
  if (st < 0) return st;
  tally.add(st);
  tally.fwd += 1;
  for (int v : its) tally.fwd_iters += v;
  tally.max_rel = std::max(tally.max_rel, mr);
  double D = 0.0, tv = 0.0;
  int rc = launch_project<R>(c, x, u, y_meas, (cplx_t<R> *)c.W, &D);
  if (rc || (rc = launch_tv_value<R>(c, x, &tv))) return rc;
  *F = D + tau * tv;
  return CISOR_OK;
}

template <typename R>
int gradient(Ctx &c, const R *x, const cplx_t<R> *y_meas, R *g, const cisor_ls_opts &o, SolveTally &tally,
             double *D) {
  std::vector<int> its(2 * c.T, 0);
  double mr = 0.0;
  int st = CISOR_OK;
  const int rc = launch_grad<R>(c, x, y_meas, g, D, (cplx_t<R> *)c.U, (cplx_t<R> *)c.V, o, its.data(), &mr, &st);
  if (rc) return rc;
  tally.add(st);
  tally.fwd += 1;
  tally.adj += 1;
  for (int t = 0; t < c.T; ++t) {
    tally.fwd_iters += its[t];
    tally.adj_iters += its[c.T + t];
  }
  tally.max_rel = std::max(tally.max_rel, mr);
  return CISOR_OK;
}

template <typename R>
int apg_step(Ctx &c, cisor_apg_state *s, const cplx_t<R> *y_meas, double gy, double gx, double tau, double lo,
             double hi, int inner, const cisor_ls_opts &o, cisor_apg_info *info) {
  using C = cplx_t<R>;
  const int N = c.N;
  const size_t TN = (size_t)c.T * N;
  R *buf = (R *)c.apg_buf;
  R *y = buf, *g = buf + N, *w = buf + 2 * (size_t)N, *zn = buf + 3 * (size_t)N, *vn = buf + 4 * (size_t)N;
  C *A1 = (C *)c.apg_A1, *A2 = (C *)c.apg_A2, *U = (C *)c.U, *V = (C *)c.V;
  R *x = (R *)s->x, *xp = (R *)s->x_prev, *z = (R *)s->z;
  const dim3 grid((N + 255) / 256), blk(256);
  if (s->k == 0) c.apg_fields = 0;
  // starting guesses of a run's first gradient: the context's last fields
  // (start 2, when there are any), else first-Born (or zero) forward, zero adjoint
  if (!c.fields_valid || (s->k == 0 && o.start != 2)) {
    if (o.start == 0) launch_fill<C>(c.stream, U, TN, mk<C>(0, 0));
    else launch_copy<C>(c.stream, U, (const C *)c.uin, TN);
    launch_fill<C>(c.stream, V, TN, mk<C>(0, 0));
  }
  cisor_ls_opts w2 = o;
  w2.start = 2;
  SolveTally tally;
  double D_y = 0.0, D_x = 0.0, F_z = 0.0, F_v = 0.0;
  // y_k and the accelerated estimate
  hipLaunchKernelGGL(k_apg_extrap<R>, grid, blk, 0, c.stream, x, z, xp, y, N, s->t_prev / s->t,
                     (s->t_prev - 1.0) / s->t);
  int rc = gradient<R>(c, y, y_meas, g, w2, tally, &D_y);
  if (rc) return rc;
  c.fields_valid = true;
  hipLaunchKernelGGL(k_apg_step<R>, grid, blk, 0, c.stream, y, g, w, N, gy);
  if ((rc = launch_tv_prox<R>(c, w, zn, gy * tau, lo, hi, inner))) return rc;
  // the proximal-gradient estimate from x_k (forward fields of x_k when known)
  if (c.apg_fields == 1) launch_copy<C>(c.stream, U, A1, TN);
  else if (c.apg_fields == 2) launch_copy<C>(c.stream, U, A2, TN);
  if ((rc = gradient<R>(c, x, y_meas, g, w2, tally, &D_x))) return rc;
  hipLaunchKernelGGL(k_apg_step<R>, grid, blk, 0, c.stream, x, g, w, N, gx);
  if ((rc = launch_tv_prox<R>(c, w, vn, gx * tau, lo, hi, inner))) return rc;
  // objective at both estimates, each solve started from the fields at x_k
  launch_copy<C>(c.stream, A1, U, TN);
  launch_copy<C>(c.stream, A2, U, TN);
  if ((rc = objective<R>(c, zn, y_meas, A1, tau, w2, tally, &F_z))) return rc;
  if ((rc = objective<R>(c, vn, y_meas, A2, tau, w2, tally, &F_v))) return rc;
  const bool took_z = F_z <= F_v;
  launch_copy<R>(c.stream, xp, x, (size_t)N);
  launch_copy<R>(c.stream, x, took_z ? zn : vn, (size_t)N);
  launch_copy<R>(c.stream, z, zn, (size_t)N);
  c.apg_fields = took_z ? 1 : 2;
  const double tn = (std::sqrt(4.0 * s->t * s->t + 1.0) + 1.0) / 2.0;
  s->t_prev = s->t;
  s->t = tn;
  s->k += 1;
  CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  if (info) {
    info->F = std::min(F_z, F_v);
    info->F_z = F_z;
    info->F_v = F_v;
    info->D_y = D_y;
    info->D_x = D_x;
    info->took_z = took_z ? 1 : 0;
    info->fwd_solves = tally.fwd;
    info->adj_solves = tally.adj;
    info->fwd_iters_sum = tally.fwd_iters;
    info->adj_iters_sum = tally.adj_iters;
    info->max_true_relres = tally.max_rel;
    info->status = tally.worst;
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

}  // namespace

}  // namespace cisor

using namespace cisor;

extern "C" int cisor_apg_step(cisor_ctx *h, cisor_apg_state *s, const void *y_meas, double gamma_y, double gamma_x,
                              double tau, double lo, double hi, int inner, const cisor_ls_opts *o,
                              cisor_apg_info *info) {
  if (!h || !s || !s->x || !s->x_prev || !s->z || !y_meas || !(gamma_y > 0) || !(gamma_x > 0) || !(tau >= 0) ||
      !(lo <= hi) || inner < 0 || !o || !(o->tol > 0.0) || !std::isfinite(o->tol) || o->maxit < 1 ||
      o->start < 0 || o->start > 2 || o->replace_every < 0 || o->check_every < 0 || !(s->t >= 1.0) ||
      !(s->t_prev >= 0.0) || s->k < 0)
    return CISOR_E_ARG;
  Ctx &c = *ctx_of(h);
  const size_t rs = c.precision ? sizeof(double) : sizeof(float), cs = 2 * rs;
  const size_t TN = (size_t)c.T * c.N;
  if (!c.apg_buf) {
    int rc;
    if ((!c.apg_A1 && (rc = dalloc_bytes(c.apg_A1, cs * TN))) || (!c.apg_A2 && (rc = dalloc_bytes(c.apg_A2, cs * TN))) ||
        (rc = dalloc_bytes(c.apg_buf, rs * 5 * (size_t)c.N)))   // allocated last: its presence means all three are
      return rc;
    c.apg_fields = 0;
  }
  if (c.precision == 0)
    return apg_step<float>(c, s, (const cf *)y_meas, gamma_y, gamma_x, tau, lo, hi, inner, *o, info);
  return apg_step<double>(c, s, (const cd *)y_meas, gamma_y, gamma_x, tau, lo, hi, inner, *o, info);
}
