// C ABI of the CISOR library: argument validation, context lifetime, dispatch
// on the context precision.  No exception crosses this boundary.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "conv_cfg.hpp"
#include "internal.hpp"

using namespace cisor;

struct cisor_ctx {
  Ctx c;
};

namespace {

template <typename T> int dalloc(T *&p, size_t bytes) {
  void *q = nullptr;
  if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) return CISOR_E_NOMEM;
  p = (T *)q;
  return CISOR_OK;
}

void free_all(Ctx &c) {
  void *ptrs[] = {c.Ghat, c.tw, c.H, c.uin, c.Ghat_d, c.tw_d, c.Gpm, c.Gpm_d, c.X1, c.X2, c.X1d, c.X2d, c.part, c.st,
                  c.rel_tmp, c.start_choice,
                  c.U, c.V, c.Q, c.Bv, c.W, c.gpart, c.zbuf, c.tvbuf, c.gemm_part, c.dpart,
                  c.U2, c.V2, c.S1, c.S2, c.xpart, c.rx_mask, c.apg_A1, c.apg_A2, c.apg_buf,
                  c.ws[0], c.ws[1], c.ws[2], c.ws[3], c.ws[4], c.ws[5]};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  solve_shared_free(c.sh);
  if (c.d_D) (void)hipFree(c.d_D);
  if (c.h_states) (void)hipHostFree(c.h_states);
  if (c.h_D) (void)hipHostFree(c.h_D);
}

}  // namespace

Ctx *cisor::ctx_of(cisor_ctx *h) { return h ? &h->c : nullptr; }

// Plane waves need finite, non-zero directions; point sources finite positions
// strictly outside the grid's square (cube), so no cell centre meets a source.
bool cisor::transmitters_ok(const cisor_geometry &g) {
  const int D = g.dim;
  const double half = 0.5 * g.n * g.h;
  if (g.tx_kind != 0 && g.tx_kind != 1) return false;
  const double *v = g.tx_kind == 0 ? g.tx_dir : g.tx_pos;
  if (!v) return false;
  for (int t = 0; t < g.T; ++t) {
    double nrm = 0.0, outside = 0.0;
    for (int d = 0; d < D; ++d) {
      const double a = v[D * t + d];
      if (!std::isfinite(a)) return false;
      nrm += a * a;
      outside = std::max(outside, std::fabs(a) - half);
    }
    if (g.tx_kind == 0 ? nrm == 0.0 : !(outside > 0.0)) return false;
  }
  return true;
}

namespace {

// start modes 0-3 are valid for every solve; 4 (extrapolated) only for a FISTA step
// start modes 0-3 and 5 for every solve; 4 (extrapolated) only for a FISTA
// step, which takes no caller guess (so no 5 there)
bool opts_ok(const cisor_ls_opts *o, int max_start = 3) {
  return o && o->tol > 0.0 && std::isfinite(o->tol) && o->maxit >= 1 && o->start >= 0 &&
         (o->start <= max_start || (max_start == 3 && o->start == 5)) && o->replace_every >= 0 &&
         o->check_every >= 0;
}

}  // namespace

extern "C" {

const char *cisor_status_string(int s) {
  switch (s) {
    case CISOR_OK: return "ok";
    case CISOR_NOT_CONVERGED: return "not converged (iteration cap reached; outputs written)";
    case CISOR_E_ARG: return "invalid argument";
    case CISOR_E_NOMEM: return "device allocation failed";
    case CISOR_E_DEVICE: return "HIP runtime error";
    case CISOR_E_NONFINITE: return "non-finite value in an FP64 reduction";
    case CISOR_E_UNSUPPORTED: return "unsupported configuration (no compiled FFT length, or a mode this call lacks)";
    case CISOR_E_SIZE: return "problem larger than the static work area of a non-allocating call";
    default: return "unknown status";
  }
}

int cisor_create(const cisor_geometry *g, void *stream, cisor_ctx **out) {
  if (!g || !out) return CISOR_E_ARG;
  *out = nullptr;
  if ((g->dim != 2 && g->dim != 3) || g->n < 2 || !(g->h > 0) || !(g->wavelength > 0) || !(g->eps_b > 0) ||
      g->T < 1 || g->M < 1 || !g->rx_pos || (g->precision != 0 && g->precision != 1) || !transmitters_ok(*g))
    return CISOR_E_ARG;
  const int D = g->dim;
  for (int m = 0; m < D * g->M; ++m)
    if (!std::isfinite(g->rx_pos[m])) return CISOR_E_ARG;
  const int P = fft_length_for(g->n);
  if (P == 0) return CISOR_E_UNSUPPORTED;
  if (!fft_length_supported(P)) return CISOR_E_UNSUPPORTED;
  cisor_ctx *h = new (std::nothrow) cisor_ctx();
  if (!h) return CISOR_E_NOMEM;
  Ctx &c = h->c;
  c.dim = D;
  c.n = g->n;
  c.rows = D == 2 ? g->n : g->n * g->n;
  c.N = c.rows * g->n;
  c.P = P;
  c.T = g->T;
  c.M = g->M;
  c.precision = g->precision;
  c.h = g->h;
  c.k = 2.0 * 3.14159265358979323846 / g->wavelength;
  c.eps_b = g->eps_b;
  c.kb = c.k * std::sqrt(g->eps_b);
  c.stream = (hipStream_t)stream;
  if (const char *env = std::getenv("CISOR_GRAPHS")) c.sh.use_graphs = std::atoi(env) != 0;
  c.nrb = row_blocks(P, c.rows);
  c.nub = (c.N + UPD_THREADS * UPD_EPT - 1) / (UPD_THREADS * UPD_EPT);
  c.nblk = std::max(c.nrb, c.nub);
  const size_t rs = c.precision ? sizeof(double) : sizeof(float);
  const size_t cs = 2 * rs;
  const size_t TN = (size_t)c.T * c.N;
  // FFT intermediates per transmitter: n x P (2D), max(n^2 P, n P^2) = n P^2 (3D)
  const size_t inter = (size_t)c.T * c.n * P * (D == 3 ? P : 1);
  const size_t PD = (size_t)P * P * (D == 3 ? P : 1);
  c.gemm_kchunks = (c.N + PROJ_KCHUNK - 1) / PROJ_KCHUNK;
  const size_t dblocks = proj_dpart_slots((size_t)c.M * c.T);
  int rc = CISOR_OK;
  if ((rc = dalloc(c.Ghat, cs * PD)) || (rc = dalloc(c.tw, cs * P)) || (rc = dalloc(c.H, cs * c.M * (size_t)c.N)) ||
      (rc = dalloc(c.uin, cs * TN)) || (rc = dalloc(c.Ghat_d, sizeof(cd) * PD)) ||
      (rc = dalloc(c.tw_d, sizeof(cd) * P)) || (rc = dalloc(c.X1, cs * inter)) || (rc = dalloc(c.X2, cs * inter)) ||
      (rc = dalloc(c.part, sizeof(double) * NPART * c.T * c.nblk)) || (rc = dalloc(c.st, sizeof(TxState) * c.T)) ||
      (rc = dalloc(c.rel_tmp, sizeof(double) * c.T)) ||
      (rc = dalloc(c.start_choice, sizeof(int) * c.T)) || (rc = dalloc(c.U, cs * TN)) || (rc = dalloc(c.V, cs * TN)) ||
      (rc = dalloc(c.Q, cs * TN)) || (rc = dalloc(c.Bv, cs * TN)) || (rc = dalloc(c.W, cs * c.M * c.T)) ||
      (rc = dalloc(c.gpart, std::max(rs * TN, sizeof(double) * c.N))) || (rc = dalloc(c.zbuf, rs * 2 * c.N)) ||
      (rc = dalloc(c.tvbuf, rs * 9 * c.N)) || (rc = dalloc(c.gemm_part, sizeof(cd) * c.gemm_kchunks * c.M * c.T)) ||
      (rc = dalloc(c.dpart, sizeof(double) * dblocks)))
    goto fail;
  for (int i = 0; i < 6; ++i)
    if ((rc = dalloc(c.ws[i], cs * TN))) goto fail;
  if (c.precision == 0) {
    if ((rc = dalloc(c.X1d, sizeof(cd) * inter)) || (rc = dalloc(c.X2d, sizeof(cd) * inter))) goto fail;
  }
  // the kz-major spectrum copies of the fused 3D plane path (power-of-two
  // transform lengths up to 128 only; elsewhere the column passes run)
  if (D == 3 && P <= 128 && (P & (P - 1)) == 0 &&
      ((rc = dalloc(c.Gpm, cs * PD)) || (rc = dalloc(c.Gpm_d, sizeof(cd) * PD))))
    goto fail;
  if ((rc = solve_shared_init(c.sh, 1))) goto fail;
  if ((rc = dalloc(c.d_D, sizeof(double))) ||
      hipHostMalloc((void **)&c.h_states, sizeof(TxState) * 2 * c.T) != hipSuccess ||
      hipHostMalloc((void **)&c.h_D, sizeof(double)) != hipSuccess) {
    rc = rc ? rc : CISOR_E_NOMEM;
    goto fail;
  }
  if ((rc = build_geometry(c, *g))) goto fail;
  *out = h;
  return CISOR_OK;
fail:
  free_all(c);
  delete h;
  return rc;
}

int cisor_destroy(cisor_ctx *h) {
  if (!h) return CISOR_E_ARG;
  (void)hipStreamSynchronize(h->c.stream);
  free_all(h->c);
  delete h;
  return CISOR_OK;
}

int cisor_set_stream(cisor_ctx *h, void *stream) {
  if (!h) return CISOR_E_ARG;
  h->c.stream = (hipStream_t)stream;
  return CISOR_OK;
}

int cisor_get_sizes(const cisor_ctx *h, int *N, int *T, int *M, int *P, int *precision) {
  if (!h) return CISOR_E_ARG;
  if (N) *N = h->c.N;
  if (T) *T = h->c.T;
  if (M) *M = h->c.M;
  if (P) *P = h->c.P;
  if (precision) *precision = h->c.precision;
  return CISOR_OK;
}

int cisor_get_uin(cisor_ctx *h, void *u) {
  if (!h || !u) return CISOR_E_ARG;
  Ctx &c = h->c;
  const size_t cs = c.precision ? sizeof(cd) : sizeof(cf);
  CISOR_HIP_CHECK(hipMemcpyAsync(u, c.uin, cs * c.T * c.N, hipMemcpyDeviceToDevice, c.stream));
  return CISOR_OK;
}

int cisor_get_start_choice(cisor_ctx *h, int *choice) {
  if (!h || !choice) return CISOR_E_ARG;
  Ctx &c = h->c;
  CISOR_HIP_CHECK(hipMemcpyAsync(choice, c.start_choice, sizeof(int) * c.T, hipMemcpyDeviceToHost, c.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  return CISOR_OK;
}

int cisor_get_H(cisor_ctx *h, void *H) {
  if (!h || !H) return CISOR_E_ARG;
  Ctx &c = h->c;
  const size_t cs = c.precision ? sizeof(cd) : sizeof(cf);
  CISOR_HIP_CHECK(hipMemcpyAsync(H, c.H, cs * c.M * c.N, hipMemcpyDeviceToDevice, c.stream));
  return CISOR_OK;
}

int cisor_apply_A(cisor_ctx *h, const void *f, const void *x, void *y, int adjoint) {
  if (!h || !f || !x || !y || x == y || (adjoint != 0 && adjoint != 1)) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_apply_A<float>(c, (const float *)f, (const cf *)x, (cf *)y, adjoint);
  return launch_apply_A<double>(c, (const double *)f, (const cd *)x, (cd *)y, adjoint);
}

int cisor_born_field(cisor_ctx *h, const void *f, void *u_b) {
  if (!h || !f || !u_b) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_born_field<float>(c, (const float *)f, (cf *)u_b);
  return launch_born_field<double>(c, (const double *)f, (cd *)u_b);
}

int cisor_apply_A_stage(cisor_ctx *h, const void *f, const void *x, void *y, int adjoint, int stage) {
  if (!h || (adjoint != 0 && adjoint != 1) || stage < 1 || stage > 3) return CISOR_E_ARG;
  if ((stage == 1 && (!f || !x)) || (stage == 3 && (!f || !x || !y || x == y))) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.dim != 2) return CISOR_E_UNSUPPORTED;
  if (c.precision == 0)
    return launch_conv_stage<float>(c, (const float *)f, (const cf *)x, (cf *)y, stage, adjoint);
  return launch_conv_stage<double>(c, (const double *)f, (const cd *)x, (cd *)y, stage, adjoint);
}

int cisor_solve(cisor_ctx *h, const void *f, const void *b, void *x, int adjoint, const cisor_ls_opts *o,
                int *iters) {
  if (!h || !f || !b || !x || b == x || (adjoint != 0 && adjoint != 1) || !opts_ok(o)) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return solve_batch<float>(c, (const float *)f, (const cf *)b, (cf *)x, adjoint, *o, iters, nullptr);
  return solve_batch<double>(c, (const double *)f, (const cd *)b, (cd *)x, adjoint, *o, iters, nullptr);
}

int cisor_forward(cisor_ctx *h, const void *f, void *u, void *y, const cisor_ls_opts *o, int *iters) {
  if (!h || !f || !u || !opts_ok(o)) return CISOR_E_ARG;
  Ctx &c = h->c;
  int st;
  if (c.precision == 0) {
    st = solve_batch<float>(c, (const float *)f, (const cf *)c.uin, (cf *)u, false, *o, iters, nullptr);
    if (st >= 0 && y) {
      const int rc = launch_project<float>(c, (const float *)f, (const cf *)u, nullptr, (cf *)y, nullptr);
      if (rc) return rc;
    }
  } else {
    st = solve_batch<double>(c, (const double *)f, (const cd *)c.uin, (cd *)u, false, *o, iters, nullptr);
    if (st >= 0 && y) {
      const int rc = launch_project<double>(c, (const double *)f, (const cd *)u, nullptr, (cd *)y, nullptr);
      if (rc) return rc;
    }
  }
  return st;
}

int cisor_project(cisor_ctx *h, const void *f, const void *u, const void *y_meas, void *y, double *D) {
  if (!h || !f || !u || !y) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (!y_meas && D) return CISOR_E_ARG;
  if (c.precision == 0)
    return launch_project<float>(c, (const float *)f, (const cf *)u, (const cf *)y_meas, (cf *)y, D);
  return launch_project<double>(c, (const double *)f, (const cd *)u, (const cd *)y_meas, (cd *)y, D);
}

int cisor_backproject(cisor_ctx *h, const void *w, void *q) {
  if (!h || !w || !q) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_backproject<float>(c, (const cf *)w, (cf *)q, nullptr, nullptr);
  return launch_backproject<double>(c, (const cd *)w, (cd *)q, nullptr, nullptr);
}

int cisor_grad(cisor_ctx *h, const void *f, const void *y_meas, void *grad, double *D, void *u_ws, void *v_ws,
               const cisor_ls_opts *o, int *iters) {
  if (!h || !f || !y_meas || !grad || !u_ws || !v_ws || u_ws == v_ws || !opts_ok(o)) return CISOR_E_ARG;
  Ctx &c = h->c;
  int worst = CISOR_OK, rc;
  if (c.precision == 0)
    rc = launch_grad<float>(c, (const float *)f, (const cf *)y_meas, (float *)grad, D, (cf *)u_ws, (cf *)v_ws, *o,
                            iters, nullptr, &worst);
  else
    rc = launch_grad<double>(c, (const double *)f, (const cd *)y_meas, (double *)grad, D, (cd *)u_ws, (cd *)v_ws, *o,
                             iters, nullptr, &worst);
  if (rc) return rc;
  return worst;
}

int cisor_vjp(cisor_ctx *h, const void *f, const void *u, const void *w, void *grad, void *v_ws,
              const cisor_ls_opts *o, int *iters) {
  if (!h || !f || !u || !w || !grad || !v_ws || u == v_ws || !opts_ok(o)) return CISOR_E_ARG;
  Ctx &c = h->c;
  int st = CISOR_OK, rc;
  if (c.precision == 0)
    rc = launch_vjp<float>(c, (const float *)f, (const cf *)u, (const cf *)w, (float *)grad, (cf *)v_ws, *o, iters,
                           nullptr, &st);
  else
    rc = launch_vjp<double>(c, (const double *)f, (const cd *)u, (const cd *)w, (double *)grad, (cd *)v_ws, *o, iters,
                            nullptr, &st);
  return rc ? rc : st;
}

int cisor_tv_prox(cisor_ctx *h, const void *z, void *x, double lam, double lo, double hi, int inner) {
  if (!h || !z || !x || !(lam >= 0) || !std::isfinite(lam) || !(lo <= hi) || inner < 0) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_tv_prox<float>(c, (const float *)z, (float *)x, lam, lo, hi, inner);
  return launch_tv_prox<double>(c, (const double *)z, (double *)x, lam, lo, hi, inner);
}

int cisor_set_rx_mask(cisor_ctx *h, const unsigned char *mask) {
  if (!h) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (!mask) {
    if (c.rx_mask) (void)hipFree(c.rx_mask);
    c.rx_mask = nullptr;
    return CISOR_OK;
  }
  const size_t MT = (size_t)c.M * c.T;
  std::vector<float> hm(MT);
  for (size_t i = 0; i < MT; ++i) hm[i] = mask[i] ? 1.0f : 0.0f;
  if (!c.rx_mask && hipMalloc((void **)&c.rx_mask, sizeof(float) * MT) != hipSuccess) {
    c.rx_mask = nullptr;
    return CISOR_E_NOMEM;
  }
  CISOR_HIP_CHECK(hipMemcpyAsync(c.rx_mask, hm.data(), sizeof(float) * MT, hipMemcpyHostToDevice, c.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  return CISOR_OK;
}

int cisor_tv_value(cisor_ctx *h, const void *x, double *tv) {
  if (!h || !x || !tv) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_tv_value<float>(c, (const float *)x, tv);
  return launch_tv_value<double>(c, (const double *)x, tv);
}

int cisor_fista_step(cisor_ctx *h, cisor_fista_state *s, const void *y_meas, double gamma, double tau, double alpha,
                     double lo, double hi, int inner, const cisor_ls_opts *o, cisor_step_info *info) {
  if (!h || !s || !s->f || !s->f_prev || !s->s || !y_meas || !(gamma > 0) || !(tau >= 0) || !(alpha >= 0) ||
      !(alpha <= 1) || !(lo <= hi) || inner < 0 || !opts_ok(o, 4) || !(s->t >= 1.0))
    return CISOR_E_ARG;
  Ctx &c = h->c;
  cisor_ls_opts lo_opts = *o;
  std::vector<int> iters(2 * c.T, 0);
  double D = 0.0, mr = 0.0;
  int worst = CISOR_OK, rc;
  const size_t cs = c.precision ? sizeof(cd) : sizeof(cf);
  const size_t rs = c.precision ? sizeof(double) : sizeof(float);
  // Starting guesses: the previous iteration's fields (start == 2), their
  // extrapolation along the path of evaluation points (start == 4; the
  // previous fields after one recorded iteration), the first-Born start for
  // the forward solve otherwise.  A run restarted at k == 0 forgets the path.
  const bool extrap = o->start == 4;
  if (extrap) {
    if (!c.xpart) {   // allocated last: its presence means all five are
      const size_t TN = (size_t)c.T * c.N;
      if ((!c.U2 && (rc = dalloc(c.U2, cs * TN))) || (!c.V2 && (rc = dalloc(c.V2, cs * TN))) ||
          (!c.S1 && (rc = dalloc(c.S1, rs * c.N))) || (!c.S2 && (rc = dalloc(c.S2, rs * c.N))) ||
          (rc = dalloc(c.xpart, sizeof(double) * 512)))
        return rc;
      c.hist_depth = 0;
    }
    if (s->k == 0 || !c.fields_valid) c.hist_depth = 0;
  } else {
    c.hist_depth = 0;   // the recorded path is only followed by consecutive mode-4 steps
  }
  const bool warm = (o->start == 2 || extrap) && c.fields_valid && (!extrap || c.hist_depth >= 1);
  if (!warm) {
    // u0 = u_in (first-Born start) or 0; v0 = 0
    if (o->start == 0)
      CISOR_HIP_CHECK(hipMemsetAsync(c.U, 0, cs * c.T * c.N, c.stream));
    else
      CISOR_HIP_CHECK(hipMemcpyAsync(c.U, c.uin, cs * c.T * c.N, hipMemcpyDeviceToDevice, c.stream));
    CISOR_HIP_CHECK(hipMemsetAsync(c.V, 0, cs * c.T * c.N, c.stream));
  }
  if (extrap) {
    rc = c.precision ? launch_extrapolate<double>(c, (const double *)s->s, c.hist_depth)
                     : launch_extrapolate<float>(c, (const float *)s->s, c.hist_depth);
    if (rc) return rc;
  }
  lo_opts.start = 2;
  if (c.precision == 0) {
    rc = launch_grad<float>(c, (const float *)s->s, (const cf *)y_meas, (float *)c.zbuf + 0, &D, (cf *)c.U, (cf *)c.V,
                            lo_opts, iters.data(), &mr, &worst);
  } else {
    rc = launch_grad<double>(c, (const double *)s->s, (const cd *)y_meas, (double *)c.zbuf + 0, &D, (cd *)c.U,
                             (cd *)c.V, lo_opts, iters.data(), &mr, &worst);
  }
  if (rc) return rc;
  c.fields_valid = true;
  if (extrap) c.hist_depth = std::min(c.hist_depth + 1, 2);
  // the gradient sits in zbuf[0:N]; the tail reads it before overwriting
  void *g = c.gpart;
  CISOR_HIP_CHECK(hipMemcpyAsync(g, c.zbuf, rs * c.N, hipMemcpyDeviceToDevice, c.stream));
  if (c.precision == 0)
    rc = launch_fista_tail<float>(c, s, (const float *)g, gamma, tau, alpha, lo, hi, inner);
  else
    rc = launch_fista_tail<double>(c, s, (const double *)g, gamma, tau, alpha, lo, hi, inner);
  if (rc) return rc;
  if (info) {
    info->D = D;
    info->fwd_iters_max = info->adj_iters_max = 0;
    info->fwd_iters_sum = info->adj_iters_sum = 0;
    for (int t = 0; t < c.T; ++t) {
      info->fwd_iters_max = std::max(info->fwd_iters_max, iters[t]);
      info->adj_iters_max = std::max(info->adj_iters_max, iters[c.T + t]);
      info->fwd_iters_sum += iters[t];
      info->adj_iters_sum += iters[c.T + t];
    }
    info->max_true_relres = mr;
    info->status = worst;
  }
  return worst < 0 ? worst : CISOR_OK;
}

int cisor_autotune(cisor_ctx *h, int reps, int *variant, float *times_ms) {
  if (!h || reps < 1) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.dim != 2) return CISOR_E_UNSUPPORTED;
  const int rc = autotune_columns(c, reps, times_ms);
  if (variant) *variant = c.col_variant;
  return rc;
}

int cisor_set_col_variant(cisor_ctx *h, int variant) {
  if (!h || variant < 0 || variant >= COL_VARIANTS) return CISOR_E_ARG;
  h->c.col_variant = variant;
  return CISOR_OK;
}

int cisor_born_lipschitz(cisor_ctx *h, int iters, double *L) {
  if (!h || !L || iters < 1) return CISOR_E_ARG;
  Ctx &c = h->c;
  if (c.precision == 0) return launch_born_lipschitz<float>(c, iters, L);
  return launch_born_lipschitz<double>(c, iters, L);
}

}  // extern "C"
