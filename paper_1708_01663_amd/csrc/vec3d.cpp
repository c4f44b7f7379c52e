// C ABI of the 3D vectorial model: context lifetime, host-side geometry
// (polarised plane waves, the dyadic receiver rows), argument validation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <new>
#include <thread>
#include <vector>

#include "vec3d.hpp"

using namespace cisor;
using namespace cisor::vec;

struct cisor_vec_ctx {
  VecCtx v;
  bool fields_valid = false;   // E and V hold the fields of a previous gradient
};

namespace {

using cdbl = std::complex<double>;
constexpr double kPi = 3.14159265358979323846264338327950288;

void parallel_rows(int n, const std::function<void(int, int)> &fn) {
  const int nt = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int i = 0; i < nt; ++i) {
    const int lo = (int)((long long)n * i / nt), hi = (int)((long long)n * (i + 1) / nt);
    th.emplace_back(fn, lo, hi);
  }
  for (auto &t : th) t.join();
}

template <typename T> int dalloc(T *&p, size_t bytes) {
  void *q = nullptr;
  if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) return CISOR_E_NOMEM;
  p = (T *)q;
  return CISOR_OK;
}

void free_vec(cisor_vec_ctx *h) {
  VecCtx &v = h->v;
  void *ptrs[] = {v.Ein, v.H, v.E, v.Vv, v.Q, v.B, v.Wr, v.part, v.st, v.fmask, v.rx_mask, v.f3, v.gemm_part, v.dpart,
                  v.gbuf, v.zb, v.fk,
                  v.ws[0], v.ws[1], v.ws[2], v.ws[3], v.ws[4], v.ws[5], v.ws[6], v.ws[7]};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (v.h_st) (void)hipHostFree(v.h_st);
  if (v.sub) (void)cisor_destroy(v.sub);
}

// Unit z projected transverse to the propagation direction d (unit x when d
// is along z): the incident polarisation.
void polarisation(const double d[3], double p[3]) {
  double ref[3] = {0.0, 0.0, 1.0};
  if (std::fabs(d[2]) >= 1.0 - 1e-9) ref[0] = 1.0, ref[2] = 0.0;
  const double dot = ref[0] * d[0] + ref[1] * d[1] + ref[2] * d[2];
  double nr = 0.0;
  for (int i = 0; i < 3; ++i) {
    p[i] = ref[i] - dot * d[i];
    nr += p[i] * p[i];
  }
  nr = std::sqrt(nr);
  for (int i = 0; i < 3; ++i) p[i] /= nr;
}

int upload(void *dst, const std::vector<cdbl> &src) {
  CISOR_HIP_CHECK(hipMemcpy(dst, src.data(), sizeof(cdbl) * src.size(), hipMemcpyHostToDevice));
  return CISOR_OK;
}

int build(VecCtx &v, const cisor_geometry &g) {
  const int n = v.n, N = v.N, T = v.T, M = v.M;
  const double h = v.h, k = v.k;
  std::vector<double> ax(n);
  for (int i = 0; i < n; ++i) ax[i] = (i - (n - 1) / 2.0) * h;
  // incident fields: polarised plane waves (tx_kind 0), or unit electric
  // dipoles E = Gd(r - s) p / k^2 = g(R) [a(kR) Rh Rh^T + b(kR) I] p (tx_kind 1);
  // p is z projected transverse to the direction of travel (from the source
  // towards the grid's centre for a dipole)
  std::vector<cdbl> ein((size_t)T * 3 * N);
  for (int t = 0; t < T; ++t) {
    const bool dip = g.tx_kind == 1;
    const double *v = dip ? g.tx_pos + 3 * t : g.tx_dir + 3 * t;
    double d[3] = {dip ? -v[0] : v[0], dip ? -v[1] : v[1], dip ? -v[2] : v[2]};
    const double nr = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (double &x : d) x /= nr;
    double p[3];
    polarisation(d, p);
    parallel_rows(n, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i)
        for (int j = 0; j < n; ++j)
          for (int l = 0; l < n; ++l) {
            const size_t cell = ((size_t)i * n + j) * n + l;
            if (!dip) {
              const cdbl w = std::polar(1.0, k * (d[0] * ax[i] + d[1] * ax[j] + d[2] * ax[l]));
              for (int c = 0; c < 3; ++c) ein[((size_t)t * 3 + c) * N + cell] = p[c] * w;
              continue;
            }
            const double R[3] = {ax[i] - v[0], ax[j] - v[1], ax[l] - v[2]};
            const double dd = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
            const double kd = k * dd;
            const cdbl gr = std::polar(1.0 / (4.0 * kPi * dd), kd);
            const cdbl a = cdbl(3.0 / (kd * kd) - 1.0, -3.0 / kd);
            const cdbl b = cdbl(1.0 - 1.0 / (kd * kd), 1.0 / kd);
            const double rp = (R[0] * p[0] + R[1] * p[1] + R[2] * p[2]) / dd;
            for (int c = 0; c < 3; ++c) ein[((size_t)t * 3 + c) * N + cell] = gr * (a * (R[c] / dd) * rp + b * p[c]);
          }
    });
  }
  // receiver rows: delta^3 times the third row of the dyadic Green's function
  // k^2 g(R) [a(kR) Rz Rj / R^2 + b(kR) delta_3j] at R = r_m - r_cell
  std::vector<cdbl> H((size_t)M * 3 * N);
  const double h3 = h * h * h;
  parallel_rows(M, [&](int lo, int hi) {
    for (int m = lo; m < hi; ++m) {
      const double *r = g.rx_pos + 3 * m;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          for (int l = 0; l < n; ++l) {
            const double R[3] = {r[0] - ax[i], r[1] - ax[j], r[2] - ax[l]};
            const double d = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
            const double kd = k * d;
            const cdbl gr = std::polar(1.0 / (4.0 * kPi * d), kd);
            const cdbl a = cdbl(3.0 / (kd * kd) - 1.0, -3.0 / kd);
            const cdbl b = cdbl(1.0 - 1.0 / (kd * kd), 1.0 / kd);
            const cdbl s = h3 * k * k * gr;
            const size_t cell = ((size_t)i * n + j) * n + l;
            for (int c = 0; c < 3; ++c) {
              cdbl val = a * (R[2] / d) * (R[c] / d);
              if (c == 2) val += b;
              H[(size_t)m * 3 * N + (size_t)c * N + cell] = s * val;
            }
          }
    }
  });
  int rc;
  if ((rc = upload(v.Ein, ein)) || (rc = upload(v.H, H))) return rc;
  return CISOR_OK;
}

bool opts_valid(const cisor_ls_opts *o, bool grad) {
  if (!o || !(o->tol > 0.0) || !std::isfinite(o->tol) || o->maxit < 1) return false;
  return grad ? (o->start >= 0 && o->start <= 2) : (o->start == 0 || o->start == 1 || o->start == 3);
}

}  // namespace

extern "C" {

int cisor_vec_create(const cisor_geometry *g, void *stream, cisor_vec_ctx **out) {
  if (!g || !out) return CISOR_E_ARG;
  *out = nullptr;
  if (g->dim != 3 || g->n < 2 || !(g->h > 0) || !(g->wavelength > 0) || g->T < 1 || g->M < 1 || !g->rx_pos ||
      !std::isfinite(g->h) || !std::isfinite(g->wavelength))
    return CISOR_E_ARG;
  if (g->precision != 1 || g->eps_b != 1.0) return CISOR_E_UNSUPPORTED;
  if (!transmitters_ok(*g)) return CISOR_E_ARG;
  // receivers strictly outside the grid's cube (the dyadic kernel is singular at a cell centre)
  const double half = 0.5 * g->n * g->h;
  for (int m = 0; m < g->M; ++m) {
    double outside = -1.0;
    for (int d = 0; d < 3; ++d) {
      const double a = g->rx_pos[3 * m + d];
      if (!std::isfinite(a)) return CISOR_E_ARG;
      outside = std::max(outside, std::fabs(a) - half);
    }
    if (!(outside > 0.0)) return CISOR_E_ARG;
  }
  if ((long long)3 * g->T > 1 << 20) return CISOR_E_ARG;
  // scalar context over the 3T component fields: same grid and wavelength
  // (only its convolution is used, so the directions are placeholders)
  std::vector<double> dirs((size_t)9 * g->T, 0.0);
  for (int f = 0; f < 3 * g->T; ++f) dirs[(size_t)3 * f + 2] = 1.0;
  cisor_geometry sg = *g;
  sg.T = 3 * g->T;
  sg.tx_dir = dirs.data();
  sg.tx_kind = 0;
  sg.tx_pos = nullptr;
  cisor_vec_ctx *h = new (std::nothrow) cisor_vec_ctx();
  if (!h) return CISOR_E_NOMEM;
  VecCtx &v = h->v;
  int rc = cisor_create(&sg, stream, &v.sub);
  if (rc) {
    delete h;
    return rc;
  }
  v.sc = ctx_of(v.sub);
  v.n = g->n;
  v.N = v.sc->N;
  v.T = g->T;
  v.M = g->M;
  v.h = g->h;
  v.k = v.sc->k;
  v.stream = (hipStream_t)stream;
  v.nbv = std::max(1, std::min(VMAXB, (3 * v.N + VB * 4 - 1) / (VB * 4)));
  const size_t L = (size_t)v.T * 3 * v.N;
  const size_t cs = sizeof(cd);
  for (int i = 0; i < 8 && !rc; ++i) rc = dalloc(v.ws[i], cs * L);
  if (rc || (rc = dalloc(v.Ein, cs * L)) || (rc = dalloc(v.H, cs * v.M * 3 * (size_t)v.N)) ||
      (rc = dalloc(v.E, cs * L)) || (rc = dalloc(v.Vv, cs * L)) || (rc = dalloc(v.Q, cs * L)) ||
      (rc = dalloc(v.B, cs * L)) || (rc = dalloc(v.Wr, cs * v.T * (size_t)v.M)) ||
      (rc = dalloc(v.part, sizeof(double) * VNP * v.T * v.nbv)) || (rc = dalloc(v.st, sizeof(VState) * v.T)) ||
      (rc = dalloc(v.fmask, sizeof(int) * 3 * (size_t)v.T)) ||
      (rc = dalloc(v.f3, sizeof(double) * 3 * (size_t)v.N)) || (rc = dalloc(v.gbuf, sizeof(double) * v.N)) ||
      (rc = dalloc(v.zb, sizeof(double) * v.N)) || (rc = dalloc(v.fk, sizeof(double) * v.N)) ||
      (rc = dalloc(v.gemm_part, sizeof(cd) * ((3 * (size_t)v.N + PROJ_KCHUNK - 1) / PROJ_KCHUNK) * v.M * v.T)) ||
      (rc = dalloc(v.dpart, sizeof(double) * (proj_dpart_slots((size_t)v.M * v.T) + 1))))
    goto fail;
  if (hipHostMalloc((void **)&v.h_st, sizeof(VState) * v.T) != hipSuccess) {
    rc = CISOR_E_NOMEM;
    goto fail;
  }
  if ((rc = build(v, *g))) goto fail;
  *out = h;
  return CISOR_OK;
fail:
  free_vec(h);
  delete h;
  return rc;
}

int cisor_vec_destroy(cisor_vec_ctx *h) {
  if (!h) return CISOR_E_ARG;
  (void)hipStreamSynchronize(h->v.stream);
  free_vec(h);
  delete h;
  return CISOR_OK;
}

int cisor_vec_set_stream(cisor_vec_ctx *h, void *stream) {
  if (!h) return CISOR_E_ARG;
  h->v.stream = (hipStream_t)stream;
  return cisor_set_stream(h->v.sub, stream);
}

int cisor_vec_set_rx_mask(cisor_vec_ctx *h, const unsigned char *mask) {
  if (!h) return CISOR_E_ARG;
  VecCtx &v = h->v;
  if (!mask) {
    if (v.rx_mask) (void)hipFree(v.rx_mask);
    v.rx_mask = nullptr;
    return CISOR_OK;
  }
  const size_t MT = (size_t)v.M * v.T;
  std::vector<float> hm(MT);
  for (size_t i = 0; i < MT; ++i) hm[i] = mask[i] ? 1.0f : 0.0f;
  if (!v.rx_mask && hipMalloc((void **)&v.rx_mask, sizeof(float) * MT) != hipSuccess) {
    v.rx_mask = nullptr;
    return CISOR_E_NOMEM;
  }
  CISOR_HIP_CHECK(hipMemcpyAsync(v.rx_mask, hm.data(), sizeof(float) * MT, hipMemcpyHostToDevice, v.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(v.stream));
  return CISOR_OK;
}

int cisor_vec_get_sizes(const cisor_vec_ctx *h, int *N, int *T, int *M) {
  if (!h) return CISOR_E_ARG;
  if (N) *N = h->v.N;
  if (T) *T = h->v.T;
  if (M) *M = h->v.M;
  return CISOR_OK;
}

int cisor_vec_get_uin(cisor_vec_ctx *h, void *E) {
  if (!h || !E) return CISOR_E_ARG;
  VecCtx &v = h->v;
  CISOR_HIP_CHECK(hipMemcpyAsync(E, v.Ein, sizeof(cd) * v.T * 3 * (size_t)v.N, hipMemcpyDeviceToDevice, v.stream));
  return CISOR_OK;
}

int cisor_vec_get_H(cisor_vec_ctx *h, void *H) {
  if (!h || !H) return CISOR_E_ARG;
  VecCtx &v = h->v;
  CISOR_HIP_CHECK(hipMemcpyAsync(H, v.H, sizeof(cd) * v.M * 3 * (size_t)v.N, hipMemcpyDeviceToDevice, v.stream));
  return CISOR_OK;
}

int cisor_vec_apply_A(cisor_vec_ctx *h, const double *f, const void *x, void *y, int adjoint) {
  if (!h || !f || !x || !y || x == y || (adjoint != 0 && adjoint != 1)) return CISOR_E_ARG;
  return launch_apply(h->v, f, (const cd *)x, (cd *)y, adjoint == 1);
}

int cisor_vec_forward(cisor_vec_ctx *h, const double *f, const cisor_ls_opts *o, void *E, void *y, int *iters,
                      double *max_rel) {
  if (!h || !f || !E || !opts_valid(o, false)) return CISOR_E_ARG;
  VecCtx &v = h->v;
  const int st = launch_solve(v, f, v.Ein, (cd *)E, false, *o, iters, max_rel);
  if (st < 0) return st;
  if (y)
    if (int rc = launch_project(v, f, (const cd *)E, nullptr, (cd *)y, nullptr, nullptr)) return rc;
  return st;
}

int cisor_vec_project(cisor_vec_ctx *h, const double *f, const void *E, void *y) {
  if (!h || !f || !E || !y) return CISOR_E_ARG;
  return launch_project(h->v, f, (const cd *)E, nullptr, (cd *)y, nullptr, nullptr);
}

}  // extern "C"

namespace {

int grad_impl(cisor_vec_ctx *h, const double *f, const void *y_meas, double *grad, double *D, const cisor_ls_opts *o,
              int *iters, double *max_rel) {
  VecCtx &v = h->v;
  cisor_ls_opts so = *o;
  // start 2: the fields of the previous gradient (the first-Born guess when there are none)
  if (so.start == 2) so.start = h->fields_valid ? 3 : 1;
  h->fields_valid = false;
  double mr[2] = {0.0, 0.0};
  const int s1 = launch_solve(v, f, v.Ein, v.E, false, so, iters, &mr[0]);
  if (s1 < 0) return s1;
  int rc = launch_project(v, f, v.E, (const cd *)y_meas, nullptr, v.Wr, D);
  if (rc || (rc = launch_backproject(v, f, v.Wr, v.Q, v.B))) return rc;
  const int s2 = launch_solve(v, f, v.B, v.Vv, true, so, iters ? iters + v.T : nullptr, &mr[1]);
  if (s2 < 0) return s2;
  if ((rc = launch_gradient(v, v.E, v.Q, v.Vv, grad))) return rc;
  if (max_rel) *max_rel = std::max(mr[0], mr[1]);
  h->fields_valid = true;
  return std::max(s1, s2);
}

}  // namespace

extern "C" {

int cisor_vec_grad(cisor_vec_ctx *h, const double *f, const void *y_meas, double *grad, double *D,
                   const cisor_ls_opts *o, int *iters, double *max_rel) {
  if (!h || !f || !y_meas || !grad || !D || !opts_valid(o, true)) return CISOR_E_ARG;
  return grad_impl(h, f, y_meas, grad, D, o, iters, max_rel);
}

int cisor_vec_fista_step(cisor_vec_ctx *h, cisor_fista_state *s, const void *y_meas, double gamma, double tau,
                         double alpha, double lo, double hi, int inner, const cisor_ls_opts *o, cisor_step_info *info) {
  if (!h || !s || !s->f || !s->f_prev || !s->s || !y_meas || !(gamma > 0) || !(tau >= 0) || !(alpha >= 0) ||
      !(alpha <= 1) || !(lo <= hi) || inner < 0 || !opts_valid(o, true) || !(s->t >= 1.0) || s->k < 0)
    return CISOR_E_ARG;
  VecCtx &v = h->v;
  std::vector<int> iters(2 * v.T, 0);
  double D = 0.0, mr = 0.0;
  const int st = grad_impl(h, (const double *)s->s, y_meas, v.gbuf, &D, o, iters.data(), &mr);
  if (st < 0) return st;
  if (int rc = launch_fista_tail(v, s, v.gbuf, gamma, tau, alpha, lo, hi, inner)) return rc;
  CISOR_HIP_CHECK(hipStreamSynchronize(v.stream));
  if (info) {
    info->D = D;
    info->fwd_iters_max = info->adj_iters_max = 0;
    info->fwd_iters_sum = info->adj_iters_sum = 0;
    for (int t = 0; t < v.T; ++t) {
      info->fwd_iters_max = std::max(info->fwd_iters_max, iters[t]);
      info->adj_iters_max = std::max(info->adj_iters_max, iters[v.T + t]);
      info->fwd_iters_sum += iters[t];
      info->adj_iters_sum += iters[v.T + t];
    }
    info->max_true_relres = mr;
    info->status = st;
  }
  return st;
}

}  // extern "C"
