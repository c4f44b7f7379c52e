// Batched CISOR: many independent reconstructions with uneven grid sizes and
// transmitter counts, stepped together (relaxed FISTA, eqs. algo1-algo3, on
// every problem at once).
//
// Problems that share a grid (n, h, wavelength, eps_b) share one kernel
// spectrum and form a group.  A group is one operator context whose fields are
// the fields of all its problems, stacked transmitter-major ([sum T_p][N]); the
// contrast is read per field through a pointer table, so one launch of each
// FFT stage covers every field of every problem of the group.  Each group
// runs on a stream of its own; a step forks the groups from the caller's
// stream and joins them back.  The solver chunks (ten BiCGSTAB iterations of
// every open system of every group, the FP64 residual check and the count of
// open systems) are captured once as one graph with one branch per group, and
// so are the non-solver parts of a step (projection, misfit, back-projection;
// gradient terms, prox, momentum).  All buffers come from one device arena.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "conv_cfg.hpp"
#include "internal.hpp"

using namespace cisor;

namespace {

struct Problem {
  int group = 0, row0 = 0;      // group and first field row inside it
  int n = 0, N = 0, T = 0, M = 0;
  Ctx view;                     // problem-sized view: group tables, own H, W, GEMM and prox buffers
  void *f = nullptr, *f_prev = nullptr, *s = nullptr, *grad = nullptr, *y = nullptr, *fin = nullptr;
  double gamma = 0.0, tau = 0.0;
  bool has_data = false;
  double t = 1.0;               // host mirror of the device t_k
  int k = 0;
};

struct Group {
  Ctx c;                        // operator over the stacked fields of its problems
  std::vector<int> probs;
  bool own_stream = false;
  const void **frow_s = nullptr;   // device [T]: s of each field's problem
  const void **frow_in = nullptr;  // device [T]: input contrast of each field's problem
  TxState *h_states = nullptr;     // pinned host [2T]: final forward / adjoint solver states of a step
};

struct Arena {
  char *base = nullptr;
  size_t off = 0;
  template <typename T> void take(T *&p, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(bytes, 16);
  }
};

}  // namespace

struct cisor_batch {
  int precision = 0;
  hipStream_t stream = nullptr;
  std::vector<Group> groups;
  std::vector<Problem> probs;
  std::vector<cisor_geometry> geoms;
  SolveShared sh;        // solver chunk graphs and counters
  SolveShared step_sh;   // graphs of the non-solver parts of a step
  void *arena = nullptr;
  size_t arena_bytes = 0;
  double *D_dev = nullptr, *t_dev = nullptr;
  bool fields_valid = false;
  int hist_depth = 0;    // FISTA evaluation points recorded for start mode 4 (0, 1, 2)
};

namespace {

// Assign every buffer of the batch from the arena (base == nullptr: measure).
void layout(cisor_batch &b, Arena &A) {
  const size_t rs = b.precision ? sizeof(double) : sizeof(float), cs = 2 * rs;
  for (Group &g : b.groups) {
    Ctx &c = g.c;
    const size_t T = c.T, N = c.N, P = c.P, TN = T * N, inter = T * c.n * P;
    A.take(c.Ghat, cs * P * P);
    A.take(c.tw, cs * P);
    A.take(c.Ghat_d, sizeof(cd) * P * P);
    A.take(c.tw_d, sizeof(cd) * P);
    A.take(c.X1, cs * inter);
    A.take(c.X2, cs * inter);
    if (b.precision == 0) {
      A.take(c.X1d, sizeof(cd) * inter);
      A.take(c.X2d, sizeof(cd) * inter);
    }
    A.take(c.part, sizeof(double) * NPART * T * c.nblk);
    A.take(c.st, sizeof(TxState) * T);
    A.take(c.rel_tmp, sizeof(double) * T);
    A.take(c.start_choice, sizeof(int) * T);
    for (int i = 0; i < 6; ++i) A.take(c.ws[i], cs * TN);
    A.take(c.uin, cs * TN);
    A.take(c.U, cs * TN);
    A.take(c.V, cs * TN);
    A.take(c.U2, cs * TN);
    A.take(c.V2, cs * TN);
    A.take(c.Q, cs * TN);
    A.take(c.Bv, cs * TN);
    A.take(c.gpart, std::max(rs * TN, sizeof(double) * N));
    A.take(g.frow_s, sizeof(void *) * T);
    A.take(g.frow_in, sizeof(void *) * T);
    for (int pi : g.probs) {
      Problem &p = b.probs[pi];
      Ctx &v = p.view;
      const size_t off = (size_t)p.row0 * N * cs;
      auto at = [&](void *base) { return base ? (void *)((char *)base + off) : nullptr; };
      v.uin = at(c.uin);
      v.U = at(c.U);
      v.V = at(c.V);
      v.U2 = at(c.U2);
      v.V2 = at(c.V2);
      v.Q = at(c.Q);
      v.Bv = at(c.Bv);
      v.Ghat = c.Ghat;
      v.tw = c.tw;
      v.Ghat_d = c.Ghat_d;
      v.tw_d = c.tw_d;
      v.gemm_kchunks = (p.N + PROJ_KCHUNK - 1) / PROJ_KCHUNK;
      A.take(v.H, cs * p.M * N);
      A.take(v.W, cs * p.M * p.T);
      A.take(v.gemm_part, sizeof(cd) * v.gemm_kchunks * p.M * p.T);
      A.take(v.dpart, sizeof(double) * proj_dpart_slots((size_t)p.M * p.T));
      A.take(v.zbuf, rs * 2 * N);
      A.take(v.tvbuf, rs * 9 * N);
      A.take(v.S1, rs * N);
      A.take(v.S2, rs * N);
      A.take(v.xpart, sizeof(double) * 512);
      A.take(p.f, rs * N);
      A.take(p.f_prev, rs * N);
      A.take(p.s, rs * N);
      A.take(p.grad, rs * N);
      A.take(p.fin, rs * N);
      A.take(p.y, cs * p.M * p.T);
    }
  }
  A.take(b.D_dev, sizeof(double) * b.probs.size());
  A.take(b.t_dev, sizeof(double) * b.probs.size());
}

void batch_free(cisor_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (Group &g : b->groups) {
    if (g.own_stream && g.c.stream) {
      (void)hipStreamSynchronize(g.c.stream);
      (void)hipStreamDestroy(g.c.stream);
    }
    if (g.h_states) (void)hipHostFree(g.h_states);
  }
  solve_shared_free(b->sh);
  solve_shared_free(b->step_sh);
  if (b->arena) (void)hipFree(b->arena);
  delete b;
}

bool same_grid(const cisor_geometry &a, const cisor_geometry &b) {
  return a.n == b.n && a.h == b.h && a.wavelength == b.wavelength && a.eps_b == b.eps_b;
}

// Step 1 of a batched FISTA iteration after the forward solves: projection,
// misfit D (device), back-projection and right-hand sides of the adjoint solves.
template <typename R> int launch_mid(cisor_batch &b, hipStream_t main) {
  using C = cplx_t<R>;
  const int G = (int)b.groups.size();
  return fork_join(b.step_sh, main, G, [&](int gi) { return b.groups[gi].c.stream; }, [&](int gi) -> int {
    for (int pi : b.groups[gi].probs) {
      Problem &p = b.probs[pi];
      Ctx &v = p.view;
      int rc = launch_project<R>(v, (const R *)p.s, (const C *)v.U, (const C *)p.y, (C *)v.W, nullptr, b.D_dev + pi);
      if (rc) return rc;
      if ((rc = launch_backproject<R>(v, (const C *)v.W, (C *)v.Q, (const R *)p.s, (C *)v.Bv))) return rc;
    }
    return CISOR_OK;
  });
}

// Step 2 after the adjoint solves: per group the terms Re{conj(u)(q + G^H v)}
// in one launch over all fields, then per problem the sum over its
// transmitters, the gradient step, the prox and the momentum.
template <typename R>
int launch_tail(cisor_batch &b, hipStream_t main, double alpha, double lo, double hi, int inner) {
  using C = cplx_t<R>;
  const int G = (int)b.groups.size();
  return fork_join(b.step_sh, main, G, [&](int gi) { return b.groups[gi].c.stream; }, [&](int gi) -> int {
    Group &g = b.groups[gi];
    ConvArgs<R, R> a{};
    fill_tables<R>(g.c, a.Ghat, a.tw, a.X1, a.X2);
    a.x = (const C *)g.c.V;
    a.u = (const C *)g.c.U;
    a.q = (const C *)g.c.Q;
    a.gpart = (R *)g.c.gpart;
    int rc = launch_conv<R, R, PRO_X, EPI_GRAD>(g.c, a, true);
    if (rc) return rc;
    for (int pi : g.probs) {
      Problem &p = b.probs[pi];
      const R *gp = (const R *)g.c.gpart + (size_t)p.row0 * p.N;
      if ((rc = launch_sum_rows<R>(p.view, gp, (R *)p.grad, p.T))) return rc;
      if ((rc = launch_fista_tail_dev<R>(p.view, (R *)p.f, (R *)p.f_prev, (R *)p.s, (const R *)p.grad,
                                         b.t_dev + pi, p.gamma, p.tau, alpha, lo, hi, inner)))
        return rc;
    }
    return CISOR_OK;
  });
}

std::vector<Ctx *> all_ctxs(cisor_batch &b) {
  std::vector<Ctx *> v;
  for (Group &g : b.groups) v.push_back(&g.c);
  for (Problem &p : b.probs) v.push_back(&p.view);
  return v;
}

// Run `launch` (enqueueing from `main`) as a cached graph, or directly.
template <typename Fn> int run_step_part(cisor_batch &b, GraphKey key, Fn &&launch) {
  // views and groups share streams; point the views at their group's stream
  // for the capture exactly as the groups are
  const int g = graph_run(b.step_sh, key, b.stream, all_ctxs(b), launch);
  if (g < 0) return g;
  if (g == 1) return launch(b.stream);
  return CISOR_OK;
}

template <typename R>
int batch_step(cisor_batch &b, double alpha, double lo, double hi, int inner, const cisor_ls_opts &o,
               cisor_step_info *info) {
  using C = cplx_t<R>;
  const int G = (int)b.groups.size();
  // starts as in cisor_fista_step: previous fields (2), their extrapolation
  // along each problem's path (4, previous fields after one recorded step)
  const bool extrap = o.start == 4;
  if (!b.fields_valid || !extrap) b.hist_depth = 0;
  const bool warm = (o.start == 2 || (extrap && b.hist_depth >= 1)) && b.fields_valid;
  if (!warm) {
    for (Group &g : b.groups) {
      const size_t TN = (size_t)g.c.T * g.c.N;
      if (o.start == 0)
        launch_fill<C>(b.stream, (C *)g.c.U, TN, mk<C>(0, 0));
      else
        launch_copy<C>(b.stream, (C *)g.c.U, (const C *)g.c.uin, TN);
      launch_fill<C>(b.stream, (C *)g.c.V, TN, mk<C>(0, 0));
    }
  }
  if (extrap) {
    for (Problem &p : b.probs) {
      Ctx v = p.view;
      v.stream = b.stream;
      const int rc = launch_extrapolate<R>(v, (const R *)p.s, b.hist_depth);
      if (rc) return rc;
    }
  }
  cisor_ls_opts so = o;
  so.start = 2;
  std::vector<std::vector<int>> itf(G), ita(G);
  std::vector<SolveJob> jobs(G);
  for (int gi = 0; gi < G; ++gi) {
    Group &g = b.groups[gi];
    g.c.frow = (const void *const *)g.frow_s;
    itf[gi].assign(g.c.T, 0);
    ita[gi].assign(g.c.T, 0);
    jobs[gi].c = &g.c;
    jobs[gi].b = g.c.uin;
    jobs[gi].x = g.c.U;
    jobs[gi].iters = itf[gi].data();
    jobs[gi].host_states = g.h_states;
  }
  // forward solves A u = u_in of every field of every problem (final states
  // collected after the step's one synchronisation)
  int rc = solve_multi<R>(jobs.data(), G, b.sh, b.stream, false, so);
  if (rc < 0) return rc;
  std::vector<SolveJob> fjobs = jobs;
  GraphKey km;
  km.ptrs = {&b};
  km.vals = {1.0};   // tag: projection part
  rc = run_step_part(b, km, [&](hipStream_t m) { return launch_mid<R>(b, m); });
  if (rc) return rc;
  // adjoint solves A^H v = f q
  for (int gi = 0; gi < G; ++gi) {
    jobs[gi].b = b.groups[gi].c.Bv;
    jobs[gi].x = b.groups[gi].c.V;
    jobs[gi].iters = ita[gi].data();
    jobs[gi].host_states = b.groups[gi].h_states + b.groups[gi].c.T;
  }
  if ((rc = solve_multi<R>(jobs.data(), G, b.sh, b.stream, true, so)) < 0) return rc;
  GraphKey kt;
  kt.ptrs = {&b};
  kt.vals = {2.0, alpha, lo, hi, (double)inner};   // tag: tail part
  for (const Problem &p : b.probs) {
    kt.vals.push_back(p.gamma);
    kt.vals.push_back(p.tau);
  }
  rc = run_step_part(b, kt, [&](hipStream_t m) { return launch_tail<R>(b, m, alpha, lo, hi, inner); });
  if (rc) return rc;
  b.fields_valid = true;
  if (extrap) b.hist_depth = std::min(b.hist_depth + 1, 2);
  std::vector<double> D(b.probs.size(), 0.0);
  CISOR_HIP_CHECK(hipMemcpyAsync(D.data(), b.D_dev, sizeof(double) * D.size(), hipMemcpyDeviceToHost, b.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(b.stream));
  std::vector<double> fwd_rel(G);
  std::vector<int> fwd_status(G);
  int st_f = CISOR_OK, st_a = CISOR_OK;
  for (int gi = 0; gi < G; ++gi) {
    const int sf = solve_collect(fjobs[gi], b.groups[gi].h_states);
    const int sa = solve_collect(jobs[gi], b.groups[gi].h_states + b.groups[gi].c.T);
    fwd_rel[gi] = fjobs[gi].max_rel;
    fwd_status[gi] = sf;
    if (sf < 0 && st_f >= 0) st_f = sf;
    if (sa < 0 && st_a >= 0) st_a = sa;
  }
  for (size_t pi = 0; pi < b.probs.size(); ++pi) {
    Problem &p = b.probs[pi];
    p.t = (std::sqrt(4.0 * p.t * p.t + 1.0) + 1.0) / 2.0;
    p.k += 1;
    if (!info) continue;
    cisor_step_info &in = info[pi];
    in.D = D[pi];
    in.fwd_iters_max = in.adj_iters_max = 0;
    in.fwd_iters_sum = in.adj_iters_sum = 0;
    const int gi = p.group;
    for (int t = 0; t < p.T; ++t) {
      const int r = p.row0 + t;
      in.fwd_iters_max = std::max(in.fwd_iters_max, itf[gi][r]);
      in.adj_iters_max = std::max(in.adj_iters_max, ita[gi][r]);
      in.fwd_iters_sum += itf[gi][r];
      in.adj_iters_sum += ita[gi][r];
    }
    in.max_true_relres = std::max(jobs[gi].max_rel, fwd_rel[gi]);
    in.status = (fwd_status[gi] != CISOR_OK) ? fwd_status[gi] : jobs[gi].status;
  }
  return (st_f < 0) ? st_f : (st_a < 0 ? st_a : CISOR_OK);
}

template <typename R>
int batch_forward(cisor_batch &b, const void *const *f, void *const *u, void *const *y, const cisor_ls_opts &o,
                  int *iters) {
  using C = cplx_t<R>;
  const int G = (int)b.groups.size();
  for (size_t pi = 0; pi < b.probs.size(); ++pi)
    launch_copy<R>(b.stream, (R *)b.probs[pi].fin, (const R *)f[pi], (size_t)b.probs[pi].N);
  std::vector<std::vector<int>> it(G);
  std::vector<SolveJob> jobs(G);
  for (int gi = 0; gi < G; ++gi) {
    Group &g = b.groups[gi];
    g.c.frow = (const void *const *)g.frow_in;
    it[gi].assign(g.c.T, 0);
    jobs[gi].c = &g.c;
    jobs[gi].b = g.c.uin;
    jobs[gi].x = g.c.U;
    jobs[gi].iters = it[gi].data();
  }
  cisor_ls_opts so = o;
  if (so.start == 2) {  // caller guesses: copy them into the stacked fields
    for (size_t pi = 0; pi < b.probs.size(); ++pi) {
      const Problem &p = b.probs[pi];
      if (u[pi]) launch_copy<C>(b.stream, (C *)p.view.U, (const C *)u[pi], (size_t)p.T * p.N);
    }
  }
  const int st = solve_multi<R>(jobs.data(), G, b.sh, b.stream, false, so);
  b.fields_valid = false;   // U no longer holds the fields of the FISTA iterate
  if (st < 0) return st;
  int off = 0;
  for (size_t pi = 0; pi < b.probs.size(); ++pi) {
    Problem &p = b.probs[pi];
    if (u[pi]) launch_copy<C>(b.stream, (C *)u[pi], (const C *)p.view.U, (size_t)p.T * p.N);
    if (y && y[pi]) {
      Ctx v = p.view;
      v.stream = b.stream;
      int rc = launch_project<R>(v, (const R *)p.fin, (const C *)p.view.U, nullptr, (C *)y[pi], nullptr);
      if (rc) return rc;
    }
    if (iters)
      for (int t = 0; t < p.T; ++t) iters[off + t] = it[p.group][p.row0 + t];
    off += p.T;
  }
  CISOR_HIP_CHECK(hipStreamSynchronize(b.stream));
  return st;
}

// start modes 0-3 for every solve; 4 (extrapolated) only for a FISTA step
bool opts_valid(const cisor_ls_opts *o, int max_start = 3) {
  return o && o->tol > 0.0 && std::isfinite(o->tol) && o->maxit >= 1 && o->start >= 0 && o->start <= max_start &&
         o->replace_every >= 0 && o->check_every >= 0;
}

}  // namespace

extern "C" {

int cisor_batch_create(const cisor_geometry *geoms, int count, void *stream, cisor_batch **out) {
  if (!geoms || !out || count < 1) return CISOR_E_ARG;
  *out = nullptr;
  const int prec = geoms[0].precision;
  for (int i = 0; i < count; ++i) {
    const cisor_geometry &g = geoms[i];
    if (g.dim != 2 || g.n < 2 || !(g.h > 0) || !(g.wavelength > 0) || !(g.eps_b > 0) || g.T < 1 || g.M < 1 ||
        !g.rx_pos || g.precision != prec || (prec != 0 && prec != 1) || !transmitters_ok(g))
      return CISOR_E_ARG;
    for (int q = 0; q < 2 * g.M; ++q)
      if (!std::isfinite(g.rx_pos[q])) return CISOR_E_ARG;
    const int P = fft_length_for(g.n);
    if (P == 0 || !fft_length_supported(P)) return CISOR_E_UNSUPPORTED;
  }
  cisor_batch *b = new (std::nothrow) cisor_batch();
  if (!b) return CISOR_E_NOMEM;
  b->precision = prec;
  b->stream = (hipStream_t)stream;
  b->geoms.assign(geoms, geoms + count);
  b->probs.resize(count);
  // group problems with the same grid, in order of first appearance
  for (int i = 0; i < count; ++i) {
    int gi = -1;
    for (size_t k = 0; k < b->groups.size(); ++k)
      if (same_grid(geoms[b->groups[k].probs[0]], geoms[i])) gi = (int)k;
    if (gi < 0) {
      b->groups.emplace_back();
      gi = (int)b->groups.size() - 1;
    }
    b->groups[gi].probs.push_back(i);
  }
  const bool multi_stream = !(std::getenv("CISOR_BATCH_STREAMS") && std::atoi(std::getenv("CISOR_BATCH_STREAMS")) == 0);
  int rc = CISOR_OK;
  for (size_t gi = 0; gi < b->groups.size() && !rc; ++gi) {
    Group &g = b->groups[gi];
    const cisor_geometry &g0 = geoms[g.probs[0]];
    Ctx &c = g.c;
    c.dim = 2;
    c.n = g0.n;
    c.rows = g0.n;
    c.N = g0.n * g0.n;
    c.P = fft_length_for(g0.n);
    c.precision = prec;
    c.h = g0.h;
    c.k = 2.0 * 3.14159265358979323846 / g0.wavelength;
    c.eps_b = g0.eps_b;
    c.kb = c.k * std::sqrt(g0.eps_b);
    c.T = 0;
    for (int pi : g.probs) {
      Problem &p = b->probs[pi];
      p.group = (int)gi;
      p.row0 = c.T;
      p.n = c.n;
      p.N = c.N;
      p.T = geoms[pi].T;
      p.M = geoms[pi].M;
      c.T += p.T;
    }
    c.nrb = row_blocks(c.P, c.rows);
    c.nub = (c.N + UPD_THREADS * UPD_EPT - 1) / (UPD_THREADS * UPD_EPT);
    c.nblk = std::max(c.nrb, c.nub);
    if (multi_stream && b->groups.size() > 1) {
      if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) rc = CISOR_E_DEVICE;
      g.own_stream = true;
    } else {
      c.stream = b->stream;
    }
    for (int pi : g.probs) {
      Problem &p = b->probs[pi];
      Ctx &v = p.view;
      v.dim = 2;
      v.n = c.n;
      v.rows = c.rows;
      v.N = c.N;
      v.P = c.P;
      v.T = p.T;
      v.M = p.M;
      v.precision = prec;
      v.h = c.h;
      v.k = c.k;
      v.kb = c.kb;
      v.eps_b = c.eps_b;
      v.stream = c.stream;
    }
  }
  if (const char *env = std::getenv("CISOR_GRAPHS")) b->sh.use_graphs = b->step_sh.use_graphs = std::atoi(env) != 0;
  for (Group &g : b->groups)
    if (!rc && hipHostMalloc((void **)&g.h_states, sizeof(TxState) * 2 * g.c.T) != hipSuccess) rc = CISOR_E_NOMEM;
  if (!rc) rc = solve_shared_init(b->sh, (int)b->groups.size());
  if (!rc) rc = solve_shared_init(b->step_sh, std::max<int>(2, (int)b->groups.size()));
  if (rc) {
    batch_free(b);
    return rc;
  }
  Arena A;
  layout(*b, A);
  b->arena_bytes = A.off;
  if (hipMalloc(&b->arena, A.off) != hipSuccess) {
    b->arena = nullptr;
    batch_free(b);
    return CISOR_E_NOMEM;
  }
  A = Arena{(char *)b->arena, 0};
  layout(*b, A);
  // geometry: incident fields and receiver matrices per problem, one spectrum per group
  for (size_t gi = 0; gi < b->groups.size() && !rc; ++gi) {
    Group &g = b->groups[gi];
    bool first = true;
    std::vector<const void *> ts(g.c.T), ti(g.c.T);
    for (int pi : g.probs) {
      Problem &p = b->probs[pi];
      if ((rc = build_geometry(p.view, geoms[pi], first))) break;
      first = false;
      for (int t = 0; t < p.T; ++t) {
        ts[p.row0 + t] = p.s;
        ti[p.row0 + t] = p.fin;
      }
    }
    if (!rc && (hipMemcpy(g.frow_s, ts.data(), sizeof(void *) * ts.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(g.frow_in, ti.data(), sizeof(void *) * ti.size(), hipMemcpyHostToDevice) != hipSuccess))
      rc = CISOR_E_DEVICE;
  }
  if (rc) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return CISOR_OK;
}

int cisor_batch_destroy(cisor_batch *b) {
  if (!b) return CISOR_E_ARG;
  batch_free(b);
  return CISOR_OK;
}

int cisor_batch_set_stream(cisor_batch *b, void *stream) {
  if (!b) return CISOR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  for (Group &g : b->groups) {
    if (g.own_stream) continue;
    g.c.stream = s;
    for (int pi : g.probs) b->probs[pi].view.stream = s;
  }
  b->stream = s;
  return CISOR_OK;
}

int cisor_batch_get_sizes(const cisor_batch *b, int p, int *N, int *T, int *M, int *P, int *group) {
  if (!b || p < 0 || p >= (int)b->probs.size()) return CISOR_E_ARG;
  const Problem &q = b->probs[p];
  if (N) *N = q.N;
  if (T) *T = q.T;
  if (M) *M = q.M;
  if (P) *P = b->groups[q.group].c.P;
  if (group) *group = q.group;
  return CISOR_OK;
}

int cisor_batch_num_groups(const cisor_batch *b, int *groups) {
  if (!b || !groups) return CISOR_E_ARG;
  *groups = (int)b->groups.size();
  return CISOR_OK;
}

int cisor_batch_set_problem(cisor_batch *b, int p, const void *y_meas, double gamma, double tau) {
  if (!b || p < 0 || p >= (int)b->probs.size() || !y_meas || !(gamma > 0) || !std::isfinite(gamma) ||
      !(tau >= 0) || !std::isfinite(tau))
    return CISOR_E_ARG;
  Problem &q = b->probs[p];
  const size_t rs = b->precision ? sizeof(double) : sizeof(float);
  const size_t cs = 2 * rs;
  CISOR_HIP_CHECK(hipMemcpyAsync(q.y, y_meas, cs * q.M * q.T, hipMemcpyDeviceToDevice, b->stream));
  // f = f_prev = s = 0, t = 1, k = 0
  if (b->precision == 0) {
    launch_fill<float>(b->stream, (float *)q.f, (size_t)q.N, 0.0f);
    launch_fill<float>(b->stream, (float *)q.f_prev, (size_t)q.N, 0.0f);
    launch_fill<float>(b->stream, (float *)q.s, (size_t)q.N, 0.0f);
  } else {
    launch_fill<double>(b->stream, (double *)q.f, (size_t)q.N, 0.0);
    launch_fill<double>(b->stream, (double *)q.f_prev, (size_t)q.N, 0.0);
    launch_fill<double>(b->stream, (double *)q.s, (size_t)q.N, 0.0);
  }
  launch_fill<double>(b->stream, b->t_dev + p, 1, 1.0);
  q.gamma = gamma;
  q.tau = tau;
  q.has_data = true;
  q.t = 1.0;
  q.k = 0;
  b->fields_valid = false;
  CISOR_HIP_CHECK(hipStreamSynchronize(b->stream));
  return CISOR_OK;
}

int cisor_batch_fista_step(cisor_batch *b, double alpha, double lo, double hi, int inner, const cisor_ls_opts *o,
                           cisor_step_info *info) {
  if (!b || !(alpha >= 0) || !(alpha <= 1) || !(lo <= hi) || inner < 0 || !opts_valid(o, 4)) return CISOR_E_ARG;
  for (const Problem &p : b->probs)
    if (!p.has_data) return CISOR_E_ARG;
  if (b->precision == 0) return batch_step<float>(*b, alpha, lo, hi, inner, *o, info);
  return batch_step<double>(*b, alpha, lo, hi, inner, *o, info);
}

int cisor_batch_get_f(cisor_batch *b, int p, void *f) {
  if (!b || !f || p < 0 || p >= (int)b->probs.size()) return CISOR_E_ARG;
  const Problem &q = b->probs[p];
  const size_t rs = b->precision ? sizeof(double) : sizeof(float);
  CISOR_HIP_CHECK(hipMemcpyAsync(f, q.f, rs * q.N, hipMemcpyDeviceToDevice, b->stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(b->stream));
  return CISOR_OK;
}

int cisor_batch_forward(cisor_batch *b, const void *const *f, void *const *u, void *const *y,
                        const cisor_ls_opts *o, int *iters) {
  if (!b || !f || !u || !opts_valid(o) || o->start == 3) return CISOR_E_ARG;
  for (size_t p = 0; p < b->probs.size(); ++p)
    if (!f[p] || (o->start == 2 && !u[p])) return CISOR_E_ARG;
  if (b->precision == 0) return batch_forward<float>(*b, f, u, y, *o, iters);
  return batch_forward<double>(*b, f, u, y, *o, iters);
}

int cisor_batch_born_lipschitz(cisor_batch *b, int p, int iters, double *L) {
  if (!b || !L || iters < 1 || p < 0 || p >= (int)b->probs.size()) return CISOR_E_ARG;
  Problem &q = b->probs[p];
  // a synchronous call on the batch stream; the power iteration's FP64
  // scratch (N doubles) borrows the group's gradient-term buffer
  Ctx v = q.view;
  v.stream = b->stream;
  v.gpart = b->groups[q.group].c.gpart;
  CISOR_HIP_CHECK(hipDeviceSynchronize());
  if (b->precision == 0) return launch_born_lipschitz<float>(v, iters, L);
  return launch_born_lipschitz<double>(v, iters, L);
}

int cisor_batch_autotune(cisor_batch *b, int reps, int *variants, float *times_ms) {
  if (!b || reps < 1) return CISOR_E_ARG;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Ctx &c = b->groups[gi].c;
    int rc = autotune_columns(c, reps, times_ms ? times_ms + gi * COL_VARIANTS : nullptr);
    if (rc) return rc;
    if (variants) variants[gi] = c.col_variant;
  }
  return CISOR_OK;
}

}  // extern "C"
