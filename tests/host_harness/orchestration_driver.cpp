// Drives the library's host orchestration against the host-only HIP stand-in
// (hip_stub.cpp): a batch of uneven 2D problems stepped through relaxed-FISTA
// iterations (start modes 2 and 4), a batched forward solve, and a single
// context's gradient, forward and FISTA calls.  Kernels do not run, so no
// number is checked here; what is checked is the host side: AddressSanitizer
// watches every host access and every copy into or out of the stand-in's
// device memory, and the stand-in counts breaches of the stream, event and
// graph rules.  Exit status 0 only when there are none.
//
// Usage: orchestration_driver <problems file> <steps>
//   problems file: one "n T" pair per line (grid side, transmitters; M = 4 T).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/cisor.h"

extern "C" {
typedef struct cisor_batch cisor_batch;
int cisor_batch_create(const cisor_geometry *, int, void *, cisor_batch **);
int cisor_batch_destroy(cisor_batch *);
int cisor_batch_autotune(cisor_batch *, int, int *, float *);
int cisor_batch_set_problem(cisor_batch *, int, const void *, double, double);
int cisor_batch_fista_step(cisor_batch *, double, double, double, int, const cisor_ls_opts *, cisor_step_info *);
int cisor_batch_forward(cisor_batch *, const void *const *, void *const *, void *const *, const cisor_ls_opts *,
                        int *);
int cisor_batch_num_groups(const cisor_batch *, int *);
void hip_stub_report(long long *out);
}

static const double kPi = 3.14159265358979323846;

struct Geo {
  std::vector<double> tx, rx;
  cisor_geometry g{};
};

static Geo make_geo(int n, int T, int M) {
  Geo G;
  const double h = 0.1, R = n * h;   // receivers on a ring of twice the half-width
  for (int t = 0; t < T; ++t) {
    G.tx.push_back(std::cos(2 * kPi * t / T));
    G.tx.push_back(std::sin(2 * kPi * t / T));
  }
  for (int m = 0; m < M; ++m) {
    G.rx.push_back(R * std::cos(2 * kPi * m / M));
    G.rx.push_back(R * std::sin(2 * kPi * m / M));
  }
  G.g.dim = 2;
  G.g.n = n;
  G.g.h = h;
  G.g.wavelength = 1.0;
  G.g.eps_b = 1.0;
  G.g.T = T;
  G.g.M = M;
  G.g.precision = 0;
  G.g.tx_kind = 0;
  return G;
}

#define EXPECT_OK(call)                                                         \
  do {                                                                          \
    const int _rc = (call);                                                     \
    if (_rc < 0) {                                                              \
      std::fprintf(stderr, "[driver] %s returned %d\n", #call, _rc);           \
      return 2;                                                                 \
    }                                                                           \
  } while (0)

int main(int argc, char **argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: %s problems_file steps\n", argv[0]);
    return 2;
  }
  FILE *fp = std::fopen(argv[1], "r");
  if (!fp) return 2;
  std::vector<Geo> geos;
  int n, T;
  while (std::fscanf(fp, "%d %d", &n, &T) == 2) geos.push_back(make_geo(n, T, 4 * T));
  std::fclose(fp);
  const int steps = std::atoi(argv[2]);
  std::vector<cisor_geometry> gs;
  for (Geo &G : geos) {
    G.g.tx_dir = G.tx.data();
    G.g.rx_pos = G.rx.data();
    gs.push_back(G.g);
  }
  const int P = (int)gs.size();
  cisor_batch *b = nullptr;
  EXPECT_OK(cisor_batch_create(gs.data(), P, nullptr, &b));
  int groups = 0;
  cisor_batch_num_groups(b, &groups);
  std::vector<int> variants(groups);
  std::vector<float> times(10 * groups);
  EXPECT_OK(cisor_batch_autotune(b, 2, variants.data(), times.data()));
  std::vector<void *> y(P), f(P), u(P);
  for (int p = 0; p < P; ++p) {
    const size_t N = (size_t)gs[p].n * gs[p].n;
    hipMalloc(&y[p], 8 * (size_t)gs[p].T * gs[p].M);
    hipMalloc(&f[p], 4 * N);
    hipMalloc(&u[p], 8 * (size_t)gs[p].T * N);
    EXPECT_OK(cisor_batch_set_problem(b, p, y[p], 1e-3, 5e-4));
  }
  std::vector<cisor_step_info> info(P);
  cisor_ls_opts o{1e-6, 20000, 2, 50, 10};
  for (int k = 0; k < steps; ++k) EXPECT_OK(cisor_batch_fista_step(b, 0.96, 0.0, 2.0, 100, &o, info.data()));
  o.start = 4;
  for (int k = 0; k < steps; ++k) EXPECT_OK(cisor_batch_fista_step(b, 0.96, 0.0, 2.0, 100, &o, info.data()));
  o.start = 1;
  std::vector<int> iters(4096 * 8);
  EXPECT_OK(cisor_batch_forward(b, f.data(), u.data(), y.data(), &o, iters.data()));
  EXPECT_OK(cisor_batch_destroy(b));

  // one context: gradient, forward, FISTA steps with every start mode
  Geo G = make_geo(24, 5, 12);
  G.g.tx_dir = G.tx.data();
  G.g.rx_pos = G.rx.data();
  cisor_ctx *c = nullptr;
  EXPECT_OK(cisor_create(&G.g, nullptr, &c));
  void *fc, *yc, *uc, *vc, *gc, *s, *fp2, *fpr;
  const size_t N = 24 * 24;
  hipMalloc(&fc, 4 * N);
  hipMalloc(&gc, 4 * N);
  hipMalloc(&yc, 8 * 5 * 12);
  hipMalloc(&uc, 8 * 5 * N);
  hipMalloc(&vc, 8 * 5 * N);
  hipMalloc(&s, 4 * N);
  hipMalloc(&fp2, 4 * N);
  hipMalloc(&fpr, 4 * N);
  double D = 0;
  int it2[10];
  cisor_ls_opts oc{1e-6, 20000, 1, 50, 10};
  EXPECT_OK(cisor_grad(c, fc, yc, gc, &D, uc, vc, &oc, it2));
  EXPECT_OK(cisor_forward(c, fc, uc, yc, &oc, it2));
  cisor_fista_state st{fp2, fpr, s, 1.0, 0};
  cisor_step_info si;
  for (int start : {2, 4, 1, 0})
    for (int k = 0; k < steps; ++k) {
      oc.start = start;
      EXPECT_OK(cisor_fista_step(c, &st, yc, 1e-3, 5e-4, 0.96, 0.0, 2.0, 100, &oc, &si));
    }
  EXPECT_OK(cisor_destroy(c));
  for (void *q : {fc, gc, yc, uc, vc, s, fp2, fpr}) hipFree(q);
  for (int p = 0; p < P; ++p) {
    hipFree(y[p]);
    hipFree(f[p]);
    hipFree(u[p]);
  }

  long long r[7];
  hip_stub_report(r);
  std::printf("groups %d problems %d violations %lld kernel_launches %lld graph_launches %lld graphs_instantiated %lld "
              "graph_execs_destroyed %lld count_reads %lld captures %lld\n",
              groups, P, r[0], r[1], r[2], r[3], r[4], r[5], r[6]);
  return r[0] == 0 ? 0 : 1;
}
