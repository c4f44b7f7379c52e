// Kernels of the 3D vectorial model (appendix on 3D imaging), complex128.
//
// The convolution by the scalar kernel G is the scalar 3D FFT convolution,
// applied to the 3T component fields at once.  What the vectorial model adds
// runs here:
//   * the grad-div stencil D (eq. 3DA_def), fused into the kernel that
//     consumes the convolution (forward operator) or produces its input
//     (adjoint operator);
//   * a BiCGSTAB over the 3N unknowns of each transmitter's system, the T
//     systems in lock step, its scalars kept on the device and its dot
//     products reduced in FP64 in a fixed order;
//   * the receiver projection with the third row of the dyadic Green's
//     function (eq. discrete0_measurement), its adjoint, and the gradient of
//     eq. 3Dg_def / eq. 3Dgradient.
#include <cmath>

#include "vec3d.hpp"

namespace cisor {
namespace vec {

namespace {

enum : int { DOT_NONE = 0, DOT_V = 1, DOT_T = 2, DOT_TR = 3 };
enum : int { PH_TR = 0, PH_BETA = 1, PH_ALPHA = 2, PH_S = 3, PH_OMEGA = 4, PH_R = 5 };
constexpr int NO_MASK = -1;

__device__ __forceinline__ cd czero() { return mk<cd>(0.0, 0.0); }

// Unsigned division by a fixed divisor d >= 2 as a multiply-high and shifts
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// x / d = (t + ((x - t) >> 1)) >> (l - 1), t = mulhi(m, x), for every 32-bit x.
struct Div {
  unsigned m, s;
};
Div make_div(unsigned d) {
  unsigned l = 0;
  while ((1ull << l) < d) ++l;
  return Div{(unsigned)(((1ull << 32) * ((1ull << l) - d)) / d + 1), l - 1};
}
__device__ __forceinline__ int udiv(int x, Div f) {
  const unsigned t = __umulhi((unsigned)x, f.m);
  return (int)((t + (((unsigned)x - t) >> 1)) >> f.s);
}

struct FieldArgs {
  int n, N, T, nbv;
  double c2;              // 1 / (delta^2 k^2)
  const double *f;        // contrast [N]
  const cd *x;            // operand field (or iterate)
  const cd *b;            // right-hand side (true-residual step)
  const cd *Y;            // convolution output
  cd *rhat;
  cd *out, *pre;          // output field; convolution input
  cd *r, *p, *v, *s, *t;  // BiCGSTAB vectors
  double *part;           // [T][nbv][VNP]
  Div dN, dn2, dn;        // division by N, n^2, n
  const VState *st;
  int need;               // status a system must have for its blocks to run (NO_MASK: all)
};

// (D F)^(A) at cell q times delta^2: the second difference of F^(A) along axis
// A plus, for each other axis B, the four-corner cross difference of F^(B)
// over 4 (corners at q + sa e_A + sb e_B weighted sa sb / 4).  Neighbours
// outside the grid read as zero; the component is a template argument so
// every stride and flag is indexed statically.
template <int A>
__device__ __forceinline__ cd graddiv_c(const cd *F, int n, int N, const int (&q)[3], int cell) {
  const int st[3] = {n * n, n, 1};
  bool lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = q[d] > 0;
    hi[d] = q[d] < n - 1;
  }
  auto ld = [&](int comp, bool ok, int off) { return ok ? F[(size_t)comp * N + cell + off] : czero(); };
  const cd ce = F[(size_t)A * N + cell];
  const cd up = ld(A, hi[A], st[A]);
  const cd dn = ld(A, lo[A], -st[A]);
  double re = up.x + dn.x - 2.0 * ce.x, im = up.y + dn.y - 2.0 * ce.y;
#pragma unroll
  for (int B = 0; B < 3; ++B) {
    if (B == A) continue;
    const cd pp = ld(B, hi[A] && hi[B], st[A] + st[B]);
    const cd pm = ld(B, hi[A] && lo[B], st[A] - st[B]);
    const cd mp = ld(B, lo[A] && hi[B], -st[A] + st[B]);
    const cd mm = ld(B, lo[A] && lo[B], -st[A] - st[B]);
    re += 0.25 * ((pp.x + mm.x) - (pm.x + mp.x));
    im += 0.25 * ((pp.y + mm.y) - (pm.y + mp.y));
  }
  return mk<cd>(re, im);
}

__device__ __forceinline__ cd graddiv(const cd *F, int n, int N, int a, const int (&q)[3], int cell) {
  switch (a) {
    case 0: return graddiv_c<0>(F, n, N, q, cell);
    case 1: return graddiv_c<1>(F, n, N, q, cell);
    default: return graddiv_c<2>(F, n, N, q, cell);
  }
}

// Component, cell and cell coordinates of element e of a system's [3][N] field.
__device__ __forceinline__ void split(const FieldArgs &a, int e, int &c, int &cell, int (&q)[3]) {
  c = udiv(e, a.dN);
  cell = e - c * a.N;
  q[0] = udiv(cell, a.dn2);
  const int r = cell - q[0] * a.n * a.n;
  q[1] = udiv(r, a.dn);
  q[2] = r - q[1] * a.n;
}

__device__ __forceinline__ int cell_of(const FieldArgs &a, int e) { return e - udiv(e, a.dN) * a.N; }

__device__ __forceinline__ bool skip_system(const FieldArgs &a, int t) {
  return a.need != NO_MASK && a.st && a.st[t].status != a.need;
}

template <int NV>
__device__ __forceinline__ void write_partials(const FieldArgs &a, int t, double (&acc)[NV]) {
  __shared__ double scratch[16 * NV];
  block_sum<NV>(acc, scratch);
  if (threadIdx.x == 0) {
    double *dst = a.part + ((size_t)t * a.nbv + blockIdx.x) * VNP;
#pragma unroll
    for (int i = 0; i < NV; ++i) dst[i] = acc[i];
  }
}

// Convolution input of the operator: f x (forward) or x + D x / k^2 (adjoint).
template <bool ADJ>
__global__ void __launch_bounds__(VB) k_vpre(FieldArgs a) {
  const int t = blockIdx.y;
  if (skip_system(a, t)) return;
  const int L = 3 * a.N;
  const cd *X = a.x + (size_t)t * L;
  cd *W = a.pre + (size_t)t * L;
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    if constexpr (ADJ) {
      int c, cell, q[3];
      split(a, e, c, cell, q);
      const cd d = graddiv(X, a.n, a.N, c, q, cell);
      W[e] = mk<cd>(X[e].x + a.c2 * d.x, X[e].y + a.c2 * d.y);
    } else {
      W[e] = cscale(X[e], a.f[cell_of(a, e)]);
    }
  }
}

// out = x - Z with Z = Y + D Y / k^2 (forward) or f Y (adjoint); DOT_TR
// writes the residual b - (x - Z) instead.  Dot products per DOT mode:
//   DOT_V: <rhat, out>;  DOT_T: ||out||^2, <out, x>;  DOT_TR: ||out||^2, ||b||^2.
template <bool ADJ, int DOT>
__global__ void __launch_bounds__(VB) k_vpost(FieldArgs a) {
  const int t = blockIdx.y;
  if (skip_system(a, t)) return;
  if (DOT == DOT_T && a.st && a.st[t].sbreak) return;
  const int L = 3 * a.N;
  const size_t base = (size_t)t * L;
  const cd *Yt = a.Y + base;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    cd Z;
    if constexpr (ADJ) {
      Z = cscale(Yt[e], a.f[cell_of(a, e)]);
    } else {
      int c, cell, q[3];
      split(a, e, c, cell, q);
      const cd d = graddiv(Yt, a.n, a.N, c, q, cell);
      Z = mk<cd>(Yt[e].x + a.c2 * d.x, Yt[e].y + a.c2 * d.y);
    }
    const cd xv = a.x[base + e];
    cd o = csub(xv, Z);
    if constexpr (DOT == DOT_TR) {
      const cd bv = a.b[base + e];
      o = csub(bv, o);
      acc[1] += bv.x * bv.x + bv.y * bv.y;
    }
    a.out[base + e] = o;
    if constexpr (DOT == DOT_V) {
      const cd h = a.rhat[base + e];
      acc[0] += h.x * o.x + h.y * o.y;
      acc[1] += h.x * o.y - h.y * o.x;
    } else if constexpr (DOT == DOT_T) {
      acc[0] += o.x * o.x + o.y * o.y;
      acc[1] += o.x * xv.x + o.y * xv.y;
      acc[2] += o.x * xv.y - o.y * xv.x;
    } else if constexpr (DOT == DOT_TR) {
      acc[0] += o.x * o.x + o.y * o.y;
    }
  }
  if constexpr (DOT != DOT_NONE) write_partials<3>(a, t, acc);
}

// p = r + beta (p - omega v); forward operator input f p.
template <bool FWD>
__global__ void __launch_bounds__(VB) k_vpupd(FieldArgs a) {
  const int t = blockIdx.y;
  if (a.st[t].status != V_ITER) return;
  const cd be = a.st[t].beta, om = a.st[t].omega;
  const int L = 3 * a.N;
  const size_t base = (size_t)t * L;
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    const size_t g = base + e;
    const cd pv = cadd(a.r[g], cmul(be, csub(a.p[g], cmul(om, a.v[g]))));
    a.p[g] = pv;
    if constexpr (FWD) a.pre[g] = cscale(pv, a.f[cell_of(a, e)]);
  }
}

// s = r - alpha v and ||s||^2; forward operator input f s.
template <bool FWD>
__global__ void __launch_bounds__(VB) k_vsupd(FieldArgs a) {
  const int t = blockIdx.y;
  if (a.st[t].status != V_ITER) return;
  const cd al = a.st[t].alpha;
  const int L = 3 * a.N;
  const size_t base = (size_t)t * L;
  double acc[1] = {0.0};
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    const size_t g = base + e;
    const cd sv = csub(a.r[g], cmul(al, a.v[g]));
    a.s[g] = sv;
    if constexpr (FWD) a.pre[g] = cscale(sv, a.f[cell_of(a, e)]);
    acc[0] += sv.x * sv.x + sv.y * sv.y;
  }
  write_partials<1>(a, t, acc);
}

// x += alpha p + omega s, r = s - omega t (or x += alpha p, r = s when the
// iteration ended after s); ||r||^2 and <rhat, r>.
__global__ void __launch_bounds__(VB) k_vxr(FieldArgs a, cd *x) {
  const int t = blockIdx.y;
  if (a.st[t].status != V_ITER) return;
  const cd al = a.st[t].alpha, om = a.st[t].omega;
  const bool sb = a.st[t].sbreak != 0;
  const int L = 3 * a.N;
  const size_t base = (size_t)t * L;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    const size_t g = base + e;
    const cd sv = a.s[g];
    cd xv = cadd(x[g], cmul(al, a.p[g]));
    cd rv = sv;
    if (!sb) {
      xv = cadd(xv, cmul(om, sv));
      rv = csub(sv, cmul(om, a.t[g]));
    }
    x[g] = xv;
    a.r[g] = rv;
    const cd h = a.rhat[g];
    acc[0] += rv.x * rv.x + rv.y * rv.y;
    acc[1] += h.x * rv.x + h.y * rv.y;
    acc[2] += h.x * rv.y - h.y * rv.x;
  }
  write_partials<3>(a, t, acc);
}

// After a true-residual step: restarted systems take rhat = r, p = v = 0;
// systems with a zero right-hand side take x = 0.
__global__ void __launch_bounds__(VB) k_vrestart(FieldArgs a, cd *x) {
  const int t = blockIdx.y;
  if (!a.st[t].restart) return;
  const bool zb = a.st[t].zero_b != 0;
  const int L = 3 * a.N;
  const size_t base = (size_t)t * L;
  for (int e = blockIdx.x * VB + threadIdx.x; e < L; e += a.nbv * VB) {
    const size_t g = base + e;
    if (zb) {
      x[g] = czero();
    } else {
      a.rhat[g] = a.r[g];
      a.p[g] = czero();
      a.v[g] = czero();
    }
  }
}

__global__ void k_vstate_init(VState *st, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  VState s{};
  s.status = V_TR;
  st[t] = s;
}

__device__ __forceinline__ cd cdiv(cd a, cd b) {
  const double d = b.x * b.x + b.y * b.y;
  return mk<cd>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool cis_zero(cd a) { return a.x == 0.0 && a.y == 0.0; }

// One system per block: sum the block partials in a fixed order and advance
// the system's BiCGSTAB scalars for phase PH.
template <int PH>
__global__ void __launch_bounds__(VB) k_vscalar(VState *st, const double *part, int nbv, double tol, int maxit) {
  const int t = blockIdx.x;
  const int want = PH == PH_TR ? V_TR : V_ITER;
  if (st[t].status != want) return;
  if (PH == PH_OMEGA && st[t].sbreak) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nbv; b += VB) {
    const double *src = part + ((size_t)t * nbv + b) * VNP;
    if (PH != PH_BETA) {
      acc[0] += src[0];
      acc[1] += src[1];
      acc[2] += src[2];
    }
  }
  __shared__ double scratch[16 * 3];
  block_sum<3>(acc, scratch);
  if (threadIdx.x != 0) return;
  VState s = st[t];
  const cd one = mk<cd>(1.0, 0.0);
  if constexpr (PH == PH_TR) {
    const double rn = acc[0], bn = acc[1];
    s.rnorm2 = rn;
    s.bnorm2 = bn;
    if (!std::isfinite(rn) || !std::isfinite(bn)) {
      s.status = V_NONFINITE;
    } else if (bn == 0.0) {
      s.zero_b = 1;
      s.restart = 1;
      s.rel = 0.0;
      s.status = V_DONE;
    } else {
      s.rel = std::sqrt(rn / bn);
      if (s.rel <= tol) {
        s.status = V_DONE;
      } else if (s.iters >= maxit) {
        s.status = V_CAP;
      } else {
        s.status = V_ITER;
        s.restart = 1;
        s.sbreak = 0;
        s.rho_next = mk<cd>(rn, 0.0);
        s.rho_old = one;
        s.alpha = one;
        s.omega = one;
      }
    }
  } else if constexpr (PH == PH_BETA) {
    s.restart = 0;
    s.iters += 1;
    s.rho = s.rho_next;
    if (cis_zero(s.rho)) {
      s.status = V_TR;
    } else {
      s.beta = cmul(cdiv(s.rho, s.rho_old), cdiv(s.alpha, s.omega));
    }
  } else if constexpr (PH == PH_ALPHA) {
    const cd d = mk<cd>(acc[0], acc[1]);
    if (!std::isfinite(d.x) || !std::isfinite(d.y)) {
      s.status = V_NONFINITE;
    } else if (cis_zero(d)) {
      s.status = V_TR;
    } else {
      s.alpha = cdiv(s.rho, d);
    }
  } else if constexpr (PH == PH_S) {
    if (!std::isfinite(acc[0])) s.status = V_NONFINITE;
    else if (std::sqrt(acc[0] / s.bnorm2) <= 0.5 * tol) s.sbreak = 1;
  } else if constexpr (PH == PH_OMEGA) {
    if (!std::isfinite(acc[0]) || !std::isfinite(acc[1]) || !std::isfinite(acc[2])) s.status = V_NONFINITE;
    else if (acc[0] == 0.0) s.sbreak = 1;
    else s.omega = mk<cd>(acc[1] / acc[0], acc[2] / acc[0]);
  } else {  // PH_R
    const double rn = acc[0];
    s.rnorm2 = rn;
    s.rho_next = mk<cd>(acc[1], acc[2]);
    s.rho_old = s.rho;
    if (!std::isfinite(rn)) {
      s.status = V_NONFINITE;
    } else if (s.sbreak || std::sqrt(rn / s.bnorm2) <= 0.5 * tol || cis_zero(s.omega) || s.iters >= maxit) {
      s.status = V_TR;
    }
    s.sbreak = 0;
  }
  st[t] = s;
}

// f3 = [f, f, f]: the contrast of each component field.
__global__ void __launch_bounds__(VB) k_vrep3(const double *f, double *f3, int N) {
  const int i = blockIdx.x * VB + threadIdx.x;
  if (i >= N) return;
  const double v = f[i];
  f3[i] = v;
  f3[i + N] = v;
  f3[(size_t)i + 2 * N] = v;
}

// grad[cell] = sum_t sum_c Re(conj(E) (q + Y)) at (t, c, cell).
__global__ void __launch_bounds__(VB) k_vgrad(const cd *E, const cd *q, const cd *Y, double *grad, int N, int T) {
  const int cell = blockIdx.x * VB + threadIdx.x;
  if (cell >= N) return;
  double g = 0.0;
  for (int t = 0; t < T; ++t)
    for (int c = 0; c < 3; ++c) {
      const size_t i = ((size_t)t * 3 + c) * N + cell;
      const cd u = E[i], z = cadd(q[i], Y[i]);
      g += u.x * z.x + u.y * z.y;
    }
  grad[cell] = g;
}

__global__ void __launch_bounds__(VB) k_vgstep(const double *s, const double *g, double *z, int N, double gamma) {
  const int q = blockIdx.x * VB + threadIdx.x;
  if (q < N) z[q] = s[q] - gamma * g[q];
}

// f_prev <- f, f <- f_k, s <- f_k + c (f_k - f)
__global__ void __launch_bounds__(VB) k_vmomentum(double *f, double *f_prev, double *s, const double *fk, int N,
                                                  double c) {
  const int q = blockIdx.x * VB + threadIdx.x;
  if (q >= N) return;
  const double fo = f[q], fn = fk[q];
  f_prev[q] = fo;
  f[q] = fn;
  s[q] = fn + c * (fn - fo);
}

FieldArgs field_args(VecCtx &v) {
  FieldArgs a{};
  a.n = v.n;
  a.N = v.N;
  a.T = v.T;
  a.nbv = v.nbv;
  a.c2 = 1.0 / (v.h * v.h * v.k * v.k);
  a.dN = make_div((unsigned)v.N);
  a.dn2 = make_div((unsigned)(v.n * v.n));
  a.dn = make_div((unsigned)v.n);
  a.part = v.part;
  a.st = v.st;
  a.need = NO_MASK;
  a.r = v.ws[0];
  a.rhat = v.ws[1];
  a.p = v.ws[2];
  a.v = v.ws[3];
  a.s = v.ws[4];
  a.t = v.ws[5];
  a.pre = v.ws[6];
  a.Y = v.ws[7];
  return a;
}

int last_error() { return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE; }

// Per component field: 1 where the system's status is `need`.
__global__ void __launch_bounds__(64) k_vfield_mask(const VState *st, int need, int *fmask, int T) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < 3 * T) fmask[i] = st[i / 3].status == need ? 1 : 0;
}

// Convolution of the 3T component fields: Y = G pre (forward) or G^H pre.
// With need != NO_MASK only the systems whose status is `need` are
// transformed (the field kernels around it skip the others too, so their Y
// is never read).
int convolve(VecCtx &v, const cd *in, cd *out, bool adjoint, int need) {
  v.sc->stream = v.stream;
  const int *mask = nullptr;
  if (need != NO_MASK) {
    hipLaunchKernelGGL(k_vfield_mask, dim3((3 * v.T + 63) / 64), dim3(64), 0, v.stream, v.st, need, v.fmask, v.T);
    mask = v.fmask;
  }
  return launch_apply_G<double>(*v.sc, in, out, adjoint, mask);
}

// out = A x (DOT_NONE), the residual b - A x (DOT_TR), ... for systems with status `need`.
template <int DOT>
int operator_pass(VecCtx &v, FieldArgs a, const cd *x, cd *out, bool adjoint) {
  const dim3 grid(v.nbv, v.T);
  a.x = x;
  if (adjoint) hipLaunchKernelGGL(k_vpre<true>, grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL(k_vpre<false>, grid, dim3(VB), 0, v.stream, a);
  if (int rc = last_error()) return rc;
  if (int rc = convolve(v, a.pre, v.ws[7], adjoint, a.need)) return rc;
  a.out = out;
  if (adjoint) hipLaunchKernelGGL((k_vpost<true, DOT>), grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL((k_vpost<false, DOT>), grid, dim3(VB), 0, v.stream, a);
  return last_error();
}

template <int PH>
void scalar_step(VecCtx &v, const cisor_ls_opts &o) {
  hipLaunchKernelGGL(k_vscalar<PH>, dim3(v.T), dim3(VB), 0, v.stream, v.st, v.part, v.nbv, o.tol, o.maxit);
}

// One BiCGSTAB iteration of every system whose status is V_ITER.
int iteration(VecCtx &v, const double *f, cd *x, bool adjoint, const cisor_ls_opts &o) {
  FieldArgs a = field_args(v);
  a.f = f;
  const dim3 grid(v.nbv, v.T);
  scalar_step<PH_BETA>(v, o);
  if (adjoint) hipLaunchKernelGGL(k_vpupd<false>, grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL(k_vpupd<true>, grid, dim3(VB), 0, v.stream, a);
  a.need = V_ITER;
  // v = A p
  if (adjoint) {
    a.x = a.p;
    hipLaunchKernelGGL(k_vpre<true>, grid, dim3(VB), 0, v.stream, a);
  }
  if (int rc = last_error()) return rc;
  if (int rc = convolve(v, a.pre, v.ws[7], adjoint, a.need)) return rc;
  a.x = a.p;
  a.out = a.v;
  if (adjoint) hipLaunchKernelGGL((k_vpost<true, DOT_V>), grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL((k_vpost<false, DOT_V>), grid, dim3(VB), 0, v.stream, a);
  scalar_step<PH_ALPHA>(v, o);
  // s = r - alpha v
  if (adjoint) hipLaunchKernelGGL(k_vsupd<false>, grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL(k_vsupd<true>, grid, dim3(VB), 0, v.stream, a);
  scalar_step<PH_S>(v, o);
  // t = A s
  if (adjoint) {
    a.x = a.s;
    hipLaunchKernelGGL(k_vpre<true>, grid, dim3(VB), 0, v.stream, a);
  }
  if (int rc = last_error()) return rc;
  if (int rc = convolve(v, a.pre, v.ws[7], adjoint, a.need)) return rc;
  a.x = a.s;
  a.out = a.t;
  if (adjoint) hipLaunchKernelGGL((k_vpost<true, DOT_T>), grid, dim3(VB), 0, v.stream, a);
  else hipLaunchKernelGGL((k_vpost<false, DOT_T>), grid, dim3(VB), 0, v.stream, a);
  scalar_step<PH_OMEGA>(v, o);
  hipLaunchKernelGGL(k_vxr, grid, dim3(VB), 0, v.stream, a, x);
  scalar_step<PH_R>(v, o);
  return last_error();
}

int read_states(VecCtx &v) {
  CISOR_HIP_CHECK(hipMemcpyAsync(v.h_st, v.st, sizeof(VState) * v.T, hipMemcpyDeviceToHost, v.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(v.stream));
  return CISOR_OK;
}

}  // namespace

int launch_apply(VecCtx &v, const double *f, const cd *x, cd *y, bool adjoint) {
  FieldArgs a = field_args(v);
  a.f = f;
  return operator_pass<DOT_NONE>(v, a, x, y, adjoint);
}

int launch_solve(VecCtx &v, const double *f, const cd *b, cd *x, bool adjoint, const cisor_ls_opts &o, int *iters,
                 double *max_rel) {
  const size_t L = (size_t)v.T * 3 * v.N;
  hipLaunchKernelGGL(k_vstate_init, dim3((v.T + 63) / 64), dim3(64), 0, v.stream, v.st, v.T);
  if (o.start == 0) launch_fill<cd>(v.stream, x, L, mk<cd>(0.0, 0.0));
  else if (o.start == 1) launch_copy<cd>(v.stream, x, b, L);
  if (int rc = last_error()) return rc;
  FieldArgs a = field_args(v);
  a.f = f;
  a.b = b;
  const dim3 grid(v.nbv, v.T);
  // Each true-residual step ends every system (done, capped) or restarts it
  // with iters < maxit; each iteration raises iters of the systems it runs,
  // and a system reaching maxit goes back to a true-residual step.
  bool running = true;
  for (int outer = 0; running && outer <= o.maxit + 1; ++outer) {
    a.need = V_TR;
    if (int rc = operator_pass<DOT_TR>(v, a, x, a.r, adjoint)) return rc;
    scalar_step<PH_TR>(v, o);
    hipLaunchKernelGGL(k_vrestart, grid, dim3(VB), 0, v.stream, a, x);
    if (int rc = last_error()) return rc;
    if (int rc = read_states(v)) return rc;
    running = false;
    for (int t = 0; t < v.T; ++t) running |= v.h_st[t].status == V_ITER;
    for (int inner = 0; running && inner <= o.maxit; ++inner) {
      if (int rc = iteration(v, f, x, adjoint, o)) return rc;
      if (int rc = read_states(v)) return rc;
      bool any_tr = false, any_iter = false;
      for (int t = 0; t < v.T; ++t) {
        any_tr |= v.h_st[t].status == V_TR;
        any_iter |= v.h_st[t].status == V_ITER;
      }
      if (any_tr) break;
      running = any_iter;
    }
    if (!running) {
      for (int t = 0; t < v.T; ++t) running |= v.h_st[t].status == V_TR;
    }
  }
  int worst = CISOR_OK;
  double mr = 0.0;
  for (int t = 0; t < v.T; ++t) {
    const VState &s = v.h_st[t];
    if (iters) iters[t] = s.iters;
    mr = std::max(mr, s.rel);
    if (s.status == V_NONFINITE) worst = CISOR_E_NONFINITE;
    else if (s.status != V_DONE && worst == CISOR_OK) worst = CISOR_NOT_CONVERGED;
  }
  if (max_rel) *max_rel = mr;
  return worst;
}

// The projection Ht (I_3 x diag f) E is the scalar path's contraction with
// K = 3N receiver-row entries and the contrast repeated per component, so its
// split-K kernels (FP64 partial tiles summed in a fixed order, masks, D) serve
// here on a view of the vectorial buffers.
namespace {
Ctx gemm_view(VecCtx &v) {
  Ctx c;
  c.dim = 3;
  c.n = v.n;
  c.N = 3 * v.N;
  c.T = v.T;
  c.M = v.M;
  c.precision = 1;
  c.stream = v.stream;
  c.H = v.H;
  c.gemm_part = v.gemm_part;
  c.dpart = v.dpart;
  c.rx_mask = v.rx_mask;
  return c;
}
void replicate_f(VecCtx &v, const double *f) {
  hipLaunchKernelGGL(k_vrep3, dim3((v.N + VB - 1) / VB), dim3(VB), 0, v.stream, f, v.f3, v.N);
}
}  // namespace

int launch_project(VecCtx &v, const double *f, const cd *E, const cd *y_meas, cd *y, cd *w, double *D) {
  replicate_f(v, f);
  Ctx c = gemm_view(v);
  return cisor::launch_project<double>(c, v.f3, E, y_meas, y_meas ? w : y, D, nullptr);
}

int launch_backproject(VecCtx &v, const double *f, const cd *w, cd *q, cd *rhs) {
  replicate_f(v, f);
  Ctx c = gemm_view(v);
  return cisor::launch_backproject<double>(c, w, q, v.f3, rhs);
}

int launch_gradient(VecCtx &v, const cd *E, const cd *q, const cd *V, double *grad) {
  FieldArgs a = field_args(v);
  a.x = V;
  hipLaunchKernelGGL(k_vpre<true>, dim3(v.nbv, v.T), dim3(VB), 0, v.stream, a);
  if (int rc = last_error()) return rc;
  if (int rc = convolve(v, a.pre, v.ws[7], true, NO_MASK)) return rc;
  hipLaunchKernelGGL(k_vgrad, dim3((v.N + VB - 1) / VB), dim3(VB), 0, v.stream, E, q, v.ws[7], grad, v.N, v.T);
  return last_error();
}

int launch_fista_tail(VecCtx &v, cisor_fista_state *s, const double *grad, double gamma, double tau, double alpha,
                      double lo, double hi, int inner) {
  const dim3 grid((v.N + VB - 1) / VB), blk(VB);
  hipLaunchKernelGGL(k_vgstep, grid, blk, 0, v.stream, (const double *)s->s, grad, v.zb, v.N, gamma);
  if (int rc = last_error()) return rc;
  v.sc->stream = v.stream;
  if (int rc = launch_tv_prox<double>(*v.sc, v.zb, v.fk, gamma * tau, lo, hi, inner)) return rc;
  const double tk = s->t, tn = (std::sqrt(4.0 * tk * tk + 1.0) + 1.0) / 2.0;
  hipLaunchKernelGGL(k_vmomentum, grid, blk, 0, v.stream, (double *)s->f, (double *)s->f_prev, (double *)s->s, v.fk,
                     v.N, alpha * (tk - 1.0) / tn);
  s->t = tn;
  s->k += 1;
  return last_error();
}

}  // namespace vec
}  // namespace cisor
