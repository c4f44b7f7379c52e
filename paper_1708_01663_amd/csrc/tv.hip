// Proximal map of lam * TV_iso + box (eq. R_def; step eq. algo1 with
// lam = gamma * tau) by the fast gradient projection (FGP) method of Beck and
// Teboulle (2009) applied to the dual problem.
//
// With grad the forward difference (zero last difference) and div = -grad^T:
//   x(r)    = clip(z + lam div r, lo, hi)                 primal of the dual point r
//   p_k     = P_disk(r_k + grad x(r_k) / (8 lam))          projected dual ascent, 2D
//   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
//   r_{k+1} = p_k + ((t_k - 1) / t_{k+1}) (p_k - p_{k-1})
// starting from p_0 = r_1 = 0, t_1 = 1; the output is clip(z + lam div p_K).
//
// The inner iterations run in launches of up to eight (temporal blocking): a
// block stages a 16 x 16 tile plus an 8-pixel halo of z and both duals in
// LDS, iterates there, and writes the exact tile back, which cuts the launches
// per prox from 100 to 13.  The state (z and four dual arrays, 20 bytes per
// pixel in FP32) stays resident in L2 between launches at n <= 512.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace cisor {

constexpr int TVB = 16;

// div r at (i, j) from LDS-resident r1 (x-component) and r2 (y-component),
// with the last-index components treated as zero.
template <typename R>
__device__ __forceinline__ R tv_div(const R (*r1)[TVB + 2], const R (*r2)[TVB + 2], int li, int lj, int gi, int gj,
                                    int n) {
  const R a = (gi < n - 1) ? r1[li][lj] : R(0);
  const R b = (gi > 0) ? r1[li - 1][lj] : R(0);
  const R c = (gj < n - 1) ? r2[li][lj] : R(0);
  const R d = (gj > 0) ? r2[li][lj - 1] : R(0);
  return a - b + c - d;
}

// KB consecutive FGP iterations per launch (temporal blocking).  A block owns
// a TVB x TVB output tile and stages the tile plus a KB-pixel halo of z, the
// momentum dual r and the previous dual p in LDS.  One FGP iteration reads
// its neighbours at distance one, so after m iterations the values in the
// staged region are exact at least m pixels away from its edge; after kb <= KB
// iterations the tile itself is exact and is written back.
constexpr int TVK = 8;
constexpr int TVS = TVB + 2 * TVK;
struct TvWeights {
  double w[TVK];
};

// One thread per staged pixel (TVS x TVS = 1024): the block's iterations are
// latency-bound, so more waves per CU matter more than fewer threads.
constexpr int TV_THREADS = TVS * TVS;

template <typename R>
__global__ void __launch_bounds__(TV_THREADS) k_fgp_block(const R *z, const R *rin, const R *pin, R *pout, R *rout, int n,
                                                   R lam, R lo, R hi, R inv_step, TvWeights mw, int kb) {
  __shared__ R sz[TVS][TVS], s1[TVS][TVS], s2[TVS][TVS], q1[TVS][TVS], q2[TVS][TVS], sx[TVS][TVS];
  const int N = n * n;
  const int gi0 = blockIdx.y * TVB - TVK, gj0 = blockIdx.x * TVB - TVK;
  for (int idx = threadIdx.x; idx < TVS * TVS; idx += blockDim.x) {
    const int li = idx / TVS, lj = idx % TVS;
    const int gi = gi0 + li, gj = gj0 + lj;
    R a = 0, b = 0, c = 0, d = 0, e = 0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      const size_t g = (size_t)gi * n + gj;
      a = z[g];
      b = rin[g];
      c = rin[N + g];
      d = pin[g];
      e = pin[N + g];
    }
    sz[li][lj] = a;
    s1[li][lj] = b;
    s2[li][lj] = c;
    q1[li][lj] = d;
    q2[li][lj] = e;
  }
  __syncthreads();
  for (int m = 0; m < kb; ++m) {
    // primal x(r) = clip(z + lam div r) on the region still exact
    for (int idx = threadIdx.x; idx < TVS * TVS; idx += blockDim.x) {
      const int li = idx / TVS, lj = idx % TVS;
      const int gi = gi0 + li, gj = gj0 + lj;
      R xv = 0;
      if (gi >= 0 && gi < n && gj >= 0 && gj < n && li > 0 && lj > 0) {
        const R a = (gi < n - 1) ? s1[li][lj] : R(0);
        const R b = (gi > 0) ? s1[li - 1][lj] : R(0);
        const R c = (gj < n - 1) ? s2[li][lj] : R(0);
        const R d = (gj > 0) ? s2[li][lj - 1] : R(0);
        xv = fmin(fmax(sz[li][lj] + lam * (a - b + c - d), lo), hi);
      }
      sx[li][lj] = xv;
    }
    __syncthreads();
    // dual step, projection and momentum (each pixel reads and writes only
    // its own r and p, and its neighbours' x)
    const R w = (R)mw.w[m];
    for (int idx = threadIdx.x; idx < TVS * TVS; idx += blockDim.x) {
      const int li = idx / TVS, lj = idx % TVS;
      const int gi = gi0 + li, gj = gj0 + lj;
      if (!(gi >= 0 && gi < n && gj >= 0 && gj < n) || li + 1 >= TVS || lj + 1 >= TVS) continue;
      const R x0 = sx[li][lj];
      const R g1 = (gi < n - 1) ? sx[li + 1][lj] - x0 : R(0);
      const R g2 = (gj < n - 1) ? sx[li][lj + 1] - x0 : R(0);
      R a = s1[li][lj] + g1 * inv_step;
      R b = s2[li][lj] + g2 * inv_step;
      const R nrm = sqrt(a * a + b * b);
      if (nrm > R(1)) {
        a /= nrm;
        b /= nrm;
      }
      const R o1 = q1[li][lj], o2 = q2[li][lj];
      q1[li][lj] = a;
      q2[li][lj] = b;
      s1[li][lj] = a + w * (a - o1);
      s2[li][lj] = b + w * (b - o2);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < TVB * TVB; idx += blockDim.x) {
    const int li = idx / TVB + TVK, lj = idx % TVB + TVK;
    const int gi = gi0 + li, gj = gj0 + lj;
    if (gi >= n || gj >= n) continue;
    const size_t g = (size_t)gi * n + gj;
    pout[g] = q1[li][lj];
    pout[N + g] = q2[li][lj];
    rout[g] = s1[li][lj];
    rout[N + g] = s2[li][lj];
  }
}

template <typename R>
__global__ void __launch_bounds__(TVB *TVB) k_fgp_final(const R *z, const R *p, R *x, int n, R lam, R lo, R hi) {
  __shared__ R s1[TVB + 2][TVB + 2];
  __shared__ R s2[TVB + 2][TVB + 2];
  const int N = n * n;
  const int i0 = blockIdx.y * TVB - 1, j0 = blockIdx.x * TVB - 1;
  for (int idx = threadIdx.x; idx < (TVB + 2) * (TVB + 2); idx += TVB * TVB) {
    const int li = idx / (TVB + 2), lj = idx % (TVB + 2);
    const int gi = i0 + li, gj = j0 + lj;
    R a = 0, b = 0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      a = p[(size_t)gi * n + gj];
      b = p[N + (size_t)gi * n + gj];
    }
    s1[li][lj] = a;
    s2[li][lj] = b;
  }
  __syncthreads();
  const int li = threadIdx.x / TVB + 1, lj = threadIdx.x % TVB + 1;
  const int gi = i0 + li, gj = j0 + lj;
  if (gi >= n || gj >= n) return;
  const size_t e = (size_t)gi * n + gj;
  x[e] = fmin(fmax(z[e] + lam * tv_div<R>(s1, s2, li, lj, gi, gj, n), lo), hi);
}

template <typename R> __global__ void k_clip(const R *z, R *x, int N, R lo, R hi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) x[i] = fmin(fmax(z[i], lo), hi);
}
template <typename R> __global__ void k_zero_real(R *x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = 0;
}

// ---------------------------------------------------------------- 3D volumes
// The same FGP on an n^3 volume (voxel q = (i n + j) n + l, axes of strides
// n^2, n, 1): dual step 1 / (12 lam) (||grad||^2 <= 4 d with d = 3), the dual
// projected voxel by voxel onto the unit ball of R^3.  One FGP iteration is
// two launches over the volume: the primal point x(r), then the dual ascent
// with its momentum, updated in place (each thread reads and writes only its
// own voxel's duals).

// div r at voxel (i, j, l), last-index components treated as zero; r is [3][N].
template <typename R>
__device__ __forceinline__ double tv3_div(const R *r, int q, int i, int j, int l, int n, int N) {
  const int st[3] = {n * n, n, 1}, ix[3] = {i, j, l};
  double d = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R *ra = r + (size_t)a * N;
    if (ix[a] < n - 1) d += (double)ra[q];
    if (ix[a] > 0) d -= (double)ra[q - st[a]];
  }
  return d;
}

template <typename R>
__global__ void __launch_bounds__(256) k_fgp3_x(const R *z, const R *r, R *x, int n, double lam, double lo,
                                                double hi) {
  const int N = n * n * n;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int i = q / (n * n), j = (q / n) % n, l = q % n;
  const double v = (double)z[q] + lam * tv3_div<R>(r, q, i, j, l, n, N);
  x[q] = (R)fmin(fmax(v, lo), hi);
}

template <typename R>
__global__ void __launch_bounds__(256) k_fgp3_dual(const R *x, R *p, R *r, int n, double inv_step, double w) {
  const int N = n * n * n;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const int st[3] = {n * n, n, 1};
  const int ix[3] = {q / (n * n), (q / n) % n, q % n};
  const double xc = (double)x[q];
  double v[3], nrm = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double g = ix[a] < n - 1 ? (double)x[q + st[a]] - xc : 0.0;
    v[a] = (double)r[(size_t)a * N + q] + g * inv_step;
    nrm += v[a] * v[a];
  }
  const double sc = 1.0 / fmax(1.0, sqrt(nrm));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double pn = v[a] * sc;
    const size_t e = (size_t)a * N + q;
    r[e] = (R)(pn + w * (pn - (double)p[e]));
    p[e] = (R)pn;
  }
}

// The prox on a dim-dimensional grid of side n from the work area `work` of
// 9 N reals (2D: a copy of z and two ping-pong pairs of [2][N] duals; 3D: a
// copy of z, the primal point and [3][N] p and r), enqueued on stream s.  Every
// launch is a kernel (no memset or copy call), so the prox can be captured in
// a graph, and the work area needs no initial contents: the duals are zeroed
// here on every call.
template <typename R>
static void tv_prox3_run(hipStream_t s, int n, R *work, const R *z, R *x, double lam, double lo, double hi,
                         int iters) {
  const int N = n * n * n;
  // buffers: zc (copy of z, so x may alias z), xw (primal of the dual point), p, r ([3][N] each)
  R *zc = work, *xw = work + N, *p = work + 2 * (size_t)N, *r = p + 3 * (size_t)N;
  launch_copy<R>(s, zc, z, (size_t)N);
  hipLaunchKernelGGL(k_zero_real<R>, dim3(256), dim3(256), 0, s, p, (size_t)6 * N);
  const dim3 grid((N + 255) / 256), blk(256);
  const double inv_step = 1.0 / (12.0 * lam);
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    hipLaunchKernelGGL(k_fgp3_x<R>, grid, blk, 0, s, zc, r, xw, n, lam, lo, hi);
    hipLaunchKernelGGL(k_fgp3_dual<R>, grid, blk, 0, s, xw, p, r, n, inv_step, (t - 1.0) / tn);
    t = tn;
  }
  hipLaunchKernelGGL(k_fgp3_x<R>, grid, blk, 0, s, zc, p, x, n, lam, lo, hi);
}

template <typename R>
static int tv_prox_run(hipStream_t s, int dim, int n, R *work, const R *z, R *x, double lam, double lo, double hi,
                       int iters) {
  const int N = dim == 3 ? n * n * n : n * n;
  if (lam <= 0.0 || iters == 0) {
    // no regulariser, or a zero dual: x = clip(z)
    hipLaunchKernelGGL(k_clip<R>, dim3((N + 255) / 256), dim3(256), 0, s, z, x, N, (R)lo, (R)hi);
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  }
  if (dim == 3) {
    tv_prox3_run<R>(s, n, work, z, x, lam, lo, hi, iters);
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  }
  // buffers: zc (copy of z, so x may alias z), pA, pB, rA, rB; each dual is [2][N]
  R *zc = work;
  R *pA = work + N, *pB = pA + 2 * (size_t)N, *rA = pB + 2 * (size_t)N, *rB = rA + 2 * (size_t)N;
  launch_copy<R>(s, zc, z, (size_t)N);
  hipLaunchKernelGGL(k_zero_real<R>, dim3(256), dim3(256), 0, s, pA, (size_t)8 * N);
  const dim3 grid((n + TVB - 1) / TVB, (n + TVB - 1) / TVB);
  const R inv_step = (R)(1.0 / (8.0 * lam));
  double t = 1.0;
  R *pin = pA, *pout = pB, *rin = rA, *rout = rB;
  for (int k0 = 0; k0 < iters; k0 += TVK) {
    const int kb = std::min(TVK, iters - k0);
    TvWeights mw{};
    for (int m = 0; m < kb; ++m) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      mw.w[m] = (t - 1.0) / tn;
      t = tn;
    }
    hipLaunchKernelGGL(k_fgp_block<R>, grid, dim3(TV_THREADS), 0, s, zc, rin, pin, pout, rout, n, (R)lam, (R)lo,
                       (R)hi, inv_step, mw, kb);
    std::swap(pin, pout);
    std::swap(rin, rout);
  }
  hipLaunchKernelGGL(k_fgp_final<R>, grid, dim3(TVB * TVB), 0, s, zc, pin, x, n, (R)lam, (R)lo, (R)hi);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template <typename R>
int launch_tv_prox(Ctx &c, const R *z, R *x, double lam, double lo, double hi, int iters) {
  return tv_prox_run<R>(c.stream, c.dim, c.n, (R *)c.tvbuf, z, x, lam, lo, hi, iters);
}

// Isotropic TV of an n x n image (the regulariser of eq. R_def): the sum over
// pixels of the Euclidean norm of the forward differences, zero at the last
// index of each axis.  FP64 block partials, summed on the host in block order.
constexpr int TVV_BLOCKS = 512;
template <typename R> __global__ void __launch_bounds__(256) k_tv_value_part(const R *x, int n, double *part) {
  __shared__ double scratch[16];
  double v[1] = {0.0};
  const int N = n * n;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < N; q += gridDim.x * 256) {
    const int i = q / n, j = q - i * n;
    const double c = (double)x[q];
    const double gi = (i + 1 < n) ? (double)x[q + n] - c : 0.0;
    const double gj = (j + 1 < n) ? (double)x[q + 1] - c : 0.0;
    v[0] += sqrt(gi * gi + gj * gj);
  }
  block_sum<1>(v, scratch);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// The same sum over the voxels of an n^3 volume.
template <typename R> __global__ void __launch_bounds__(256) k_tv3_value_part(const R *x, int n, double *part) {
  __shared__ double scratch[16];
  double v[1] = {0.0};
  const int N = n * n * n;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < N; q += gridDim.x * 256) {
    const int st[3] = {n * n, n, 1};
    const int ix[3] = {q / (n * n), (q / n) % n, q % n};
    const double c = (double)x[q];
    double s2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double g = ix[a] + 1 < n ? (double)x[q + st[a]] - c : 0.0;
      s2 += g * g;
    }
    v[0] += sqrt(s2);
  }
  block_sum<1>(v, scratch);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename R> int launch_tv_value(Ctx &c, const R *x, double *tv) {
  // partials in the gradient-term buffer, which holds at least N doubles
  const int nb = std::min(TVV_BLOCKS, (c.N + 255) / 256);
  double *part = (double *)c.gpart;
  if (c.dim == 3)
    hipLaunchKernelGGL(k_tv3_value_part<R>, dim3(nb), dim3(256), 0, c.stream, x, c.n, part);
  else
    hipLaunchKernelGGL(k_tv_value_part<R>, dim3(nb), dim3(256), 0, c.stream, x, c.n, part);
  std::vector<double> h(nb);
  CISOR_HIP_CHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, c.stream));
  CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  double s = 0.0;
  for (double v : h) s += v;
  *tv = s;
  return std::isfinite(s) ? CISOR_OK : CISOR_E_NONFINITE;
}

template int launch_tv_value<float>(Ctx &, const float *, double *);
template int launch_tv_value<double>(Ctx &, const double *, double *);
template int launch_tv_prox<float>(Ctx &, const float *, float *, double, double, double, int);
template int launch_tv_prox<double>(Ctx &, const double *, double *, double, double, double, int);

}  // namespace cisor

// ------------------------------------------------ the non-allocating prox
// cisor_tv_prox_noalloc runs the same kernels as cisor_tv_prox on a work area
// that lives in this file-scope device array instead of a context buffer, so
// it calls no allocator.  Each GPU holds its own copy of the array; its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and kept, and only that address is ever handed to kernels (the
// array's name is a host-side stand-in in host code).
static __device__ __align__(256) unsigned char scratch[CISOR_TV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CISOR_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CISOR_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CISOR_OK;
}
}  // namespace

extern "C" int cisor_tv_prox_noalloc(int dim, int n, int precision, const void *z, void *x, double lam, double lo,
                                     double hi, int inner_iters, void *stream) {
  if ((dim != 2 && dim != 3) || n < 1 || (precision != 0 && precision != 1) || !z || !x || !(lam >= 0) ||
      !std::isfinite(lam) || !(lo <= hi) || inner_iters < 0)
    return CISOR_E_ARG;
  const long long N = dim == 3 ? (long long)n * n * n : (long long)n * n;
  if (N > CISOR_TV_NOALLOC_MAX_N) return CISOR_E_SIZE;
  void *work = nullptr;
  if (int rc = scratch_of_current_device(&work)) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (precision == 0)
    return cisor::tv_prox_run<float>(s, dim, n, (float *)work, (const float *)z, (float *)x, lam, lo, hi,
                                     inner_iters);
  return cisor::tv_prox_run<double>(s, dim, n, (double *)work, (const double *)z, (double *)x, lam, lo, hi,
                                    inner_iters);
}
