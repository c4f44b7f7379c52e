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
// One launch per inner iteration: each thread owns one pixel and recomputes
// the three primal values it needs (its own and its +x, +y neighbours) from
// the previous dual, so a single pass produces the new dual and momentum
// point; a 16 x 16 tile plus a one-pixel halo of the momentum dual is staged
// in LDS.  The state (z and four dual arrays, 20 bytes per pixel in FP32)
// stays resident in L2 across the inner iterations at n <= 512.
#include <cmath>
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

// One FGP iteration.  rin: momentum dual r_k [2][N]; pold: p_{k-1} [2][N];
// pout: p_k; rout: r_{k+1}.  Tile (i, j) covers rows bi*16.., cols bj*16...
template <typename R>
__global__ void __launch_bounds__(TVB *TVB) k_fgp_iter(const R *z, const R *rin, const R *pold, R *pout, R *rout,
                                                       int n, R lam, R lo, R hi, R inv_step, R mom) {
  __shared__ R s1[TVB + 2][TVB + 2];
  __shared__ R s2[TVB + 2][TVB + 2];
  const int N = n * n;
  const int i0 = blockIdx.y * TVB - 1, j0 = blockIdx.x * TVB - 1;
  // stage r over the tile with a one-pixel halo on every side
  for (int idx = threadIdx.x; idx < (TVB + 2) * (TVB + 2); idx += TVB * TVB) {
    const int li = idx / (TVB + 2), lj = idx % (TVB + 2);
    const int gi = i0 + li, gj = j0 + lj;
    R a = 0, b = 0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      a = rin[(size_t)gi * n + gj];
      b = rin[N + (size_t)gi * n + gj];
    }
    s1[li][lj] = a;
    s2[li][lj] = b;
  }
  __syncthreads();
  const int li = threadIdx.x / TVB + 1, lj = threadIdx.x % TVB + 1;
  const int gi = i0 + li, gj = j0 + lj;
  if (gi >= n || gj >= n) return;
  const size_t e = (size_t)gi * n + gj;
  const R x0 = fmin(fmax(z[e] + lam * tv_div<R>(s1, s2, li, lj, gi, gj, n), lo), hi);
  R g1 = 0, g2 = 0;
  if (gi < n - 1) {
    const R x1 = fmin(fmax(z[e + n] + lam * tv_div<R>(s1, s2, li + 1, lj, gi + 1, gj, n), lo), hi);
    g1 = x1 - x0;
  }
  if (gj < n - 1) {
    const R x2 = fmin(fmax(z[e + 1] + lam * tv_div<R>(s1, s2, li, lj + 1, gi, gj + 1, n), lo), hi);
    g2 = x2 - x0;
  }
  R q1 = s1[li][lj] + g1 * inv_step;
  R q2 = s2[li][lj] + g2 * inv_step;
  const R nrm = sqrt(q1 * q1 + q2 * q2);
  if (nrm > R(1)) {
    q1 /= nrm;
    q2 /= nrm;
  }
  const R o1 = pold[e], o2 = pold[N + e];
  pout[e] = q1;
  pout[N + e] = q2;
  rout[e] = q1 + mom * (q1 - o1);
  rout[N + e] = q2 + mom * (q2 - o2);
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

template <typename R>
int launch_tv_prox(Ctx &c, const R *z, R *x, double lam, double lo, double hi, int iters) {
  const int n = c.n, N = c.N;
  if (lam <= 0.0 || iters == 0) {
    if (lam <= 0.0) {
      hipLaunchKernelGGL(k_clip<R>, dim3((N + 255) / 256), dim3(256), 0, c.stream, z, x, N, (R)lo, (R)hi);
    } else {
      // zero dual: x = clip(z)
      hipLaunchKernelGGL(k_clip<R>, dim3((N + 255) / 256), dim3(256), 0, c.stream, z, x, N, (R)lo, (R)hi);
    }
    return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
  }
  // buffers: zc (copy of z, so x may alias z), pA, pB, rA, rB; each dual is [2][N]
  R *base = (R *)c.tvbuf;
  R *zc = base;
  R *pA = base + N, *pB = pA + 2 * (size_t)N, *rA = pB + 2 * (size_t)N, *rB = rA + 2 * (size_t)N;
  CISOR_HIP_CHECK(hipMemcpyAsync(zc, z, sizeof(R) * N, hipMemcpyDeviceToDevice, c.stream));
  hipLaunchKernelGGL(k_zero_real<R>, dim3(256), dim3(256), 0, c.stream, pA, (size_t)8 * N);
  const dim3 grid((n + TVB - 1) / TVB, (n + TVB - 1) / TVB);
  const R inv_step = (R)(1.0 / (8.0 * lam));
  double t = 1.0;
  R *pin = pA, *pout = pB, *rin = rA, *rout = rB;
  for (int k = 0; k < iters; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const R mom = (R)((t - 1.0) / tn);
    hipLaunchKernelGGL(k_fgp_iter<R>, grid, dim3(TVB * TVB), 0, c.stream, zc, rin, pin, pout, rout, n, (R)lam,
                       (R)lo, (R)hi, inv_step, mom);
    std::swap(pin, pout);
    std::swap(rin, rout);
    t = tn;
  }
  hipLaunchKernelGGL(k_fgp_final<R>, grid, dim3(TVB * TVB), 0, c.stream, zc, pin, x, n, (R)lam, (R)lo, (R)hi);
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template int launch_tv_prox<float>(Ctx &, const float *, float *, double, double, double, int);
template int launch_tv_prox<double>(Ctx &, const double *, double *, double, double, double, int);

}  // namespace cisor
