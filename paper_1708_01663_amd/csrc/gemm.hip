// Receiver projection and its adjoint (the one dense contraction of the path).
//
//   projection      y_t = H diag(u_t) f           (eq. Z_def), [T][M]
//   misfit          w_t = y_t - y_meas,t, D = 1/2 sum |w|^2 (eq. D_def, FP64)
//   back-projection q_t = H^H w_t, b_t = f q_t    (right-hand side of eq. u_and_v)
//
// The projection contracts over the N pixels (K = N, large) into a small
// M x T output, so it is split over K: each block produces a partial tile,
// and a second kernel sums the partials in FP64 in a fixed order.  The FP32
// path runs on the matrix cores (v_mfma_f32_32x32x2_f32) as a real GEMM on
// the interleaved complex operands, with Gauss's three real products per
// complex product (four without); the FP64 path uses plain FMA.
#include <vector>

#include "internal.hpp"

namespace cisor {

constexpr int PJ_KCHUNK = PROJ_KCHUNK;  // pixels per split-K chunk
constexpr int PJ_MT = 32;        // receivers per block tile
constexpr int PJ_TT = 64;        // transmitters per block tile

// ---------------------------------------------------------------- generic (FMA) projection
// Block: 256 threads; tile = 32 receivers x up to 64 transmitters, one K chunk.
// Each thread accumulates 8 (m, t) pairs.
template <typename R>
__global__ void __launch_bounds__(256) k_project_fma(const cplx_t<R> *H, const R *f, const cplx_t<R> *u, cd *part,
                                                     int M, int N, int T) {
  using C = cplx_t<R>;
  constexpr int KS = 32;  // pixels staged per step
  __shared__ C sh[PJ_MT][KS + 1];
  __shared__ C su[PJ_TT][KS + 1];
  const int m0 = blockIdx.x * PJ_MT, t0 = blockIdx.y * PJ_TT, kc = blockIdx.z;
  const int k0 = kc * PJ_KCHUNK;
  const int kend = min(k0 + PJ_KCHUNK, N);
  const int tm = threadIdx.x % PJ_MT;     // receiver within tile
  const int tg = threadIdx.x / PJ_MT;     // 0..7: transmitter group
  double accr[8] = {0}, acci[8] = {0};
  for (int kb = k0; kb < kend; kb += KS) {
    for (int i = threadIdx.x; i < PJ_MT * KS; i += 256) {
      const int mm = i / KS, kk = i % KS;
      const int m = m0 + mm, k = kb + kk;
      sh[mm][kk] = (m < M && k < kend) ? H[(size_t)m * N + k] : mk<C>(0, 0);
    }
    for (int i = threadIdx.x; i < PJ_TT * KS; i += 256) {
      const int tt = i / KS, kk = i % KS;
      const int t = t0 + tt, k = kb + kk;
      C val = mk<C>(0, 0);
      if (t < T && k < kend) val = cscale(u[(size_t)t * N + k], f[k]);
      su[tt][kk] = val;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KS; ++kk) {
      const C h = sh[tm][kk];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const C x = su[tg + 8 * j][kk];
        accr[j] += (double)h.x * x.x - (double)h.y * x.y;
        acci[j] += (double)h.x * x.y + (double)h.y * x.x;
      }
    }
    __syncthreads();
  }
  const int m = m0 + tm;
  if (m >= M) return;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int t = t0 + tg + 8 * j;
    if (t < T) part[((size_t)kc * T + t) * M + m] = mk<cd>(accr[j], acci[j]);
  }
}

// ---------------------------------------------------------------- MFMA projection (FP32)
// Real GEMM view: for a receiver row m and a transmitter column t,
//   Re y = sum_q Hr*Xr - Hi*Xi,  Im y = sum_q Hr*Xi + Hi*Xr,   X = f u.
// v_mfma_f32_32x32x2f32 multiplies a 32x2 A block by a 2x32 B block: lane l
// supplies A[l%32][l/32] and B[l/32][l%32] and holds C[8*(r/4) + 4*(l/32) + r%4][l%32]
// in accumulator register r.  A block of 4 waves covers 64 receivers x 64
// transmitters (one 32x32 quadrant per wave) for one K chunk.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int KS>
__global__ void __launch_bounds__(256) k_project_mfma(const cf *H, const float *f, const cf *u, cd *part, int M,
                                                      int N, int T) {
  constexpr int PER = 64 * KS / 256;   // tile elements per thread and operand
  __shared__ cf sh[64][KS + 1];
  __shared__ cf su[64][KS + 1];
  const int m0 = blockIdx.x * 64, kc = blockIdx.z;
  const int k0 = kc * PJ_KCHUNK;
  const int kend = min(k0 + PJ_KCHUNK, N);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave & 1, wt = wave >> 1;
  // three real products per complex one (Gauss): P1 = Hr Xr, P2 = Hi Xi,
  // P3 = (Hr + Hi)(Xr + Xi); Re = P1 - P2, Im = P3 - P1 - P2
  floatx16 acc1 = {0}, acc2 = {0}, acc3 = {0};
  // the next step's H and f u elements are loaded into registers while the
  // current step runs on the matrix cores
  cf rh[PER], ru[PER];
  auto load = [&](int kb) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int mm = i / KS, kk = i % KS;
      const int m = m0 + mm, k = kb + kk;
      rh[e] = (m < M && k < kend) ? H[(size_t)m * N + k] : mk<cf>(0, 0);
      ru[e] = (mm < T && k < kend) ? cscale(u[(size_t)mm * N + k], f[k]) : mk<cf>(0, 0);
    }
  };
  load(k0);
  for (int kb = k0; kb < kend; kb += KS) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = threadIdx.x + 256 * e;
      sh[i / KS][i % KS] = rh[e];
      su[i / KS][i % KS] = ru[e];
    }
    __syncthreads();
    if (kb + KS < kend) load(kb + KS);
    const int am = wm * 32 + (lane & 31);
    const int bt = wt * 32 + (lane & 31);
    const int kl = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < KS; kk += 2) {
      const cf a = sh[am][kk + kl];
      const cf b = su[bt][kk + kl];
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x + a.y, b.x + b.y, acc3, 0, 0, 0);
    }
    __syncthreads();
  }
  const int t = wt * 32 + (lane & 31);
  if (t >= T) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
    const double p1 = acc1[r], p2 = acc2[r], p3 = acc3[r];
    if (m < M) part[((size_t)kc * T + t) * M + m] = mk<cd>(p1 - p2, p3 - p1 - p2);
  }
}

// Narrow variant for at most 16 transmitters (one 16-wide transmitter tile),
// on v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and holds C[4*(l/16) + r][l%16] in accumulator register r.  Four waves own
// 16 receivers each (64 per block) against the same 16 transmitters, so no
// matrix-core work is spent on absent transmitters and H is still read once.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int PJ_NARROW_T = 16;   // transmitters of the narrow projection tiles

template <int KS>
__global__ void __launch_bounds__(256) k_project_mfma16(const cf *H, const float *f, const cf *u, cd *part, int M,
                                                        int N, int T) {
  constexpr int PH = 64 * KS / 256, PU = PJ_NARROW_T * KS / 256;
  static_assert(PH * 256 == 64 * KS && PU * 256 == PJ_NARROW_T * KS, "tile loads must cover the tiles");
  __shared__ cf sh[64][KS + 1];
  __shared__ cf su[PJ_NARROW_T][KS + 1];
  const int m0 = blockIdx.x * 64, kc = blockIdx.z;
  const int k0 = kc * PJ_KCHUNK;
  const int kend = min(k0 + PJ_KCHUNK, N);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  floatx4 acc1 = {0}, acc2 = {0}, acc3 = {0};   // Gauss's three products, as in k_project_mfma
  cf rh[PH], ru[PU];
  auto load = [&](int kb) {
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int mm = i / KS, kk = i % KS;
      const int m = m0 + mm, k = kb + kk;
      rh[e] = (m < M && k < kend) ? H[(size_t)m * N + k] : mk<cf>(0, 0);
    }
#pragma unroll
    for (int e = 0; e < PU; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int tt = i / KS, kk = i % KS;
      const int k = kb + kk;
      ru[e] = (tt < T && k < kend) ? cscale(u[(size_t)tt * N + k], f[k]) : mk<cf>(0, 0);
    }
  };
  load(k0);
  for (int kb = k0; kb < kend; kb += KS) {
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      sh[i / KS][i % KS] = rh[e];
    }
#pragma unroll
    for (int e = 0; e < PU; ++e) {
      const int i = threadIdx.x + 256 * e;
      su[i / KS][i % KS] = ru[e];
    }
    __syncthreads();
    if (kb + KS < kend) load(kb + KS);
    const int am = wave * 16 + (lane & 15);
    const int bt = lane & 15;
    const int kl = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const cf a = sh[am][kk + kl];
      const cf b = su[bt][kk + kl];
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, acc3, 0, 0, 0);
    }
    __syncthreads();
  }
  const int t = lane & 15;
  if (t >= T) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + wave * 16 + 4 * (lane >> 4) + r;
    const double p1 = acc1[r], p2 = acc2[r], p3 = acc3[r];
    if (m < M) part[((size_t)kc * T + t) * M + m] = mk<cd>(p1 - p2, p3 - p1 - p2);
  }
}

// Sum the split-K partials in FP64, form y (or w = y - y_meas) and block
// partials of |w|^2.  A block owns PROJ_REDUCE_OUT outputs; its 256 threads
// are RD_LANES chunk lanes per output, lane l summing chunks l, l + RD_LANES, ...,
// and the lanes' sums are added in lane order: a fixed order, independent of
// timing, with short dependent chains even for thousands of chunks.
constexpr int RD_LANES = 256 / PROJ_REDUCE_OUT;

template <typename R>
__global__ void __launch_bounds__(256) k_project_reduce(const cd *part, int kchunks, const cplx_t<R> *y_meas,
                                                        cplx_t<R> *y, double *dpart, int MT,
                                                        const float *__restrict__ mask) {
  using C = cplx_t<R>;
  __shared__ double lr[RD_LANES][PROJ_REDUCE_OUT], li[RD_LANES][PROJ_REDUCE_OUT];
  __shared__ double scratch[16];
  const int o = threadIdx.x % PROJ_REDUCE_OUT, l = threadIdx.x / PROJ_REDUCE_OUT;
  const int i = blockIdx.x * PROJ_REDUCE_OUT + o;
  double sr = 0.0, si = 0.0;
  if (i < MT) {
    for (int k = l; k < kchunks; k += RD_LANES) {
      const cd p = part[(size_t)k * MT + i];
      sr += p.x;
      si += p.y;
    }
  }
  lr[l][o] = sr;
  li[l][o] = si;
  __syncthreads();
  double acc[1] = {0.0};
  if (l == 0 && i < MT) {
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int j = 0; j < RD_LANES; ++j) {
      ar += lr[j][o];
      ai += li[j][o];
    }
    if (y_meas) {
      const C ym = y_meas[i];
      ar -= ym.x;
      ai -= ym.y;
      if (mask && mask[i] == 0.0f) ar = ai = 0.0;   // a switched-off receiver has no datum
    }
    y[i] = mk<C>((R)ar, (R)ai);
    acc[0] = ar * ar + ai * ai;
  }
  block_sum<1>(acc, scratch);
  if (threadIdx.x == 0) dpart[blockIdx.x] = acc[0];
}

// D = 1/2 sum of the n block partials: each of the 64 lanes sums a strided
// subset, lane 0 adds the 64 sums in lane order.
__global__ void __launch_bounds__(64) k_sum_dpart(const double *dpart, int n, double *out) {
  __shared__ double ls[64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += dpart[i];
  ls[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int j = 0; j < 64; ++j) t += ls[j];
  out[0] = 0.5 * t;
}

template <typename R>
int launch_project(Ctx &c, const R *f, const cplx_t<R> *u, const cplx_t<R> *y_meas, cplx_t<R> *y,
                   double *D_host, double *D_dev) {
  const int kchunks = (c.N + PJ_KCHUNK - 1) / PJ_KCHUNK;
  cd *part = (cd *)c.gemm_part;
  if constexpr (std::is_same<R, float>::value) {
    if (c.T <= PJ_NARROW_T) {
      dim3 g((c.M + 63) / 64, 1, kchunks);
      hipLaunchKernelGGL(k_project_mfma16<32>, g, dim3(256), 0, c.stream, (const cf *)c.H, f, u, part, c.M, c.N,
                         c.T);
    } else if (c.T <= 64) {
      dim3 g((c.M + 63) / 64, 1, kchunks);
      hipLaunchKernelGGL(k_project_mfma<32>, g, dim3(256), 0, c.stream, (const cf *)c.H, f, u, part, c.M, c.N,
                         c.T);
    } else {
      dim3 g((c.M + PJ_MT - 1) / PJ_MT, (c.T + PJ_TT - 1) / PJ_TT, kchunks);
      hipLaunchKernelGGL(k_project_fma<float>, g, dim3(256), 0, c.stream, (const cf *)c.H, f, u, part, c.M, c.N,
                         c.T);
    }
  } else {
    dim3 g((c.M + PJ_MT - 1) / PJ_MT, (c.T + PJ_TT - 1) / PJ_TT, kchunks);
    hipLaunchKernelGGL(k_project_fma<double>, g, dim3(256), 0, c.stream, (const cd *)c.H, f, u, part, c.M, c.N,
                       c.T);
  }
  const int MT = c.M * c.T;
  const int nb = (MT + PROJ_REDUCE_OUT - 1) / PROJ_REDUCE_OUT;
  hipLaunchKernelGGL(k_project_reduce<R>, dim3(nb), dim3(256), 0, c.stream, part, kchunks, y_meas, y, c.dpart, MT,
                     (const float *)c.rx_mask);
  if (D_dev) hipLaunchKernelGGL(k_sum_dpart, dim3(1), dim3(64), 0, c.stream, c.dpart, nb, D_dev);
  if (D_host) {
    hipLaunchKernelGGL(k_sum_dpart, dim3(1), dim3(64), 0, c.stream, c.dpart, nb, c.dpart + nb);
    CISOR_HIP_CHECK(hipMemcpyAsync(D_host, c.dpart + nb, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    CISOR_HIP_CHECK(hipStreamSynchronize(c.stream));
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

// ---------------------------------------------------------------- back-projection
// q[t][k] = sum_m conj(H[m][k]) w[t][m]; optional b = f q.  Block: 256 pixels
// x all transmitters in groups of 16; w staged in LDS per receiver chunk.
template <typename R>
__global__ void __launch_bounds__(256) k_backproject(const cplx_t<R> *H, const cplx_t<R> *w, cplx_t<R> *q,
                                                     const R *f, cplx_t<R> *b, int M, int N, int T) {
  using C = cplx_t<R>;
  constexpr int TG = 16, MS = 64;
  __shared__ C sw[TG][MS];
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int t0 = blockIdx.y * TG;
  R accr[TG] = {0}, acci[TG] = {0};
  for (int mb = 0; mb < M; mb += MS) {
    for (int i = threadIdx.x; i < TG * MS; i += 256) {
      const int tt = i / MS, mm = i % MS;
      sw[tt][mm] = (t0 + tt < T && mb + mm < M) ? w[(size_t)(t0 + tt) * M + mb + mm] : mk<C>(0, 0);
    }
    __syncthreads();
    if (k < N) {
      const int mmax = min(MS, M - mb);
      for (int mm = 0; mm < mmax; ++mm) {
        const C h = H[(size_t)(mb + mm) * N + k];
#pragma unroll
        for (int j = 0; j < TG; ++j) {
          const C x = sw[j][mm];
          accr[j] += h.x * x.x + h.y * x.y;
          acci[j] += h.x * x.y - h.y * x.x;
        }
      }
    }
    __syncthreads();
  }
  if (k >= N) return;
#pragma unroll
  for (int j = 0; j < TG; ++j) {
    const int t = t0 + j;
    if (t < T) {
      const C val = mk<C>(accr[j], acci[j]);
      q[(size_t)t * N + k] = val;
      if (b) b[(size_t)t * N + k] = cscale(val, f[k]);
    }
  }
}

// ---------------------------------------------------------------- MFMA back-projection (FP32)
// Q[t][k] = sum_m W[t][m] conj(H[m][k]) as real GEMMs on v_mfma_f32_32x32x2f32:
//   Re Q = sum Wr Hr + Wi Hi,  Im Q = sum Wi Hr - Wr Hi,
// rows = transmitters (A operand: lane l supplies W[l%32][m + l/32]), columns =
// pixels (B operand: H[m + l/32][l%32]).  A block of four waves owns 64
// transmitters x 128 pixels; wave w holds transmitter half w%2 and pixel half
// w/2 (two 32-pixel column blocks), so H is read from HBM exactly once per
// 64 transmitters.  W and H are staged in LDS 16 receivers at a time.
constexpr int BP_MS = 16, BP_PT = 128, BP_TT = 64;

__global__ void __launch_bounds__(256) k_backproject_mfma(const cf *H, const cf *w, cf *q, const float *f, cf *b,
                                                          int M, int N, int T) {
  constexpr int PW = BP_TT * BP_MS / 256, PH = BP_MS * BP_PT / 256;
  __shared__ cf sw[BP_TT][BP_MS + 1];
  __shared__ cf shh[BP_MS][BP_PT + 1];
  const int k0 = blockIdx.x * BP_PT, t0 = blockIdx.y * BP_TT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wt = wave & 1, wp = wave >> 1;
  // Gauss's three products: P1 = Wr Hr, P2 = Wi Hi, P3 = (Wr + Wi)(Hr - Hi);
  // Re = P1 + P2, Im = P3 - P1 + P2
  floatx16 acc1[2] = {{0}, {0}}, acc2[2] = {{0}, {0}}, acc3[2] = {{0}, {0}};
  // next step's W and H staged in registers during the current step's MFMAs
  cf rw[PW], rh[PH];
  auto load = [&](int m0) {
#pragma unroll
    for (int e = 0; e < PW; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int tt = i / BP_MS, mm = i % BP_MS;
      const int t = t0 + tt, m = m0 + mm;
      rw[e] = (t < T && m < M) ? w[(size_t)t * M + m] : mk<cf>(0, 0);
    }
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int mm = i / BP_PT, kk = i % BP_PT;
      const int m = m0 + mm, k = k0 + kk;
      rh[e] = (m < M && k < N) ? H[(size_t)m * N + k] : mk<cf>(0, 0);
    }
  };
  load(0);
  for (int m0 = 0; m0 < M; m0 += BP_MS) {
#pragma unroll
    for (int e = 0; e < PW; ++e) {
      const int i = threadIdx.x + 256 * e;
      sw[i / BP_MS][i % BP_MS] = rw[e];
    }
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      shh[i / BP_PT][i % BP_PT] = rh[e];
    }
    __syncthreads();
    if (m0 + BP_MS < M) load(m0 + BP_MS);
    const int ar = wt * 32 + (lane & 31);
    const int kl = lane >> 5;
#pragma unroll
    for (int mm = 0; mm < BP_MS; mm += 2) {
      const cf a = sw[ar][mm + kl];
      const float as = a.x + a.y;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const cf h = shh[mm + kl][wp * 64 + j * 32 + (lane & 31)];
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, h.x, acc1[j], 0, 0, 0);
        acc2[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, h.y, acc2[j], 0, 0, 0);
        acc3[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as, h.x - h.y, acc3[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = k0 + wp * 64 + j * 32 + (lane & 31);
    if (k >= N) continue;
    const float fk = b ? f[k] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = t0 + wt * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
      if (t >= T) continue;
      const double p1 = acc1[j][r], p2 = acc2[j][r], p3 = acc3[j][r];
      const cf val = mk<cf>((float)(p1 + p2), (float)(p3 - p1 + p2));
      q[(size_t)t * N + k] = val;
      if (b) b[(size_t)t * N + k] = mk<cf>(val.x * fk, val.y * fk);
    }
  }
}

// Narrow variant for at most 16 transmitters on v_mfma_f32_16x16x4f32 (lane
// layout as in k_project_mfma16): rows = the 16 transmitters (A operand
// W[l%16][m + l/16]), columns = pixels (B operand H[m + l/16][l%16]).  Each of
// the four waves owns 16 pixels (64 per block), so every pixel column of H is
// read once and no matrix-core work is spent on absent transmitters.
constexpr int BP16_PT = 64;

__global__ void __launch_bounds__(256) k_backproject_mfma16(const cf *H, const cf *w, cf *q, const float *f, cf *b,
                                                            int M, int N, int T) {
  constexpr int PH = BP_MS * BP16_PT / 256;
  static_assert(PH * 256 == BP_MS * BP16_PT && PJ_NARROW_T * BP_MS == 256, "tile loads must cover the tiles");
  __shared__ cf sw[PJ_NARROW_T][BP_MS + 1];
  __shared__ cf shh[BP_MS][BP16_PT + 1];
  const int k0 = blockIdx.x * BP16_PT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  floatx4 acc1 = {0}, acc2 = {0}, acc3 = {0};   // Gauss's three products, as in k_backproject_mfma
  cf rw, rh[PH];
  auto load = [&](int m0) {
    {
      const int tt = threadIdx.x / BP_MS, mm = threadIdx.x % BP_MS;
      const int m = m0 + mm;
      rw = (tt < T && m < M) ? w[(size_t)tt * M + m] : mk<cf>(0, 0);
    }
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      const int mm = i / BP16_PT, kk = i % BP16_PT;
      const int m = m0 + mm, k = k0 + kk;
      rh[e] = (m < M && k < N) ? H[(size_t)m * N + k] : mk<cf>(0, 0);
    }
  };
  load(0);
  for (int m0 = 0; m0 < M; m0 += BP_MS) {
    sw[threadIdx.x / BP_MS][threadIdx.x % BP_MS] = rw;
#pragma unroll
    for (int e = 0; e < PH; ++e) {
      const int i = threadIdx.x + 256 * e;
      shh[i / BP16_PT][i % BP16_PT] = rh[e];
    }
    __syncthreads();
    if (m0 + BP_MS < M) load(m0 + BP_MS);
    const int ar = lane & 15;
    const int kl = lane >> 4;
#pragma unroll
    for (int mm = 0; mm < BP_MS; mm += 4) {
      const cf a = sw[ar][mm + kl];
      const cf h = shh[mm + kl][wave * 16 + (lane & 15)];
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, h.x, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, h.y, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, h.x - h.y, acc3, 0, 0, 0);
    }
    __syncthreads();
  }
  const int k = k0 + wave * 16 + (lane & 15);
  if (k >= N) return;
  const float fk = b ? f[k] : 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int t = 4 * (lane >> 4) + r;
    if (t >= T) continue;
    const double p1 = acc1[r], p2 = acc2[r], p3 = acc3[r];
    const cf val = mk<cf>((float)(p1 + p2), (float)(p3 - p1 + p2));
    q[(size_t)t * N + k] = val;
    if (b) b[(size_t)t * N + k] = mk<cf>(val.x * fk, val.y * fk);
  }
}

template <typename R>
int launch_backproject(Ctx &c, const cplx_t<R> *w, cplx_t<R> *q, const R *f, cplx_t<R> *b) {
  if constexpr (std::is_same<R, float>::value) {
    if (c.T <= PJ_NARROW_T) {
      dim3 g((c.N + BP16_PT - 1) / BP16_PT);
      hipLaunchKernelGGL(k_backproject_mfma16, g, dim3(256), 0, c.stream, (const cf *)c.H, w, q, f, b, c.M, c.N,
                         c.T);
      return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
    }
    dim3 g((c.N + BP_PT - 1) / BP_PT, (c.T + BP_TT - 1) / BP_TT);
    hipLaunchKernelGGL(k_backproject_mfma, g, dim3(256), 0, c.stream, (const cf *)c.H, w, q, f, b, c.M, c.N, c.T);
  } else {
    dim3 g((c.N + 255) / 256, (c.T + 15) / 16);
    hipLaunchKernelGGL(k_backproject<R>, g, dim3(256), 0, c.stream, (const cplx_t<R> *)c.H, w, q, f, b, c.M, c.N,
                       c.T);
  }
  return hipGetLastError() == hipSuccess ? CISOR_OK : CISOR_E_DEVICE;
}

template int launch_project<float>(Ctx &, const float *, const cf *, const cf *, cf *, double *, double *);
template int launch_project<double>(Ctx &, const double *, const cd *, const cd *, cd *, double *, double *);
template int launch_backproject<float>(Ctx &, const cf *, cf *, const float *, cf *);
template int launch_backproject<double>(Ctx &, const cd *, cd *, const double *, cd *);

}  // namespace cisor
