// Shared device/host helpers of the CISOR HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <type_traits>

namespace cisor {

// Complex storage types: interleaved {re, im}, naturally aligned.
struct __align__(8) cf {
  float x, y;
};
struct __align__(16) cd {
  double x, y;
};
template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = cf; };
template <> struct cplx_of<double> { using type = cd; };
template <typename R> using cplx_t = typename cplx_of<R>::type;
template <typename C> struct real_of;
template <> struct real_of<cf> { using type = float; };
template <> struct real_of<cd> { using type = double; };
template <typename C> using real_t = typename real_of<C>::type;

template <typename C> __host__ __device__ __forceinline__ C mk(real_t<C> re, real_t<C> im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return mk<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cscale(C a, real_t<C> s) { return mk<C>(a.x * s, a.y * s); }
// multiply by (s * i), s = +-1
template <typename C> __device__ __forceinline__ C cmul_si(C a, int s) {
  return s > 0 ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

// Convert between complex storage types.
template <typename Cd, typename Cs> __device__ __forceinline__ Cd ccast(Cs a) {
  return mk<Cd>(static_cast<real_t<Cd>>(a.x), static_cast<real_t<Cd>>(a.y));
}

// Wavefront-wide sum (64 lanes) of a double; every lane receives the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of NV doubles per thread; result valid in thread 0.  The
// reduction order is fixed, so results are bitwise reproducible.  For NV a
// power of two the wave stage is a reduce-scatter: each exchange with the lane
// `off` away halves the values a lane still carries (the lane with that bit
// set keeps the upper half), until every lane carries one value, whose sum the
// remaining exchanges complete: NV - 1 + 6 - log2(NV) exchanges instead of 6 NV
// (10 instead of 48 for NV = 8).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *scratch /* >= NV * 16 */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  constexpr bool POW2 = (NV & (NV - 1)) == 0 && NV <= 64;
  // (the scatter needs every lane of every wave: blocks with a partial last
  // wave, as some row kernels of non-power-of-two lengths have, sum per value)
  if (POW2 && blockDim.x % 64 == 0) {
    constexpr int L = NV <= 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : NV == 16 ? 4 : NV == 32 ? 5 : 6;
    int k = 0;   // index of the value this lane ends up carrying
#pragma unroll
    for (int st = 0; st < L; ++st) {
      const int off = 32 >> st, half = NV >> (st + 1);
      const bool up = (lane & off) != 0;
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const double send = up ? v[j] : v[j + half];
        const double keep = up ? v[j + half] : v[j];
        v[j] = keep + __shfl_xor(send, off, 64);
      }
      k += up ? half : 0;
    }
#pragma unroll
    for (int off = 32 >> L; off >= 1; off >>= 1) v[0] += __shfl_xor(v[0], off, 64);
    __syncthreads();
    if ((lane & ((64 >> L) - 1)) == 0) scratch[wid * NV + k] = v[0];
  } else {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) scratch[wid * NV + i] = v[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += scratch[w * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

}  // namespace cisor

#define CISOR_HIP_CHECK(expr)                                                              \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      std::fprintf(stderr, "cisor: HIP error %s at %s:%d: %s\n", hipGetErrorName(_e),      \
                   __FILE__, __LINE__, #expr);                                             \
      return CISOR_E_DEVICE;                                                               \
    }                                                                                      \
  } while (0)
