// Host-side (FP64) construction of the discretised scattering operators.
//
// Discretisation ("Problem Formulation", eqs. discrete2D_measurement and
// discrete2D_constraint): f u is taken constant on each pixel and the pixel
// replaced by the disk of equal area, radius a = h / sqrt(pi).  Integrating
// k^2 g, g = (i/4) H0^(1)(k_b r) the outgoing 2D Green's function, over that
// disk gives (Graf's addition theorem for the off-diagonal cells, the
// antiderivative x H1(x) of x H0(x) for the self cell):
//   K(0)   = ((i pi/2) k_b a H1^(1)(k_b a) - 1) / eps_b
//   K(rho) = (i pi/2) k_b a J1(k_b a) H0^(1)(k_b rho) / eps_b      (rho >= a)
// G[p,q] = K(|r_p - r_q|) is applied as a circular convolution on the (2n)^2
// grid (offset j stands for distance j or 2n - j, offset n is unused), so its
// spectrum Ghat = FFT2(K_c) is all the device needs.  H[m,q] = K(|r_m - r_q|).
// Reading of the paper: the printed 2D Green's function carries -j/4; the
// outgoing solution consistent with the 3D exp(+j k r) convention is +i/4,
// which is the one used here.
#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace cisor {

using cdbl = std::complex<double>;
static const double kPi = 3.14159265358979323846264338327950288;

// Hankel function H0^(1)(x) = J0(x) + i Y0(x), x > 0.  For x >= 25 the
// Hankel asymptotic expansion sqrt(2/(pi x)) e^{i(x - pi/4)} sum_k i^k a_k / x^k
// with a_k = prod_{j<=k} (-(2j-1)^2) / (k! 8^k) is summed until its terms drop
// below 1e-17; otherwise the standard-library cylindrical Bessel functions are
// used.
static cdbl hankel1_0(double x) {
  if (x >= 25.0) {
    cdbl sum(1.0, 0.0), term(1.0, 0.0);
    const cdbl iu(0.0, 1.0);
    for (int k = 1; k < 40; ++k) {
      const double a = -((2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k * x);
      term *= iu * a;
      sum += term;
      if (std::abs(term) < 1e-17) break;
    }
    return std::sqrt(2.0 / (kPi * x)) * std::exp(iu * (x - kPi / 4.0)) * sum;
  }
  return cdbl(std::cyl_bessel_j(0.0, x), std::cyl_neumann(0.0, x));
}

static cdbl hankel1_1(double x) { return cdbl(std::cyl_bessel_j(1.0, x), std::cyl_neumann(1.0, x)); }

struct Kernel2D {
  double kb, a, c;
  cdbl self_val, off_coef;
  Kernel2D(double k, double h, double eps_b) {
    kb = k * std::sqrt(eps_b);
    a = h / std::sqrt(kPi);
    c = 1.0 / eps_b;
    const double ka = kb * a;
    const cdbl ihalfpi(0.0, kPi / 2.0);
    self_val = c * (ihalfpi * ka * hankel1_1(ka) - 1.0);
    off_coef = c * ihalfpi * ka * std::cyl_bessel_j(1.0, ka);
  }
  cdbl operator()(double rho) const { return rho == 0.0 ? self_val : off_coef * hankel1_0(kb * rho); }
};

// In-place Stockham FFT of length P = 2^a 3^b (FP64, host), sign -1 forward.
static void host_fft(std::vector<cdbl> &x, int sign) {
  const int P = (int)x.size();
  std::vector<int> rad;
  int m = P;
  while (m % 4 == 0) {
    rad.push_back(4);
    m /= 4;
  }
  while (m % 2 == 0) {
    rad.push_back(2);
    m /= 2;
  }
  while (m % 3 == 0) {
    rad.push_back(3);
    m /= 3;
  }
  std::vector<cdbl> y(P);
  int Ns = 1;
  for (int R : rad) {
    for (int j = 0; j < P / R; ++j) {
      const int k = j % Ns;
      cdbl v[4];
      for (int r = 0; r < R; ++r)
        v[r] = x[j + r * (P / R)] * std::polar(1.0, sign * 2.0 * kPi * r * k / (double)(Ns * R));
      const int base = (j / Ns) * Ns * R + k;
      for (int q = 0; q < R; ++q) {
        cdbl s = 0;
        for (int r = 0; r < R; ++r) s += v[r] * std::polar(1.0, sign * 2.0 * kPi * r * q / (double)R);
        y[base + q * Ns] = s;
      }
    }
    x.swap(y);
    Ns *= R;
  }
}

static void fft2(std::vector<cdbl> &a, int P) {
  std::vector<cdbl> line(P);
  for (int i = 0; i < P; ++i) {
    for (int j = 0; j < P; ++j) line[j] = a[(size_t)i * P + j];
    host_fft(line, -1);
    for (int j = 0; j < P; ++j) a[(size_t)i * P + j] = line[j];
  }
  for (int j = 0; j < P; ++j) {
    for (int i = 0; i < P; ++i) line[i] = a[(size_t)i * P + j];
    host_fft(line, -1);
    for (int i = 0; i < P; ++i) a[(size_t)i * P + j] = line[i];
  }
}

template <typename R> static int upload(Ctx &c, void *dst, const std::vector<cdbl> &src) {
  std::vector<cplx_t<R>> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = mk<cplx_t<R>>((R)src[i].real(), (R)src[i].imag());
  CISOR_HIP_CHECK(hipMemcpy(dst, tmp.data(), sizeof(cplx_t<R>) * tmp.size(), hipMemcpyHostToDevice));
  return CISOR_OK;
}

static void parallel_for(int n, const std::function<void(int, int)> &fn) {
  int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min(nth, std::max(1, n));
  std::vector<std::thread> th;
  for (int w = 0; w < nth; ++w) th.emplace_back([&, w] { fn((int)((long)n * w / nth), (int)((long)n * (w + 1) / nth)); });
  for (auto &t : th) t.join();
}

// 3D: the ball of equal volume, radius a = h (3/(4 pi))^(1/3), replaces each
// voxel; integrating k^2 exp(i k_b r)/(4 pi r) over it gives (mean-value
// property of Helmholtz solutions off the diagonal, a radial integral on it)
//   K(0) = ((1 - i k_b a) exp(i k_b a) - 1) / eps_b
//   K(d) = (4 pi / k_b) (sin k_b a - k_b a cos k_b a) exp(i k_b d) / (4 pi d) / eps_b.
struct Kernel3D {
  double kb, a, c;
  cdbl self_val;
  double off_coef;
  Kernel3D(double k, double h, double eps_b) {
    kb = k * std::sqrt(eps_b);
    a = h * std::cbrt(3.0 / (4.0 * kPi));
    c = 1.0 / eps_b;
    const double ka = kb * a;
    self_val = c * ((1.0 - cdbl(0.0, ka)) * std::exp(cdbl(0.0, ka)) - 1.0);
    off_coef = c * (4.0 * kPi / kb) * (std::sin(ka) - ka * std::cos(ka));
  }
  cdbl operator()(double d) const {
    return d == 0.0 ? self_val : off_coef * std::exp(cdbl(0.0, kb * d)) / (4.0 * kPi * d);
  }
};

static void fft3(std::vector<cdbl> &a, int P) {
  std::vector<cdbl> line(P);
  const size_t P2 = (size_t)P * P;
  for (int axis = 0; axis < 3; ++axis) {
    const size_t stride = axis == 0 ? P2 : (axis == 1 ? (size_t)P : 1);
    for (size_t o = 0; o < P2; ++o) {
      // the two other coordinates of the line
      const size_t i1 = o / P, i2 = o % P;
      size_t base;
      if (axis == 0) base = i1 * P + i2;
      else if (axis == 1) base = i1 * P2 + i2;
      else base = i1 * P2 + i2 * P;
      for (int j = 0; j < P; ++j) line[j] = a[base + j * stride];
      host_fft(line, -1);
      for (int j = 0; j < P; ++j) a[base + j * stride] = line[j];
    }
  }
}

template <typename R> static int upload_H3(Ctx &c, const cisor_geometry &g, const Kernel3D &ker,
                                            const std::vector<double> &ax) {
  const int n = c.n, M = c.M;
  const size_t N = c.N;
  const int chunk = 32;
  std::vector<cplx_t<R>> buf((size_t)chunk * N);
  bool bad = false;
  for (int m0 = 0; m0 < M; m0 += chunk) {
    const int m1 = std::min(M, m0 + chunk);
    parallel_for(m1 - m0, [&](int lo, int hi) {
      for (int mm = lo; mm < hi; ++mm) {
        const int m = m0 + mm;
        const double rx = g.rx_pos[3 * m], ry = g.rx_pos[3 * m + 1], rz = g.rx_pos[3 * m + 2];
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j)
            for (int l = 0; l < n; ++l) {
              const double dx = rx - ax[i], dy = ry - ax[j], dz = rz - ax[l];
              const double rho = std::sqrt(dx * dx + dy * dy + dz * dz);
              if (rho < ker.a) bad = true;
              const cdbl v = ker(rho);
              buf[(size_t)mm * N + ((size_t)i * n + j) * n + l] = mk<cplx_t<R>>((R)v.real(), (R)v.imag());
            }
      }
    });
    if (bad) return CISOR_E_ARG;
    CISOR_HIP_CHECK(hipMemcpy((cplx_t<R> *)c.H + (size_t)m0 * N, buf.data(), sizeof(cplx_t<R>) * (m1 - m0) * N,
                              hipMemcpyHostToDevice));
  }
  return CISOR_OK;
}

static int build_geometry_3d(Ctx &c, const cisor_geometry &g) {
  const int n = c.n, P = c.P, T = c.T;
  const size_t N = c.N;
  const double h = c.h;
  const Kernel3D ker(c.k, h, c.eps_b);
  std::vector<double> ax(n);
  for (int i = 0; i < n; ++i) ax[i] = (i - (n - 1) / 2.0) * h;
  std::vector<cdbl> uin((size_t)T * N);
  for (int t = 0; t < T; ++t) {
    if (g.tx_kind == 1) {   // unit point source exp(i k_b d) / (4 pi d)
      const double *s = g.tx_pos + 3 * t;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          for (int l = 0; l < n; ++l) {
            const double dd = std::sqrt((ax[i] - s[0]) * (ax[i] - s[0]) + (ax[j] - s[1]) * (ax[j] - s[1]) +
                                        (ax[l] - s[2]) * (ax[l] - s[2]));
            uin[(size_t)t * N + ((size_t)i * n + j) * n + l] = std::polar(1.0 / (4 * kPi * dd), c.kb * dd);
          }
      continue;
    }
    double d[3] = {g.tx_dir[3 * t], g.tx_dir[3 * t + 1], g.tx_dir[3 * t + 2]};
    const double nr = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (double &x : d) x /= nr;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l)
          uin[(size_t)t * N + ((size_t)i * n + j) * n + l] =
              std::polar(1.0, c.kb * (d[0] * ax[i] + d[1] * ax[j] + d[2] * ax[l]));
  }
  std::vector<cdbl> uniq((size_t)n * n * n);
  parallel_for(n, [&](int lo, int hi) {
    for (int d1 = lo; d1 < hi; ++d1)
      for (int d2 = 0; d2 < n; ++d2)
        for (int d3 = 0; d3 < n; ++d3)
          uniq[((size_t)d1 * n + d2) * n + d3] =
              ker(h * std::sqrt((double)d1 * d1 + (double)d2 * d2 + (double)d3 * d3));
  });
  const size_t P2 = (size_t)P * P;
  std::vector<cdbl> G(P2 * P, cdbl(0, 0));
  auto dist = [&](int j) { return j < n ? j : (j > P - n ? P - j : -1); };
  for (int j1 = 0; j1 < P; ++j1) {
    const int d1 = dist(j1);
    if (d1 < 0) continue;
    for (int j2 = 0; j2 < P; ++j2) {
      const int d2 = dist(j2);
      if (d2 < 0) continue;
      for (int j3 = 0; j3 < P; ++j3) {
        const int d3 = dist(j3);
        if (d3 < 0) continue;
        G[j1 * P2 + (size_t)j2 * P + j3] = uniq[((size_t)d1 * n + d2) * n + d3];
      }
    }
  }
  fft3(G, P);
  // kz-major copy for the plane kernel: Gp[kz][kx][ky] = G[kx][ky][kz]
  std::vector<cdbl> Gp(c.Gpm ? G.size() : 0);
  for (int kx = 0; c.Gpm && kx < P; ++kx)
    for (int ky = 0; ky < P; ++ky)
      for (int kz = 0; kz < P; ++kz) Gp[((size_t)kz * P + kx) * P + ky] = G[((size_t)kx * P + ky) * P + kz];
  std::vector<cdbl> tw(P);
  for (int m = 0; m < P; ++m) tw[m] = std::polar(1.0, -2.0 * kPi * m / P);
  int rc;
  if (c.precision == 0) {
    if ((rc = upload<float>(c, c.uin, uin)) || (rc = upload<float>(c, c.Ghat, G)) ||
        (rc = upload<float>(c, c.tw, tw)) || (rc = upload_H3<float>(c, g, ker, ax)))
      return rc;
  } else {
    if ((rc = upload<double>(c, c.uin, uin)) || (rc = upload<double>(c, c.Ghat, G)) ||
        (rc = upload<double>(c, c.tw, tw)) || (rc = upload_H3<double>(c, g, ker, ax)))
      return rc;
  }
  if ((rc = upload<double>(c, c.Ghat_d, G)) || (rc = upload<double>(c, c.tw_d, tw))) return rc;
  if (c.Gpm && (c.precision == 0 ? (rc = upload<float>(c, c.Gpm, Gp)) : (rc = upload<double>(c, c.Gpm, Gp))))
    return rc;
  if (c.Gpm_d && (rc = upload<double>(c, c.Gpm_d, Gp))) return rc;
  return CISOR_OK;
}

int build_geometry(Ctx &c, const cisor_geometry &g, bool spectrum) {
  if (c.dim == 3) return build_geometry_3d(c, g);
  const int n = c.n, N = c.N, P = c.P, T = c.T, M = c.M;
  const double h = c.h;
  const Kernel2D ker(c.k, h, c.eps_b);
  // pixel centres
  std::vector<double> ax(n);
  for (int i = 0; i < n; ++i) ax[i] = (i - (n - 1) / 2.0) * h;
  // incident fields: plane waves, or the unit point source (i/4) H0(k_b |r - s|)
  std::vector<cdbl> uin((size_t)T * N);
  for (int t = 0; t < T; ++t) {
    if (g.tx_kind == 1) {
      const double sx = g.tx_pos[2 * t], sy = g.tx_pos[2 * t + 1];
      parallel_for(n, [&](int a, int b) {
        for (int i = a; i < b; ++i)
          for (int j = 0; j < n; ++j)
            uin[(size_t)t * N + (size_t)i * n + j] =
                cdbl(0.0, 0.25) * hankel1_0(c.kb * std::hypot(ax[i] - sx, ax[j] - sy));
      });
      continue;
    }
    double dx = g.tx_dir[2 * t], dy = g.tx_dir[2 * t + 1];
    const double nr = std::sqrt(dx * dx + dy * dy);
    dx /= nr;
    dy /= nr;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        uin[(size_t)t * N + (size_t)i * n + j] = std::polar(1.0, c.kb * (dx * ax[i] + dy * ax[j]));
  }
  // padded kernel and its spectrum
  std::vector<cdbl> uniq(spectrum ? (size_t)n * n : 0);
  if (spectrum)
    parallel_for(n, [&](int a, int b) {
      for (int d1 = a; d1 < b; ++d1)
        for (int d2 = 0; d2 < n; ++d2)
          uniq[(size_t)d1 * n + d2] = ker(h * std::sqrt((double)d1 * d1 + (double)d2 * d2));
    });
  std::vector<cdbl> G(spectrum ? (size_t)P * P : 0, cdbl(0, 0));
  for (int j1 = 0; spectrum && j1 < P; ++j1) {
    if (j1 >= n && j1 <= P - n) continue;
    const int d1 = j1 < n ? j1 : P - j1;
    for (int j2 = 0; j2 < P; ++j2) {
      if (j2 >= n && j2 <= P - n) continue;
      const int d2 = j2 < n ? j2 : P - j2;
      G[(size_t)j1 * P + j2] = uniq[(size_t)d1 * n + d2];
    }
  }
  if (spectrum) fft2(G, P);
  // receiver matrix
  std::vector<cdbl> H((size_t)M * N);
  bool bad = false;
  parallel_for(M, [&](int a, int b) {
    for (int m = a; m < b; ++m) {
      const double rx = g.rx_pos[2 * m], ry = g.rx_pos[2 * m + 1];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const double rho = std::hypot(rx - ax[i], ry - ax[j]);
          if (rho < ker.a) bad = true;
          H[(size_t)m * N + (size_t)i * n + j] = ker(rho);
        }
    }
  });
  if (bad) return CISOR_E_ARG;
  // twiddles exp(-2 pi i m / P)
  std::vector<cdbl> tw(P);
  for (int m = 0; m < P; ++m) tw[m] = std::polar(1.0, -2.0 * kPi * m / P);
  int rc;
  if (c.precision == 0) {
    if ((rc = upload<float>(c, c.uin, uin)) || (rc = upload<float>(c, c.H, H))) return rc;
    if (spectrum && ((rc = upload<float>(c, c.Ghat, G)) || (rc = upload<float>(c, c.tw, tw)))) return rc;
  } else {
    if ((rc = upload<double>(c, c.uin, uin)) || (rc = upload<double>(c, c.H, H))) return rc;
    if (spectrum && ((rc = upload<double>(c, c.Ghat, G)) || (rc = upload<double>(c, c.tw, tw)))) return rc;
  }
  if (spectrum && ((rc = upload<double>(c, c.Ghat_d, G)) || (rc = upload<double>(c, c.tw_d, tw)))) return rc;
  return CISOR_OK;
}

}  // namespace cisor
