// plan.cpp -- host-side construction of an MSM plan in FP64.
//
// Geometry of the level grids, the softening polynomial, the restriction
// taps J, the quasi-interpolation sequence omega', the per-level stencils K^l
// and the dense top-level kernel, including the Ewald treatment of the
// infinite-range top kernel on periodic axes.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <sstream>

#include "msm.h"

namespace msm {

namespace {

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Centred cardinal B-spline at integer argument from the truncated-power
// form M_p(x) = 1/(p-1)! sum_j (-1)^j C(p,j) (x-j)_+^(p-1).
long double bspline_at(int p, long double x) {
  long double s = 0.0L, fact = 1.0L;
  for (int i = 2; i < p; ++i) fact *= i;
  for (int j = 0; j <= p; ++j) {
    long double t = x - j;
    if (t > 0) s += ((j & 1) ? -1.0L : 1.0L) * binom(p, j) * powl(t, p - 1);
  }
  return s / fact;
}

}  // namespace

// gamma(rho) for rho < 1 is the degree-(p-1) Taylor polynomial of s^(-1/2)
// about s = 1 at s = rho^2 (Sec. "Splitting for Coulomb kernels").  Expanded
// in powers of t = rho^2: c_k = sum_{j>=k} C(-1/2, j) C(j, k) (-1)^(j-k).
// The kernel r^-nu is split the same way, with s^(-nu/2) (nu = 1: Coulomb).
void softener_coefficients(int p, double* c, int nu) {
  std::vector<double> b(p);
  double v = 1.0;
  for (int j = 0; j < p; ++j) {
    b[j] = v;  // C(-nu/2, j)
    v *= (-0.5 * nu - j) / (j + 1.0);
  }
  for (int k = 0; k < p; ++k) {
    double s = 0.0;
    for (int j = k; j < p; ++j) s += b[j] * binom(j, k) * (((j - k) & 1) ? -1.0 : 1.0);
    c[k] = s;
  }
}

static double gamma_t(const double* c, int p, double rho, int nu = 1) {
  if (rho >= 1.0) return nu == 1 ? 1.0 / rho : std::pow(rho, -nu);
  double t = rho * rho, s = c[p - 1];
  for (int k = p - 2; k >= 0; --k) s = s * t + c[k];
  return s;
}

// Partial kernels k_l, 1 <= l <= L (eq. coulomb_splitting_with_softener) of
// r^-nu: gamma(r/a_l)/a_l^nu - gamma(r/a_{l+1})/a_{l+1}^nu, a_l = 2^(l-1) a.
static double split_kernel(const double* c, int p, int l, int L, double a, double r,
                           int nu = 1) {
  double s0 = std::ldexp(a, l - 1);
  if (l == L) return gamma_t(c, p, r / s0, nu) / std::pow(s0, nu);
  double s1 = std::ldexp(a, l);
  if (r >= s1) return 0.0;
  return gamma_t(c, p, r / s0, nu) / std::pow(s0, nu) - gamma_t(c, p, r / s1, nu) / std::pow(s1, nu);
}

// Quasi-interpolation sequence (eq. kernel_stencil_by_conv_with_universal_coeff).
// The kernel is interpolated in both arguments, so the exact sequence has the
// symbol 1/Bhat(theta)^2, Bhat = sum_n Phi_p(n) e^{i n theta}.  Bhat is a
// polynomial in z = sin^2(theta/2) (cos n theta = T_n(1-2z)); omega'(z) is the
// degree-M Taylor truncation of 1/Bhat(z)^2, and z^k expands to
// 4^-k sum_j (-1)^j C(2k,k+j) e^{ij theta}.
std::vector<double> quasi_sequence(int p, int M) {
  const int half = p / 2;
  // Chebyshev polynomials T_n(1-2z) as coefficient vectors in z
  std::vector<std::vector<long double>> T(half);
  T[0] = {1.0L};
  if (half > 1) T[1] = {1.0L, -2.0L};
  for (int n = 2; n < half; ++n) {
    std::vector<long double> t(n + 1, 0.0L);
    for (size_t i = 0; i < T[n - 1].size(); ++i) {
      t[i] += 2.0L * T[n - 1][i];
      t[i + 1] += -4.0L * T[n - 1][i];
    }
    for (size_t i = 0; i < T[n - 2].size(); ++i) t[i] -= T[n - 2][i];
    T[n] = t;
  }
  std::vector<long double> B(half, 0.0L);
  for (int n = 0; n < half; ++n) {
    long double phi = bspline_at(p, (long double)n + half);
    long double w = (n == 0) ? phi : 2.0L * phi;
    for (size_t i = 0; i < T[n].size(); ++i) B[i] += w * T[n][i];
  }
  std::vector<long double> B2(M + 1, 0.0L);
  for (int i = 0; i < half; ++i)
    for (int j = 0; j < half; ++j)
      if (i + j <= M) B2[i + j] += B[i] * B[j];
  std::vector<long double> inv(M + 1, 0.0L);
  inv[0] = 1.0L / B2[0];
  for (int k = 1; k <= M; ++k) {
    long double s = 0.0L;
    for (int j = 1; j <= k; ++j) s += B2[j] * inv[k - j];
    inv[k] = -s / B2[0];
  }
  std::vector<double> om(M + 1);
  for (int j = 0; j <= M; ++j) {
    long double s = 0.0L;
    for (int k = j; k <= M; ++k)
      s += inv[k] * ldexpl(1.0L, -2 * k) * ((j & 1) ? -1.0L : 1.0L) * binom(2 * k, k + j);
    om[j] = (double)s;
  }
  return om;
}

// Separable convolution of a [n2][n1][n0] box with omega' along one axis.
// Periodic: circular over the axis length; free: the output box shrinks by M
// at both ends.
static void conv_axis(const std::vector<double>& in, const int nin[3], int axis, bool circular,
                      const std::vector<double>& om, std::vector<double>& out, int nout[3]) {
  const int M = (int)om.size() - 1;
  for (int k = 0; k < 3; ++k) nout[k] = nin[k];
  if (!circular) nout[axis] = nin[axis] - 2 * M;
  out.assign((size_t)nout[0] * nout[1] * nout[2], 0.0);
  const long long stride[3] = {1, nin[0], (long long)nin[0] * nin[1]};
  const long long ostride[3] = {1, nout[0], (long long)nout[0] * nout[1]};
  for (int z = 0; z < nout[2]; ++z)
    for (int y = 0; y < nout[1]; ++y)
      for (int x = 0; x < nout[0]; ++x) {
        int o[3] = {x, y, z};
        double s = 0.0;
        for (int k = -M; k <= M; ++k) {
          int i[3] = {x, y, z};
          if (circular) {
            int n = nin[axis];
            i[axis] = ((o[axis] - k) % n + n) % n;
          } else {
            i[axis] = o[axis] + M - k;
          }
          s += om[std::abs(k)] * in[i[0] * stride[0] + i[1] * stride[1] + i[2] * stride[2]];
        }
        out[x * ostride[0] + y * ostride[1] + z * ostride[2]] = s;
      }
}

static void inverse3(const double A[9], double B[9]) {
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

// Distance of the grid offset d: |A d| for a grid whose steps are the columns
// of A, else |h o d|.
static double offset_length(const double* A, const double h[3], double dx, double dy, double dz) {
  if (!A) {
    const double x = dx * h[0], y = dy * h[1], z = dz * h[2];
    return std::sqrt(x * x + y * y + z * z);
  }
  double v[3];
  for (int k = 0; k < 3; ++k) v[k] = A[3 * k] * dx + A[3 * k + 1] * dy + A[3 * k + 2] * dz;
  return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// Largest |d_k| with a grid offset of length below r: r / h_k, or r times the
// length of row k of A^{-1} (the component of A^{-1} x is at most that
// row's length times |x|).
static double offset_reach(const double* A, const double h[3], int k, double r) {
  if (!A) return r / h[k];
  double B[9];
  inverse3(A, B);
  return r * std::sqrt(B[3 * k] * B[3 * k] + B[3 * k + 1] * B[3 * k + 1] + B[3 * k + 2] * B[3 * k + 2]);
}

// Unfolded K^1 on |d_k| <= W_k = R_k + M, R_k = ceil(2a/h_k) - 1 (k_1 vanishes
// for r >= 2a; on a triclinic grid the reach of 2a along each grid axis).
void level1_stencil(int p, int M, double a, const double h[3], int W[3], std::vector<double>& K,
                    const double* gcoef, const double* A, int nu) {
  int R[3], ns[3];
  for (int k = 0; k < 3; ++k) {
    R[k] = (int)std::ceil(offset_reach(A, h, k, 2.0 * a) - 1e-12) - 1;
    if (R[k] < 0) R[k] = 0;
    W[k] = R[k] + M;
    ns[k] = 2 * (R[k] + 2 * M) + 1;  // samples padded by M for the free-axis passes
  }
  std::vector<double> s((size_t)ns[0] * ns[1] * ns[2], 0.0);
  for (int z = 0; z < ns[2]; ++z)
    for (int y = 0; y < ns[1]; ++y)
      for (int x = 0; x < ns[0]; ++x) {
        const double r = offset_length(A, h, x - R[0] - 2 * M, y - R[1] - 2 * M, z - R[2] - 2 * M);
        s[((size_t)z * ns[1] + y) * ns[0] + x] = split_kernel(gcoef, p, 1, 2, a, r, nu);
      }
  std::vector<double> om = quasi_sequence(p, M), t1, t2;
  int n1[3], n2[3], n3[3];
  conv_axis(s, ns, 0, false, om, t1, n1);
  conv_axis(t1, n1, 1, false, om, t2, n2);
  conv_axis(t2, n2, 2, false, om, K, n3);
}

// The ball of the factored level-1 stencil on an orthorhombic grid: S^1(d) =
// k_1(|h o d|) on |d_k| <= R_k, [2R_2+1][2R_1+1][2R_0+1] (K^1 = omega' x
// omega' x omega' * S^1, eq. kernel_stencil_by_conv_with_universal_coeff).
void level1_samples(int p, double a, const double h[3], const int R[3], const double* gcoef,
                    std::vector<double>& S, int nu) {
  const int n0 = 2 * R[0] + 1, n1 = 2 * R[1] + 1, n2 = 2 * R[2] + 1;
  S.assign((size_t)n0 * n1 * n2, 0.0);
  for (int z = 0; z < n2; ++z)
    for (int y = 0; y < n1; ++y)
      for (int x = 0; x < n0; ++x)
        S[((size_t)z * n1 + y) * n0 + x] =
            split_kernel(gcoef, p, 1, 2, a, offset_length(nullptr, h, x - R[0], y - R[1], z - R[2]),
                         nu);
}

// ---------------------------------------------------------------------------
// Ewald sums for the periodic top level.  psi is the potential of a unit
// charge and all its periodic images with tin-foil boundary conditions (and a
// neutralising background in 3-D).  reg: at a lattice point return the
// regular part lim (psi - 1/r).
// ---------------------------------------------------------------------------
static double ewald3d(const double box[3], const double x[3]) {
  const double V = box[0] * box[1] * box[2];
  const double alpha = 1.25 * std::sqrt(M_PI) / std::cbrt(V);
  const double xr = 6.7;  // erfc(6.7) < 4e-21
  const double rc = xr / alpha, kc = 2.0 * alpha * xr;
  double real = 0.0;
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    nr[k] = (int)std::ceil((rc + std::fabs(x[k])) / box[k]) + 1;
    nk[k] = (int)std::ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  }
  for (int i = -nr[0]; i <= nr[0]; ++i)
    for (int j = -nr[1]; j <= nr[1]; ++j)
      for (int k = -nr[2]; k <= nr[2]; ++k) {
        double d[3] = {x[0] + i * box[0], x[1] + j * box[1], x[2] + k * box[2]};
        double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r == 0.0)
          real += -2.0 * alpha / std::sqrt(M_PI);
        else if (r < rc)
          real += std::erfc(alpha * r) / r;
      }
  double rec = 0.0;
  for (int i = -nk[0]; i <= nk[0]; ++i)
    for (int j = -nk[1]; j <= nk[1]; ++j)
      for (int k = -nk[2]; k <= nk[2]; ++k) {
        if (!i && !j && !k) continue;
        double g[3] = {2 * M_PI * i / box[0], 2 * M_PI * j / box[1], 2 * M_PI * k / box[2]};
        double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (g2 >= kc * kc) continue;
        rec += std::exp(-g2 / (4 * alpha * alpha)) / g2 * std::cos(g[0] * x[0] + g[1] * x[1] + g[2] * x[2]);
      }
  return real + 4.0 * M_PI / V * rec - M_PI / (alpha * alpha * V);
}

// Slab, x and y periodic, z free (Parry's 2-D Ewald sum).  alpha is fixed at
// 3/min(Lx, Ly): the constant of a non-neutral slab depends on it.
static double ewald2d(const double box[3], const double x[3]) {
  const double A = box[0] * box[1];
  const double alpha = 3.0 / std::min(box[0], box[1]);
  const double xr = 6.7, rc = xr / alpha, kc = 2.0 * alpha * xr;
  const double z = x[2];
  double real = 0.0;
  int nr[2], nk[2];
  for (int k = 0; k < 2; ++k) {
    nr[k] = (int)std::ceil((rc + std::fabs(x[k])) / box[k]) + 1;
    nk[k] = (int)std::ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  }
  for (int i = -nr[0]; i <= nr[0]; ++i)
    for (int j = -nr[1]; j <= nr[1]; ++j) {
      double d[3] = {x[0] + i * box[0], x[1] + j * box[1], z};
      double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (r == 0.0)
        real += -2.0 * alpha / std::sqrt(M_PI);
      else if (r < rc)
        real += std::erfc(alpha * r) / r;
    }
  double rec = 0.0;
  for (int i = -nk[0]; i <= nk[0]; ++i)
    for (int j = -nk[1]; j <= nk[1]; ++j) {
      if (!i && !j) continue;
      double g0 = 2 * M_PI * i / box[0], g1 = 2 * M_PI * j / box[1];
      double g = std::sqrt(g0 * g0 + g1 * g1);
      if (g >= kc) continue;
      double u = g / (2 * alpha);
      double t = 0.0;
      if (g * z < 700.0) t += std::exp(g * z) * std::erfc(u + alpha * z);
      if (-g * z < 700.0) t += std::exp(-g * z) * std::erfc(u - alpha * z);
      rec += std::cos(g0 * x[0] + g1 * x[1]) / g * t;
    }
  double k0 = -(2.0 * M_PI / A) *
              (z * std::erf(alpha * z) + std::exp(-alpha * alpha * z * z) / (alpha * std::sqrt(M_PI)));
  return real + M_PI / A * rec + k0;
}

// One periodic axis ax (length L, coordinate z along it, distance rho from
// it), two free axes: the 1-D Ewald sum.  Real space is erfc(alpha r)/r over
// the images along the axis.  Fourier space along the axis: the m = 0 term is
// (1/L) [gamma_E + 2 ln(alpha L) - Ein(alpha^2 rho^2)], the logarithm of a
// line charge with its constant chosen so that psi -> -(2/L) ln(rho/L) far
// from the axis, for every alpha; the m != 0 terms are (2/L) cos(k z) F with
// the incomplete Bessel function F = int_0^inf exp(-b e^t - c e^-t) dt,
// b = k^2/(4 alpha^2), c = alpha^2 rho^2, taken by tanh-sinh quadrature over
// the t-range where the exponent stays below 46.  alpha = 2/L.
static double ein(double x) {  // int_0^x (1 - e^-v)/v dv
  if (x > 0.75) return 0.57721566490153286061 + std::log(x) - std::expint(-x);
  double t = -1.0, s = 0.0;
  for (int k = 1; k < 60; ++k) {
    t *= -x / k;
    s += t / k;
  }
  return s;
}

// int_0^inf e^{-wt} exp(-b e^t - c e^-t) dt by tanh-sinh quadrature over the
// t-range where the exponent stays below 46: bounded by b e^t + c e^-t when
// b > 0, by w t and c e^-t when b = 0 (then w > 0).
static double exp_integral(double w, double b, double c) {
  const double E = 46.0;
  double lo, hi;
  if (b > 0.0) {
    const double D = E * E - 4.0 * b * c;
    if (D <= 0.0) return 0.0;
    hi = std::log((E + std::sqrt(D)) / (2.0 * b));
    lo = std::max(0.0, std::log((E - std::sqrt(D)) / (2.0 * b)));
  } else {
    hi = E / w;
    lo = c > E ? std::log(c / E) : 0.0;
  }
  if (hi <= lo) return 0.0;
  const double mid = 0.5 * (hi + lo), half = 0.5 * (hi - lo), step = 1.0 / 32.0;
  double sum = 0.0;
  for (int k = -112; k <= 112; ++k) {  // |u| <= 3.5: weights below 1e-30 beyond
    const double u = k * step, v = 0.5 * M_PI * std::sinh(u);
    const double wt = 0.5 * M_PI * std::cosh(u) / (std::cosh(v) * std::cosh(v));
    const double t = mid + half * std::tanh(v);
    sum += wt * std::exp(-w * t - b * std::exp(t) - c * std::exp(-t));
  }
  return sum * half * step;
}

static double incomplete_bessel(double b, double c) { return exp_integral(0.0, b, c); }

static double ewald1d(const double box[3], int ax, const double x[3]) {
  const double L = box[ax], z = x[ax];
  const double alpha = 2.0 / L;
  double rho2 = 0.0;
  for (int k = 0; k < 3; ++k)
    if (k != ax) rho2 += x[k] * x[k];
  const double rc = 6.7 / alpha;
  const int nr = (int)std::ceil((rc + std::fabs(z)) / L) + 1;
  double val = 0.0;
  for (int i = -nr; i <= nr; ++i) {
    const double dz = z + i * L, r = std::sqrt(rho2 + dz * dz);
    if (r == 0.0)
      val += -2.0 * alpha / std::sqrt(M_PI);
    else if (r < rc)
      val += std::erfc(alpha * r) / r;
  }
  const double c = alpha * alpha * rho2;
  val += (0.57721566490153286061 + 2.0 * std::log(alpha * L) - ein(c)) / L;
  for (int m = 1;; ++m) {
    const double k = 2.0 * M_PI * m / L, b = k * k / (4.0 * alpha * alpha);
    if (b > 46.0) break;
    val += 2.0 / L * std::cos(k * z) * incomplete_bessel(b, c);
  }
  return val;
}

// Lattice sum of r^-6 over a 3-D periodic box by the Ewald method: with
// r^-6 = (1/2) int_0^inf t^2 e^{-r^2 t} dt split at t = alpha^2, real space
// keeps e^{-y}(1 + y + y^2/2)/r^6 (y = alpha^2 r^2), Fourier space the rest,
// pi^{3/2} alpha^3 / (3V) [(1 - 2 b^2) e^{-b^2} + 2 sqrt(pi) b^3 erfc(b)]
// per wave vector k (b = |k| / (2 alpha), k = 0 included).  The sum
// converges absolutely: no boundary term.  At x = 0 the n = 0 term is left
// out (its real-space part tends to -alpha^6/6 after r^-6 is removed).
static double ewald3d_r6(const double box[3], const double x[3]) {
  const double V = box[0] * box[1] * box[2];
  const double alpha = 1.3 / std::cbrt(V);
  const double rc = 7.2 / alpha, bc = 6.8;  // dropped terms below 1e-18 of the sum
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    nr[k] = (int)std::ceil((rc + std::fabs(x[k])) / box[k]) + 1;
    nk[k] = (int)std::ceil(2.0 * alpha * bc * box[k] / (2.0 * M_PI)) + 1;
  }
  double val = 0.0;
  for (int i = -nr[0]; i <= nr[0]; ++i)
    for (int j = -nr[1]; j <= nr[1]; ++j)
      for (int k = -nr[2]; k <= nr[2]; ++k) {
        const double d[3] = {x[0] + i * box[0], x[1] + j * box[1], x[2] + k * box[2]};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) {
          val -= std::pow(alpha, 6) / 6.0;
        } else if (r2 < rc * rc) {
          const double y = alpha * alpha * r2;
          val += std::exp(-y) * (1.0 + y + 0.5 * y * y) / (r2 * r2 * r2);
        }
      }
  double rec = 0.0;
  for (int i = -nk[0]; i <= nk[0]; ++i)
    for (int j = -nk[1]; j <= nk[1]; ++j)
      for (int k = -nk[2]; k <= nk[2]; ++k) {
        const double g[3] = {2 * M_PI * i / box[0], 2 * M_PI * j / box[1], 2 * M_PI * k / box[2]};
        const double b = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) / (2.0 * alpha);
        if (b >= bc) continue;
        const double w = (1.0 - 2.0 * b * b) * std::exp(-b * b) +
                         2.0 * std::sqrt(M_PI) * b * b * b * std::erfc(b);
        rec += w * std::cos(g[0] * x[0] + g[1] * x[1] + g[2] * x[2]);
      }
  return val + std::pow(M_PI, 1.5) * alpha * alpha * alpha / (3.0 * V) * rec;
}

// Lattice sums of r^-6 over two periodic axes (slab, free axis f) or one
// (line): real space e^{-y}(1 + y + y^2/2)/r^6 over the images as in 3-D;
// the smooth rest (1/2) int_0^{alpha^2} t^2 e^{-r^2 t} dt summed over the
// periodic axes by Poisson summation, where the 2-D (1-D) transform of
// e^{-t rho^2} is (pi/t) e^{-k^2/4t} (sqrt(pi/t) e^{-k^2/4t}).  With t =
// alpha^2 e^{-u} every Fourier term, k = 0 included, is alpha^4 (alpha^5)
// times int_0^inf e^{-w u} exp(-b e^u - c e^-u) du with w = 2 (5/2),
// b = k^2/(4 alpha^2) and c = alpha^2 z^2 (alpha^2 rho^2).
static double r6_real(double alpha, double r2) {
  const double y = alpha * alpha * r2;
  return std::exp(-y) * (1.0 + y + 0.5 * y * y) / (r2 * r2 * r2);
}

static double ewald2d_r6(const double box[3], int f, const double x[3]) {
  const int a0 = f == 0 ? 1 : 0, a1 = f == 2 ? 1 : 2;
  const double La = box[a0], Lb = box[a1], z = x[f];
  const double alpha = 1.5 / std::min(La, Lb), rc = 7.2 / alpha;
  const int na = (int)std::ceil((rc + std::fabs(x[a0])) / La) + 1;
  const int nb = (int)std::ceil((rc + std::fabs(x[a1])) / Lb) + 1;
  double val = 0.0;
  for (int i = -na; i <= na; ++i)
    for (int j = -nb; j <= nb; ++j) {
      const double da = x[a0] + i * La, db = x[a1] + j * Lb, r2 = da * da + db * db + z * z;
      if (r2 == 0.0)
        val -= std::pow(alpha, 6) / 6.0;
      else if (r2 < rc * rc)
        val += r6_real(alpha, r2);
    }
  const double c = alpha * alpha * z * z;
  const int ma = (int)std::ceil(2.0 * alpha * std::sqrt(46.0) * La / (2.0 * M_PI)) + 1;
  const int mb = (int)std::ceil(2.0 * alpha * std::sqrt(46.0) * Lb / (2.0 * M_PI)) + 1;
  double rec = 0.0;
  for (int i = -ma; i <= ma; ++i)
    for (int j = -mb; j <= mb; ++j) {
      const double ka = 2.0 * M_PI * i / La, kb = 2.0 * M_PI * j / Lb;
      const double b = (ka * ka + kb * kb) / (4.0 * alpha * alpha);
      if (b > 46.0) continue;
      rec += std::cos(ka * x[a0] + kb * x[a1]) * exp_integral(2.0, b, c);
    }
  return val + M_PI / (2.0 * La * Lb) * std::pow(alpha, 4) * rec;
}

static double ewald1d_r6(const double box[3], int ax, const double x[3]) {
  const double L = box[ax], z = x[ax];
  const double alpha = 1.0 / L, rc = 7.2 / alpha;
  double rho2 = 0.0;
  for (int k = 0; k < 3; ++k)
    if (k != ax) rho2 += x[k] * x[k];
  const int nr = (int)std::ceil((rc + std::fabs(z)) / L) + 1;
  double val = 0.0;
  for (int i = -nr; i <= nr; ++i) {
    const double dz = z + i * L, r2 = rho2 + dz * dz;
    if (r2 == 0.0)
      val -= std::pow(alpha, 6) / 6.0;
    else if (r2 < rc * rc)
      val += r6_real(alpha, r2);
  }
  const double c = alpha * alpha * rho2;
  double rec = exp_integral(2.5, 0.0, c);
  for (int m = 1;; ++m) {
    const double k = 2.0 * M_PI * m / L, b = k * k / (4.0 * alpha * alpha);
    if (b > 46.0) break;
    rec += 2.0 * std::cos(k * z) * exp_integral(2.5, b, c);
  }
  return val + std::sqrt(M_PI) / (2.0 * L) * std::pow(alpha, 5) * rec;
}

static double ewald_r6_axes(const HostPlan& P, const double x[3]) {
  const int np = P.periodic[0] + P.periodic[1] + P.periodic[2];
  if (np == 3) return ewald3d_r6(P.box, x);
  if (np == 1) return ewald1d_r6(P.box, P.periodic[0] ? 0 : (P.periodic[1] ? 1 : 2), x);
  return ewald2d_r6(P.box, !P.periodic[0] ? 0 : (!P.periodic[1] ? 1 : 2), x);
}

// Ewald potential for the periodic axes of the plan (not triclinic): all
// three, two (the free axis moved to z for the slab sum), or one.
static double ewald_axes(const HostPlan& P, const double x[3]) {
  const int np = P.periodic[0] + P.periodic[1] + P.periodic[2];
  if (np == 3) return ewald3d(P.box, x);
  if (np == 1) return ewald1d(P.box, P.periodic[0] ? 0 : (P.periodic[1] ? 1 : 2), x);
  const int f = !P.periodic[0] ? 0 : (!P.periodic[1] ? 1 : 2);
  const int a0 = f == 0 ? 1 : 0, a1 = f == 2 ? 1 : 2;
  const double b[3] = {P.box[a0], P.box[a1], P.box[f]}, y[3] = {x[a0], x[a1], x[f]};
  return ewald2d(b, y);
}

// The 3-D sum for the lattice {H n}: real space over the lattice vectors,
// reciprocal space over k = 2 pi H^{-T} m, V = |det H| (tin-foil boundary,
// neutralising background; alpha balances the two sums).
static double ewald3d_cell(const double H[9], const double Hinv[9], const double x[3]) {
  const double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                     H[2] * (H[3] * H[7] - H[4] * H[6]);
  const double V = std::fabs(det);
  const double alpha = 1.25 * std::sqrt(M_PI) / std::cbrt(V);
  const double rc = 6.7 / alpha, kc = 2.0 * alpha * 6.7;  // erfc(6.7) < 4e-21
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    const double* b = Hinv + 3 * k;
    const double bk = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double sk = b[0] * x[0] + b[1] * x[1] + b[2] * x[2];
    nr[k] = (int)std::ceil(rc * bk + std::fabs(sk)) + 1;
    const double ak = std::sqrt(H[k] * H[k] + H[3 + k] * H[3 + k] + H[6 + k] * H[6 + k]);
    nk[k] = (int)std::ceil(kc * ak / (2.0 * M_PI)) + 1;
  }
  double real = 0.0;
  for (int i = -nr[0]; i <= nr[0]; ++i)
    for (int j = -nr[1]; j <= nr[1]; ++j)
      for (int k = -nr[2]; k <= nr[2]; ++k) {
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = x[c] + H[3 * c] * i + H[3 * c + 1] * j + H[3 * c + 2] * k;
        const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r == 0.0) {
          real -= 2.0 * alpha / std::sqrt(M_PI);
          continue;
        }
        if (r < rc) real += std::erfc(alpha * r) / r;
      }
  double rec = 0.0;
  for (int i = -nk[0]; i <= nk[0]; ++i)
    for (int j = -nk[1]; j <= nk[1]; ++j)
      for (int k = -nk[2]; k <= nk[2]; ++k) {
        if (i == 0 && j == 0 && k == 0) continue;
        double g[3];
        for (int c = 0; c < 3; ++c) g[c] = 2.0 * M_PI * (Hinv[c] * i + Hinv[3 + c] * j + Hinv[6 + c] * k);
        const double k2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (k2 > kc * kc) continue;
        rec += std::exp(-k2 / (4.0 * alpha * alpha)) * std::cos(g[0] * x[0] + g[1] * x[1] + g[2] * x[2]) / k2;
      }
  return real + 4.0 * M_PI / V * rec - M_PI / (alpha * alpha * V);
}

// The lattice sum of r^-6 over {H n}: the terms of ewald3d_r6 with images H n
// and wave vectors 2 pi H^{-T} m, V = |det H|.
static double ewald3d_cell_r6(const double H[9], const double Hinv[9], const double x[3]) {
  const double V = std::fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                             H[2] * (H[3] * H[7] - H[4] * H[6]));
  const double alpha = 1.3 / std::cbrt(V);
  const double rc = 7.2 / alpha, bc = 6.8;
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    const double* b = Hinv + 3 * k;
    const double bk = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    nr[k] = (int)std::ceil(rc * bk + std::fabs(b[0] * x[0] + b[1] * x[1] + b[2] * x[2])) + 1;
    const double ak = std::sqrt(H[k] * H[k] + H[3 + k] * H[3 + k] + H[6 + k] * H[6 + k]);
    nk[k] = (int)std::ceil(2.0 * alpha * bc * ak / (2.0 * M_PI)) + 1;
  }
  double val = 0.0;
  for (int i = -nr[0]; i <= nr[0]; ++i)
    for (int j = -nr[1]; j <= nr[1]; ++j)
      for (int k = -nr[2]; k <= nr[2]; ++k) {
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = x[c] + H[3 * c] * i + H[3 * c + 1] * j + H[3 * c + 2] * k;
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0)
          val -= std::pow(alpha, 6) / 6.0;
        else if (r2 < rc * rc)
          val += r6_real(alpha, r2);
      }
  double rec = 0.0;
  for (int i = -nk[0]; i <= nk[0]; ++i)
    for (int j = -nk[1]; j <= nk[1]; ++j)
      for (int k = -nk[2]; k <= nk[2]; ++k) {
        double g[3];
        for (int c = 0; c < 3; ++c) g[c] = 2.0 * M_PI * (Hinv[c] * i + Hinv[3 + c] * j + Hinv[6 + c] * k);
        const double b = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) / (2.0 * alpha);
        if (b >= bc) continue;
        const double w = (1.0 - 2.0 * b * b) * std::exp(-b * b) +
                         2.0 * std::sqrt(M_PI) * b * b * b * std::erfc(b);
        rec += w * std::cos(g[0] * x[0] + g[1] * x[1] + g[2] * x[2]);
      }
  return val + std::pow(M_PI, 1.5) * alpha * alpha * alpha / (3.0 * V) * rec;
}

// Top-level kernel summed over periodic images: G(x) = psi(x) - sum_j s(|x+j|)
// with s(r) = 1/r - gamma(r/R)/R for r < R (zero beyond), R = 2^(L-1) a, i.e.
// the periodic sum of k_L(r) = gamma(r/R)/R with the 1/r tail Ewald-summed.
static double periodic_top_G(const HostPlan& P, const double x[3]) {
  const double R = std::ldexp(P.a, P.L - 1);
  if (P.tri) {  // x Cartesian; images x + H j
    const int nu = P.nu;
    const double Rn = std::pow(R, nu);
    double val = nu == 1 ? ewald3d_cell(P.H, P.Hinv, x) : ewald3d_cell_r6(P.H, P.Hinv, x);
    int ni[3];
    for (int k = 0; k < 3; ++k) {
      const double* b = P.Hinv + 3 * k;
      const double bk = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      ni[k] = (int)std::ceil(R * bk + std::fabs(b[0] * x[0] + b[1] * x[1] + b[2] * x[2])) + 1;
    }
    for (int i = -ni[0]; i <= ni[0]; ++i)
      for (int j = -ni[1]; j <= ni[1]; ++j)
        for (int k = -ni[2]; k <= ni[2]; ++k) {
          double d[3];
          for (int c = 0; c < 3; ++c)
            d[c] = x[c] + P.H[3 * c] * i + P.H[3 * c + 1] * j + P.H[3 * c + 2] * k;
          const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          if (r == 0.0)
            val += P.gamma0 / Rn;
          else if (r < R)
            val -= std::pow(r, -nu) - gamma_t(P.gcoef, P.p, r / R, nu) / Rn;
        }
    return val;
  }
  // kernel r^-nu (Coulomb or r^-6), every set of periodic axes
  const int nu = P.nu;
  const double Rn = std::pow(R, nu);
  double val = nu == 1 ? ewald_axes(P, x) : ewald_r6_axes(P, x);
  int ni[3];
  for (int k = 0; k < 3; ++k)
    ni[k] = P.periodic[k] ? (int)std::ceil((R + std::fabs(x[k])) / P.box[k]) + 1 : 0;
  for (int i = -ni[0]; i <= ni[0]; ++i)
    for (int j = -ni[1]; j <= ni[1]; ++j)
      for (int k = -ni[2]; k <= ni[2]; ++k) {
        double d[3] = {x[0] + i * P.box[0], x[1] + j * P.box[1], x[2] + k * P.box[2]};
        double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r == 0.0)
          val += P.gamma0 / Rn;  // regular part: psi - r^-nu already taken, + gamma(0)/R^nu
        else if (r < R)
          val -= std::pow(r, -nu) - gamma_t(P.gcoef, P.p, r / R, nu) / Rn;
      }
  return val;
}

// Dense top kernel of a free-space system: offsets |d_k| <= n_k - 1.
void free_top_kernel(int p, int M, double a, int L, const double hL[3], const int n[3],
                     const std::vector<double>& omega, const double* gcoef,
                     std::vector<double>& K, int nu) {
  int ns[3];
  for (int k = 0; k < 3; ++k) ns[k] = 2 * (n[k] - 1 + M) + 1;
  std::vector<double> s((size_t)ns[0] * ns[1] * ns[2]);
  const double R = std::ldexp(a, L - 1);
  for (int z = 0; z < ns[2]; ++z)
    for (int y = 0; y < ns[1]; ++y)
      for (int x = 0; x < ns[0]; ++x) {
        double dx = (x - (ns[0] - 1) / 2) * hL[0], dy = (y - (ns[1] - 1) / 2) * hL[1],
               dz = (z - (ns[2] - 1) / 2) * hL[2];
        double r = std::sqrt(dx * dx + dy * dy + dz * dz);
        s[((size_t)z * ns[1] + y) * ns[0] + x] = gamma_t(gcoef, p, r / R, nu) / std::pow(R, nu);
      }
  std::vector<double> t1, t2;
  int n1[3], n2[3], n3[3];
  conv_axis(s, ns, 0, false, omega, t1, n1);
  conv_axis(t1, n1, 1, false, omega, t2, n2);
  conv_axis(t2, n2, 2, false, omega, K, n3);
}

int build_host_plan(HostPlan& P, const double box_in[3], unsigned periodic_mask, int order,
                    double h, double a, int levels, int precision, int max_n, int M,
                    const double* cell, const int* ntop_fixed, double skin, int nu) {
  if ((!box_in && !cell) || !(h > 0) || !(a > 0) || levels < 1 || levels > kMaxLevels ||
      max_n < 0)
    return MSM_ERR_INVALID_ARG;
  if (precision != MSM_FP32 && precision != MSM_FP64) return MSM_ERR_INVALID_ARG;
  // edges: the box lengths, or the lattice vector lengths of a cell (whose
  // grids live in the unit cube, box (1, 1, 1))
  double box[3], edge[3], width[3];
  P.tri = cell != nullptr;
  if (P.tri) {
    if (periodic_mask != 7) return MSM_ERR_UNSUPPORTED;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(cell[k])) return MSM_ERR_INVALID_ARG;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) P.H[3 * r + c] = cell[3 * c + r];  // columns a, b, c
    const double det = P.H[0] * (P.H[4] * P.H[8] - P.H[5] * P.H[7]) -
                       P.H[1] * (P.H[3] * P.H[8] - P.H[5] * P.H[6]) +
                       P.H[2] * (P.H[3] * P.H[7] - P.H[4] * P.H[6]);
    if (!(std::fabs(det) > 0)) return MSM_ERR_INVALID_ARG;
    inverse3(P.H, P.Hinv);
    for (int k = 0; k < 3; ++k) {
      box[k] = 1.0;
      edge[k] = std::sqrt(cell[3 * k] * cell[3 * k] + cell[3 * k + 1] * cell[3 * k + 1] +
                          cell[3 * k + 2] * cell[3 * k + 2]);
      const double* b = P.Hinv + 3 * k;
      width[k] = 1.0 / std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    }
  } else {
    for (int k = 0; k < 3; ++k) {
      if (!(box_in[k] > 0) || !std::isfinite(box_in[k])) return MSM_ERR_INVALID_ARG;
      box[k] = edge[k] = width[k] = box_in[k];
    }
  }
  if (order != 4 && order != 6 && order != 8) return MSM_ERR_UNSUPPORTED;
  // kernels r^-nu: Coulomb (1) and dispersion (6), every geometry (the
  // periodic top level by the lattice sums of each)
  if (nu != 1 && nu != 6) return MSM_ERR_INVALID_ARG;
  P.nu = nu;
  if (periodic_mask > 7) return MSM_ERR_INVALID_ARG;
  if (M < 0) M = order;
  if (M > 24) return MSM_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k) {
    P.box[k] = box[k];
    P.periodic[k] = (periodic_mask >> k) & 1;
    // minimum image: the cutoff within half the box (half the cell's width
    // V / |face| across each axis of a triclinic cell)
    if (P.periodic[k] && a > 0.5 * width[k] * (1.0 + 1e-12)) return MSM_ERR_CUTOFF_TOO_LARGE;
  }
  P.p = order;
  P.L = levels;
  P.M = M;
  P.h_req = h;
  P.a = a;
  P.precision = precision;
  P.max_n = max_n;
  softener_coefficients(order, P.gcoef, nu);
  P.gamma0 = P.gcoef[0];
  P.self_const = P.gamma0 / std::pow(a, nu);
  P.omega = quasi_sequence(order, M);
  for (int n = -order / 2; n <= order / 2; ++n)
    P.J[n + order / 2] = std::ldexp(binom(order, n + order / 2), 1 - order);

  // level geometry
  for (int l = 1; l <= levels; ++l) {
    LevelGeom& g = P.lev[l - 1];
    g.G = 1;
    for (int k = 0; k < 3; ++k) {
      if (P.periodic[k]) {
        double q = edge[k] / std::ldexp(h, levels - 1);
        long long ntop = (long long)std::floor(q + 0.5);
        if (ntop < 1) ntop = 1;
        if (ntop_fixed) ntop = ntop_fixed[k];
        long long n1 = ntop << (levels - 1);
        if (n1 > (1 << 14)) return MSM_ERR_GRID;
        g.n[k] = (int)(n1 >> (l - 1));
        g.lo[k] = 0;
        g.h[k] = box[k] / g.n[k];
      } else {
        double hl = std::ldexp(h, l - 1);
        int hi = (int)std::ceil(box[k] / hl - 1e-9) + order / 2 - 1;
        if (hi > (1 << 14)) return MSM_ERR_GRID;
        g.lo[k] = -order / 2 + 1;
        g.n[k] = hi - g.lo[k] + 1;
        g.h[k] = hl;
      }
      g.G *= g.n[k];
    }
    if (g.G > (1LL << 30)) return MSM_ERR_GRID;
  }

  // Cartesian step of one grid point along each grid axis at level l (columns):
  // H diag(h_l) in a triclinic cell
  auto steps = [&](int l, double A[9]) {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A[3 * r + c] = P.H[3 * r + c] * P.lev[l - 1].h[c];
  };
  double A1[9];
  if (P.tri) steps(1, A1);
  const double* A1p = P.tri ? A1 : nullptr;

  // level-1 stencil, unfolded
  std::vector<double> K1;
  level1_stencil(order, M, a, P.lev[0].h, P.W1, K1, P.gcoef, A1p, nu);
  const int u[3] = {2 * P.W1[0] + 1, 2 * P.W1[1] + 1, 2 * P.W1[2] + 1};

  // levels 1..L-1: K^l = K^1 / 2^((l-1) nu) (Sec. "Splitting for Coulomb
  // kernels": k_l(r) = 2^-(l-1)nu k_1(r / 2^(l-1)) on a grid twice as coarse),
  // folded onto periodic axes, cropped on free axes.
  for (int l = 1; l < levels; ++l) {
    LevelGeom& g = P.lev[l - 1];
    const double scale = std::ldexp(1.0, -(l - 1) * nu);
    for (int k = 0; k < 3; ++k) {
      const int W = P.W1[k];
      if (P.periodic[k]) {
        if (2 * W + 1 <= g.n[k]) {
          g.off[k] = -W;
          g.len[k] = 2 * W + 1;
        } else {
          g.off[k] = -(g.n[k] / 2);
          g.len[k] = g.n[k];
        }
      } else {
        int w = std::min(W, g.n[k] - 1);
        g.off[k] = -w;
        g.len[k] = 2 * w + 1;
      }
    }
    g.K.assign((size_t)g.len[0] * g.len[1] * g.len[2], 0.0);
    for (int z = 0; z < u[2]; ++z)
      for (int y = 0; y < u[1]; ++y)
        for (int x = 0; x < u[0]; ++x) {
          int d[3] = {x - P.W1[0], y - P.W1[1], z - P.W1[2]};
          int idx[3];
          bool keep = true;
          for (int k = 0; k < 3; ++k) {
            int e = d[k] - g.off[k];
            if (P.periodic[k]) {
              e = ((e % g.n[k]) + g.n[k]) % g.n[k];
              if (e >= g.len[k]) keep = false;  // cannot happen when folded
            } else if (e < 0 || e >= g.len[k]) {
              keep = false;
            }
            idx[k] = e;
          }
          if (!keep) continue;
          g.K[((size_t)idx[2] * g.len[1] + idx[1]) * g.len[0] + idx[0]] +=
              scale * K1[((size_t)z * u[1] + y) * u[0] + x];
        }
  }

  // factored form for the intermediate levels: S^l = S^1 / 2^(l-1) with
  // S^1(d) = k_1(|h_1 o d|) on |d_k| <= R_k (the same R as for K^1)
  {
    int R[3];
    for (int k = 0; k < 3; ++k) R[k] = P.W1[k] - M;
    const LevelGeom& g1 = P.lev[0];
    std::vector<double> S1((size_t)(2 * R[0] + 1) * (2 * R[1] + 1) * (2 * R[2] + 1));
    for (int z = -R[2]; z <= R[2]; ++z)
      for (int y = -R[1]; y <= R[1]; ++y)
        for (int x = -R[0]; x <= R[0]; ++x) {
          const double r = offset_length(A1p, g1.h, x, y, z);
          S1[((size_t)(z + R[2]) * (2 * R[1] + 1) + (y + R[1])) * (2 * R[0] + 1) + (x + R[0])] =
              split_kernel(P.gcoef, order, 1, 2, a, r, nu);
        }
    for (int l = 1; l < levels; ++l) {
      LevelGeom& g = P.lev[l - 1];
      const double scale = std::ldexp(1.0, -(l - 1) * nu);
      g.Gext = 1;
      for (int k = 0; k < 3; ++k) {
        if (P.periodic[k]) {
          g.next[k] = g.n[k];
          g.shift[k] = 0;
          if (2 * R[k] + 1 <= g.n[k]) {
            g.s_off[k] = -R[k];
            g.s_len[k] = 2 * R[k] + 1;
          } else {
            g.s_off[k] = -(g.n[k] / 2);
            g.s_len[k] = g.n[k];
          }
        } else {
          g.next[k] = g.n[k] + 2 * M;
          g.shift[k] = -M;
          int w = std::min(R[k], g.n[k] - 1 + M);
          g.s_off[k] = -w;
          g.s_len[k] = 2 * w + 1;
        }
        g.Gext *= g.next[k];
      }
      g.S.assign((size_t)g.s_len[0] * g.s_len[1] * g.s_len[2], 0.0);
      for (int z = -R[2]; z <= R[2]; ++z)
        for (int y = -R[1]; y <= R[1]; ++y)
          for (int x = -R[0]; x <= R[0]; ++x) {
            const int d[3] = {x, y, z};
            int idx[3];
            bool keep = true;
            for (int k = 0; k < 3; ++k) {
              int e = d[k] - g.s_off[k];
              if (P.periodic[k]) e = ((e % g.n[k]) + g.n[k]) % g.n[k];
              else if (e < 0 || e >= g.s_len[k]) keep = false;
              idx[k] = e;
            }
            if (!keep) continue;
            g.S[((size_t)idx[2] * g.s_len[1] + idx[1]) * g.s_len[0] + idx[0]] +=
                scale * S1[((size_t)(z + R[2]) * (2 * R[1] + 1) + (y + R[1])) * (2 * R[0] + 1) +
                           (x + R[0])];
          }
      long long nnzK = 0, nnzS = 0;
      for (double v : g.K) nnzK += (v != 0.0);
      for (double v : g.S) nnzS += (v != 0.0);
      // work: taps x outputs; the factored form adds (2M+1) taps per axis
      const double direct = (double)nnzK * g.G;
      const double fact = (double)nnzS * g.Gext + 3.0 * (2 * M + 1) * g.G;
      // MSM_FACTORED=0 keeps every level on the direct stencil (tests compare both)
      const char* env = std::getenv("MSM_FACTORED");
      const bool allow = !(env && env[0] == '0');
      g.factored = allow && fact < 0.8 * direct;
    }
  }

  // top level: dense over every top-grid pair
  {
    LevelGeom& g = P.lev[levels - 1];
    const int Mq = M;
    int next[3];
    for (int k = 0; k < 3; ++k) {
      if (P.periodic[k]) {
        g.off[k] = -(g.n[k] / 2);
        g.len[k] = g.n[k];
        next[k] = g.n[k];  // table over residues 0..n-1
      } else {
        g.off[k] = -(g.n[k] - 1);
        g.len[k] = 2 * g.n[k] - 1;
        next[k] = 2 * (g.n[k] - 1 + Mq) + 1;  // offsets -(n-1+M)..(n-1+M)
      }
    }
    std::vector<double> T((size_t)next[0] * next[1] * next[2]);
    const bool anyp = P.periodic[0] || P.periodic[1] || P.periodic[2];
    const double R = std::ldexp(a, levels - 1);
    double AL[9];
    if (P.tri) steps(levels, AL);
    for (int z = 0; z < next[2]; ++z)
      for (int y = 0; y < next[1]; ++y)
        for (int x = 0; x < next[0]; ++x) {
          int i3[3] = {x, y, z}, d[3];
          double xv[3];
          for (int k = 0; k < 3; ++k) {
            d[k] = P.periodic[k] ? i3[k] : i3[k] - (g.n[k] - 1 + Mq);
            xv[k] = d[k] * g.h[k];
          }
          if (P.tri)  // Cartesian offset of the grid step d
            for (int k = 0; k < 3; ++k) xv[k] = AL[3 * k] * d[0] + AL[3 * k + 1] * d[1] + AL[3 * k + 2] * d[2];
          double val;
          if (anyp) {
            val = periodic_top_G(P, xv);
          } else {
            double r = std::sqrt(xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2]);
            val = gamma_t(P.gcoef, P.p, r / R, nu) / std::pow(R, nu);
          }
          T[((size_t)z * next[1] + y) * next[0] + x] = val;
        }
    std::vector<double> a1 = T, a2;
    int na[3] = {next[0], next[1], next[2]}, nb[3];
    for (int ax = 0; ax < 3; ++ax) {
      conv_axis(a1, na, ax, P.periodic[ax] != 0, P.omega, a2, nb);
      a1.swap(a2);
      for (int k = 0; k < 3; ++k) na[k] = nb[k];
    }
    // a1 now indexed by residue (periodic) or by d + (n-1) (free)
    g.K.assign((size_t)g.len[0] * g.len[1] * g.len[2], 0.0);
    for (int z = 0; z < g.len[2]; ++z)
      for (int y = 0; y < g.len[1]; ++y)
        for (int x = 0; x < g.len[0]; ++x) {
          int i3[3] = {x, y, z}, s[3];
          for (int k = 0; k < 3; ++k) {
            int d = g.off[k] + i3[k];
            s[k] = P.periodic[k] ? ((d % g.n[k]) + g.n[k]) % g.n[k] : d + (g.n[k] - 1);
          }
          g.K[((size_t)z * g.len[1] + y) * g.len[0] + x] =
              a1[((size_t)s[2] * na[1] + s[1]) * na[0] + s[0]];
        }
  }

  P.skin = skin;
  for (int k = 0; k < 3; ++k) P.width[k] = width[k];
  cell_list_geometry(P);
  return MSM_OK;
}

// cell list (triclinic: in the unit cube, as many cells per axis as the
// cell's width across that axis holds whole cutoffs plus the skin)
void cell_list_geometry(HostPlan& P) {
  for (int k = 0; k < 3; ++k) {
    int n = (int)std::floor(P.width[k] / (P.a + P.skin));
    if (n < 1) n = 1;
    if (n > 1024) n = 1024;
    P.nc[k] = n;
    P.cs[k] = P.box[k] / n;
  }
}

// ---------------------------------------------------------------------------
// Cell derivatives of a triclinic plan (dE/dH at fixed fractional
// coordinates).  Level l < L: E_l = 1/2 sum_m q~_m (S^l * w)_m with
// w = omega' * q~ (eq. kernel_stencil_by_conv_with_universal_coeff) and
// S^l(d) = k_l(|A_l d|), A_l = H diag(1/N_l); at fixed d, d/dH of k_l(|x|)
// with x = A_l d is k_l'(|x|)/|x| x (H^{-1} x)^T, so the level contributes
// 1/2 sum_m q~_m (T^l_ab * w)_m (H^{-T}) with T^l_ab(d) = k_l'(r)/r x_a x_b;
// and T^l = T^1 / 2^((l-1) nu) as for S (kernel r^-nu).

// d gamma / d rho from the coefficients in t = rho^2 (kernel rho^-nu)
static double gamma_t_d1(const double* c, int p, double rho, int nu) {
  if (rho >= 1.0) return -nu * std::pow(rho, -nu - 1);
  const double t = rho * rho;
  double s = 2.0 * (p - 1) * c[p - 1];
  for (int k = p - 2; k >= 1; --k) s = s * t + 2.0 * k * c[k];
  return rho * s;
}

void cell_stress_stencils(const HostPlan& P, int l, std::vector<double> T[6]) {
  const LevelGeom& g1 = P.lev[0];
  const LevelGeom& g = P.lev[l - 1];
  int R[3];
  for (int k = 0; k < 3; ++k) R[k] = P.W1[k] - P.M;
  double A1[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) A1[3 * r + c] = P.H[3 * r + c] * g1.h[c];
  const size_t vol = (size_t)g.s_len[0] * g.s_len[1] * g.s_len[2];
  for (int i = 0; i < 6; ++i) T[i].assign(vol, 0.0);
  const int nu = P.nu;
  const double scale = std::ldexp(1.0, -(l - 1) * nu), a = P.a;
  for (int z = -R[2]; z <= R[2]; ++z)
    for (int y = -R[1]; y <= R[1]; ++y)
      for (int x = -R[0]; x <= R[0]; ++x) {
        const int d[3] = {x, y, z};
        double v[3];
        for (int k = 0; k < 3; ++k) v[k] = A1[3 * k] * x + A1[3 * k + 1] * y + A1[3 * k + 2] * z;
        const double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (r == 0.0 || r >= 2.0 * a) continue;  // k_1 vanishes beyond 2a
        // k_1 = gamma(r/a)/a^nu - gamma(r/2a)/(2a)^nu
        const double kp = gamma_t_d1(P.gcoef, P.p, r / a, nu) / std::pow(a, nu + 1) -
                          gamma_t_d1(P.gcoef, P.p, r / (2.0 * a), nu) / std::pow(2.0 * a, nu + 1);
        const double f = scale * kp / r;
        int idx[3];
        for (int k = 0; k < 3; ++k) {
          const int e = d[k] - g.s_off[k];
          idx[k] = ((e % g.n[k]) + g.n[k]) % g.n[k];
        }
        const size_t o = ((size_t)idx[2] * g.s_len[1] + idx[1]) * g.s_len[0] + idx[0];
        T[0][o] += f * v[0] * v[0];
        T[1][o] += f * v[1] * v[1];
        T[2][o] += f * v[2] * v[2];
        T[3][o] += f * v[0] * v[1];
        T[4][o] += f * v[0] * v[2];
        T[5][o] += f * v[1] * v[2];
      }
}

// The top level's K^L differentiated in H_rc at fixed fractional offsets, by
// central differences of plans built for H +- eps e_rc with the grid counts
// held (the top table includes the triclinic Ewald sum, whose every part
// depends on the cell); dK[3 r + c] has K^L's layout.
int top_cell_derivative(const HostPlan& P, std::vector<double> dK[9]) {
  const int L = P.L;
  int ntop[3];
  for (int k = 0; k < 3; ++k) ntop[k] = P.lev[L - 1].n[k];
  double scale = 0.0;
  for (int k = 0; k < 9; ++k) scale = std::max(scale, std::fabs(P.H[k]));
  const double eps = 1e-5 * scale;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      std::vector<double> Kpm[2];
      for (int sgn = 0; sgn < 2; ++sgn) {
        double cell[9];  // rows: lattice vectors (columns of H)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) cell[3 * k + j] = P.H[3 * j + k];
        cell[3 * c + r] += sgn == 0 ? eps : -eps;
        HostPlan Q;
        const int rc = build_host_plan(Q, nullptr, 7, P.p, P.h_req, P.a, P.L, P.precision,
                                       P.max_n, P.M, cell, ntop, P.skin, P.nu);
        if (rc != MSM_OK) return rc;
        const LevelGeom& q = Q.lev[L - 1];
        for (int k = 0; k < 3; ++k)
          if (q.len[k] != P.lev[L - 1].len[k] || q.off[k] != P.lev[L - 1].off[k])
            return MSM_ERR_GRID;
        Kpm[sgn] = q.K;
      }
      dK[3 * r + c].resize(Kpm[0].size());
      for (size_t i = 0; i < Kpm[0].size(); ++i)
        dK[3 * r + c][i] = (Kpm[0][i] - Kpm[1][i]) / (2.0 * eps);
    }
  return MSM_OK;
}

std::string describe_json(const HostPlan& P) {
  std::ostringstream o;
  o.precision(17);
  o << "{\"box\":[" << P.box[0] << "," << P.box[1] << "," << P.box[2] << "],";
  o << "\"periodic\":[" << P.periodic[0] << "," << P.periodic[1] << "," << P.periodic[2] << "],";
  if (P.tri) {  // lattice vectors a, b, c as rows (the grids' box is the unit cube)
    o << "\"cell\":[";
    for (int c = 0; c < 3; ++c)
      o << (c ? "," : "") << "[" << P.H[c] << "," << P.H[3 + c] << "," << P.H[6 + c] << "]";
    o << "],";
  }
  o << "\"order\":" << P.p << ",\"levels\":" << P.L << ",\"M\":" << P.M << ",\"h\":" << P.h_req
    << ",\"cutoff\":" << P.a << ",\"precision\":\"" << (P.precision ? "fp64" : "fp32") << "\",";
  o << "\"max_n\":" << P.max_n << ",\"self_const\":" << P.self_const << ",\"kernel_power\":"
    << P.nu << ",";
  o << "\"gamma_t_coeffs\":[";
  for (int k = 0; k < P.p; ++k) o << (k ? "," : "") << P.gcoef[k];
  o << "],\"omega\":[";
  for (size_t k = 0; k < P.omega.size(); ++k) o << (k ? "," : "") << P.omega[k];
  o << "],\"J\":[";
  for (int k = 0; k <= P.p; ++k) o << (k ? "," : "") << P.J[k];
  o << "],\"cells\":[" << P.nc[0] << "," << P.nc[1] << "," << P.nc[2] << "],\"skin\":" << P.skin
    << ",";
  o << "\"stencil1_halfwidth\":[" << P.W1[0] << "," << P.W1[1] << "," << P.W1[2] << "],";
  o << "\"levels_info\":[";
  for (int l = 0; l < P.L; ++l) {
    const LevelGeom& g = P.lev[l];
    long long nnz = 0;
    for (double v : g.K) nnz += (v != 0.0);
    o << (l ? "," : "") << "{\"n\":[" << g.n[0] << "," << g.n[1] << "," << g.n[2] << "],\"lo\":["
      << g.lo[0] << "," << g.lo[1] << "," << g.lo[2] << "],\"h\":[" << g.h[0] << "," << g.h[1]
      << "," << g.h[2] << "],\"stencil_off\":[" << g.off[0] << "," << g.off[1] << "," << g.off[2]
      << "],\"stencil_len\":[" << g.len[0] << "," << g.len[1] << "," << g.len[2]
      << "],\"stencil_nnz\":" << nnz;
    if (g.factored) {
      long long snz = 0;
      for (double v : g.S) snz += (v != 0.0);
      o << ",\"factored\":true,\"samples_len\":[" << g.s_len[0] << "," << g.s_len[1] << ","
        << g.s_len[2] << "],\"samples_nnz\":" << snz << ",\"ext\":[" << g.next[0] << ","
        << g.next[1] << "," << g.next[2] << "]";
    }
    o << "}";
  }
  o << "]}";
  return o.str();
}

}  // namespace msm
