// device.hpp -- device helpers shared by the libmsm HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace msm {

// Sticky error bits (mirrors MSM_ERR_OUT_OF_DOMAIN / MSM_ERR_NONFINITE).
constexpr int kFlagDomain = 1;
constexpr int kFlagNonfinite = 2;

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};
template <typename T>
using vec4_t = typename Vec4<T>::type;

__device__ inline float rsqrt_t(float x) { return __frsqrt_rn(x); }
__device__ inline double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// Geometry of one level grid as the kernels see it.
template <typename T>
struct GridDev {
  int n[3];    // points per axis
  int lo[3];   // grid index of array element 0
  int per[3];  // 1 = periodic axis (index wraps modulo n)
  T h[3];      // spacing
  T inv_h[3];
  double hd[3];  // spacing in FP64 (grid coordinates of particles)
  // triclinic cell: particle coordinates are fractional, s = H^{-1} r, and
  // a gradient in s is taken back to r through H^{-T} (Hi = H^{-1}, row-major)
  int tri;
  double Hi[9];
};

// Grid-frame coordinates of a particle at Cartesian x (in place): x itself,
// or on a triclinic grid its fractional coordinates s = H^{-1} x, formed in
// FP64.
template <typename T, typename V>
__device__ inline void grid_frame(const GridDev<T>& g, V* x) {
  if (!g.tri) return;
  const double a = (double)x[0], b = (double)x[1], c = (double)x[2];
  x[0] = (V)(g.Hi[0] * a + g.Hi[1] * b + g.Hi[2] * c);
  x[1] = (V)(g.Hi[3] * a + g.Hi[4] * b + g.Hi[5] * c);
  x[2] = (V)(g.Hi[6] * a + g.Hi[7] * b + g.Hi[8] * c);
}

// grad_r = H^{-T} grad_s on a triclinic grid (in place; no-op otherwise).
template <typename T, typename V>
__device__ inline void grid_to_cartesian(const GridDev<T>& g, V& x, V& y, V& z) {
  if (!g.tri) return;
  const V a = x, b = y, c = z;
  x = (V)g.Hi[0] * a + (V)g.Hi[3] * b + (V)g.Hi[6] * c;
  y = (V)g.Hi[1] * a + (V)g.Hi[4] * b + (V)g.Hi[7] * c;
  z = (V)g.Hi[2] * a + (V)g.Hi[5] * b + (V)g.Hi[8] * c;
}

// Fractional grid coordinate of x on an axis of spacing h: returns the
// integer part (floor of x/h) and f in [0,1), with the rounding error of the
// quotient folded back in (x - u h is exact under fma).
template <typename T>
__device__ inline int grid_coord(T x, T h, T& f) {
  T u = x / h;
  T r = fma(-u, h, x);
  T fl = floor(u);
  f = (u - fl) + r / h;
  int base = (int)fl;
  if (f < T(0)) {
    f += T(1);
    base -= 1;
  } else if (f >= T(1)) {
    f -= T(1);
    base += 1;
  }
  return base;
}

// Centred cardinal B-spline weights of order P at the p grid points
// m = base - P/2 + 1 + k, k = 0..P-1, for fractional offset f (de Boor's
// triangular recurrence on uniform knots):
//   B^(k)_j = [(f + k - 1 - j) B^(k-1)_{j-1} + (j + 1 - f) B^(k-1)_j] / (k - 1)
// with w_k = B^(P)_k, dw_k/du = B^(P-1)_{k-1} - B^(P-1)_k and
// d2w_k/du2 = B^(P-2)_{k-2} - 2 B^(P-2)_{k-1} + B^(P-2)_k.
template <int P, typename T>
__device__ inline void bspline_weights(T f, T* w, T* dw, T* d2w) {
  T B[P];
  B[0] = T(1);
#pragma unroll
  for (int j = 1; j < P; ++j) B[j] = T(0);
  T Bm1[P], Bm2[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    Bm1[j] = T(0);
    Bm2[j] = T(0);
  }
#pragma unroll
  for (int k = 2; k <= P; ++k) {
    if (k == P - 1) {
#pragma unroll
      for (int j = 0; j < P; ++j) Bm2[j] = B[j];
    }
    if (k == P) {
#pragma unroll
      for (int j = 0; j < P; ++j) Bm1[j] = B[j];
    }
    const T inv = T(1) / T(k - 1);
    T nb[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j < k) {
        T left = (j >= 1) ? B[j - 1] : T(0);
        T right = (j < k - 1) ? B[j] : T(0);
        nb[j] = ((f + T(k - 1 - j)) * left + (T(j + 1) - f) * right) * inv;
      } else {
        nb[j] = T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) B[j] = nb[j];
  }
#pragma unroll
  for (int j = 0; j < P; ++j) w[j] = B[j];
  if (dw) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      T a = (j >= 1) ? Bm1[j - 1] : T(0);
      T b = (j < P - 1) ? Bm1[j] : T(0);
      dw[j] = a - b;
    }
  }
  if (d2w) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      T a = (j >= 2) ? Bm2[j - 2] : T(0);
      T b = (j >= 1 && j - 1 < P - 2) ? Bm2[j - 1] : T(0);
      T c = (j < P - 2) ? Bm2[j] : T(0);
      d2w[j] = a - T(2) * b + c;
    }
  }
}

// Array index of grid point m (absolute index) on one axis, or -1 if the
// point lies outside a free-axis grid.
__device__ inline int axis_index(int m, int n, int lo, int per) {
  if (per) {
    int r = m % n;
    return r < 0 ? r + n : r;
  }
  int i = m - lo;
  return (i >= 0 && i < n) ? i : -1;
}

__device__ inline int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

}  // namespace msm
