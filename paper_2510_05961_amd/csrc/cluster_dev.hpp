// cluster_dev.hpp -- device helpers of the short-range pair kernels: the
// neighbour-cell walk with periodic image shifts, box gaps and cluster boxes.
#pragma once

#include "kernels.hpp"

namespace msm {

// Neighbour cell along one axis at offset o in {-1, 0, 1}: the cell index
// (or -1 outside a free axis) and the image shift in units of the box edge.
__device__ inline int neighbour_shift(int c, int o, int nc, int per, int& sh) {
  const int v = c + o;
  sh = 0;
  if (per) {
    if (v < 0) {
      sh = -1;
      return v + nc;
    }
    if (v >= nc) {
      sh = 1;
      return v - nc;
    }
    return v;
  }
  return (v >= 0 && v < nc) ? v : -1;
}

// Cartesian image shift of a neighbour cell reached across sh periods:
// sh o box, or H sh in a triclinic cell.
template <typename T>
__device__ inline void image_shift(const PairParams<T>& pp, int shx, int shy, int shz, T& sx,
                                   T& sy, T& sz) {
  if (pp.tri) {
    sx = pp.H[0] * (T)shx + pp.H[1] * (T)shy + pp.H[2] * (T)shz;
    sy = pp.H[3] * (T)shx + pp.H[4] * (T)shy + pp.H[5] * (T)shz;
    sz = pp.H[6] * (T)shx + pp.H[7] * (T)shy + pp.H[8] * (T)shz;
  } else {
    sx = (T)shx * pp.box[0];
    sy = (T)shy * pp.box[1];
    sz = (T)shz * pp.box[2];
  }
}

template <typename T>
__device__ inline T box_gap2(T jlo_x, T jlo_y, T jlo_z, T jhi_x, T jhi_y, T jhi_z, T ilo_x,
                             T ilo_y, T ilo_z, T ihi_x, T ihi_y, T ihi_z) {
  const T gx = max(T(0), max(jlo_x - ihi_x, ilo_x - jhi_x));
  const T gy = max(T(0), max(jlo_y - ihi_y, ilo_y - jhi_y));
  const T gz = max(T(0), max(jlo_z - ihi_z, ilo_z - jhi_z));
  return gx * gx + gy * gy + gz * gz;
}

// A wave-uniform value held in a VGPR: one VALU instruction may read only
// one SGPR, so the leading Horner coefficient lives in a VGPR (loaded once)
// instead of being copied from its SGPR at every pair block.
__device__ inline float in_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}
__device__ inline double in_vgpr(double x) {
  double r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

// Box of i-cluster ic: the union of its j-groups' boxes (an empty second
// group is left out).
template <typename T>
__device__ inline void cluster_box(const vec4_t<T>* cbox, int ic, int m, vec4_t<T>& lo,
                                   vec4_t<T>& hi) {
  lo = cbox[4 * (size_t)ic];
  hi = cbox[4 * (size_t)ic + 1];
  if (m > kGroupSize) {
    const vec4_t<T> l2 = cbox[4 * (size_t)ic + 2], h2 = cbox[4 * (size_t)ic + 3];
    lo.x = min(lo.x, l2.x);
    lo.y = min(lo.y, l2.y);
    lo.z = min(lo.z, l2.z);
    hi.x = max(hi.x, h2.x);
    hi.y = max(hi.y, h2.y);
    hi.z = max(hi.z, h2.z);
  }
}

}  // namespace msm
