// backward.hip -- adjoint kernels of the MSM (vector-Jacobian product of the
// forward outputs E, F and phi = dE/dq with respect to charges and positions).
//
// For L = gE * U + sum_i v_i . F_i (v = cotangent of the forces):
//  * dU/dq_i = phi_i and dU/dr_i = -F_i are the forward's own outputs;
//  * the long-range force is F_i = -q_i sum_m e_m grad phi_m(r_i) with
//    e = A q~ and A = K^1 + I(K^2 + ...)I^T symmetric (eq. u_oneplus_nested_eval),
//    so with the dipole grid D_m = sum_i q_i v_i . grad phi_m(r_i):
//      d(v.F)/dq_i = -sum_m [(A D)_m phi_m(r_i) + e_m v_i . grad phi_m(r_i)]
//      d(v.F)/dr_i = -q_i sum_m [(A D)_m grad phi_m(r_i) + e_m (Hess phi_m(r_i)) v_i]
//    i.e. one more anterpolation (of D), one more grid pass, and one
//    interpolation with B-spline Hessians;
//  * the short-range force F0_i = q_i sum_j q_j f(r) d_ij, f = -k0'(r)/r, gives
//      d(v.F0)/dq_i = sum_j q_j f (v_i - v_j) . d_ij
//      d(v.F0)/dr_i = sum_j q_i q_j [f (v_i - v_j) + (f'/r) ((v_i - v_j) . d_ij) d_ij]
//    with f = 1/r^3 + 2 P'(t)/a^3 and f'/r = -3/r^5 + 4 P''(t)/a^5.
// A cotangent w of phi adds sum_i w_i phi_i = w^T G q, bilinear in (w, q)
// with the same symmetric G as U = q^T G q / 2:
//  * d/dq_i = (G w)_i: the potential of charges w, i.e. w_i enters the
//    adjoint grid source like a charge (source S = D - W, W_m = sum_i w_i
//    phi_m(r_i), so that -(A S) gives -(A D) + (A W)), plus the short-range
//    sum_j w_j k0(r_ij) and the self term -w_i gamma(0)/a;
//  * d/dr_i = w_i grad phi^q(r_i) + q_i grad phi^w(r_i): the first from the
//    forward's e (its gradient moments), the second from A S as above, and
//    in the pair sum -sum_j (w_i q_j + q_i w_j) f d_ij.
#include <algorithm>
#include <cmath>

#include "brick.hpp"
#include "kernels.hpp"

namespace msm {

// Cotangents in sorted order: v from the caller's [n][3] force cotangent in
// x, y, z (zero without one), the cotangent w of phi in .w (zero without one).
// On a triclinic grid v is taken to the grid frame, H^{-1} v, so that
// v . grad_r = (H^{-1} v) . grad_s.
template <typename T>
__global__ void k_gather_v(int n, const int* __restrict__ perm, const T* __restrict__ gF,
                           const T* __restrict__ gphi, GridDev<T> g, vec4_t<T>* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  vec4_t<T> t;
  t.x = gF ? gF[3 * o] : T(0);
  t.y = gF ? gF[3 * o + 1] : T(0);
  t.z = gF ? gF[3 * o + 2] : T(0);
  t.w = gphi ? gphi[o] : T(0);
  if (g.tri) {
    const T a = t.x, b = t.y, c = t.z;
    t.x = (T)g.Hi[0] * a + (T)g.Hi[1] * b + (T)g.Hi[2] * c;
    t.y = (T)g.Hi[3] * a + (T)g.Hi[4] * b + (T)g.Hi[5] * c;
    t.z = (T)g.Hi[6] * a + (T)g.Hi[7] * b + (T)g.Hi[8] * c;
  }
  v[i] = t;
}

// The adjoint grid source S_m = sum_i [q_i v_i . grad phi_m(r_i) - w_i phi_m(r_i)]
// (the dipole grid, less the grid charge of the phi cotangent) in the brick
// form of the forward anterpolation: one workgroup per super-cell (as in the
// forward), 64-bit fixed-point sums in LDS (exact integer adds; the
// power-of-two scale bounds every sum by 2^62, since |contribution| <=
// |q| (|vx| + |vy| + |vz|) max(1/h) + |w| for B-spline weights in [0, 1] and
// derivatives in [-1/h, 1/h]), then one atomic per non-zero point.  Bricks
// larger than brick_cap points fall back to per-particle atomics.
template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_anterp_dipole_brick(const int* __restrict__ start, const vec4_t<T>* __restrict__ sorted,
                          const vec4_t<T>* __restrict__ v, GridDev<T> g, CellGrid cg,
                          BrickGeom bg, int brick_cap, T* __restrict__ grid) {
  extern __shared__ long long brick[];
  __shared__ double bsum[4];
  __shared__ BrickRuns runs;
  int c0[3], c1[3], nruns;
  const int part = blockIdx.x % bg.split, stride = blockDim.x * bg.split;  // (as the forward)
  const int count = brick_runs(blockIdx.x / bg.split, start, cg, bg, c0, c1, runs, nruns);
  if (count <= part * (int)blockDim.x) return;
  int lo[3], ext[3];
  const int vol = brick_box<P>(c0, c1, cg, g.hd, lo, ext);
  const bool staged = vol <= brick_cap;
  const double ih[3] = {1.0 / g.hd[0], 1.0 / g.hd[1], 1.0 / g.hd[2]};
  const double ihmax = fmax(ih[0], fmax(ih[1], ih[2]));
  double scale = 1.0;
  if (staged) {
    for (int b = threadIdx.x; b < vol; b += blockDim.x) brick[b] = 0;
    double bound = 0.0;
    for (int j = part * blockDim.x + threadIdx.x; j < count; j += stride) {
      const int i = brick_particle(runs, nruns, j);
      const vec4_t<T> vi = v[i];
      bound += fabs((double)sorted[i].w) *
                   (fabs((double)vi.x) + fabs((double)vi.y) + fabs((double)vi.z)) * ihmax +
               fabs((double)vi.w);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bound += __shfl_xor(bound, o);
    if ((threadIdx.x & 63) == 0) bsum[threadIdx.x >> 6] = bound;
    __syncthreads();
    int ex;
    (void)frexp(bsum[0] + bsum[1] + bsum[2] + bsum[3], &ex);
    scale = ldexp(1.0, 62 - max(ex, -900));
  }
  for (int jp = part * blockDim.x + threadIdx.x; jp < count; jp += stride) {
    const int i = brick_particle(runs, nruns, jp);
    const vec4_t<T> pi = sorted[i];
    const vec4_t<T> vi = v[i];
    double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    grid_frame(g, xs);
    double w[3][P], dw[3][P];
    int m0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double f;
      m0[k] = grid_coord<double>(xs[k], g.hd[k], f) - P / 2 + 1;
      bspline_weights<P, double>(f, w[k], dw[k], nullptr);
#pragma unroll
      for (int j = 0; j < P; ++j) dw[k][j] *= ih[k];
    }
    bool inside = staged;
#pragma unroll
    for (int k = 0; k < 3; ++k) inside = inside && m0[k] >= lo[k] && m0[k] + P - 1 < lo[k] + ext[k];
    const double qd = (double)pi.w;
    const double vx = (double)vi.x, vy = (double)vi.y, vz = (double)vi.z, wd = (double)vi.w;
    if (inside) {
      const double qs = qd * scale, ws = wd * scale;
      const int b0 = ((m0[2] - lo[2]) * ext[1] + (m0[1] - lo[1])) * ext[0] + (m0[0] - lo[0]);
#pragma unroll
      for (int c = 0; c < P; ++c) {
#pragma unroll
        for (int b = 0; b < P; ++b) {
          const double syz = qs * vx * w[1][b] * w[2][c];
          const double tyz = (qs * (vy * dw[1][b] * w[2][c] + vz * w[1][b] * dw[2][c])) -
                             ws * w[1][b] * w[2][c];
          const int row = b0 + (c * ext[1] + b) * ext[0];
#pragma unroll
          for (int a = 0; a < P; ++a)
            atomicAdd((unsigned long long*)&brick[row + a],
                      (unsigned long long)__double2ll_rn(syz * dw[0][a] + tyz * w[0][a]));
        }
      }
    } else {
      int idx[3][P];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < P; ++j) idx[k][j] = axis_index(m0[k] + j, g.n[k], g.lo[k], g.per[k]);
#pragma unroll
      for (int c = 0; c < P; ++c) {
        if (idx[2][c] < 0) continue;
#pragma unroll
        for (int b = 0; b < P; ++b) {
          if (idx[1][b] < 0) continue;
          const double syz = qd * vx * w[1][b] * w[2][c];
          const double tyz = (qd * (vy * dw[1][b] * w[2][c] + vz * w[1][b] * dw[2][c])) -
                             wd * w[1][b] * w[2][c];
          const long long row = ((long long)idx[2][c] * g.n[1] + idx[1][b]) * g.n[0];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            if (idx[0][a] < 0) continue;
            atomicAdd(&grid[row + idx[0][a]], (T)(syz * dw[0][a] + tyz * w[0][a]));
          }
        }
      }
    }
  }
  if (!staged) return;
  __syncthreads();
  const double inv_scale = 1.0 / scale;  // a power of two
  for (int b = threadIdx.x; b < vol; b += blockDim.x) {
    const long long sum = brick[b];
    if (sum == 0) continue;
    const int bx = b % ext[0], by = (b / ext[0]) % ext[1], bz = b / (ext[0] * ext[1]);
    const int ix = axis_index(lo[0] + bx, g.n[0], g.lo[0], g.per[0]);
    const int iy = axis_index(lo[1] + by, g.n[1], g.lo[1], g.per[1]);
    const int iz = axis_index(lo[2] + bz, g.n[2], g.lo[2], g.per[2]);
    if (ix < 0 || iy < 0 || iz < 0) continue;
    atomicAdd(&grid[((long long)iz * g.n[1] + iy) * g.n[0] + ix], (T)((double)sum * inv_scale));
  }
}

// Interpolation adjoint with B-spline Hessians, combined with the gE terms,
// the phi-cotangent terms and the short-range VJP, scattered to the caller's
// order.
template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_interp_vjp(int n, const vec4_t<T>* __restrict__ sorted, const vec4_t<T>* __restrict__ v,
                 const int* __restrict__ perm, GridDev<T> g, const T* __restrict__ psi,
                 const T* __restrict__ psiD, const T* __restrict__ save_phi,
                 const T* __restrict__ save_F, const T* __restrict__ gq_sr,
                 const T* __restrict__ gr_sr, const double* __restrict__ gE, double self_const,
                 T* __restrict__ grad_q, T* __restrict__ grad_pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const vec4_t<T> pi = sorted[i];
  const vec4_t<T> vi = v[i];
  T xs[3] = {pi.x, pi.y, pi.z};
  grid_frame(g, xs);
  T w[3][P], dw[3][P], d2w[3][P];
  int idx[3][P];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T f;
    const int base = grid_coord(xs[k], g.h[k], f);
    bspline_weights<P, T>(f, w[k], dw[k], d2w[k]);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      idx[k][j] = axis_index(base - P / 2 + 1 + j, g.n[k], g.lo[k], g.per[k]);
      dw[k][j] *= g.inv_h[k];
      d2w[k][j] *= g.inv_h[k] * g.inv_h[k];
    }
  }
  // moments of psi (M_abc: derivative orders in x, y, z) and of psiD (N_abc)
  T M000 = 0, M100 = 0, M010 = 0, M001 = 0, M200 = 0, M020 = 0, M002 = 0, M110 = 0, M101 = 0,
    M011 = 0;
  T N000 = 0, N100 = 0, N010 = 0, N001 = 0;
  // rows of p consecutive grid values (no wrap, inside a free axis): one
  // vector load each
  const bool run = idx[0][0] >= 0 && idx[0][P - 1] == idx[0][0] + P - 1;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    if (idx[2][c] < 0) continue;
    T Y00 = 0, Y10 = 0, Y01 = 0, Y20 = 0, Y02 = 0, Y11 = 0, Z0 = 0, Z1x = 0, Z1y = 0;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      if (idx[1][b] < 0) continue;
      const long long row = ((long long)idx[2][c] * g.n[1] + idx[1][b]) * g.n[0];
      T S0 = 0, S1 = 0, S2 = 0, D0 = 0, D1 = 0;
      T pv[P], pd[P];
      if (run) {
        __builtin_memcpy(pv, psi + row + idx[0][0], sizeof(pv));
        __builtin_memcpy(pd, psiD + row + idx[0][0], sizeof(pd));
      } else {
#pragma unroll
        for (int a = 0; a < P; ++a) {
          pv[a] = idx[0][a] >= 0 ? psi[row + idx[0][a]] : T(0);
          pd[a] = idx[0][a] >= 0 ? psiD[row + idx[0][a]] : T(0);
        }
      }
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const T e = pv[a];
        const T ed = pd[a];
        S0 += e * w[0][a];
        S1 += e * dw[0][a];
        S2 += e * d2w[0][a];
        D0 += ed * w[0][a];
        D1 += ed * dw[0][a];
      }
      const T wy = w[1][b], dwy = dw[1][b], d2wy = d2w[1][b];
      Y00 += S0 * wy;
      Y10 += S1 * wy;
      Y01 += S0 * dwy;
      Y20 += S2 * wy;
      Y02 += S0 * d2wy;
      Y11 += S1 * dwy;
      Z0 += D0 * wy;
      Z1x += D1 * wy;
      Z1y += D0 * dwy;
    }
    const T wz = w[2][c], dwz = dw[2][c], d2wz = d2w[2][c];
    M000 += Y00 * wz;
    M100 += Y10 * wz;
    M010 += Y01 * wz;
    M001 += Y00 * dwz;
    M200 += Y20 * wz;
    M020 += Y02 * wz;
    M002 += Y00 * d2wz;
    M110 += Y11 * wz;
    M101 += Y10 * dwz;
    M011 += Y01 * dwz;
    N000 += Z0 * wz;
    N100 += Z1x * wz;
    N010 += Z1y * wz;
    N001 += Z0 * dwz;
  }
  (void)M000;
  const T vx = vi.x, vy = vi.y, vz = vi.z, wi = vi.w, qi = pi.w;
  const T sq = N000 + vx * M100 + vy * M010 + vz * M001;
  // q_i grad(phi of A S) + q_i Hess(e) v_i - w_i grad(e), all in the grid frame
  T sx = qi * (N100 + vx * M200 + vy * M110 + vz * M101) - wi * M100;
  T sy = qi * (N010 + vx * M110 + vy * M020 + vz * M011) - wi * M010;
  T sz = qi * (N001 + vx * M101 + vy * M011 + vz * M002) - wi * M001;
  // (triclinic: v is in the grid frame; the gradient goes back through H^{-T})
  grid_to_cartesian(g, sx, sy, sz);
  const T ge = gE ? (T)(*gE) : T(0);
  const int o = perm[i];
  if (grad_q) grad_q[o] = ge * save_phi[i] + gq_sr[i] - sq - (T)(self_const * (double)wi);
  if (grad_pos) {
    grad_pos[3 * o] = -ge * save_F[3 * i] + gr_sr[3 * i] - sx;
    grad_pos[3 * o + 1] = -ge * save_F[3 * i + 1] + gr_sr[3 * i + 1] - sy;
    grad_pos[3 * o + 2] = -ge * save_F[3 * i + 2] + gr_sr[3 * i + 2] - sz;
  }
}

// Without a force cotangent: grad_q = gE phi, grad_pos = -gE F.
template <typename T>
__global__ void k_grad_energy_only(int n, const int* __restrict__ perm,
                                   const T* __restrict__ save_phi, const T* __restrict__ save_F,
                                   const double* __restrict__ gE, T* __restrict__ grad_q,
                                   T* __restrict__ grad_pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ge = gE ? (T)(*gE) : T(0);
  const int o = perm[i];
  if (grad_q) grad_q[o] = ge * save_phi[i];
  if (grad_pos) {
    grad_pos[3 * o] = -ge * save_F[3 * i];
    grad_pos[3 * o + 1] = -ge * save_F[3 * i + 1];
    grad_pos[3 * o + 2] = -ge * save_F[3 * i + 2];
  }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_gather_v(int n, const int* perm, const T* gF, const T* gphi, const GridDev<T>& g,
                     vec4_t<T>* v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_v<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, gF, gphi, g,
                     v);
}

template <typename T>
void launch_anterp_dipole(int p, int n, int ncell, const int* start, const CellGrid& cg,
                          const vec4_t<T>* sorted, const vec4_t<T>* v, const GridDev<T>& g,
                          T* grid, hipStream_t s) {
  if (n <= 0) return;
  const BrickGeom bg = brick_geom(p, n, ncell, cg, g.hd);
  const int bc = brick_lds_cap(p, bg, cg, g.hd);
  const size_t lds = (size_t)bc * sizeof(long long);
  const unsigned nb = (unsigned)bg.nsc[0] * bg.nsc[1] * bg.nsc[2] * bg.split;
  switch (p) {
    case 4: hipLaunchKernelGGL((k_anterp_dipole_brick<T, 4>), dim3(nb), dim3(256), lds, s, start, sorted, v, g, cg, bg, bc, grid); break;
    case 6: hipLaunchKernelGGL((k_anterp_dipole_brick<T, 6>), dim3(nb), dim3(256), lds, s, start, sorted, v, g, cg, bg, bc, grid); break;
    case 8: hipLaunchKernelGGL((k_anterp_dipole_brick<T, 8>), dim3(nb), dim3(256), lds, s, start, sorted, v, g, cg, bg, bc, grid); break;
  }
}

template <typename T>
void launch_interp_vjp(int p, int n, const vec4_t<T>* sorted, const vec4_t<T>* v, const int* perm,
                       const GridDev<T>& g, const T* psi, const T* psiD, const T* save_phi,
                       const T* save_F, const T* gq_sr, const T* gr_sr, const double* gE,
                       double self_const, T* grad_q, T* grad_pos, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (n + 255) / 256;
  switch (p) {
    case 4: hipLaunchKernelGGL((k_interp_vjp<T, 4>), dim3(nb), dim3(256), 0, s, n, sorted, v, perm, g, psi, psiD, save_phi, save_F, gq_sr, gr_sr, gE, self_const, grad_q, grad_pos); break;
    case 6: hipLaunchKernelGGL((k_interp_vjp<T, 6>), dim3(nb), dim3(256), 0, s, n, sorted, v, perm, g, psi, psiD, save_phi, save_F, gq_sr, gr_sr, gE, self_const, grad_q, grad_pos); break;
    case 8: hipLaunchKernelGGL((k_interp_vjp<T, 8>), dim3(nb), dim3(256), 0, s, n, sorted, v, perm, g, psi, psiD, save_phi, save_F, gq_sr, gr_sr, gE, self_const, grad_q, grad_pos); break;
  }
}

template <typename T>
void launch_grad_energy_only(int n, const int* perm, const T* save_phi, const T* save_F,
                             const double* gE, T* grad_q, T* grad_pos, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_grad_energy_only<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, perm,
                     save_phi, save_F, gE, grad_q, grad_pos);
}

#define MSM_INST_BACKWARD(T)                                                                      \
  template void launch_gather_v<T>(int, const int*, const T*, const T*, const GridDev<T>&,        \
                                   vec4_t<T>*, hipStream_t);                                       \
  template void launch_anterp_dipole<T>(int, int, int, const int*, const CellGrid&,                \
                                        const vec4_t<T>*, const vec4_t<T>*, const GridDev<T>&, T*,  \
                                        hipStream_t);                                             \
  template void launch_interp_vjp<T>(int, int, const vec4_t<T>*, const vec4_t<T>*, const int*,    \
                                     const GridDev<T>&, const T*, const T*, const T*, const T*,   \
                                     const T*, const T*, const double*, double, T*, T*,           \
                                     hipStream_t);                                                 \
  template void launch_grad_energy_only<T>(int, const int*, const T*, const T*, const double*,    \
                                           T*, T*, hipStream_t);
MSM_INST_BACKWARD(float)
MSM_INST_BACKWARD(double)

}  // namespace msm
