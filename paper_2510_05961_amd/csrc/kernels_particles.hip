// kernels_particles.hip -- particle-side kernels of the MSM forward pass:
// cell binning (count, scan, scatter), the short-range pair sum over the cell
// list, anterpolation onto the level-1 grid, and interpolation fused with the
// final combination of short- and long-range parts and the FP64 energy sum.
#include "kernels.hpp"

namespace msm {

// ---------------------------------------------------------------------------
// a1: binning.  Periodic coordinates are wrapped into [0, box); free ones are
// checked against [0, box] (flag + clamp, so every later index stays in
// bounds); non-finite values are flagged and replaced by 0.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_bin_count(int n, const T* __restrict__ pos, const T* __restrict__ q,
                            BinParams<T> bp, int* __restrict__ cell_of, int* __restrict__ rank,
                            int* __restrict__ counts, vec4_t<T>* __restrict__ wrapped,
                            int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  T qi = q[i];
  int bad = 0;
  if (!isfinite(qi)) {
    bad |= kFlagNonfinite;
    qi = T(0);
  }
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T v = x[k];
    if (!isfinite(v)) {
      bad |= kFlagNonfinite;
      v = T(0);
    }
    if (bp.per[k]) {
      v = v - bp.box[k] * floor(v / bp.box[k]);
      if (!(v >= T(0) && v < bp.box[k])) v = T(0);
    } else if (v < T(0) || v > bp.box[k]) {
      bad |= kFlagDomain;
      v = v < T(0) ? T(0) : bp.box[k];
    }
    x[k] = v;
    int ci = (int)(v / bp.cs[k]);
    c[k] = ci < 0 ? 0 : (ci >= bp.nc[k] ? bp.nc[k] - 1 : ci);
  }
  if (bad) atomicOr(flag, bad);
  const int cell = (c[2] * bp.nc[1] + c[1]) * bp.nc[0] + c[0];
  cell_of[i] = cell;
  rank[i] = atomicAdd(&counts[cell], 1);
  vec4_t<T> w;
  w.x = x[0];
  w.y = x[1];
  w.z = x[2];
  w.w = qi;
  wrapped[i] = w;
}

// Exclusive scan of the cell counts into start[0..ncell] (one workgroup).
__global__ void __launch_bounds__(1024) k_scan(int ncell, const int* __restrict__ counts,
                                               int* __restrict__ start) {
  __shared__ int buf[1024];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ncell; base += 1024) {
    int v = (base + t < ncell) ? counts[base + t] : 0;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int add = (t >= off) ? buf[t - off] : 0;
      __syncthreads();
      buf[t] += add;
      __syncthreads();
    }
    if (base + t < ncell) start[base + t] = carry + buf[t] - v;
    __syncthreads();
    if (t == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (t == 0) start[ncell] = carry;
}

template <typename T>
__global__ void k_bin_scatter(int n, const int* __restrict__ cell_of, const int* __restrict__ rank,
                              const int* __restrict__ start, const vec4_t<T>* __restrict__ wrapped,
                              vec4_t<T>* __restrict__ sorted, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dst = start[cell_of[i]] + rank[i];
  sorted[dst] = wrapped[i];
  perm[dst] = i;
}

// ---------------------------------------------------------------------------
// a2: short-range pair sum (eq. U_zero).  One workgroup per home cell; the
// particles of each neighbour cell are staged through LDS in tiles and every
// thread sweeps the tile for its own home particle:
//   phi0_i = sum_j q_j k0(r),  F0_i = q_i sum_j q_j (1/r^3 + 2 P'(t)/a^3) d_ij,
// k0(r) = 1/r - P(t)/a, t = r^2/a^2, P the softening polynomial in t.
// ---------------------------------------------------------------------------
// Cell index along one axis at offset o in {-1, 0, 1} from cell c, or -1 when
// that neighbour does not exist or repeats one already visited: periodic axes
// with one cell visit only o = 0, with two cells only o = 0 and o = 1.
__device__ inline int neighbour_cell(int c, int o, int nc, int per) {
  if (per) {
    if (nc == 1) return o == 0 ? 0 : -1;
    if (nc == 2) return o < 0 ? -1 : (c + o) & 1;
    const int v = c + o;
    return v < 0 ? v + nc : (v >= nc ? v - nc : v);
  }
  const int v = c + o;
  return (v >= 0 && v < nc) ? v : -1;
}

template <typename T, int P>
__global__ void __launch_bounds__(kPairThreads)
    k_pair(const vec4_t<T>* __restrict__ sorted, const int* __restrict__ start, PairParams<T> pp,
           double* __restrict__ phi0, T* __restrict__ F0) {
  __shared__ vec4_t<T> tile[kPairThreads];
  const int cell = blockIdx.x;
  const int cx = cell % pp.nc[0];
  const int cy = (cell / pp.nc[0]) % pp.nc[1];
  const int cz = cell / (pp.nc[0] * pp.nc[1]);
  const int i_beg = start[cell], i_end = start[cell + 1];
  for (int ib = i_beg; ib < i_end; ib += kPairThreads) {
    const int i = ib + (int)threadIdx.x;
    const bool active = i < i_end;
    vec4_t<T> pi;
    if (active) pi = sorted[i];
    else {
      pi.x = pi.y = pi.z = pi.w = T(0);
    }
    double ph = 0.0;  // the potential is carried in FP64 up to the energy sum
    T fx = T(0), fy = T(0), fz = T(0);
    // neighbour cells: offsets -1..1 per axis, each distinct cell once
    for (int oz = -1; oz <= 1; ++oz) {
      const int nz = neighbour_cell(cz, oz, pp.nc[2], pp.per[2]);
      if (nz < 0) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        const int ny = neighbour_cell(cy, oy, pp.nc[1], pp.per[1]);
        if (ny < 0) continue;
        for (int ox = -1; ox <= 1; ++ox) {
          const int nx = neighbour_cell(cx, ox, pp.nc[0], pp.per[0]);
          if (nx < 0) continue;
          const int nc_ = (nz * pp.nc[1] + ny) * pp.nc[0] + nx;
          const int j_beg = start[nc_], j_end = start[nc_ + 1];
          for (int jb = j_beg; jb < j_end; jb += kPairThreads) {
            __syncthreads();
            if (jb + (int)threadIdx.x < j_end) tile[threadIdx.x] = sorted[jb + threadIdx.x];
            __syncthreads();
            const int cnt = min(kPairThreads, j_end - jb);
            for (int jj = 0; jj < cnt; ++jj) {
              const vec4_t<T> pj = tile[jj];
              T dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
              if (pp.per[0]) dx -= pp.box[0] * rint(dx * pp.inv_box[0]);
              if (pp.per[1]) dy -= pp.box[1] * rint(dy * pp.inv_box[1]);
              if (pp.per[2]) dz -= pp.box[2] * rint(dz * pp.inv_box[2]);
              const T r2 = dx * dx + dy * dy + dz * dz;
              if (r2 < pp.a2 && jb + jj != i) {
                const T rinv = rsqrt_t(r2);
                const T t = r2 * pp.inv_a2;
                T Pt = pp.c[P - 1], dP = pp.dc[P - 2];
#pragma unroll
                for (int k = P - 2; k >= 0; --k) Pt = Pt * t + pp.c[k];
#pragma unroll
                for (int k = P - 3; k >= 0; --k) dP = dP * t + pp.dc[k];
                ph += (double)(pj.w * (rinv - Pt * pp.inv_a));
                const T fs = pj.w * (rinv * rinv * rinv + T(2) * dP * pp.inv_a3);
                fx += fs * dx;
                fy += fs * dy;
                fz += fs * dz;
              }
            }
          }
        }
      }
    }
    if (active) {
      phi0[i] = ph;
      F0[3 * i] = pi.w * fx;
      F0[3 * i + 1] = pi.w * fy;
      F0[3 * i + 2] = pi.w * fz;
    }
  }
}

// ---------------------------------------------------------------------------
// a3: anterpolation (eq. grid_charge): q~^1_m += q_i phi_m(r_i) over the p^3
// grid points of each particle (particles are in cell order, so neighbouring
// threads update neighbouring grid points).
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ void k_anterp(int n, const vec4_t<T>* __restrict__ sorted, GridDev<T> g,
                         T* __restrict__ grid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const vec4_t<T> pi = sorted[i];
  const double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
  // weights in FP64: they enter the grid self-energy quadratically
  double w[3][P];
  int idx[3][P];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double f;
    const int base = grid_coord<double>(xs[k], g.hd[k], f);
    bspline_weights<P, double>(f, w[k], nullptr, nullptr);
#pragma unroll
    for (int j = 0; j < P; ++j) idx[k][j] = axis_index(base - P / 2 + 1 + j, g.n[k], g.lo[k], g.per[k]);
  }
  const double qi = (double)pi.w;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    if (idx[2][c] < 0) continue;
    const double wz = qi * w[2][c];
#pragma unroll
    for (int b = 0; b < P; ++b) {
      if (idx[1][b] < 0) continue;
      const double wyz = wz * w[1][b];
      const long long row = ((long long)idx[2][c] * g.n[1] + idx[1][b]) * g.n[0];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        if (idx[0][a] < 0) continue;
        atomicAdd(&grid[row + idx[0][a]], (T)(wyz * w[0][a]));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// a8 + a9: interpolation of e^{1+} (eqs. analytic_uoneplus_position_grad,
// analytic_uoneplus_charge_grad), combined with the short-range part and the
// self term, scattered back to the caller's particle order, and the energy
// E = 1/2 sum_i q_i phi_i summed in FP64.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_interp(int n, const vec4_t<T>* __restrict__ sorted, const int* __restrict__ perm,
             GridDev<T> g, const T* __restrict__ e1, const double* __restrict__ phi0,
             const T* __restrict__ F0, double self_const, T* __restrict__ dEdq, T* __restrict__ F,
             T* __restrict__ save_phi, T* __restrict__ save_F, double* __restrict__ energy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double ep = 0.0;
  if (i < n) {
    const vec4_t<T> pi = sorted[i];
    const double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    // weights and sums in FP64 (the energy needs the grid self-interaction
    // below FP32 rounding); outputs are rounded to T at the end
    double w[3][P], dw[3][P];
    int idx[3][P];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double f;
      const int base = grid_coord<double>(xs[k], g.hd[k], f);
      bspline_weights<P, double>(f, w[k], dw[k], nullptr);
      const double ih = 1.0 / g.hd[k];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        idx[k][j] = axis_index(base - P / 2 + 1 + j, g.n[k], g.lo[k], g.per[k]);
        dw[k][j] *= ih;
      }
    }
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      if (idx[2][c] < 0) continue;
#pragma unroll
      for (int b = 0; b < P; ++b) {
        if (idx[1][b] < 0) continue;
        const long long row = ((long long)idx[2][c] * g.n[1] + idx[1][b]) * g.n[0];
        double sv = 0.0, sd = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a) {
          if (idx[0][a] < 0) continue;
          const double e = (double)e1[row + idx[0][a]];
          sv += e * w[0][a];
          sd += e * dw[0][a];
        }
        v += sv * w[1][b] * w[2][c];
        gx += sd * w[1][b] * w[2][c];
        gy += sv * dw[1][b] * w[2][c];
        gz += sv * w[1][b] * dw[2][c];
      }
    }
    const double qd = (double)pi.w;
    const T qi = pi.w;
    const double phid = phi0[i] + v - qd * self_const;
    const T phi = (T)phid;
    const T fx = (T)((double)F0[3 * i] - qd * gx), fy = (T)((double)F0[3 * i + 1] - qd * gy),
            fz = (T)((double)F0[3 * i + 2] - qd * gz);
    const int o = perm[i];
    if (dEdq) dEdq[o] = phi;
    if (F) {
      F[3 * o] = fx;
      F[3 * o + 1] = fy;
      F[3 * o + 2] = fz;
    }
    if (save_phi) save_phi[i] = phi;
    if (save_F) {
      save_F[3 * i] = fx;
      save_F[3 * i + 1] = fy;
      save_F[3 * i + 2] = fz;
    }
    ep = 0.5 * qd * phid;
    (void)qi;
  }
  // wavefront then workgroup reduction in FP64
  for (int off = 32; off > 0; off >>= 1) ep += __shfl_down(ep, off, 64);
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = ep;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    atomicAdd(energy, s);
  }
}

// ---------------------------------------------------------------------------
// explicit instantiation through launch helpers
// ---------------------------------------------------------------------------
template <typename T>
void launch_binning(int n, const T* pos, const T* q, const BinParams<T>& bp, int ncell,
                    int* cell_of, int* rank, int* counts, vec4_t<T>* wrapped, int* start,
                    vec4_t<T>* sorted, int* perm, int* flag, hipStream_t s) {
  const int nb = (n + 255) / 256;
  if (n > 0)
    hipLaunchKernelGGL(k_bin_count<T>, dim3(nb), dim3(256), 0, s, n, pos, q, bp, cell_of, rank,
                       counts, wrapped, flag);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ncell, counts, start);
  if (n > 0)
    hipLaunchKernelGGL(k_bin_scatter<T>, dim3(nb), dim3(256), 0, s, n, cell_of, rank, start,
                       wrapped, sorted, perm);
}

template <typename T>
void launch_pair(int p, int ncell, const vec4_t<T>* sorted, const int* start,
                 const PairParams<T>& pp, double* phi0, T* F0, hipStream_t s) {
  if (ncell <= 0) return;
  switch (p) {
    case 4: hipLaunchKernelGGL((k_pair<T, 4>), dim3(ncell), dim3(kPairThreads), 0, s, sorted, start, pp, phi0, F0); break;
    case 6: hipLaunchKernelGGL((k_pair<T, 6>), dim3(ncell), dim3(kPairThreads), 0, s, sorted, start, pp, phi0, F0); break;
    case 8: hipLaunchKernelGGL((k_pair<T, 8>), dim3(ncell), dim3(kPairThreads), 0, s, sorted, start, pp, phi0, F0); break;
  }
}

template <typename T>
void launch_anterp(int p, int n, const vec4_t<T>* sorted, const GridDev<T>& g, T* grid,
                   hipStream_t s) {
  if (n <= 0) return;
  const int nb = (n + 255) / 256;
  switch (p) {
    case 4: hipLaunchKernelGGL((k_anterp<T, 4>), dim3(nb), dim3(256), 0, s, n, sorted, g, grid); break;
    case 6: hipLaunchKernelGGL((k_anterp<T, 6>), dim3(nb), dim3(256), 0, s, n, sorted, g, grid); break;
    case 8: hipLaunchKernelGGL((k_anterp<T, 8>), dim3(nb), dim3(256), 0, s, n, sorted, g, grid); break;
  }
}

template <typename T>
void launch_interp(int p, int n, const vec4_t<T>* sorted, const int* perm, const GridDev<T>& g,
                   const T* e1, const double* phi0, const T* F0, double self_const, T* dEdq,
                   T* F, T* save_phi, T* save_F, double* energy, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (n + 255) / 256;
  switch (p) {
    case 4: hipLaunchKernelGGL((k_interp<T, 4>), dim3(nb), dim3(256), 0, s, n, sorted, perm, g, e1, phi0, F0, self_const, dEdq, F, save_phi, save_F, energy); break;
    case 6: hipLaunchKernelGGL((k_interp<T, 6>), dim3(nb), dim3(256), 0, s, n, sorted, perm, g, e1, phi0, F0, self_const, dEdq, F, save_phi, save_F, energy); break;
    case 8: hipLaunchKernelGGL((k_interp<T, 8>), dim3(nb), dim3(256), 0, s, n, sorted, perm, g, e1, phi0, F0, self_const, dEdq, F, save_phi, save_F, energy); break;
  }
}

#define MSM_INST_PARTICLES(T)                                                                    \
  template void launch_binning<T>(int, const T*, const T*, const BinParams<T>&, int, int*, int*, \
                                  int*, vec4_t<T>*, int*, vec4_t<T>*, int*, int*, hipStream_t);  \
  template void launch_pair<T>(int, int, const vec4_t<T>*, const int*, const PairParams<T>&,      \
                               double*, T*, hipStream_t);                                        \
  template void launch_anterp<T>(int, int, const vec4_t<T>*, const GridDev<T>&, T*, hipStream_t); \
  template void launch_interp<T>(int, int, const vec4_t<T>*, const int*, const GridDev<T>&,      \
                                 const T*, const double*, const T*, double, T*, T*, T*, T*,       \
                                 double*, hipStream_t);
MSM_INST_PARTICLES(float)
MSM_INST_PARTICLES(double)

}  // namespace msm
