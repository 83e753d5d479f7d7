// kernels_particles.hip -- particle-side kernels of the MSM forward pass:
// cell binning (count, scan, scatter), anterpolation onto the level-1 grid, and interpolation fused with the
// final combination of short- and long-range parts and the FP64 energy sum.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "brick.hpp"
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
  // kCountCopies counters per cell spread the atomic traffic of dense cells
  const int slot = cell * kCountCopies + (i & (kCountCopies - 1));
  cell_of[i] = slot;
  rank[i] = atomicAdd(&counts[slot], 1);
  vec4_t<T> w;
  w.x = x[0];
  w.y = x[1];
  w.z = x[2];
  w.w = qi;
  wrapped[i] = w;
}

// Exclusive scans of the cell counts into start[0..ncell] and of the
// per-cell cluster counts ceil(count / 8) into cl_start[0..ncell] (one
// workgroup).  The kCountCopies counters of every cell are replaced in place
// by the offset of their first particle (the scatter's base per slot).
__global__ void __launch_bounds__(1024) k_scan(int ncell, int* __restrict__ counts,
                                               int* __restrict__ start,
                                               int* __restrict__ cl_start) {
  __shared__ int buf[1024], cbuf[1024];
  __shared__ int carry, ccarry;
  const int t = threadIdx.x;
  if (t == 0) {
    carry = 0;
    ccarry = 0;
  }
  __syncthreads();
  for (int base = 0; base < ncell; base += 1024) {
    const int cell = base + t;
    int sub[kCountCopies];
    int v = 0;
#pragma unroll
    for (int k = 0; k < kCountCopies; ++k) {
      sub[k] = cell < ncell ? counts[cell * kCountCopies + k] : 0;
      v += sub[k];
    }
    const int cv = (v + 7) / 8;
    buf[t] = v;
    cbuf[t] = cv;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = (t >= off) ? buf[t - off] : 0;
      const int cadd = (t >= off) ? cbuf[t - off] : 0;
      __syncthreads();
      buf[t] += add;
      cbuf[t] += cadd;
      __syncthreads();
    }
    if (cell < ncell) {
      int o = carry + buf[t] - v;
      start[cell] = o;
      cl_start[cell] = ccarry + cbuf[t] - cv;
#pragma unroll
      for (int k = 0; k < kCountCopies; ++k) {
        counts[cell * kCountCopies + k] = o;
        o += sub[k];
      }
    }
    __syncthreads();
    if (t == 1023) {
      carry += buf[1023];
      ccarry += cbuf[1023];
    }
    __syncthreads();
  }
  if (t == 0) {
    start[ncell] = carry;
    cl_start[ncell] = ccarry;
  }
}

// Zeroes up to kZeroJobs buffers (4-byte words) in one launch.
__global__ void k_zero_multi(ZeroJobs jobs) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int j = 0; j < jobs.n; ++j) {
    unsigned* p = reinterpret_cast<unsigned*>(jobs.ptr[j]);
    const long long w = jobs.words[j];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < w; i += stride) p[i] = 0u;
  }
}

void launch_zero_multi(const ZeroJobs& jobs, hipStream_t s) {
  long long maxw = 0;
  for (int j = 0; j < jobs.n; ++j) maxw = jobs.words[j] > maxw ? jobs.words[j] : maxw;
  if (maxw == 0) return;
  long long nb = (maxw + 255) / 256;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_zero_multi, dim3((unsigned)nb), dim3(256), 0, s, jobs);
}

// Scatter to cell order; the same threads also clear the accumulators of
// the rest of the pass (zero: up to kZeroJobs buffers of 4-byte words).
template <typename T>
__global__ void k_bin_scatter(int n, const int* __restrict__ cell_of, const int* __restrict__ rank,
                              const int* __restrict__ slot_base,
                              const vec4_t<T>* __restrict__ wrapped,
                              vec4_t<T>* __restrict__ sorted, int* __restrict__ perm,
                              ZeroJobs zero) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int j = 0; j < zero.n; ++j) {
    unsigned* p = reinterpret_cast<unsigned*>(zero.ptr[j]);
    for (long long k = i; k < zero.words[j]; k += stride) p[k] = 0u;
  }
  if (i >= n) return;
  const int dst = slot_base[cell_of[i]] + rank[i];
  sorted[dst] = wrapped[i];
  perm[dst] = i;
}

// ---------------------------------------------------------------------------
// a3: anterpolation (eq. grid_charge): q~^1_m += q_i phi_m(r_i) over the p^3
// grid points of each particle, B-spline weights in FP64.
// ---------------------------------------------------------------------------
// Staged per super-cell (kc^3 cells of the cell list, kc > 1 where cells are
// sparse): one workgroup accumulates the charges of its cells into an LDS
// brick covering every grid point they can touch, then adds the brick to
// the grid with one atomic per non-zero point (coalesced along x, and
// conflicting only where neighbouring bricks overlap).  The
// brick holds 64-bit fixed-point sums: every contribution is rounded to a
// multiple of 2^-S with 2^S sum_cell |q_i| < 2^62 (no sum can overflow, since
// B-spline weights lie in [0, 1]), and integer LDS adds are exact, so the
// brick does not depend on the order of the adds; the rounding is below 2^-62
// of the brick's total |q| per contribution.  A brick larger than brick_cap
// points (cells much wider than h) falls back to per-particle global atomics.

template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_anterp_brick(const int* __restrict__ start, const vec4_t<T>* __restrict__ sorted,
                   GridDev<T> g, CellGrid cg, BrickGeom bg, int brick_cap,
                   T* __restrict__ grid) {
  extern __shared__ long long brick[];
  __shared__ double qsum[4];
  __shared__ BrickRuns runs;
  int c0[3], c1[3], nruns;
  const int count = brick_runs(blockIdx.x, start, cg, bg, c0, c1, runs, nruns);
  if (count == 0) return;
  int lo[3], ext[3];
  const int vol = brick_box<P>(c0, c1, cg, g.hd, lo, ext);
  const bool staged = vol <= brick_cap;
  double scale = 1.0;
  if (staged) {
    for (int b = threadIdx.x; b < vol; b += blockDim.x) brick[b] = 0;
    double aq = 0.0;
    for (int j = threadIdx.x; j < count; j += blockDim.x)
      aq += fabs((double)sorted[brick_particle(runs, nruns, j)].w);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) aq += __shfl_xor(aq, o);
    if ((threadIdx.x & 63) == 0) qsum[threadIdx.x >> 6] = aq;
    __syncthreads();
    int ex;
    (void)frexp(qsum[0] + qsum[1] + qsum[2] + qsum[3], &ex);  // total < 2^ex
    scale = ldexp(1.0, 62 - max(ex, -900));  // stays a finite power of two
  }
  for (int jp = threadIdx.x; jp < count; jp += blockDim.x) {
    const vec4_t<T> pi = sorted[brick_particle(runs, nruns, jp)];
    const double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    double w[3][P];
    int m0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double f;
      m0[k] = grid_coord<double>(xs[k], g.hd[k], f) - P / 2 + 1;
      bspline_weights<P, double>(f, w[k], nullptr, nullptr);
    }
    const double qi = (double)pi.w;
    const double qs = qi * scale;
    bool inside = staged;
#pragma unroll
    for (int k = 0; k < 3; ++k) inside = inside && m0[k] >= lo[k] && m0[k] + P - 1 < lo[k] + ext[k];
    if (inside) {
      const int b0 = ((m0[2] - lo[2]) * ext[1] + (m0[1] - lo[1])) * ext[0] + (m0[0] - lo[0]);
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const double wz = qs * w[2][c];
#pragma unroll
        for (int b = 0; b < P; ++b) {
          const double wyz = wz * w[1][b];
          const int row = b0 + (c * ext[1] + b) * ext[0];
#pragma unroll
          for (int a = 0; a < P; ++a)
            atomicAdd((unsigned long long*)&brick[row + a],
                      (unsigned long long)__double2ll_rn(wyz * w[0][a]));
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
  }
  if (!staged) return;
  __syncthreads();
  const double inv_scale = 1.0 / scale;  // a power of two
  for (int b = threadIdx.x; b < vol; b += blockDim.x) {
    const long long s = brick[b];
    if (s == 0) continue;
    const T v = (T)((double)s * inv_scale);
    const int bx = b % ext[0], by = (b / ext[0]) % ext[1], bz = b / (ext[0] * ext[1]);
    const int ix = axis_index(lo[0] + bx, g.n[0], g.lo[0], g.per[0]);
    const int iy = axis_index(lo[1] + by, g.n[1], g.lo[1], g.per[1]);
    const int iz = axis_index(lo[2] + bz, g.n[2], g.lo[2], g.per[2]);
    if (ix < 0 || iy < 0 || iz < 0) continue;
    atomicAdd(&grid[((long long)iz * g.n[1] + iy) * g.n[0] + ix], v);
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
    // the P points of a row are consecutive in memory unless the row wraps
    // or leaves a free axis: then one vector load per row
    const bool run = idx[0][0] >= 0 && idx[0][P - 1] == idx[0][0] + P - 1;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      if (idx[2][c] < 0) continue;
#pragma unroll
      for (int b = 0; b < P; ++b) {
        if (idx[1][b] < 0) continue;
        const long long row = ((long long)idx[2][c] * g.n[1] + idx[1][b]) * g.n[0];
        T ev[P];
        if (run) {
          __builtin_memcpy(ev, e1 + row + idx[0][0], sizeof(ev));
        } else {
#pragma unroll
          for (int a = 0; a < P; ++a) ev[a] = idx[0][a] >= 0 ? e1[row + idx[0][a]] : T(0);
        }
        double sv = 0.0, sd = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a) {
          const double e = (double)ev[a];
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
                    int* cl_start, vec4_t<T>* sorted, int* perm, int* flag,
                    const ZeroJobs& zero, hipStream_t s) {
  const int nb = (n + 255) / 256;
  if (n > 0)
    hipLaunchKernelGGL(k_bin_count<T>, dim3(nb), dim3(256), 0, s, n, pos, q, bp, cell_of, rank,
                       counts, wrapped, flag);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ncell, counts, start, cl_start);
  if (n > 0)
    hipLaunchKernelGGL(k_bin_scatter<T>, dim3(nb), dim3(256), 0, s, n, cell_of, rank, counts,
                       wrapped, sorted, perm, zero);
  else
    launch_zero_multi(zero, s);
}

BrickGeom brick_geom(int p, int n, int ncell, const CellGrid& cg, const double hd[3]) {
  // LDS for the largest brick of kc^3 cells: per axis at most
  // ceil(kc cs / h) + p + 3 points (one more for the rounding of cs / h)
  auto cap = [&](int kc) {
    long long c = 1;
    for (int k = 0; k < 3; ++k) c *= (long long)std::ceil(kc * cg.cs[k] / hd[k]) + p + 4;
    return c;
  };
  auto bricks = [&](int kc) {
    long long m = 1;
    for (int k = 0; k < 3; ++k) m *= (cg.nc[k] + kc - 1) / kc;
    return m;
  };
  // grow the super-cell while clearing and flushing its brick (2 cap) costs
  // more than the charges' p^3 contributions, the brick fits and at least
  // kMinBricks workgroups remain
  constexpr long long kMinBricks = 4096;
  const double per_cell = (double)n / std::max(ncell, 1) * p * p * p;
  int kc = 1;
  const char* env = std::getenv("MSM_BRICK_CELLS");
  if (env && std::atoi(env) > 0) {
    const int want = std::min(std::atoi(env), kBrickMaxCells);
    while (kc < want && cap(kc + 1) <= kBrickMax) ++kc;
  } else {
    while (kc < kBrickMaxCells && cap(kc + 1) <= kBrickMax && bricks(kc + 1) >= kMinBricks &&
           2.0 * cap(kc) > per_cell * kc * kc * kc)
      ++kc;
  }
  BrickGeom bg;
  bg.kc = kc;
  for (int k = 0; k < 3; ++k) bg.nsc[k] = (cg.nc[k] + kc - 1) / kc;
  return bg;
}

// brick LDS in elements: the largest brick of this geometry, at most kBrickMax
int brick_lds_cap(int p, const BrickGeom& bg, const CellGrid& cg, const double hd[3]) {
  long long c = 1;
  for (int k = 0; k < 3; ++k) c *= (long long)std::ceil(bg.kc * cg.cs[k] / hd[k]) + p + 4;
  return (int)std::min<long long>(c, kBrickMax);
}

template <typename T>
void launch_anterp(int p, int n, int ncell, const int* start, const CellGrid& cg,
                   const vec4_t<T>* sorted, const GridDev<T>& g, T* grid, hipStream_t s) {
  if (n <= 0) return;
  const BrickGeom bg = brick_geom(p, n, ncell, cg, g.hd);
  const int bc = brick_lds_cap(p, bg, cg, g.hd);
  const size_t lds = (size_t)bc * sizeof(long long);
  const unsigned nb = (unsigned)bg.nsc[0] * bg.nsc[1] * bg.nsc[2];
  switch (p) {
    case 4: hipLaunchKernelGGL((k_anterp_brick<T, 4>), dim3(nb), dim3(256), lds, s, start, sorted, g, cg, bg, bc, grid); break;
    case 6: hipLaunchKernelGGL((k_anterp_brick<T, 6>), dim3(nb), dim3(256), lds, s, start, sorted, g, cg, bg, bc, grid); break;
    case 8: hipLaunchKernelGGL((k_anterp_brick<T, 8>), dim3(nb), dim3(256), lds, s, start, sorted, g, cg, bg, bc, grid); break;
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
                                  int*, vec4_t<T>*, int*, int*, vec4_t<T>*, int*, int*,         \
                                  const ZeroJobs&, hipStream_t);                                \
  template void launch_anterp<T>(int, int, int, const int*, const CellGrid&, const vec4_t<T>*,   \
                                 const GridDev<T>&, T*, hipStream_t);                             \
  template void launch_interp<T>(int, int, const vec4_t<T>*, const int*, const GridDev<T>&,      \
                                 const T*, const double*, const T*, double, T*, T*, T*, T*,       \
                                 double*, hipStream_t);
MSM_INST_PARTICLES(float)
MSM_INST_PARTICLES(double)

}  // namespace msm
