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
// Verlet skin.  The cell list (cell edge >= a + skin) is rebuilt only when
// some charge has moved more than skin/2 since the last rebuild: a pair
// within the cutoff then still lies in neighbouring cells of that cell list,
// so only the positions in it are refreshed.  Every kernel is launched on
// every call and reads the decision from device memory (a graph of the
// call replays unchanged).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void skin_keep(const SkinDev<T>& sk, int i, const T (&raw)[3],
                                 const vec4_t<T>& w) {
  vec4_t<T> r, d;
  r.x = raw[0];
  r.y = raw[1];
  r.z = raw[2];
  r.w = T(0);
  d.x = raw[0] - w.x;
  d.y = raw[1] - w.y;
  d.z = raw[2] - w.z;
  d.w = T(0);
  sk.ref[i] = r;
  sk.shift[i] = d;
}

// rebuild = force (a new n, a call with a workspace, a new cell or skin)
__global__ void k_skin_begin(int* __restrict__ state, int force) {
  if (threadIdx.x == 0) {
    if (force) state[kSkinForce] = 1;
    state[kSkinRebuild] = state[kSkinForce];
    state[kSkinCalls] += 1;
  }
}

// ... or any displacement beyond skin/2 (non-finite ones included)
template <typename T>
__global__ void k_skin_check(int n, const T* __restrict__ pos, SkinDev<T> sk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool far = false;
  if (i < n) {
    const vec4_t<T> r = sk.ref[i];
    const T dx = pos[3 * i] - r.x, dy = pos[3 * i + 1] - r.y, dz = pos[3 * i + 2] - r.z;
    far = !(dx * dx + dy * dy + dz * dz <= sk.half2);
  }
  if (__ballot(far) != 0 && (threadIdx.x & 63) == 0) atomicOr(&sk.state[kSkinRebuild], 1);
}

// No rebuild: the cell-ordered list gets the new positions, moved by each
// charge's wrap of the last rebuild (continuous across periodic faces, so
// the cell list and its image shifts stay valid), and the new charges.
template <typename T>
__global__ void k_skin_refresh(int n, const T* __restrict__ pos, const T* __restrict__ q,
                               const int* __restrict__ perm, BinParams<T> bp, SkinDev<T> sk,
                               vec4_t<T>* __restrict__ sorted, int* __restrict__ flag) {
  if (sk.state[kSkinRebuild]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const vec4_t<T> d = sk.shift[o];
  T x[3] = {pos[3 * o] - d.x, pos[3 * o + 1] - d.y, pos[3 * o + 2] - d.z};
  T qi = q[o];
  int bad = 0;
  if (!isfinite(qi)) {
    bad |= kFlagNonfinite;
    qi = T(0);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!bp.tri && !bp.per[k] && (x[k] < T(0) || x[k] > bp.box[k])) {
      bad |= kFlagDomain;
      x[k] = x[k] < T(0) ? T(0) : bp.box[k];
    }
  if (bad) atomicOr(flag, bad);
  vec4_t<T> w;
  w.x = x[0];
  w.y = x[1];
  w.z = x[2];
  w.w = qi;
  sorted[i] = w;
}

// ---------------------------------------------------------------------------
// a1: binning.  Periodic coordinates are wrapped into [0, box); free ones are
// checked against [0, box] (flag + clamp, so every later index stays in
// bounds); non-finite values are flagged and replaced by 0.
// ---------------------------------------------------------------------------
//
// With a Verlet skin (sk != null, the plan's SkinState) the binning kernels
// run only on calls that rebuild the cell list; the count kernel then also
// keeps each caller's position and its wrap (raw minus wrapped) for the
// refresh of later calls, and marks the rebuild as done.
template <typename T>
__global__ void k_bin_count(int n, const T* __restrict__ pos, const T* __restrict__ q,
                            BinParams<T> bp, int* __restrict__ cell_of, int* __restrict__ rank,
                            int* __restrict__ counts, vec4_t<T>* __restrict__ wrapped,
                            int* __restrict__ flag, SkinDev<T> sk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (sk.state) {
    if (!sk.state[kSkinRebuild]) return;
    if (i == 0) {
      sk.state[kSkinForce] = sk.keep_force;
      sk.state[kSkinRebuilds] += 1;
    }
  }
  if (i >= n) return;
  T x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  T qi = q[i];
  int bad = 0;
  if (!isfinite(qi)) {
    bad |= kFlagNonfinite;
    qi = T(0);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!isfinite(x[k])) {
      bad |= kFlagNonfinite;
      x[k] = T(0);
    }
  if (bp.tri) {
    // the cell from the fractional coordinates s = H^{-1} r (FP64); the
    // position is wrapped by the whole lattice vectors floor(s) and stays
    // Cartesian (unchanged inside the cell)
    const double r[3] = {(double)x[0], (double)x[1], (double)x[2]};
    double sf[3], nw[3];
    int ct[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sf[k] = bp.Hi[3 * k] * r[0] + bp.Hi[3 * k + 1] * r[1] + bp.Hi[3 * k + 2] * r[2];
      nw[k] = floor(sf[k]);
      const int ci = (int)((sf[k] - nw[k]) * (double)bp.nc[k]);
      ct[k] = ci < 0 ? 0 : (ci >= bp.nc[k] ? bp.nc[k] - 1 : ci);
    }
    vec4_t<T> w;
    if (nw[0] != 0.0 || nw[1] != 0.0 || nw[2] != 0.0) {
      w.x = (T)(r[0] - (bp.H[0] * nw[0] + bp.H[1] * nw[1] + bp.H[2] * nw[2]));
      w.y = (T)(r[1] - (bp.H[3] * nw[0] + bp.H[4] * nw[1] + bp.H[5] * nw[2]));
      w.z = (T)(r[2] - (bp.H[6] * nw[0] + bp.H[7] * nw[1] + bp.H[8] * nw[2]));
    } else {
      w.x = x[0];
      w.y = x[1];
      w.z = x[2];
    }
    w.w = qi;
    if (bad) atomicOr(flag, bad);
    const int cell = (ct[2] * bp.nc[1] + ct[1]) * bp.nc[0] + ct[0];
    const int slot = cell * kCountCopies + (i & (kCountCopies - 1));
    cell_of[i] = slot;
    rank[i] = atomicAdd(&counts[slot], 1);
    wrapped[i] = w;
    if (sk.state) {
      const T raw[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
      skin_keep(sk, i, raw, w);
    }
    return;
  }
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T v = x[k];
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
  if (sk.state) {
    const T raw[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    skin_keep(sk, i, raw, w);
  }
}

// Exclusive scans of the cell counts into start[0..ncell] and of the
// per-cell cluster counts ceil(count / 8) into cl_start[0..ncell] (one
// workgroup).  The kCountCopies counters of every cell are replaced in place
// by the offset of their first particle (the scatter's base per slot).
// Inclusive scan of (v, cv) over the 1024 threads of a workgroup.
__device__ inline void scan1024(int& v, int& cv, int* buf, int* cbuf) {
  const int t = threadIdx.x;
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
  v = buf[t];
  cv = cbuf[t];
}

// Counts of one cell (its kCountCopies counters) and its cluster count.
__device__ inline int cell_count(int cell, int ncell, const int* counts, int (&sub)[kCountCopies]) {
  int v = 0;
#pragma unroll
  for (int k = 0; k < kCountCopies; ++k) {
    sub[k] = cell < ncell ? counts[cell * kCountCopies + k] : 0;
    v += sub[k];
  }
  return v;
}

// Writes the cell's start, cluster offset and per-slot scatter bases.
__device__ inline void cell_store(int cell, int o, int co, int* counts, int* start, int* cl_start,
                                  const int (&sub)[kCountCopies]) {
  start[cell] = o;
  cl_start[cell] = co;
#pragma unroll
  for (int k = 0; k < kCountCopies; ++k) {
    counts[cell * kCountCopies + k] = o;
    o += sub[k];
  }
}

__global__ void __launch_bounds__(1024) k_scan(int ncell, int* __restrict__ counts,
                                               int* __restrict__ start,
                                               int* __restrict__ cl_start,
                                               const int* __restrict__ gate) {
  if (gate && !gate[kSkinRebuild]) return;
  __shared__ int buf[1024], cbuf[1024];
  int carry = 0, ccarry = 0;  // the same in every thread
  for (int base = 0; base < ncell; base += 1024) {
    const int cell = base + threadIdx.x;
    int sub[kCountCopies];
    const int v = cell_count(cell, ncell, counts, sub), cv = (v + 7) / 8;
    int sv = v, scv = cv;
    scan1024(sv, scv, buf, cbuf);
    if (cell < ncell) cell_store(cell, carry + sv - v, ccarry + scv - cv, counts, start, cl_start, sub);
    carry += buf[1023];
    ccarry += cbuf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    start[ncell] = carry;
    cl_start[ncell] = ccarry;
  }
}

// Many cells: the same scan in three launches over blocks of 1024 cells
// (block totals; their exclusive scan in one workgroup; the blocks' own
// scans plus their offsets).  tmp holds 2 ints per block.
__global__ void __launch_bounds__(1024) k_scan_totals(int ncell, const int* __restrict__ counts,
                                                      int* __restrict__ tmp,
                                                      const int* __restrict__ gate) {
  if (gate && !gate[kSkinRebuild]) return;
  __shared__ int buf[1024], cbuf[1024];
  const int cell = blockIdx.x * 1024 + threadIdx.x;
  int sub[kCountCopies];
  int v = cell_count(cell, ncell, counts, sub), cv = (v + 7) / 8;
  scan1024(v, cv, buf, cbuf);
  if (threadIdx.x == 1023) {
    tmp[2 * blockIdx.x] = v;
    tmp[2 * blockIdx.x + 1] = cv;
  }
}

__global__ void __launch_bounds__(1024) k_scan_offsets(int nblk, int* __restrict__ tmp,
                                                       const int* __restrict__ gate) {
  if (gate && !gate[kSkinRebuild]) return;
  __shared__ int buf[1024], cbuf[1024];
  int carry = 0, ccarry = 0;
  for (int base = 0; base < nblk; base += 1024) {
    const int b = base + threadIdx.x;
    const int v = b < nblk ? tmp[2 * b] : 0, cv = b < nblk ? tmp[2 * b + 1] : 0;
    int sv = v, scv = cv;
    scan1024(sv, scv, buf, cbuf);
    __syncthreads();  // every thread has read tmp before it is overwritten
    if (b < nblk) {
      tmp[2 * b] = carry + sv - v;
      tmp[2 * b + 1] = ccarry + scv - cv;
    }
    carry += buf[1023];
    ccarry += cbuf[1023];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_scan_apply(int ncell, int* __restrict__ counts,
                                                     int* __restrict__ start,
                                                     int* __restrict__ cl_start,
                                                     const int* __restrict__ tmp,
                                                     const int* __restrict__ gate) {
  if (gate && !gate[kSkinRebuild]) return;
  __shared__ int buf[1024], cbuf[1024];
  const int cell = blockIdx.x * 1024 + threadIdx.x;
  int sub[kCountCopies];
  const int v = cell_count(cell, ncell, counts, sub), cv = (v + 7) / 8;
  int sv = v, scv = cv;
  scan1024(sv, scv, buf, cbuf);
  const int o = tmp[2 * blockIdx.x], co = tmp[2 * blockIdx.x + 1];
  if (cell < ncell) cell_store(cell, o + sv - v, co + scv - cv, counts, start, cl_start, sub);
  if (cell == ncell - 1) {
    start[ncell] = o + sv;
    cl_start[ncell] = co + scv;
  }
}

int scan_tmp_ints(int ncell) { return 2 * ((ncell + 1023) / 1024); }
constexpr int kScanOneBlock = 16384;  // up to this many cells: k_scan alone

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
                              ZeroJobs zero, const int* __restrict__ gate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int j = 0; j < zero.n; ++j) {
    unsigned* p = reinterpret_cast<unsigned*>(zero.ptr[j]);
    for (long long k = i; k < zero.words[j]; k += stride) p[k] = 0u;
  }
  if (i >= n || (gate && !gate[kSkinRebuild])) return;
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
  // brick blockIdx.x / split; this workgroup takes every split-th block of
  // 256 of its charges
  const int part = blockIdx.x % bg.split, stride = blockDim.x * bg.split;
  const int count = brick_runs(blockIdx.x / bg.split, start, cg, bg, c0, c1, runs, nruns);
  if (count <= part * (int)blockDim.x) return;
  int lo[3], ext[3];
  const int vol = brick_box<P>(c0, c1, cg, g.hd, lo, ext);
  const bool staged = vol <= brick_cap;
  double scale = 1.0;
  if (staged) {
    for (int b = threadIdx.x; b < vol; b += blockDim.x) brick[b] = 0;
    double aq = 0.0;
    for (int j = part * blockDim.x + threadIdx.x; j < count; j += stride)
      aq += fabs((double)sorted[brick_particle(runs, nruns, j)].w);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) aq += __shfl_xor(aq, o);
    if ((threadIdx.x & 63) == 0) qsum[threadIdx.x >> 6] = aq;
    __syncthreads();
    int ex;
    (void)frexp(qsum[0] + qsum[1] + qsum[2] + qsum[3], &ex);  // total < 2^ex
    scale = ldexp(1.0, 62 - max(ex, -900));  // stays a finite power of two
  }
  for (int jp = part * blockDim.x + threadIdx.x; jp < count; jp += stride) {
    const vec4_t<T> pi = sorted[brick_particle(runs, nruns, jp)];
    double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    grid_frame(g, xs);
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
    double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    grid_frame(g, xs);
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
    grid_to_cartesian(g, gx, gy, gz);
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
                    int* cl_start, vec4_t<T>* sorted, int* perm, int* flag, int* scan_tmp,
                    const ZeroJobs& zero, const SkinDev<T>& sk, int force, hipStream_t s) {
  const int nb = (n + 255) / 256;
  const int* gate = sk.state;
  if (sk.state) {
    hipLaunchKernelGGL(k_skin_begin, dim3(1), dim3(64), 0, s, sk.state, force);
    if (n > 0) hipLaunchKernelGGL(k_skin_check<T>, dim3(nb), dim3(256), 0, s, n, pos, sk);
  }
  if (n > 0)
    hipLaunchKernelGGL(k_bin_count<T>, dim3(nb), dim3(256), 0, s, n, pos, q, bp, cell_of, rank,
                       counts, wrapped, flag, sk);
  if (ncell <= kScanOneBlock || !scan_tmp) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ncell, counts, start, cl_start, gate);
  } else {
    const int nblk = (ncell + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_totals, dim3(nblk), dim3(1024), 0, s, ncell, counts, scan_tmp, gate);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, nblk, scan_tmp, gate);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(1024), 0, s, ncell, counts, start, cl_start,
                       scan_tmp, gate);
  }
  if (n > 0)
    hipLaunchKernelGGL(k_bin_scatter<T>, dim3(nb), dim3(256), 0, s, n, cell_of, rank, counts,
                       wrapped, sorted, perm, zero, gate);
  else
    launch_zero_multi(zero, s);
  if (sk.state && n > 0)
    hipLaunchKernelGGL(k_skin_refresh<T>, dim3(nb), dim3(256), 0, s, n, pos, q, perm, bp, sk,
                       sorted, flag);
}

// Large level-1 grids: one workgroup owns a tile of kTileX x kTileY x kTileZ
// grid points and gathers every charge whose support meets it, from the
// cells around the tile (periodic images included: a cell reached across a
// periodic face shifts its charges' grid indices by one period).  The tile
// is summed in LDS in the same 64-bit fixed point as the bricks (scale from
// the total |q| of the gathered cells) and written with plain stores, so
// HBM sees each grid value once, with no atomics and no clearing.  A charge
// is spread by every tile its support meets (about two at p = 4) and read by
// every tile whose margin its cell meets.
constexpr int kTileX = 32, kTileY = 8, kTileZ = 8;
constexpr int kTileRuns = 256;  // cell runs per tile (x segments of cell rows)
constexpr int kTileSegs = 8;    // x segments per cell row (periodic splits)

template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_anterp_tile(const int* __restrict__ start, const vec4_t<T>* __restrict__ sorted,
                  GridDev<T> g, CellGrid cg, T* __restrict__ grid) {
  __shared__ long long acc[kTileX * kTileY * kTileZ];
  __shared__ int rbeg[kTileRuns], roff[kTileRuns + 1], rsh[kTileRuns][3];
  __shared__ double qsum[4];
  const int T3[3] = {kTileX, kTileY, kTileZ};
  int nt[3], t0[3], t1[3];
  for (int k = 0; k < 3; ++k) nt[k] = (g.n[k] + T3[k] - 1) / T3[k];
  {
    const int b = blockIdx.x;
    const int ti[3] = {b % nt[0], (b / nt[0]) % nt[1], b / (nt[0] * nt[1])};
    for (int k = 0; k < 3; ++k) {
      t0[k] = ti[k] * T3[k];
      t1[k] = min(g.n[k], t0[k] + T3[k]);
    }
  }
  // cells whose charges can reach grid indices [t0, t1): a charge touches
  // the tile only if its coordinate lies in [(t0 + lo - P/2 - 1) h,
  // (t1 + lo + P/2) h) (its first support point is floor(x/h) - P/2 + 1,
  // give or take one for the rounding of grid_coord); one more grid spacing
  // on each side covers the rounding of the binning.  Free axes are clipped
  // to the grid of cells.
  int clo[3], chi[3];
  for (int k = 0; k < 3; ++k) {
    const double a0 = (double)(t0[k] + g.lo[k] - P / 2 - 2) * g.hd[k];
    const double a1 = (double)(t1[k] + g.lo[k] + P / 2 + 1) * g.hd[k];
    clo[k] = (int)floor(a0 / cg.cs[k]);
    chi[k] = (int)floor(a1 / cg.cs[k]);
    if (!g.per[k]) {
      clo[k] = max(clo[k], 0);
      chi[k] = min(chi[k], cg.nc[k] - 1);
    }
  }
  // x segments: consecutive cells of one periodic image
  int sa[kTileSegs], sb[kTileSegs], ss[kTileSegs], nseg = 0;
  for (int c = clo[0]; c <= chi[0] && nseg < kTileSegs;) {
    const int img = g.per[0] ? (c >= 0 ? c / cg.nc[0] : -((-c + cg.nc[0] - 1) / cg.nc[0])) : 0;
    const int e = min(chi[0], (img + 1) * cg.nc[0] - 1);
    sa[nseg] = c - img * cg.nc[0];
    sb[nseg] = e - img * cg.nc[0];
    ss[nseg] = img * g.n[0];
    ++nseg;
    c = e + 1;
  }
  const int ny = max(chi[1] - clo[1] + 1, 0), nz = max(chi[2] - clo[2] + 1, 0);
  const int nruns = ny * nz * nseg;  // <= kTileRuns (checked by the host)
  for (int i = threadIdx.x; i < kTileX * kTileY * kTileZ; i += blockDim.x) acc[i] = 0;
  if (threadIdx.x < nruns) {
    const int r = threadIdx.x, sg = r % nseg, row = r / nseg;
    int cy = clo[1] + row % ny, cz = clo[2] + row / ny, sy = 0, sz = 0;
    if (g.per[1]) {
      sy = cy >= 0 ? cy / cg.nc[1] : -((-cy + cg.nc[1] - 1) / cg.nc[1]);
      cy -= sy * cg.nc[1];
    }
    if (g.per[2]) {
      sz = cz >= 0 ? cz / cg.nc[2] : -((-cz + cg.nc[2] - 1) / cg.nc[2]);
      cz -= sz * cg.nc[2];
    }
    const int rowc = (cz * cg.nc[1] + cy) * cg.nc[0];
    const int b = start[rowc + sa[sg]];
    rbeg[r] = b;
    roff[r + 1] = start[rowc + sb[sg] + 1] - b;
    rsh[r][0] = ss[sg];
    rsh[r][1] = sy * g.n[1];
    rsh[r][2] = sz * g.n[2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    roff[0] = 0;
    for (int r = 0; r < nruns; ++r) {
      a += roff[r + 1];
      roff[r + 1] = a;
    }
  }
  __syncthreads();
  const int count = roff[nruns];
  auto particle = [&](int j, int& r) {
    r = 0;
#pragma unroll
    for (int step = kTileRuns / 2; step > 0; step >>= 1)
      if (r + step < nruns && roff[r + step] <= j) r += step;
    return rbeg[r] + (j - roff[r]);
  };
  double aq = 0.0;
  for (int j = threadIdx.x; j < count; j += blockDim.x) {
    int r;
    aq += fabs((double)sorted[particle(j, r)].w);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) aq += __shfl_xor(aq, o);
  if ((threadIdx.x & 63) == 0) qsum[threadIdx.x >> 6] = aq;
  __syncthreads();
  int ex;
  (void)frexp(qsum[0] + qsum[1] + qsum[2] + qsum[3], &ex);
  const double scale = ldexp(1.0, 62 - max(ex, -900));
  for (int j = threadIdx.x; j < count; j += blockDim.x) {
    int r;
    const vec4_t<T> pi = sorted[particle(j, r)];
    double xs[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
    grid_frame(g, xs);
    double w[3][P];
    bool in[3][P];
    int i0[3];  // tile-local index of support point 0 per axis
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double f;
      const int m0 = grid_coord<double>(xs[k], g.hd[k], f) - P / 2 + 1 + rsh[r][k];
      bspline_weights<P, double>(f, w[k], nullptr, nullptr);
      i0[k] = m0 - g.lo[k] - t0[k];
#pragma unroll
      for (int a = 0; a < P; ++a) in[k][a] = i0[k] + a >= 0 && i0[k] + a < t1[k] - t0[k];
    }
    const double qs = (double)pi.w * scale;
#pragma unroll
    for (int c = 0; c < P; ++c) {
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const double wyz = qs * w[2][c] * w[1][b];
        const int row = ((i0[2] + c) * kTileY + (i0[1] + b)) * kTileX + i0[0];
#pragma unroll
        for (int a = 0; a < P; ++a)
          if (in[2][c] && in[1][b] && in[0][a])
            atomicAdd((unsigned long long*)&acc[row + a],
                      (unsigned long long)__double2ll_rn(wyz * w[0][a]));
      }
    }
  }
  __syncthreads();
  const double inv_scale = 1.0 / scale;
  const int ex0 = t1[0] - t0[0], ex1 = t1[1] - t0[1], vol = ex0 * ex1 * (t1[2] - t0[2]);
  for (int i = threadIdx.x; i < vol; i += blockDim.x) {
    const int x = i % ex0, y = (i / ex0) % ex1, z = i / (ex0 * ex1);
    grid[((long long)(t0[2] + z) * g.n[1] + (t0[1] + y)) * g.n[0] + (t0[0] + x)] =
        (T)((double)acc[(z * kTileY + y) * kTileX + x] * inv_scale);
  }
}

// Whether launch_anterp takes the tiled path (large grids; the tile's
// cell runs must fit kTileRuns).  The tiled path writes every grid value,
// so the caller need not clear the grid first.
bool anterp_tiled(int p, int n, const CellGrid& cg, const int gn[3], const int gper[3],
                  const double hd[3]) {
  if (n <= 0 || cg.margin > 0) return false;
  // measured on periodic 128^3-512^3 grids: tiles win where charges are
  // sparse (0.075 per grid point: 1.6 against 3.5 ms), bricks where they are
  // dense (0.45 per point: 5.1 against 6.5 ms; 0.6: 0.96 against 1.13 ms),
  // since a tile spreads each charge of its margin again (MSM_ANTERP_TILES=1
  // / 0 forces a path)
  const char* env = std::getenv("MSM_ANTERP_TILES");
  const long long G = (long long)gn[0] * gn[1] * gn[2];
  const bool want = env && env[0] ? env[0] == '1' : (G >= (1LL << 21) && n <= 0.15 * (double)G);
  if (!want) return false;
  const int T3[3] = {kTileX, kTileY, kTileZ};
  long long runs = 1;
  for (int k = 0; k < 3; ++k) {
    // cells a tile can gather along axis k (k_anterp_tile's cell range spans
    // (ext + p + 3) h; floor at both ends adds up to two cells)
    const int ext = std::min(T3[k], gn[k]);
    const long long cells = (long long)std::ceil((ext + p + 3) * hd[k] / cg.cs[k]) + 2;
    const long long nck = std::max(cg.nc[k], 1);
    if (k == 0) {
      // consecutive cells meet at most ceil(cells / nc) + 1 periodic images
      const long long segs = gper[0] ? (cells + nck - 1) / nck + 1 : 1;
      if (segs > kTileSegs) return false;
      runs *= segs;
    } else {
      runs *= gper[k] ? cells : std::min(cells, nck);
    }
  }
  return runs <= kTileRuns;
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
  // grow the super-cell while its brick's points (each cleared, read and
  // added to HBM with a global atomic: weighed as kFlushWeight LDS adds) cost
  // more than the charges' p^3 LDS adds, the brick fits and at least
  // kMinBricks workgroups remain (a larger brick also overlaps its
  // neighbours less, so the grid takes fewer atomics per point)
  constexpr long long kMinBricks = 4096;
  constexpr double kFlushWeight = 10.0;  // (2 was 25% slower on 128^3-256^3 grids)
  const double per_cell = (double)n / std::max(ncell, 1) * p * p * p;
  int kc = 1;
  const char* env = std::getenv("MSM_BRICK_CELLS");
  if (env && std::atoi(env) > 0) {
    const int want = std::min(std::atoi(env), kBrickMaxCells);
    while (kc < want && cap(kc + 1) <= kBrickMax) ++kc;
  } else {
    while (kc < kBrickMaxCells && cap(kc + 1) <= kBrickMax && bricks(kc + 1) >= kMinBricks &&
           kFlushWeight * cap(kc) > per_cell * kc * kc * kc)
      ++kc;
  }
  BrickGeom bg;
  bg.kc = kc;
  for (int k = 0; k < 3; ++k) bg.nsc[k] = (cg.nc[k] + kc - 1) / kc;
  // few bricks (a small box, or cells of several cutoffs' worth of charges):
  // split each brick's charges over several workgroups, each with a brick
  // of its own, so that the launch still spreads over the chip; at least
  // kMinShare charges per workgroup keep the extra clears and flushes small
  constexpr long long kSplitBelow = 512, kMinShare = 128;
  const long long nb = bricks(kc);
  bg.split = 1;
  if (nb < kSplitBelow)
    bg.split = (int)std::max<long long>(
        1, std::min<long long>((kSplitBelow + nb - 1) / nb, (long long)n / (nb * kMinShare)));
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
  if (anterp_tiled(p, n, cg, g.n, g.per, g.hd)) {
    const unsigned nb = (unsigned)(((g.n[0] + kTileX - 1) / kTileX) *
                                   ((g.n[1] + kTileY - 1) / kTileY) *
                                   ((g.n[2] + kTileZ - 1) / kTileZ));
    switch (p) {
      case 4: hipLaunchKernelGGL((k_anterp_tile<T, 4>), dim3(nb), dim3(256), 0, s, start, sorted, g, cg, grid); break;
      case 6: hipLaunchKernelGGL((k_anterp_tile<T, 6>), dim3(nb), dim3(256), 0, s, start, sorted, g, cg, grid); break;
      case 8: hipLaunchKernelGGL((k_anterp_tile<T, 8>), dim3(nb), dim3(256), 0, s, start, sorted, g, cg, grid); break;
    }
    return;
  }
  const BrickGeom bg = brick_geom(p, n, ncell, cg, g.hd);
  const int bc = brick_lds_cap(p, bg, cg, g.hd);
  const size_t lds = (size_t)bc * sizeof(long long);
  const unsigned nb = (unsigned)bg.nsc[0] * bg.nsc[1] * bg.nsc[2] * bg.split;
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
                                  int*, vec4_t<T>*, int*, int*, vec4_t<T>*, int*, int*, int*,   \
                                  const ZeroJobs&, const SkinDev<T>&, int, hipStream_t);        \
  template void launch_anterp<T>(int, int, int, const int*, const CellGrid&, const vec4_t<T>*,   \
                                 const GridDev<T>&, T*, hipStream_t);                             \
  template void launch_interp<T>(int, int, const vec4_t<T>*, const int*, const GridDev<T>&,      \
                                 const T*, const double*, const T*, double, T*, T*, T*, T*,       \
                                 double*, hipStream_t);
MSM_INST_PARTICLES(float)
MSM_INST_PARTICLES(double)

}  // namespace msm
