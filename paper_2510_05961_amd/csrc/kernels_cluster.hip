// kernels_cluster.hip -- the short-range part U^0 (eq. U_zero): the cluster
// layout of the cell list, the pair sum and its vector-Jacobian product.
//
// Layout.  Binning sorts particles by cell (cells of edge >= a).  Inside
// every cell the particles are then ordered along a Morton curve of a 16^3
// sub-grid (ties broken by the caller's index, so the order is
// deterministic) and cut into clusters of 8 consecutive particles; the last
// cluster of a cell is padded with far-away zero charges.  Each half of a
// cluster (4 particles, a "j-group") keeps its bounding box.
//
// Pair sum.  One wave per i-cluster.  Over the 27 neighbour cells, the
// j-groups whose box lies within the cutoff of the i-cluster's box are
// listed, then each of their members whose distance to that box is below
// the cutoff is moved into the i-cluster's frame and put in a per-wave ring;
// the wave evaluates eight ring entries per step, lane (il, jj) =
// (lane / 8, lane % 8) taking i-member il against entry jj.  Every pair is
// evaluated from both sides (each particle's sums stay in its own lanes).
// Periodic images are handled by a uniform shift per neighbour cell (27
// offsets, each (cell, shift) combination distinct), which is exact whenever
// the cell edge is >= a and every periodic edge is >= 2a: then at most one
// image of a particle lies inside the cutoff and it lies in one of the 27
// shifted neighbour cells.
//
// Pair VJP.  As the pair sum but on j-groups (8 x 4 blocks, two groups per
// step, lane (slot, il, jl) = (lane / 32, lane / 4 % 8, lane % 4)), with the
// force cotangents of both particles.
#include "cluster_dev.hpp"

namespace msm {

constexpr int kClusterThreads = 256;  // 4 waves = 4 i-clusters per workgroup
constexpr int kGroup = kGroupSize;    // particles per j-group (half a cluster)
constexpr int kSlots = 64 / (8 * kGroup);  // j-groups per wave step
constexpr int kPrepThreads = 256;
constexpr int kPrepSortMax = 4096;    // cells larger than this keep their order
constexpr int kSmallCell = 128;       // cells up to this size are staged in LDS
constexpr int kRing = 128;            // per-wave ring of culled j particles
constexpr int kStepJ = 8;             // j particles per wave step (8 x 8 lanes)

// Cluster offsets: cl_start[c] = sum_{c' < c} ceil(count_c' / 8), one workgroup.
__global__ void __launch_bounds__(1024) k_cluster_scan(int ncell, const int* __restrict__ start,
                                                       int* __restrict__ cl_start) {
  __shared__ int buf[1024];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ncell; base += 1024) {
    const int c = base + t;
    const int v = c < ncell ? (start[c + 1] - start[c] + 7) / 8 : 0;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = (t >= off) ? buf[t - off] : 0;
      __syncthreads();
      buf[t] += add;
      __syncthreads();
    }
    if (c < ncell) cl_start[c] = carry + buf[t] - v;
    __syncthreads();
    if (t == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (t == 0) cl_start[ncell] = carry;
}

__device__ inline unsigned spread3(unsigned v) {  // 4 bits -> every third bit
  v &= 0xF;
  v = (v | (v << 4)) & 0x0C3;
  v = (v | (v << 2)) & 0x249;
  return v;
}

// One workgroup per cell.  With sort != 0 the cell's particles are put in
// Morton order of a 16^3 sub-grid, ties broken by the caller's index, in
// place (sorted[], perm[] of the segment).  Cells of up to kSmallCell
// particles are staged in LDS and sorted in one wave's registers; larger
// ones are sorted in LDS and their positions re-read from wrapped[] in the
// caller's order; cells larger than kPrepSortMax keep the cell order.  The
// cluster slots, j-group boxes and cluster info are written in both modes
// from the (possibly new) order, and the cell's binning counters are set
// back to zero (counts != nullptr).
template <typename T>
__global__ void __launch_bounds__(kPrepThreads)
    k_cluster_prep(int sort, const int* __restrict__ start, const int* __restrict__ cl_start,
                   BinParams<T> bp, const vec4_t<T>* __restrict__ wrapped,
                   vec4_t<T>* __restrict__ sorted, int* __restrict__ perm,
                   vec4_t<T>* __restrict__ cpos, vec4_t<T>* __restrict__ cbox,
                   int4* __restrict__ cinfo, int* __restrict__ counts,
                   const int* __restrict__ gate) {
  __shared__ unsigned long long key[kPrepSortMax];
  if (gate && !gate[kSkinRebuild]) return;  // (Verlet skin: the layout is kept)
  const int cell = blockIdx.x;
  const int t = threadIdx.x;
  // the binning's counters of this cell (read by the scatter, which ran
  // before this kernel) go back to zero for the next binning
  if (counts && t < kCountCopies) counts[cell * kCountCopies + t] = 0;
  const int beg = start[cell], cnt = start[cell + 1] - beg;
  const int cbeg = cl_start[cell], ncl = cl_start[cell + 1] - cbeg;
  if (cnt == 0) return;
  const int cx = cell % bp.nc[0];
  const int cy = (cell / bp.nc[0]) % bp.nc[1];
  const int cz = cell / (bp.nc[0] * bp.nc[1]);
  const T lo3[3] = {(T)cx * bp.cs[0], (T)cy * bp.cs[1], (T)cz * bp.cs[2]};
  auto morton = [&](const vec4_t<T>& v) {
    T x[3] = {v.x, v.y, v.z};
    if (bp.tri) {  // cells of a triclinic cell are in fractional coordinates
      const double a = v.x, b = v.y, c = v.z;
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = (T)(bp.Hi[3 * d] * a + bp.Hi[3 * d + 1] * b + bp.Hi[3 * d + 2] * c);
    }
    unsigned m = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int s = (int)((x[d] - lo3[d]) * (T(16) / bp.cs[d]));
      s = s < 0 ? 0 : (s > 15 ? 15 : s);
      m |= spread3((unsigned)s) << d;
    }
    return m;
  };
  if (cnt <= kSmallCell) {
    // the whole cell in LDS: one read of the cell list, a sort in the
    // registers of one wave (lane t holds elements t and t + 64 of a bitonic
    // network over 128 slots, sentinels ~0 past cnt), then every output is
    // written from LDS
    __shared__ vec4_t<T> part[kSmallCell];
    __shared__ int pidx[kSmallCell];
    for (int i = t; i < cnt; i += kPrepThreads) {
      part[i] = sorted[beg + i];
      pidx[i] = perm[beg + i];
    }
    __syncthreads();
    const bool sorting = sort && cnt > 1;
    if (sorting) {
      if (t < 64) {
        // key: Morton code | caller's index | position in the cell
        auto key_of = [&](int i) -> unsigned long long {
          if (i >= cnt) return ~0ull;
          return ((unsigned long long)morton(part[i]) << 44) |
                 ((unsigned long long)(unsigned)pidx[i] << 12) | (unsigned long long)i;
        };
        unsigned long long e0 = key_of(t), e1 = key_of(t + 64);
        for (int k = 2; k <= 128; k <<= 1) {
          for (int j = k >> 1; j > 0; j >>= 1) {
            // element i keeps the smaller of (i, i ^ j) when "i is the lower
            // index" equals "the block of size k ascends", else the larger
            const bool up0 = (t & k) == 0, up1 = ((t + 64) & k) == 0;
            if (j == 64) {
              const unsigned long long a = e0 < e1 ? e0 : e1, b = e0 < e1 ? e1 : e0;
              e0 = up0 ? a : b;
              e1 = up1 ? b : a;
            } else {
              const unsigned long long p0 = __shfl_xor(e0, j), p1 = __shfl_xor(e1, j);
              const bool lower = (t & j) == 0;
              e0 = (lower == up0) ? (e0 < p0 ? e0 : p0) : (e0 < p0 ? p0 : e0);
              e1 = (lower == up1) ? (e1 < p1 ? e1 : p1) : (e1 < p1 ? p1 : e1);
            }
          }
        }
        key[t] = e0;
        key[t + 64] = e1;
      }
      __syncthreads();
    }
    auto src_of = [&](int slot) { return sorting ? (int)(key[slot] & 0xFFFu) : slot; };
    for (int s = t; s < ncl * 8; s += kPrepThreads) {
      vec4_t<T> v;
      if (s < cnt) {
        const int q = src_of(s);
        v = part[q];
        if (sorting) {
          sorted[beg + s] = v;
          perm[beg + s] = pidx[q];
        }
      } else {  // padding: a zero charge far outside every cutoff
        v.x = v.y = v.z = T(1e15);
        v.w = T(0);
      }
      cpos[(size_t)cbeg * 8 + s] = v;
    }
    for (int h = t; h < 2 * ncl; h += kPrepThreads) {
      const int m = min(kGroup, cnt - kGroup * h);
      vec4_t<T> lo, hi;
      if (m <= 0) {
        lo.x = lo.y = lo.z = T(1e15);
        lo.w = T(0);
        hi = lo;
      } else {
        lo = part[src_of(kGroup * h)];
        hi = lo;
        for (int r = 1; r < m; ++r) {
          const vec4_t<T> v = part[src_of(kGroup * h + r)];
          lo.x = min(lo.x, v.x);
          lo.y = min(lo.y, v.y);
          lo.z = min(lo.z, v.z);
          hi.x = max(hi.x, v.x);
          hi.y = max(hi.y, v.y);
          hi.z = max(hi.z, v.z);
        }
      }
      cbox[2 * (2 * (size_t)cbeg + h)] = lo;
      cbox[2 * (2 * (size_t)cbeg + h) + 1] = hi;
    }
    for (int c = t; c < ncl; c += kPrepThreads)
      cinfo[cbeg + c] = make_int4(beg + 8 * c, min(8, cnt - 8 * c), cell, 0);
    return;
  }
  if (sort && cnt > 1 && cnt <= kPrepSortMax) {
    int npow = 1;
    while (npow < cnt) npow <<= 1;
    for (int i = t; i < npow; i += kPrepThreads) {
      unsigned long long k = ~0ull;
      if (i < cnt) k = ((unsigned long long)morton(sorted[beg + i]) << 32) | (unsigned)perm[beg + i];
      key[i] = k;
    }
    __syncthreads();
    // bitonic sort of key[0 .. npow)
    for (int k = 2; k <= npow; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < npow; i += kPrepThreads) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const unsigned long long a = key[i], b = key[ixj];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              key[i] = b;
              key[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = t; i < cnt; i += kPrepThreads) {
      const int src = (int)(key[i] & 0xFFFFFFFFu);
      sorted[beg + i] = wrapped[src];
      perm[beg + i] = src;
    }
    __syncthreads();
  }
  // padded cluster slots (read back through sorted[]: each thread reads what
  // it or another thread of this workgroup wrote before the barrier above)
  for (int s = t; s < ncl * 8; s += kPrepThreads) {
    vec4_t<T> v;
    if (s < cnt) {
      v = sorted[beg + s];
    } else {  // padding: a zero charge far outside every cutoff
      v.x = v.y = v.z = T(1e15);
      v.w = T(0);
    }
    cpos[(size_t)cbeg * 8 + s] = v;
  }
  // boxes of the j-groups (an empty group: a point far outside every cutoff)
  for (int h = t; h < 2 * ncl; h += kPrepThreads) {
    const int m = min(kGroup, cnt - kGroup * h);
    vec4_t<T> lo, hi;
    if (m <= 0) {
      lo.x = lo.y = lo.z = T(1e15);
      lo.w = T(0);
      hi = lo;
    } else {
      lo = sorted[beg + kGroup * h];
      hi = lo;
      for (int r = 1; r < m; ++r) {
        const vec4_t<T> v = sorted[beg + kGroup * h + r];
        lo.x = min(lo.x, v.x);
        lo.y = min(lo.y, v.y);
        lo.z = min(lo.z, v.z);
        hi.x = max(hi.x, v.x);
        hi.y = max(hi.y, v.y);
        hi.z = max(hi.z, v.z);
      }
    }
    cbox[2 * (2 * (size_t)cbeg + h)] = lo;
    cbox[2 * (2 * (size_t)cbeg + h) + 1] = hi;
  }
  for (int c = t; c < ncl; c += kPrepThreads)
    cinfo[cbeg + c] = make_int4(beg + 8 * c, min(8, cnt - 8 * c), cell, 0);
}

// Sum over the 8 lanes of one i-member (jl and slot: lane bits 0, 1 and 5).
template <typename V>
__device__ inline V sum_i(V v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 32);
  return v;
}

// Member r of j-group h (a 32-bit byte offset from the array base, so the
// load takes the base from scalar registers).
template <typename T>
__device__ inline vec4_t<T> group_member(const vec4_t<T>* base, int h, int r) {
  const unsigned off = ((unsigned)h * kGroup + (unsigned)r) * (unsigned)sizeof(vec4_t<T>);
  return *reinterpret_cast<const vec4_t<T>*>(reinterpret_cast<const char*>(base) + off);
}

// Visits every j-group whose box (shifted image) lies within the cutoff of
// the i-cluster's box: per neighbour cell the surviving groups are listed in
// the wave's LDS list (padded to a multiple of kSlots with null_h, a group
// of far-away zero charges), and body(h, d, sx, sy, sz, self_h) runs once per
// step with h = this lane's entry and d = load(h), the lane's j data (loaded
// one step ahead, so the memory latency overlaps the previous step's
// arithmetic); self_h is the group index at which lane (il, jl) would meet
// its own particle (-1 if none in this cell).  flush() runs after each
// neighbour cell.  The i-box is wave-uniform.
template <typename T, typename Load, typename Body, typename Flush>
__device__ inline void for_each_group_block(const PairParams<T>& pp, const int* cl_start,
                                            const vec4_t<T>* cbox, int ic, int cell,
                                            const vec4_t<T>& blo, const vec4_t<T>& bhi,
                                            int* list, int null_h, Load&& load, Body&& body,
                                            Flush&& flush) {
  const int lane = threadIdx.x & 63;
  const int slot = lane >> 5, il = (lane >> 2) & 7, jl = lane & 3;
  // the group holding i-member il, where jl is il itself
  const int own_h = (jl == (il & 3)) ? 2 * ic + (il >> 2) : -1;
  const int cx = cell % pp.nc[0];
  const int cy = (cell / pp.nc[0]) % pp.nc[1];
  const int cz = cell / (pp.nc[0] * pp.nc[1]);
  for (int oz = -1; oz <= 1; ++oz) {
    int shz;
    const int nz = neighbour_shift(cz, oz, pp.nc[2], pp.per[2], shz);
    if (nz < 0) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      int shy;
      const int ny = neighbour_shift(cy, oy, pp.nc[1], pp.per[1], shy);
      if (ny < 0) continue;
      for (int ox = -1; ox <= 1; ++ox) {
        int shx;
        const int nx = neighbour_shift(cx, ox, pp.nc[0], pp.per[0], shx);
        if (nx < 0) continue;
        T sx, sy, sz;
        image_shift(pp, shx, shy, shz, sx, sy, sz);
        // i-box moved by minus the shift of the j image
        const T ilx = blo.x - sx, ily = blo.y - sy, ilz = blo.z - sz;
        const T ihx = bhi.x - sx, ihy = bhi.y - sy, ihz = bhi.z - sz;
        // whole-cell test with a margin for the rounding of the binning and
        // for charges that moved out of their cell under a Verlet skin (the
        // cells of a triclinic cell are not boxes: skipped there)
        if (!pp.tri) {
          const T mx = pp.cs[0] * T(1e-3) + pp.margin, my = pp.cs[1] * T(1e-3) + pp.margin,
                  mz = pp.cs[2] * T(1e-3) + pp.margin;
          const T g2 = box_gap2<T>((T)nx * pp.cs[0] - mx, (T)ny * pp.cs[1] - my,
                                   (T)nz * pp.cs[2] - mz, (T)(nx + 1) * pp.cs[0] + mx,
                                   (T)(ny + 1) * pp.cs[1] + my, (T)(nz + 1) * pp.cs[2] + mz,
                                   ilx, ily, ilz, ihx, ihy, ihz);
          if (!(g2 < pp.a2)) continue;
        }
        const int ncell = (nz * pp.nc[1] + ny) * pp.nc[0] + nx;
        const int jb0 = 2 * cl_start[ncell], jb1 = 2 * cl_start[ncell + 1];
        const int self_h = ((shx | shy | shz) == 0 && ncell == cell) ? own_h : -1;
        for (int jb = jb0; jb < jb1; jb += 64) {
          const int h = jb + lane;
          bool hit = false;
          if (h < jb1) {
            const vec4_t<T> lo = cbox[2 * (size_t)h], hi = cbox[2 * (size_t)h + 1];
            hit = box_gap2<T>(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, ilx, ily, ilz, ihx, ihy, ihz) <
                  pp.a2;
          }
          const unsigned long long mask = __ballot(hit);
          if (mask == 0) continue;
          const int cnt = __popcll(mask);
          const int pos = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
          if (hit) list[pos] = h;
          if (lane >= cnt && lane < cnt + (kSlots - cnt % kSlots) % kSlots) list[lane] = null_h;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          // two steps per trip, each loading the next step's data before its
          // own arithmetic (the null group stands in past the end)
          int ha = list[slot];
          auto da = load(ha);
          for (int it = 0; it < cnt; it += 2 * kSlots) {
            const int hb = it + kSlots < cnt ? list[it + kSlots + slot] : null_h;
            const auto db = load(hb);
            body(ha, da, sx, sy, sz, self_h);
            if (it + kSlots >= cnt) break;
            ha = it + 2 * kSlots < cnt ? list[it + 2 * kSlots + slot] : null_h;
            da = load(ha);
            body(hb, db, sx, sy, sz, self_h);
          }
          // every lane's reads are issued before the next chunk's writes
          __builtin_amdgcn_wave_barrier();
        }
        flush();
      }
    }
  }
}

// Position and force cotangent of one j particle (pair VJP).
template <typename T>
struct JData {
  vec4_t<T> p, v;
};

// Visits every j particle within the cutoff of the i-cluster's box, over the
// 27 neighbour cells with their image shifts: per cell, the j-groups whose
// box lies within a of the i-box, then their members whose own distance to
// the i-box is below a.  Survivors go, moved into the i-cluster's frame
// (position + shift, charge), to the wave's LDS ring; step(head) runs on
// ring entries [head, head + 8) whenever eight are waiting, and once more at
// the end on the remainder (the rest of that step reads a far-away zero
// charge).  flush() runs after each neighbour cell.
template <typename T, typename Step, typename Flush>
__device__ inline void for_each_j_culled(const PairParams<T>& pp, const int* cl_start,
                                         const vec4_t<T>* cpos, const vec4_t<T>* cbox, int cell,
                                         const vec4_t<T>& blo, const vec4_t<T>& bhi,
                                         vec4_t<T>* ring, int* gl, const vec4_t<T>& far,
                                         Step&& step, Flush&& flush) {
  const int lane = threadIdx.x & 63, jj = lane & (kStepJ - 1);
  const int cx = cell % pp.nc[0];
  const int cy = (cell / pp.nc[0]) % pp.nc[1];
  const int cz = cell / (pp.nc[0] * pp.nc[1]);
  int head = 0, tail = 0;
  for (int oz = -1; oz <= 1; ++oz) {
    int shz;
    const int nz = neighbour_shift(cz, oz, pp.nc[2], pp.per[2], shz);
    if (nz < 0) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      int shy;
      const int ny = neighbour_shift(cy, oy, pp.nc[1], pp.per[1], shy);
      if (ny < 0) continue;
      for (int ox = -1; ox <= 1; ++ox) {
        int shx;
        const int nx = neighbour_shift(cx, ox, pp.nc[0], pp.per[0], shx);
        if (nx < 0) continue;
        T sx, sy, sz;
        image_shift(pp, shx, shy, shz, sx, sy, sz);
        // i-box moved by minus the shift of the j image
        const T ilx = blo.x - sx, ily = blo.y - sy, ilz = blo.z - sz;
        const T ihx = bhi.x - sx, ihy = bhi.y - sy, ihz = bhi.z - sz;
        if (!pp.tri) {  // whole-cell test, margins as in for_each_group_block
          const T mx = pp.cs[0] * T(1e-3) + pp.margin, my = pp.cs[1] * T(1e-3) + pp.margin,
                  mz = pp.cs[2] * T(1e-3) + pp.margin;
          const T g2 = box_gap2<T>((T)nx * pp.cs[0] - mx, (T)ny * pp.cs[1] - my,
                                   (T)nz * pp.cs[2] - mz, (T)(nx + 1) * pp.cs[0] + mx,
                                   (T)(ny + 1) * pp.cs[1] + my, (T)(nz + 1) * pp.cs[2] + mz,
                                   ilx, ily, ilz, ihx, ihy, ihz);
          if (!(g2 < pp.a2)) continue;
        }
        const int ncell = (nz * pp.nc[1] + ny) * pp.nc[0] + nx;
        const int jb0 = 2 * cl_start[ncell], jb1 = 2 * cl_start[ncell + 1];
        for (int jb = jb0; jb < jb1; jb += 64) {
          const int h = jb + lane;
          bool hit = false;
          if (h < jb1) {
            const vec4_t<T> lo = cbox[2 * (size_t)h], hi = cbox[2 * (size_t)h + 1];
            hit = box_gap2<T>(lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, ilx, ily, ilz, ihx, ihy, ihz) <
                  pp.a2;
          }
          const unsigned long long mask = __ballot(hit);
          if (mask == 0) continue;
          const int ng = __popcll(mask);
          const int pos = (int)__builtin_amdgcn_mbcnt_hi(
              (unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
          if (hit) gl[pos] = h;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          for (int e0 = 0; e0 < ng; e0 += 64 / kGroup) {
            const int e = e0 + lane / kGroup;
            bool hit2 = false;
            vec4_t<T> pj;
            if (e < ng) {
              pj = group_member<T>(cpos, gl[e], lane & (kGroup - 1));
              const T gx = max(T(0), max(ilx - pj.x, pj.x - ihx));
              const T gy = max(T(0), max(ily - pj.y, pj.y - ihy));
              const T gz = max(T(0), max(ilz - pj.z, pj.z - ihz));
              hit2 = gx * gx + gy * gy + gz * gz < pp.a2;
            }
            const unsigned long long m2 = __ballot(hit2);
            const int pos2 = (int)__builtin_amdgcn_mbcnt_hi(
                (unsigned)(m2 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m2, 0u));
            if (hit2) {
              pj.x += sx;
              pj.y += sy;
              pj.z += sz;
              ring[(tail + pos2) & (kRing - 1)] = pj;
            }
            tail += __popcll(m2);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // the waiting full steps, two per trip, each one's ring read issued
            // a step ahead.  head is a multiple of kStepJ here, so a step's
            // eight entries never wrap: lane jj reads ring[(head mod kRing) +
            // jj], a per-lane base plus a wave-uniform offset.  The read ahead
            // past the last step lands on an old slot of the ring and is unused.
            const int nst = (tail - head) / kStepJ;
            if (nst > 0) {
              const vec4_t<T>* rl = ring + jj;
              vec4_t<T> a = rl[head & (kRing - 1)];
              int st = 0;
              for (; st + 2 <= nst; st += 2) {
                const vec4_t<T> b = rl[(head + kStepJ) & (kRing - 1)];
                step(a);
                a = rl[(head + 2 * kStepJ) & (kRing - 1)];
                step(b);
                head += 2 * kStepJ;
              }
              if (st < nst) {
                step(a);
                head += kStepJ;
              }
            }
            __builtin_amdgcn_wave_barrier();
          }
        }
        flush();
      }
    }
  }
  if (tail > head) step(jj < tail - head ? ring[(head + jj) & (kRing - 1)] : far);
}

// U^0 per particle (eq. U_zero) over the culled j particles: lane (il, jj)
// = (lane / 8, lane % 8) evaluates i-member il against ring entry head + jj
// of each step.
// The self pair (the same particle, shift 0) is the only pair at distance
// exactly zero and is left out by r^2 > 0.
// r^-nu and nu r^-(nu+2) from 1/r (nu = 1: Coulomb, 6: dispersion)
template <int NU, typename T>
__device__ inline void power_terms(T rinv, T& k, T& f) {
  const T rinv2 = rinv * rinv;
  if constexpr (NU == 1) {
    k = rinv;
    f = rinv * rinv2;
  } else {
    const T r6 = rinv2 * rinv2 * rinv2;
    k = r6;
    f = T(NU) * r6 * rinv2;
  }
}

template <typename T, int P, int NU>
__global__ void __launch_bounds__(kClusterThreads)
    k_pair_pc(const int* __restrict__ cl_start, const vec4_t<T>* __restrict__ cpos,
              const vec4_t<T>* __restrict__ cbox, const int4* __restrict__ cinfo,
              PairParams<T> pp, double* __restrict__ phi0, T* __restrict__ F0) {
  __shared__ vec4_t<T> rings[kClusterThreads / 64][kRing];
  __shared__ int glists[kClusterThreads / 64][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ic = __builtin_amdgcn_readfirstlane(blockIdx.x * (kClusterThreads / 64) + wv);
  if (ic >= cl_start[pp.ncell]) return;
  const int il = lane >> 3, jj = lane & 7;
  const int4 inf = cinfo[ic];
  const vec4_t<T> pi = cpos[(size_t)ic * 8 + il];
  vec4_t<T> blo, bhi;
  cluster_box<T>(cbox, ic, inf.y, blo, bhi);
  const T e_top = in_vgpr(pp.er[P - 1]), f_top = in_vgpr(pp.fr[P - 2]);
  const T a2v = in_vgpr(pp.a2);
  vec4_t<T>* ring = rings[wv];
  vec4_t<T> far;
  far.x = far.y = far.z = T(1e15);
  far.w = T(0);
  double ph = 0.0;  // the potential is carried in FP64 up to the energy sum
  T phc = T(0);     // ... after a partial sum over one neighbour cell
  T fx = T(0), fy = T(0), fz = T(0);
  for_each_j_culled<T>(
      pp, cl_start, cpos, cbox, inf.z, blo, bhi, ring, glists[wv], far,
      [&](const vec4_t<T>& pj) {
        const T dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        const bool ok = r2 < pp.a2 && r2 > T(0);
        const T r2c = ok ? r2 : a2v;
        const T qj = ok ? pj.w : T(0);
        const T rinv = rsqrt_t(r2c);
        T pe = e_top, pf = f_top;
#pragma unroll
        for (int k = P - 2; k >= 0; --k) pe = pe * r2c + pp.er[k];
#pragma unroll
        for (int k = P - 3; k >= 0; --k) pf = pf * r2c + pp.fr[k];
        T kr, fr;
        power_terms<NU>(rinv, kr, fr);
        const T fs = qj * (fr + pf);
        phc += qj * (kr - pe);
        fx += fs * dx;
        fy += fs * dy;
        fz += fs * dz;
      },
      [&]() {
        ph += (double)phc;
        phc = T(0);
      });
  ph += (double)phc;
#pragma unroll
  for (int d = 1; d < 8; d <<= 1) {
    ph += __shfl_xor(ph, d);
    fx += __shfl_xor(fx, d);
    fy += __shfl_xor(fy, d);
    fz += __shfl_xor(fz, d);
  }
  if (jj == 0 && il < inf.y) {
    const int i = inf.x + il;
    phi0[i] = ph;
    F0[3 * (size_t)i] = pi.w * fx;
    F0[3 * (size_t)i + 1] = pi.w * fy;
    F0[3 * (size_t)i + 2] = pi.w * fz;
  }
}

// Virial of the short-range part, sum_i q_i sum_j q_j f(r) d d^T over every
// pair within a (both orders; f = -k0'(r)/r, d = r_i - r_j of the image),
// for the cell derivative: the same culled walk as k_pair_pc, six sums per
// lane, reduced over the wave and added to acc[0..5] (xx, yy, zz, xy, xz, yz)
// in FP64.  NU: the kernel r^-NU.
template <typename T, int P, int NU>
__global__ void __launch_bounds__(kClusterThreads)
    k_pair_virial(const int* __restrict__ cl_start, const vec4_t<T>* __restrict__ cpos,
                  const vec4_t<T>* __restrict__ cbox, const int4* __restrict__ cinfo,
                  PairParams<T> pp, double* __restrict__ acc) {
  __shared__ vec4_t<T> rings[kClusterThreads / 64][kRing];
  __shared__ int glists[kClusterThreads / 64][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ic = __builtin_amdgcn_readfirstlane(blockIdx.x * (kClusterThreads / 64) + wv);
  if (ic >= cl_start[pp.ncell]) return;
  const int il = lane >> 3;
  const int4 inf = cinfo[ic];
  const vec4_t<T> pi = cpos[(size_t)ic * 8 + il];
  vec4_t<T> blo, bhi;
  cluster_box<T>(cbox, ic, inf.y, blo, bhi);
  const T f_top = in_vgpr(pp.fr[P - 2]);
  const T a2v = in_vgpr(pp.a2);
  vec4_t<T> far;
  far.x = far.y = far.z = T(1e15);
  far.w = T(0);
  double v[6] = {0, 0, 0, 0, 0, 0};
  T vc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};  // one neighbour cell's part
  for_each_j_culled<T>(
      pp, cl_start, cpos, cbox, inf.z, blo, bhi, rings[wv], glists[wv], far,
      [&](const vec4_t<T>& pj) {
        const T dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        const bool ok = r2 < pp.a2 && r2 > T(0);
        const T r2c = ok ? r2 : a2v;
        const T qj = ok ? pj.w : T(0);
        const T rinv = rsqrt_t(r2c);
        T pf = f_top;
#pragma unroll
        for (int k = P - 3; k >= 0; --k) pf = pf * r2c + pp.fr[k];
        T kr, fr;
        power_terms<NU>(rinv, kr, fr);
        const T fs = qj * (fr + pf);
        vc[0] += fs * dx * dx;
        vc[1] += fs * dy * dy;
        vc[2] += fs * dz * dz;
        vc[3] += fs * dx * dy;
        vc[4] += fs * dx * dz;
        vc[5] += fs * dy * dz;
      },
      [&]() {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] += (double)vc[k];
          vc[k] = T(0);
        }
      });
  const double qi = (double)pi.w;  // zero in padding slots
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double t = (v[k] + (double)vc[k]) * qi;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) atomicAdd(&acc[k], t);
  }
}

// Cotangents in cluster-slot order (zero in padding slots): the force
// cotangent in x, y, z, the cotangent of phi in w (each zero without one).
template <typename T>
__global__ void k_gather_v_cl(int nslot_max, const int* __restrict__ cl_start, int ncell,
                              const int4* __restrict__ cinfo, const int* __restrict__ perm,
                              const T* __restrict__ gF, const T* __restrict__ gphi,
                              vec4_t<T>* __restrict__ cv) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslot_max || s >= 8 * cl_start[ncell]) return;
  const int4 inf = cinfo[s >> 3];
  const int r = s & 7;
  vec4_t<T> v;
  v.x = v.y = v.z = v.w = T(0);
  if (r < inf.y) {
    const int u = perm[inf.x + r];
    if (gF) {
      v.x = gF[3 * (size_t)u];
      v.y = gF[3 * (size_t)u + 1];
      v.z = gF[3 * (size_t)u + 2];
    }
    if (gphi) v.w = gphi[u];
  }
  cv[s] = v;
}

// VJP of the short-range part for a force cotangent v (eq. U_zero):
//   d/dq_i  sum_k v_k . F0_k   = sum_j q_j f(r) (v_i - v_j) . d_ij
//   d/dr_i  sum_k v_k . F0_k   = q_i sum_j q_j [f (v_i - v_j) + (f'/r) ((v_i - v_j) . d) d]
// with f = 1/r^3 + 2 P'(t)/a^3 and f'/r = -3/r^5 + 4 P''(t)/a^5; and, with
// W, for a cotangent w of the short-range potential phi0:
//   d/dq_i  sum_k w_k phi0_k   = sum_j w_j k0(r)
//   d/dr_i  sum_k w_k phi0_k   = -q_i sum_j w_j f d_ij - w_i sum_j q_j f d_ij.
template <typename T, int P, bool W, int NU>
__global__ void __launch_bounds__(kClusterThreads)
    k_pair_vjp_cl(const int* __restrict__ cl_start, const vec4_t<T>* __restrict__ cpos,
                  const vec4_t<T>* __restrict__ cv, const vec4_t<T>* __restrict__ cbox,
                  const int4* __restrict__ cinfo, PairParams<T> pp, int null_h,
                  T* __restrict__ gq, T* __restrict__ gr) {
  __shared__ int lists[kClusterThreads / 64][64];
  const int lane = threadIdx.x & 63;
  const int ic = __builtin_amdgcn_readfirstlane(blockIdx.x * (kClusterThreads / 64) +
                                                (int)(threadIdx.x >> 6));
  if (ic >= cl_start[pp.ncell]) return;
  const int il = (lane >> 2) & 7, jl = lane & 3;
  const int4 inf = cinfo[ic];
  const vec4_t<T> pi = cpos[(size_t)ic * 8 + il];
  const vec4_t<T> vi = cv[(size_t)ic * 8 + il];
  vec4_t<T> blo, bhi;
  cluster_box<T>(cbox, ic, inf.y, blo, bhi);
  const T f_top = in_vgpr(pp.fr[P - 2]), g_top = in_vgpr(pp.gr[P - 3]);
  const T e_top = in_vgpr(pp.er[P - 1]);
  const T a2v = in_vgpr(pp.a2);
  T sq = T(0), rx = T(0), ry = T(0), rz = T(0);
  T bx = T(0), by = T(0), bz = T(0);  // sum_j q_j f d_ij (W only)
  for_each_group_block<T>(
      pp, cl_start, cbox, ic, inf.z, blo, bhi, lists[threadIdx.x >> 6], null_h,
      [&](int h) { return JData<T>{group_member<T>(cpos, h, jl), group_member<T>(cv, h, jl)}; },
      [&](int h, const JData<T>& jd, T sx, T sy, T sz, int self_h) {
        const vec4_t<T>& pj = jd.p;
        const vec4_t<T>& vj = jd.v;
        const T dx = (pi.x - sx) - pj.x, dy = (pi.y - sy) - pj.y, dz = (pi.z - sz) - pj.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        const bool ok = r2 < pp.a2 && h != self_h;
        const T r2c = ok ? r2 : a2v;
        const T qj = ok ? pj.w : T(0);
        const T rinv = rsqrt_t(r2c);
        const T rinv2 = rinv * rinv;
        T pf = f_top, pg = g_top;
#pragma unroll
        for (int k = P - 3; k >= 0; --k) pf = pf * r2c + pp.fr[k];
#pragma unroll
        for (int k = P - 4; k >= 0; --k) pg = pg * r2c + pp.gr[k];
        // f = nu r^-(nu+2) + pf, f'/r = -nu (nu+2) r^-(nu+4) + pg
        T kr, fr;
        power_terms<NU>(rinv, kr, fr);
        const T f = fr + pf;
        const T fpr = T(-(NU + 2)) * fr * rinv2 + pg;
        const T wx = vi.x - vj.x, wy = vi.y - vj.y, wz = vi.z - vj.z;
        const T wd = wx * dx + wy * dy + wz * dz;
        const T qf = qj * f;
        const T c2 = qj * fpr * wd;
        sq += qf * wd;
        rx += qf * wx + c2 * dx;
        ry += qf * wy + c2 * dy;
        rz += qf * wz + c2 * dz;
        if constexpr (W) {
          const T wj = ok ? vj.w : T(0);
          T pe = e_top;
#pragma unroll
          for (int k = P - 2; k >= 0; --k) pe = pe * r2c + pp.er[k];
          sq += wj * (kr - pe);
          const T wf = wj * f;
          rx -= wf * dx;
          ry -= wf * dy;
          rz -= wf * dz;
          bx += qf * dx;
          by += qf * dy;
          bz += qf * dz;
        }
      },
      []() {});
  sq = sum_i(sq);
  rx = sum_i(rx);
  ry = sum_i(ry);
  rz = sum_i(rz);
  if constexpr (W) {
    bx = sum_i(bx);
    by = sum_i(by);
    bz = sum_i(bz);
  }
  if ((lane & ~0x1C) == 0 && il < inf.y) {  // slot 0, jl 0
    const int i = inf.x + il;
    gq[i] = sq;
    gr[3 * (size_t)i] = pi.w * rx - vi.w * bx;
    gr[3 * (size_t)i + 1] = pi.w * ry - vi.w * by;
    gr[3 * (size_t)i + 2] = pi.w * rz - vi.w * bz;
  }
}

// Verlet skin, a call without rebuild: the cluster slots and j-group boxes
// of the kept layout from the refreshed cell-ordered list (one thread per
// j-group; padding slots and empty groups keep their far-away values).
template <typename T>
__global__ void k_cluster_refresh(int ngroup_max, const int* __restrict__ cl_start, int ncell,
                                  const int4* __restrict__ cinfo,
                                  const vec4_t<T>* __restrict__ sorted,
                                  vec4_t<T>* __restrict__ cpos, vec4_t<T>* __restrict__ cbox,
                                  const int* __restrict__ gate) {
  if (gate[kSkinRebuild]) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= ngroup_max || h >= 2 * cl_start[ncell]) return;
  const int4 inf = cinfo[h >> 1];
  const int r0 = (h & 1) * kGroup, m = min(kGroup, inf.y - r0);
  if (m <= 0) return;
  vec4_t<T> lo = sorted[inf.x + r0], hi = lo;
  cpos[(size_t)kGroup * h] = lo;
  for (int r = 1; r < m; ++r) {
    const vec4_t<T> v = sorted[inf.x + r0 + r];
    cpos[(size_t)kGroup * h + r] = v;
    lo.x = min(lo.x, v.x);
    lo.y = min(lo.y, v.y);
    lo.z = min(lo.z, v.z);
    hi.x = max(hi.x, v.x);
    hi.y = max(hi.y, v.y);
    hi.z = max(hi.z, v.z);
  }
  cbox[2 * (size_t)h] = lo;
  cbox[2 * (size_t)h + 1] = hi;
}

int cluster_capacity(int n, int ncell) { return n / 8 + ncell + 1; }

template <typename T>
void launch_cluster_layout(int sort, int scan, int ncell, const int* start, int* cl_start,
                           const BinParams<T>& bp, const vec4_t<T>* wrapped, vec4_t<T>* sorted,
                           int* perm, vec4_t<T>* cpos, vec4_t<T>* cbox, int4* cinfo,
                           int* counts, const int* skin, int n, hipStream_t s) {
  if (ncell <= 0) return;
  if (scan) hipLaunchKernelGGL(k_cluster_scan, dim3(1), dim3(1024), 0, s, ncell, start, cl_start);
  hipLaunchKernelGGL(k_cluster_prep<T>, dim3(ncell), dim3(kPrepThreads), 0, s, sort, start,
                     cl_start, bp, wrapped, sorted, perm, cpos, cbox, cinfo, counts, skin);
  if (skin && n > 0) {
    const int ng = 2 * cluster_capacity(n, ncell);
    hipLaunchKernelGGL(k_cluster_refresh<T>, dim3((ng + 255) / 256), dim3(256), 0, s, ng,
                       cl_start, ncell, cinfo, sorted, cpos, cbox, skin);
  }
}

template <typename T>
void launch_pair_cl(int p, int n, int ncell, const int* cl_start, const vec4_t<T>* cpos,
                    const vec4_t<T>* cbox, const int4* cinfo, const PairParams<T>& pp,
                    double* phi0, T* F0, hipStream_t s) {
  if (n <= 0) return;
  const int ncl = cluster_capacity(n, ncell);
  const dim3 grid((ncl + 3) / 4), block(kClusterThreads);
  if (pp.nu == 6) {
    switch (p) {
      case 4: hipLaunchKernelGGL((k_pair_pc<T, 4, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
      case 6: hipLaunchKernelGGL((k_pair_pc<T, 6, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
      case 8: hipLaunchKernelGGL((k_pair_pc<T, 8, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
    }
    return;
  }
  switch (p) {
    case 4: hipLaunchKernelGGL((k_pair_pc<T, 4, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
    case 6: hipLaunchKernelGGL((k_pair_pc<T, 6, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
    case 8: hipLaunchKernelGGL((k_pair_pc<T, 8, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, phi0, F0); break;
  }
}

template <typename T, bool W, int NU>
void launch_pair_vjp_p(int p, dim3 grid, const int* cl_start, const vec4_t<T>* cpos,
                       const vec4_t<T>* cv, const vec4_t<T>* cbox, const int4* cinfo,
                       const PairParams<T>& pp, int nh, T* gq, T* gr, hipStream_t s) {
  const dim3 block(kClusterThreads);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_pair_vjp_cl<T, 4, W, NU>), grid, block, 0, s, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr); break;
    case 6: hipLaunchKernelGGL((k_pair_vjp_cl<T, 6, W, NU>), grid, block, 0, s, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr); break;
    case 8: hipLaunchKernelGGL((k_pair_vjp_cl<T, 8, W, NU>), grid, block, 0, s, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr); break;
  }
}

template <typename T>
void launch_pair_vjp_cl(int p, int n, int ncell, const int* cl_start, const int4* cinfo,
                        const int* perm, const T* gF, const T* gphi, const vec4_t<T>* cpos,
                        vec4_t<T>* cv, const vec4_t<T>* cbox, const PairParams<T>& pp, int nh,
                        T* gq, T* gr, hipStream_t s) {
  if (n <= 0) return;
  const int ncl = cluster_capacity(n, ncell);
  hipLaunchKernelGGL(k_gather_v_cl<T>, dim3((8 * ncl + 255) / 256), dim3(256), 0, s, 8 * ncl,
                     cl_start, ncell, cinfo, perm, gF, gphi, cv);
  const dim3 grid((ncl + 3) / 4);
  if (pp.nu == 6) {
    if (gphi)
      launch_pair_vjp_p<T, true, 6>(p, grid, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr, s);
    else
      launch_pair_vjp_p<T, false, 6>(p, grid, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr, s);
  } else if (gphi) {
    launch_pair_vjp_p<T, true, 1>(p, grid, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr, s);
  } else {
    launch_pair_vjp_p<T, false, 1>(p, grid, cl_start, cpos, cv, cbox, cinfo, pp, nh, gq, gr, s);
  }
}

template <typename T>
void launch_pair_virial(int p, int n, int ncell, const int* cl_start, const vec4_t<T>* cpos,
                        const vec4_t<T>* cbox, const int4* cinfo, const PairParams<T>& pp,
                        double* acc, hipStream_t s) {
  if (n <= 0) return;
  const int ncl = cluster_capacity(n, ncell);
  const dim3 grid((ncl + 3) / 4), block(kClusterThreads);
  if (pp.nu == 6) {
    switch (p) {
      case 4: hipLaunchKernelGGL((k_pair_virial<T, 4, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
      case 6: hipLaunchKernelGGL((k_pair_virial<T, 6, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
      case 8: hipLaunchKernelGGL((k_pair_virial<T, 8, 6>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
    }
    return;
  }
  switch (p) {
    case 4: hipLaunchKernelGGL((k_pair_virial<T, 4, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
    case 6: hipLaunchKernelGGL((k_pair_virial<T, 6, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
    case 8: hipLaunchKernelGGL((k_pair_virial<T, 8, 1>), grid, block, 0, s, cl_start, cpos, cbox, cinfo, pp, acc); break;
  }
}

#define MSM_INST_CLUSTER(T)                                                                    \
  template void launch_cluster_layout<T>(int, int, int, const int*, int*, const BinParams<T>&, \
                                         const vec4_t<T>*, vec4_t<T>*, int*, vec4_t<T>*,       \
                                         vec4_t<T>*, int4*, int*, const int*, int, hipStream_t); \
  template void launch_pair_virial<T>(int, int, int, const int*, const vec4_t<T>*,             \
                                      const vec4_t<T>*, const int4*, const PairParams<T>&,     \
                                      double*, hipStream_t);                                   \
  template void launch_pair_cl<T>(int, int, int, const int*, const vec4_t<T>*,                 \
                                  const vec4_t<T>*, const int4*, const PairParams<T>&,         \
                                  double*, T*, hipStream_t);                                   \
  template void launch_pair_vjp_cl<T>(int, int, int, const int*, const int4*, const int*,      \
                                      const T*, const T*, const vec4_t<T>*, vec4_t<T>*,        \
                                      const vec4_t<T>*, const PairParams<T>&, int, T*, T*,     \
                                      hipStream_t);
MSM_INST_CLUSTER(float)
MSM_INST_CLUSTER(double)

}  // namespace msm
