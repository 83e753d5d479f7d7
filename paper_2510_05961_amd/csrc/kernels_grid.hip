// kernels_grid.hip -- grid-side kernels of the MSM: restriction, prolongation
// and the per-level stencil convolution (also used for the dense top level).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "conv_tile.hpp"
#include "kernels.hpp"

namespace msm {

template <typename T>
struct JTaps {
  T J[9];  // J_{-p/2..p/2}
};

__device__ inline int floor_div2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

// Prolongation tap t of a fine point m whose first coarse point is
// nl = ceil((m - P/2)/2): J_{m - 2(nl + t)}.  With e = (m - P/2) mod 2 that is
// entry P - e - 2t of the table (zero when negative), so the unrolled t and
// the parity select the tap without a run-time index into the by-value table
// (which would put the table in memory and add a load per tap).
template <typename T, int P>
__device__ inline T prolong_tap(const JTaps<T>& jt, int e, int t) {
  const T even = jt.J[P - 2 * t];
  const T odd = (P - 1 - 2 * t >= 0) ? jt.J[max(P - 1 - 2 * t, 0)] : T(0);
  return e ? odd : even;
}

// ---------------------------------------------------------------------------
// a4: restriction (eq. restriction_prolongation_explicit_formulas, first line)
//   q~^{l+1}_m = sum_n J_{n-2m} q~^l_n,  J_n = J_nx J_ny J_nz, p+1 taps per axis;
// a7: prolongation, its transpose (the paper's corrected form)
//   e^l_m += sum_n J_{m-2n} e^{l+1}_n, at most p/2+1 coarse points per axis.
// A workgroup stages the fine (restriction) or coarse (prolongation) window
// of a block in LDS (periodic wrap; zeros outside a free axis) and applies
// the 1-D taps axis by axis: x, then y, then z.
// ---------------------------------------------------------------------------
constexpr int kRestrictB = 4;  // coarse points per axis per workgroup
constexpr int kProlongB = 8;   // fine points per axis per workgroup

template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_restrict_tiled(GridDev<T> f, GridDev<T> c, JTaps<T> jt, const T* __restrict__ qf,
                     T* __restrict__ qc) {
  constexpr int B = kRestrictB, W = 2 * B + P - 1;
  __shared__ T F[W * W * W];
  __shared__ T X1[W * W * B];
  __shared__ T X2[W * B * B];
  const int nbx = (c.n[0] + B - 1) / B, nby = (c.n[1] + B - 1) / B;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
  const int c0[3] = {bx * B, by * B, bz * B};
  // absolute fine index of window element 0 per axis
  int f0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) f0[k] = 2 * (c0[k] + c.lo[k]) - P / 2;
  for (int i = threadIdx.x; i < W * W * W; i += blockDim.x) {
    const int x = i % W, y = (i / W) % W, z = i / (W * W);
    const int ix = axis_index(f0[0] + x, f.n[0], f.lo[0], f.per[0]);
    const int iy = axis_index(f0[1] + y, f.n[1], f.lo[1], f.per[1]);
    const int iz = axis_index(f0[2] + z, f.n[2], f.lo[2], f.per[2]);
    F[i] = (ix < 0 || iy < 0 || iz < 0) ? T(0)
                                          : qf[((long long)iz * f.n[1] + iy) * f.n[0] + ix];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * W * B; i += blockDim.x) {
    const int x = i % B, yz = i / B;
    const T* row = F + yz * W + 2 * x;
    T sx = T(0);
#pragma unroll
    for (int t = 0; t <= P; ++t) sx += jt.J[t] * row[t];
    X1[i] = sx;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * B * B; i += blockDim.x) {
    const int x = i % B, y = (i / B) % B, z = i / (B * B);
    T sy = T(0);
#pragma unroll
    for (int t = 0; t <= P; ++t) sy += jt.J[t] * X1[(z * W + 2 * y + t) * B + x];
    X2[i] = sy;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < B * B * B; i += blockDim.x) {
    const int x = i % B, y = (i / B) % B, z = i / (B * B);
    const int gx = c0[0] + x, gy = c0[1] + y, gz = c0[2] + z;
    if (gx >= c.n[0] || gy >= c.n[1] || gz >= c.n[2]) continue;
    T s = T(0);
#pragma unroll
    for (int t = 0; t <= P; ++t) s += jt.J[t] * X2[((2 * z + t) * B + y) * B + x];
    qc[((long long)gz * c.n[1] + gy) * c.n[0] + gx] = s;
  }
}

// The coarse grid comes from ecT (grid precision) or ec64 (FP64); with ef64
// the fine result is (T) ef64 + prolongation (the level's own FP64
// convolution output, cast here), else ef += prolongation.
template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_prolong_tiled(GridDev<T> f, GridDev<T> c, JTaps<T> jt, const T* __restrict__ ecT,
                    const double* __restrict__ ec64, T* __restrict__ ef,
                    const double* __restrict__ ef64) {
  constexpr int B = kProlongB, W = B / 2 + P / 2 + 2;  // coarse window per axis
  __shared__ T C[W * W * W];
  __shared__ T X1[W * W * B];
  __shared__ T X2[W * B * B];
  const int nbx = (f.n[0] + B - 1) / B, nby = (f.n[1] + B - 1) / B;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
  const int fb[3] = {bx * B, by * B, bz * B};
  // absolute coarse index of window element 0 per axis: ceil((m0 - P/2)/2)
  int n0[3], m0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m0[k] = fb[k] + f.lo[k];
    n0[k] = -floor_div2(-(m0[k] - P / 2));
  }
  for (int i = threadIdx.x; i < W * W * W; i += blockDim.x) {
    const int x = i % W, y = (i / W) % W, z = i / (W * W);
    const int ix = axis_index(n0[0] + x, c.n[0], c.lo[0], c.per[0]);
    const int iy = axis_index(n0[1] + y, c.n[1], c.lo[1], c.per[1]);
    const int iz = axis_index(n0[2] + z, c.n[2], c.lo[2], c.per[2]);
    const long long ci = ((long long)iz * c.n[1] + iy) * c.n[0] + ix;
    C[i] = (ix < 0 || iy < 0 || iz < 0) ? T(0) : (ec64 ? (T)ec64[ci] : ecT[ci]);
  }
  __syncthreads();
  // fine point m (absolute) takes coarse n with |m - 2n| <= P/2, in order
  // of increasing n starting at ceil((m - P/2)/2); window offset of that n:
  // ceil((m - P/2)/2) - n0
  for (int i = threadIdx.x; i < W * W * B; i += blockDim.x) {
    const int x = i % B, yz = i / B;
    const int m = m0[0] + x;
    const int nl = -floor_div2(-(m - P / 2)), e = (m - P / 2) & 1;
    T sx = T(0);
#pragma unroll
    for (int t = 0; t < P / 2 + 1; ++t)
      sx += prolong_tap<T, P>(jt, e, t) * C[yz * W + (nl + t - n0[0])];
    X1[i] = sx;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * B * B; i += blockDim.x) {
    const int x = i % B, y = (i / B) % B, z = i / (B * B);
    const int m = m0[1] + y;
    const int nl = -floor_div2(-(m - P / 2)), e = (m - P / 2) & 1;
    T sy = T(0);
#pragma unroll
    for (int t = 0; t < P / 2 + 1; ++t)
      sy += prolong_tap<T, P>(jt, e, t) * X1[(z * W + (nl + t - n0[1])) * B + x];
    X2[i] = sy;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < B * B * B; i += blockDim.x) {
    const int x = i % B, y = (i / B) % B, z = i / (B * B);
    const int gx = fb[0] + x, gy = fb[1] + y, gz = fb[2] + z;
    if (gx >= f.n[0] || gy >= f.n[1] || gz >= f.n[2]) continue;
    const int m = m0[2] + z;
    const int nl = -floor_div2(-(m - P / 2)), e = (m - P / 2) & 1;
    T s = T(0);
#pragma unroll
    for (int t = 0; t < P / 2 + 1; ++t)
      s += prolong_tap<T, P>(jt, e, t) * X2[((nl + t - n0[2]) * B + y) * B + x];
    const long long fi = ((long long)gz * f.n[1] + gy) * f.n[0] + gx;
    if (ef64) ef[fi] = (T)ef64[fi] + s;
    else ef[fi] += s;
  }
}

// ---------------------------------------------------------------------------
// a5 / a6: stencil convolution e_o = sum_d K_d q_{o+shift-d} (eq.
// action_of_K_as_convolution).  A workgroup owns a (TXT R) x (TYT Q) tile of
// output points of one z-plane and a contiguous range of stencil z-planes
// (split across workgroups, FP64 atomics, when a launch needs more waves).
// For each stencil plane it stages the input window (periodic wrap or zero
// padding) through LDS, one wave per window row, and adds the plane with
// conv_plane (conv_tile.hpp): R x Q outputs per thread in registers, taps in
// chunks over padded stencil rows, workgroup-uniform coefficients.  With
// WS > 1 the workgroup holds WS copies of the TXT x TYT thread tile; copy w
// walks window rows w, w + WS, ... of every plane and the copies' sums meet
// in LDS at the end (more waves per output tile on small grids).  TI is the
// grid type (what LDS holds), TA the stencil / accumulation / output type.
// ---------------------------------------------------------------------------
template <typename TI, typename TA, int R, int Q, int TXT, int TYT, int WS>
__global__ void __launch_bounds__(TXT * TYT * WS)
    k_conv(ConvParams cp, const TA* __restrict__ K, const int2* __restrict__ rowext,
           const TI* __restrict__ q, TA* __restrict__ e) {
  constexpr int CH = kConvCH;
  constexpr int NTILE = TXT * TYT, NT = NTILE * WS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TI* lds = reinterpret_cast<TI*>(smem_raw);
  // ws (wave-uniform) selects the copy; a constant 0 without the split
  const int tt = WS > 1 ? (int)threadIdx.x % NTILE : (int)threadIdx.x;
  const int ws = WS > 1 ? (int)threadIdx.x / NTILE : 0;
  const int tx = tt % TXT, ty = tt / TXT;
  const int n0 = cp.n[0], n1 = cp.n[1], n2 = cp.n[2];
  const int o0 = cp.nout[0], o1 = cp.nout[1], o2 = cp.nout[2];
  const int lx = cp.len[0], ly = cp.len[1], lxp = cp.lxp;
  const int bx = blockIdx.x, by = blockIdx.y;
  const int z = blockIdx.z % o2, split = blockIdx.z / o2;
  const int x0 = bx * (TXT * R), y0 = by * (TYT * Q);
  const int jz0 = split * cp.dz_per_split;
  const int jz1 = min(cp.nplanes, jz0 + cp.dz_per_split);
  const int LW = cp.lds_w, LH = cp.lds_h;
  // input index of LDS element (row 0, column 0)
  const int xs = x0 + cp.shift[0] - (cp.off[0] + lx - 1) - (CH - 1);
  const int ys = y0 + cp.shift[1] - (cp.off[1] + ly - 1);
  TA acc[Q][R];
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[a][r] = TA(0);
  // input column of every window column (-1: outside a free axis), once per
  // workgroup; the staging below then needs no per-element division
  __shared__ int colsrc[kConvMaxLW];
  for (int c = threadIdx.x; c < LW; c += NT) {
    int xi = xs + c;
    if (cp.per[0]) xi = wrap_index(xi, n0);
    else if (xi < 0 || xi >= n0) xi = -1;
    colsrc[c] = xi;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int jz = jz0; jz < jz1; ++jz) {
    // input plane of stencil plane jz and, folded, of its mirror plane
    // len2-1-jz (same coefficients); a null pointer stands for an all-zero
    // plane outside a free axis (uniform over the workgroup)
    const TI* qa = nullptr;
    const TI* qb = nullptr;
    {
      int zi = z + cp.shift[2] - (cp.off[2] + jz);
      if (cp.per[2]) zi = wrap_index(zi, n2);
      if (zi >= 0 && zi < n2) qa = q + (long long)zi * n1 * n0;
      const int jm = cp.len[2] - 1 - jz;
      if (cp.fold && jm != jz) {
        int zm = z + cp.shift[2] - (cp.off[2] + jm);
        if (cp.per[2]) zm = wrap_index(zm, n2);
        if (zm >= 0 && zm < n2) qb = q + (long long)zm * n1 * n0;
      }
    }
    if (!qa && !qb) continue;
    if (!qa) {
      qa = qb;
      qb = nullptr;
    }
    __syncthreads();
    // one wave per window row, lanes along x
    for (int ry = wave; ry < LH; ry += NT >> 6) {
      int yi = ys + ry;
      bool ok = true;
      if (cp.per[1]) yi = wrap_index(yi, n1);
      else ok = (yi >= 0 && yi < n1);
      const long long ro = (long long)(ok ? yi : 0) * n0;
      TI* dst = lds + ry * LW;
      if (qb) {
        for (int c = lane; c < LW; c += 64) {
          const int xi = colsrc[c];
          dst[c] = (ok && xi >= 0) ? qa[ro + xi] + qb[ro + xi] : TI(0);
        }
      } else {
        for (int c = lane; c < LW; c += 64) {
          const int xi = colsrc[c];
          dst[c] = (ok && xi >= 0) ? qa[ro + xi] : TI(0);
        }
      }
    }
    __syncthreads();
    // plane jz of the stencil: ly + 2 kConvRowPad rows of stride lxp
    const TA* Kz = K + ((long long)jz * (ly + 2 * kConvRowPad) + kConvRowPad) * lxp;
    conv_plane<TI, TA, R, Q>(lds, LW, tx, ty, Kz, rowext + jz * ly, lx, ly, lxp, 0, lx - 1, ws,
                             Q + ly - 2, acc, WS);
  }
  if constexpr (WS > 1) {
    // copies 1..WS-1 hand their sums to copy 0 through the (no longer
    // needed) window memory: red[w][a R + r][tt]
    TA* red = reinterpret_cast<TA*>(smem_raw);
    __syncthreads();
    if (ws > 0) {
#pragma unroll
      for (int a = 0; a < Q; ++a)
#pragma unroll
        for (int r = 0; r < R; ++r) red[((ws - 1) * Q * R + a * R + r) * NTILE + tt] = acc[a][r];
    }
    __syncthreads();
    if (ws > 0) return;
#pragma unroll
    for (int w = 0; w < WS - 1; ++w)
#pragma unroll
      for (int a = 0; a < Q; ++a)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[a][r] += red[(w * Q * R + a * R + r) * NTILE + tt];
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int y = y0 + ty * Q + a;
    if (y >= o1) continue;
    TA* erow = e + ((long long)z * o1 + y) * o0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = x0 + tx * R + r;
      if (x < o0) {
        if (cp.nsplit > 1) atomicAdd(&erow[x], acc[a][r]);
        else erow[x] = acc[a][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Second half of the factored stencil: e_m = sum_k omega'_kx omega'_ky
// omega'_kz u_{m-k}, one axis per launch (x, then y, then z).  Each thread
// owns one output point and sums its 2M+1 taps in order k = -M..M; a wave
// covers 64 consecutive x, so every tap is a coalesced read (the x pass's
// neighbouring taps come from the same cache lines).  Along a periodic axis
// the input index wraps; along a free one the input lives on the extended
// domain (index m + M - k) and is zero outside it.  The passes keep no
// tile in LDS, so they run beside the level-1 convolution's workgroups.
// ---------------------------------------------------------------------------
template <typename TO, int AX>
__global__ void __launch_bounds__(256)
    k_omega_pass(OmegaPass pa, const double* __restrict__ in, TO* __restrict__ out) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= pa.out[0] || y >= pa.out[1]) return;
  const int c[3] = {x, y, z};
  const int m = c[AX], nin = pa.in[AX], M = pa.M;
  const long long stride = AX == 0 ? 1LL : AX == 1 ? (long long)pa.in[0] : (long long)pa.in[0] * pa.in[1];
  long long base = 0;
  {
    const int cx = AX == 0 ? 0 : x, cy = AX == 1 ? 0 : y, cz = AX == 2 ? 0 : z;
    base = ((long long)cz * pa.in[1] + cy) * pa.in[0] + cx;
  }
  double s = 0.0;
  for (int k = -M; k <= M; ++k) {
    int i;
    if (pa.per) {
      i = m - k;
      if (i < 0 || i >= nin) i = wrap_index(i, nin);
    } else {
      i = m + M - k;
      if (i < 0 || i >= nin) continue;
    }
    s += pa.omega[k < 0 ? -k : k] * in[base + i * stride];
  }
  out[((long long)z * pa.out[1] + y) * pa.out[0] + x] = (TO)s;
}

template <typename T>
__global__ void k_cast(const double* __restrict__ src, T* __restrict__ dst, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (T)src[i];
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, long long count, T value) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
// J: host array of the p+1 taps J_{-p/2..p/2}, passed to the kernel by value.
template <typename T>
static JTaps<T> make_taps(const double* J, int p) {
  JTaps<T> jt;
  for (int k = 0; k < 9; ++k) jt.J[k] = k <= p ? (T)J[k] : T(0);
  return jt;
}

// Large grids: streaming forms of the two passes.  A workgroup owns a
// kStreamBX x kStreamBY column of output points and walks a range of output
// planes along z.  Each input plane is staged in LDS once, filtered along x
// and y (one value per thread), and kept in a shift register of the thread
// for the z taps, so every input plane is read from HBM once per column
// (plus the x-y halo) instead of once per small cube; the next plane's
// loads are issued before the current plane's filters.  Tap orders match
// the tiled kernels above.
constexpr int kStreamBX = 32, kStreamBY = 8;  // 256 threads, one output column each
constexpr int kProlongBX = 64, kProlongBY = 4;  // prolongation: a wave per 64-point fine row

template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_restrict_stream(GridDev<T> f, GridDev<T> c, JTaps<T> jt, int zchunk,
                      const T* __restrict__ qf, T* __restrict__ qc) {
  constexpr int BX = kStreamBX, BY = kStreamBY;
  constexpr int WX = 2 * BX + P - 1, WY = 2 * BY + P - 1, NW = WX * WY;
  constexpr int NL = (NW + 255) / 256;  // window loads per thread
  __shared__ T F[NW];
  __shared__ T X1[WY * BX];
  const int nbx = (c.n[0] + BX - 1) / BX, nby = (c.n[1] + BY - 1) / BY;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
  const int cx0 = bx * BX, cy0 = by * BY;
  const int cz0 = bz * zchunk, cz1 = min(c.n[2], cz0 + zchunk);
  if (cz0 >= cz1) return;
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  // absolute fine index of window element 0 in x and y, of plane 0 in z
  const int fx0 = 2 * (cx0 + c.lo[0]) - P / 2, fy0 = 2 * (cy0 + c.lo[1]) - P / 2;
  const int fz0 = 2 * (cz0 + c.lo[2]) - P / 2;
  int off[NL];  // in-plane offset of each loaded window element, -1: zero
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = threadIdx.x + 256 * k;
    off[k] = -1;
    if (e < NW) {
      const int ix = axis_index(fx0 + e % WX, f.n[0], f.lo[0], f.per[0]);
      const int iy = axis_index(fy0 + e / WX, f.n[1], f.lo[1], f.per[1]);
      if (ix >= 0 && iy >= 0) off[k] = iy * f.n[0] + ix;
    }
  }
  const long long plane = (long long)f.n[0] * f.n[1];
  // Loads are unconditional (elements outside the grid read element 0 of a
  // valid plane and are replaced by zero when staged), so every wave keeps
  // the same number of loads in flight and the waits stay partial.
  auto load = [&](int fz, T (&r)[NL], bool& zok) {
    const int iz = axis_index(fz, f.n[2], f.lo[2], f.per[2]);
    zok = iz >= 0;
    const T* src = qf + (long long)max(iz, 0) * plane;
#pragma unroll
    for (int k = 0; k < NL; ++k) r[k] = src[max(off[k], 0)];
  };
  // fine planes fz0 .. fz0 + np - 1 in order: after plane i >= P (i - P
  // even) the last P + 1 planes are the z taps of coarse plane cz0 + (i - P)/2
  const int np = 2 * (cz1 - cz0) + P - 1;
  T ring[P + 1];
#pragma unroll
  for (int t = 0; t <= P; ++t) ring[t] = T(0);
  // plane i: stage it (loaded two planes earlier), start loading plane i + 2
  // into the same registers, filter
  auto step = [&](int i, T (&r)[NL], bool& zok) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < NW) F[e] = (zok && off[k] >= 0) ? r[k] : T(0);
    }
    __syncthreads();
    load(fz0 + min(i + 2, np - 1), r, zok);  // past the end: a spare load
    for (int j = threadIdx.x; j < WY * BX; j += 256) {
      const int x = j % BX, y = j / BX;
      const T* row = F + y * WX + 2 * x;
      T sx = T(0);
#pragma unroll
      for (int t = 0; t <= P; ++t) sx += jt.J[t] * row[t];
      X1[j] = sx;
    }
    __syncthreads();
    T sy = T(0);
#pragma unroll
    for (int t = 0; t <= P; ++t) sy += jt.J[t] * X1[(2 * ty + t) * BX + tx];
#pragma unroll
    for (int t = 0; t < P; ++t) ring[t] = ring[t + 1];
    ring[P] = sy;
    if (i >= P && ((i - P) & 1) == 0) {
      const int gz = cz0 + (i - P) / 2, gx = cx0 + tx, gy = cy0 + ty;
      if (gx < c.n[0] && gy < c.n[1]) {
        T sum = T(0);
#pragma unroll
        for (int t = 0; t <= P; ++t) sum += jt.J[t] * ring[t];
        qc[((long long)gz * c.n[1] + gy) * c.n[0] + gx] = sum;
      }
    }
  };
  T ra[NL], rb[NL];
  bool za, zb;
  load(fz0, ra, za);
  load(fz0 + 1, rb, zb);  // np >= P + 1 >= 2
  for (int i = 0; i < np; i += 2) {
    step(i, ra, za);
    if (i + 1 < np) step(i + 1, rb, zb);
  }
}

// SC / SF: type of the coarse source and of the fine term (T, or FP64 from a
// direct level's convolution buffer); fsrc may be ef itself (ef += ...).
template <typename T, int P, typename SC, typename SF>
__global__ void __launch_bounds__(256)
    k_prolong_stream(GridDev<T> f, GridDev<T> c, JTaps<T> jt, int zchunk,
                     const SC* __restrict__ csrc, const SF* fsrc, T* ef) {
  constexpr int BX = kProlongBX, BY = kProlongBY;
  constexpr int CW = BX / 2 + P / 2 + 2, CH = BY / 2 + P / 2 + 2, NC = CW * CH;
  constexpr int NL = (NC + 255) / 256;
  __shared__ T C[NC];
  __shared__ T X1[CH * BX];
  const int nbx = (f.n[0] + BX - 1) / BX, nby = (f.n[1] + BY - 1) / BY;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
  const int fx0 = bx * BX, fy0 = by * BY;
  const int fz0 = bz * zchunk, fz1 = min(f.n[2], fz0 + zchunk);
  if (fz0 >= fz1) return;
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  // absolute fine index of the column's first point; coarse window start:
  // ceil((m - P/2)/2) of that point, per axis
  const int mx0 = fx0 + f.lo[0], my0 = fy0 + f.lo[1];
  const int n0x = -floor_div2(-(mx0 - P / 2)), n0y = -floor_div2(-(my0 - P / 2));
  int off[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int e = threadIdx.x + 256 * k;
    off[k] = -1;
    if (e < NC) {
      const int ix = axis_index(n0x + e % CW, c.n[0], c.lo[0], c.per[0]);
      const int iy = axis_index(n0y + e / CW, c.n[1], c.lo[1], c.per[1]);
      if (ix >= 0 && iy >= 0) off[k] = iy * c.n[0] + ix;
    }
  }
  const long long cplane = (long long)c.n[0] * c.n[1];
  // unconditional loads as in the restriction; sources are kept in their
  // own type until they are used
  SC r[NL];
  bool rz = false;
  auto load = [&](int nz) {
    const int iz = axis_index(nz, c.n[2], c.lo[2], c.per[2]);
    rz = iz >= 0;
    const long long base = (long long)max(iz, 0) * cplane;
#pragma unroll
    for (int k = 0; k < NL; ++k) r[k] = csrc[base + max(off[k], 0)];
  };
  // fine x and y of this thread and their first coarse point
  const int gx = fx0 + tx, gy = fy0 + ty;
  const bool own = gx < f.n[0] && gy < f.n[1];
  const int my = my0 + ty, nly = -floor_div2(-(my - P / 2)), ey = (my - P / 2) & 1;
  // coarse planes nz (absolute) in order; after plane nz the fine planes
  // 2 nz - P/2 and 2 nz - P/2 + 1 have all their z taps: ring[j] holds the
  // x-y filtered plane nz - j
  const int mz_lo = fz0 + f.lo[2], mz_hi = fz1 - 1 + f.lo[2];
  const int nz_lo = -floor_div2(-(mz_lo - P / 2)), nz_hi = floor_div2(mz_hi + P / 2);
  T ring[P / 2 + 1];
#pragma unroll
  for (int j = 0; j <= P / 2; ++j) ring[j] = T(0);
  const long long fplane = (long long)f.n[0] * f.n[1];
  // fine values that coarse plane nz completes (planes 2 nz - P/2 and
  // 2 nz - P/2 + 1 of this column), or 0 outside the workgroup's range
  // (read unconditionally at a clamped index; only written points use them)
  const long long fcol = (long long)min(gy, f.n[1] - 1) * f.n[0] + min(gx, f.n[0] - 1);
  auto fine_load = [&](int nz, SF& v0, SF& v1) {
    const int me = 2 * nz - P / 2;
    const int z0 = min(max(me - f.lo[2], 0), f.n[2] - 1);
    const int z1 = min(max(me + 1 - f.lo[2], 0), f.n[2] - 1);
    v0 = fsrc[(long long)z0 * fplane + fcol];
    v1 = fsrc[(long long)z1 * fplane + fcol];
  };
  // coarse plane nz: its fine values v0, v1 were read two planes earlier;
  // after the outputs they are reused for plane nz + 2
  auto step = [&](int nz, SF& v0, SF& v1) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < NC) C[e] = (rz && off[k] >= 0) ? (T)r[k] : T(0);
    }
    __syncthreads();
    load(min(nz + 1, nz_hi));  // past the end: a spare load
    for (int j = threadIdx.x; j < CH * BX; j += 256) {
      const int x = j % BX, cy = j / BX;
      const int m = mx0 + x;
      const int nl = -floor_div2(-(m - P / 2)), e = (m - P / 2) & 1;
      T sx = T(0);
#pragma unroll
      for (int t = 0; t < P / 2 + 1; ++t)
        sx += prolong_tap<T, P>(jt, e, t) * C[cy * CW + (nl + t - n0x)];
      X1[j] = sx;
    }
    __syncthreads();
    T sy = T(0);
#pragma unroll
    for (int t = 0; t < P / 2 + 1; ++t)
      sy += prolong_tap<T, P>(jt, ey, t) * X1[(nly + t - n0y) * BX + tx];
#pragma unroll
    for (int j = P / 2; j > 0; --j) ring[j] = ring[j - 1];
    ring[0] = sy;
    // coarse planes in increasing order: fine plane me takes nz - P/2 .. nz
    // (J index 2j), plane me + 1 takes nz - P/2 + 1 .. nz (J index 2j + 1)
    const int me = 2 * nz - P / 2;
    const long long fi0 = (long long)(me - f.lo[2]) * fplane + (long long)gy * f.n[0] + gx;
    if (own && me >= mz_lo && me <= mz_hi) {
      T s0 = T(0);
#pragma unroll
      for (int j = P / 2; j >= 0; --j) s0 += jt.J[2 * j] * ring[j];
      ef[fi0] = (T)v0 + s0;
    }
    if (own && me + 1 >= mz_lo && me + 1 <= mz_hi) {
      T s1 = T(0);
#pragma unroll
      for (int j = P / 2 - 1; j >= 0; --j) s1 += jt.J[2 * j + 1] * ring[j];
      ef[fi0 + fplane] = (T)v1 + s1;
    }
    fine_load(nz + 2, v0, v1);  // past the end: a spare load
  };
  SF va0, va1, vb0, vb1;
  load(nz_lo);
  fine_load(nz_lo, va0, va1);
  fine_load(nz_lo + 1, vb0, vb1);
  for (int nz = nz_lo; nz <= nz_hi; nz += 2) {
    step(nz, va0, va1);
    if (nz + 1 <= nz_hi) step(nz + 1, vb0, vb1);
  }
}

// Streaming passes for fine grids of at least this many points
// (MSM_GRID_STREAM=1 / 0 forces them on / off).
constexpr long long kStreamMinFine = 1LL << 21;
static bool use_stream(long long fine_points) {
  const char* e = std::getenv("MSM_GRID_STREAM");
  if (e && e[0] == '1') return true;
  if (e && e[0] == '0') return false;
  return fine_points >= kStreamMinFine;
}
// z planes per workgroup: at least 4, and enough chunks for about 2048
// workgroups over the (x, y) columns
static int stream_zchunk(long long columns, int nz) {
  const long long want = std::max<long long>(1, (2048 + columns - 1) / columns);
  return std::max<int>(4, (int)((nz + want - 1) / want));
}

template <typename T>
void launch_restrict(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                     const T* qf, T* qc, hipStream_t s) {
  JTaps<T> jt = make_taps<T>(J, p);
  if (use_stream((long long)fine.n[0] * fine.n[1] * fine.n[2])) {
    const long long cols = (long long)((coarse.n[0] + kStreamBX - 1) / kStreamBX) *
                           ((coarse.n[1] + kStreamBY - 1) / kStreamBY);
    const int zc = stream_zchunk(cols, coarse.n[2]);
    const unsigned nb = (unsigned)(cols * ((coarse.n[2] + zc - 1) / zc));
    switch (p) {
      case 4: hipLaunchKernelGGL((k_restrict_stream<T, 4>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, qf, qc); break;
      case 6: hipLaunchKernelGGL((k_restrict_stream<T, 6>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, qf, qc); break;
      case 8: hipLaunchKernelGGL((k_restrict_stream<T, 8>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, qf, qc); break;
    }
    return;
  }
  constexpr int B = kRestrictB;
  const long long nb = (long long)((coarse.n[0] + B - 1) / B) * ((coarse.n[1] + B - 1) / B) *
                       ((coarse.n[2] + B - 1) / B);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_restrict_tiled<T, 4>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
    case 6: hipLaunchKernelGGL((k_restrict_tiled<T, 6>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
    case 8: hipLaunchKernelGGL((k_restrict_tiled<T, 8>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
  }
}

template <typename T>
void launch_prolong(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                    const T* ecT, const double* ec64, T* ef, const double* ef64,
                    hipStream_t s) {
  JTaps<T> jt = make_taps<T>(J, p);
  if (use_stream((long long)fine.n[0] * fine.n[1] * fine.n[2])) {
    const long long cols = (long long)((fine.n[0] + kProlongBX - 1) / kProlongBX) *
                           ((fine.n[1] + kProlongBY - 1) / kProlongBY);
    const int zc = stream_zchunk(cols, fine.n[2]);
    const unsigned nb = (unsigned)(cols * ((fine.n[2] + zc - 1) / zc));
    auto go = [&](auto csrc, auto fsrc) {
      using SC = std::remove_const_t<std::remove_pointer_t<decltype(csrc)>>;
      using SF = std::remove_const_t<std::remove_pointer_t<decltype(fsrc)>>;
      switch (p) {
        case 4: hipLaunchKernelGGL((k_prolong_stream<T, 4, SC, SF>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, csrc, fsrc, ef); break;
        case 6: hipLaunchKernelGGL((k_prolong_stream<T, 6, SC, SF>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, csrc, fsrc, ef); break;
        case 8: hipLaunchKernelGGL((k_prolong_stream<T, 8, SC, SF>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, zc, csrc, fsrc, ef); break;
      }
    };
    if (ec64) {
      if (ef64) go(ec64, ef64);
      else go(ec64, (const T*)ef);
    } else {
      if (ef64) go(ecT, ef64);
      else go(ecT, (const T*)ef);
    }
    return;
  }
  constexpr int B = kProlongB;
  const long long nb = (long long)((fine.n[0] + B - 1) / B) * ((fine.n[1] + B - 1) / B) *
                       ((fine.n[2] + B - 1) / B);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_prolong_tiled<T, 4>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, ecT, ec64, ef, ef64); break;
    case 6: hipLaunchKernelGGL((k_prolong_tiled<T, 6>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, ecT, ec64, ef, ef64); break;
    case 8: hipLaunchKernelGGL((k_prolong_tiled<T, 8>), dim3((unsigned)nb), dim3(256), 0, s, fine, coarse, jt, ecT, ec64, ef, ef64); break;
  }
}

// Tile shapes {R, Q, TXT, TYT, WS}: 0 = 64 x 64 outputs, 256 threads; 1 =
// 32 x 32 outputs, 4 x 64 threads splitting the stencil rows; 2 = 16 x 16
// outputs (R = Q = 2), 4 x 64 threads splitting the stencil rows.
struct ConvShape {
  int R, Q, TXT, TYT, WS;
  double eff;  // relative multiply-add throughput of the shape
};
static const ConvShape kShapes[3] = {
    {4, 4, 16, 16, 1, 1.0}, {4, 4, 8, 8, 4, 0.9}, {2, 2, 8, 8, 4, 0.55}};
constexpr int kNumShapes = 3;

int conv_row_stride(int len0) { return len0 + kConvCH - 1; }

// LDS of k_conv: the staged window (tsize bytes per point) or, reusing it
// at the end, the row-split reduction buffer (FP64 accumulators), plus the
// static column table
static size_t conv_lds_total(const ConvShape& sh, size_t window_bytes) {
  const size_t red = (size_t)(sh.WS - 1) * sh.Q * sh.R * sh.TXT * sh.TYT * sizeof(double);
  return std::max(window_bytes, red) + sizeof(int) * kConvMaxLW;
}

ConvParams make_conv_params(const int n[3], const int nout[3], const int shift[3],
                            const int per[3], const int off[3], const int len[3], int tsize,
                            int fold) {
  ConvParams cp;
  cp.fold = fold && len[2] > 1;
  cp.nplanes = cp.fold ? (len[2] + 1) / 2 : len[2];
  for (int k = 0; k < 3; ++k) {
    cp.n[k] = n[k];
    cp.nout[k] = nout[k];
    cp.shift[k] = shift[k];
    cp.per[k] = per[k];
    cp.off[k] = off[k];
    cp.len[k] = len[k];
  }
  cp.lxp = conv_row_stride(len[0]);
  // shape: fewest padded outputs per unit throughput, penalised when the
  // launch cannot reach 2048 waves even with one stencil plane per split
  double best = 0;
  int pick = -1;
  for (int c = 0; c < kNumShapes; ++c) {
    const ConvShape& sh = kShapes[c];
    const int TX = sh.TXT * sh.R, TY = sh.TYT * sh.Q;
    const size_t lds =
        conv_lds_total(sh, (size_t)(TX + len[0] - 1 + kConvCH - 1) * (TY + len[1] - 1) * tsize);
    if (lds > 64 * 1024 || TX + len[0] - 1 + kConvCH - 1 > kConvMaxLW) continue;
    const double tiles = (double)((nout[0] + TX - 1) / TX) * ((nout[1] + TY - 1) / TY) * nout[2];
    const double waves = tiles * cp.nplanes * (sh.TXT * sh.TYT * sh.WS / 64);
    double cost = tiles * TX * TY / sh.eff;
    if (waves < 2048) cost *= 2048.0 / waves;
    if (pick < 0 || cost < best) {
      best = cost;
      pick = c;
    }
  }
  if (pick < 0) pick = 2;
  const ConvShape& sh = kShapes[pick];
  const int TX = sh.TXT * sh.R, TY = sh.TYT * sh.Q;
  cp.shape = pick;
  cp.lds_w = TX + len[0] - 1 + kConvCH - 1;
  cp.lds_h = TY + len[1] - 1;
  // waves wanted per launch (the stencil z-planes are split across
  // workgroups until the launch has this many); MSM_CONV_WAVES overrides
  static const long long target = [] {
    const char* e = getenv("MSM_CONV_WAVES");
    const long long v = e ? atoll(e) : 0;
    return v > 0 ? v : 8192LL;
  }();
  const long long wpb = sh.TXT * sh.TYT * sh.WS / 64;
  const long long blocks =
      (long long)((nout[0] + TX - 1) / TX) * ((nout[1] + TY - 1) / TY) * nout[2];
  long long want = (target + blocks * wpb - 1) / (blocks * wpb);
  if (want < 1) want = 1;
  if (want > cp.nplanes) want = cp.nplanes;
  cp.dz_per_split = (int)((cp.nplanes + want - 1) / want);
  cp.nsplit = (cp.nplanes + cp.dz_per_split - 1) / cp.dz_per_split;
  return cp;
}

size_t conv_lds_bytes(const ConvParams& cp, int tsize) {
  return conv_lds_total(kShapes[cp.shape], (size_t)cp.lds_w * cp.lds_h * tsize);
}

template <typename TI, typename TA>
void launch_conv(const ConvParams& cp, const TA* K, const int2* rowext, const TI* q, TA* e,
                 hipStream_t s) {
  const ConvShape& sh = kShapes[cp.shape];
  const size_t lds = conv_lds_total(sh, (size_t)cp.lds_w * cp.lds_h * sizeof(TI)) -
                     sizeof(int) * kConvMaxLW;
  const int TX = sh.TXT * sh.R, TY = sh.TYT * sh.Q;
  dim3 grid((cp.nout[0] + TX - 1) / TX, (cp.nout[1] + TY - 1) / TY, cp.nout[2] * cp.nsplit);
  switch (cp.shape) {
    case 0: hipLaunchKernelGGL((k_conv<TI, TA, 4, 4, 16, 16, 1>), grid, dim3(256), lds, s, cp, K, rowext, q, e); break;
    case 1: hipLaunchKernelGGL((k_conv<TI, TA, 4, 4, 8, 8, 4>), grid, dim3(256), lds, s, cp, K, rowext, q, e); break;
    default: hipLaunchKernelGGL((k_conv<TI, TA, 2, 2, 8, 8, 4>), grid, dim3(256), lds, s, cp, K, rowext, q, e); break;
  }
}

template <typename TO, int AX>
static void omega_pass(const OmegaParams& op, const int in[3], const int out[3],
                       const double* u, TO* e, hipStream_t s) {
  OmegaPass pa;
  for (int k = 0; k < 3; ++k) {
    pa.in[k] = in[k];
    pa.out[k] = out[k];
  }
  pa.per = op.per[AX];
  pa.M = op.M;
  for (int k = 0; k < 25; ++k) pa.omega[k] = op.omega[k];
  dim3 grid((out[0] + 63) / 64, (out[1] + 3) / 4, out[2]);
  hipLaunchKernelGGL((k_omega_pass<TO, AX>), grid, dim3(64, 4), 0, s, pa, u, e);
}

// u (extended grid next) -> t (n0, next1, next2) -> u (n0, n1, next2) -> e
template <typename TO>
void launch_omega(const OmegaParams& op, double* u, double* t, TO* e, hipStream_t s) {
  const int d0[3] = {op.next[0], op.next[1], op.next[2]};
  const int d1[3] = {op.n[0], op.next[1], op.next[2]};
  const int d2[3] = {op.n[0], op.n[1], op.next[2]};
  const int d3[3] = {op.n[0], op.n[1], op.n[2]};
  omega_pass<double, 0>(op, d0, d1, u, t, s);
  omega_pass<double, 1>(op, d1, d2, t, u, s);
  omega_pass<TO, 2>(op, d2, d3, u, e, s);
}

template <typename T>
void launch_cast(const double* src, T* dst, long long count, hipStream_t s) {
  if (count <= 0) return;
  long long nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_cast<T>, dim3((unsigned)nb), dim3(256), 0, s, src, dst, count);
}

template <typename T>
void launch_fill(T* p, long long count, T value, hipStream_t s) {
  if (count <= 0) return;
  long long nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)nb), dim3(256), 0, s, p, count, value);
}

#define MSM_INST_GRID(T)                                                                          \
  template void launch_restrict<T>(int, const GridDev<T>&, const GridDev<T>&, const double*,     \
                                   const T*, T*, hipStream_t);                                    \
  template void launch_prolong<T>(int, const GridDev<T>&, const GridDev<T>&, const double*,      \
                                  const T*, const double*, T*, const double*, hipStream_t);       \
  template void launch_omega<T>(const OmegaParams&, double*, double*, T*, hipStream_t);                    \
  template void launch_fill<T>(T*, long long, T, hipStream_t);                                    \
  template void launch_cast<T>(const double*, T*, long long, hipStream_t);
MSM_INST_GRID(float)
MSM_INST_GRID(double)
template void launch_fill<int>(int*, long long, int, hipStream_t);
template void launch_conv<float, double>(const ConvParams&, const double*, const int2*,
                                         const float*, double*, hipStream_t);
template void launch_conv<double, double>(const ConvParams&, const double*, const int2*,
                                          const double*, double*, hipStream_t);

}  // namespace msm
