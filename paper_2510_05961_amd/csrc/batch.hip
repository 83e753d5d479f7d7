// batch.hip -- the MSM for many independent free-space systems at once.
//
// Sec. "Madelung constants" evaluates one model over many structures by
// padding them to a common shape (vmap).  Here there is no padding: system s
// keeps its own box, level count and grids, its particles are the CSR range
// offsets[s]..offsets[s+1], and every stage is ONE launch over all systems:
//   system ids -> pair sums (one workgroup per system, all pairs in LDS) ->
//   anterpolation -> restriction -> stencil convolution (a task list of
//   output tiles across systems; shared K^1, K^2 = K^1/2 and one dense top
//   table per level count) -> prolongation -> interpolation with per-system
//   FP64 energies.
// An intermediate level may run factored (K^l = omega' x omega' x omega' *
// S^l, eq. kernel_stencil_by_conv_with_universal_coeff): three omega' passes
// over the charges, onto grids extended by M on every side, then the ball
// S^l of k-samples from the extended grid back to the level grid.
// The launch sequence is captured once in a hipGraph and replayed; the conv
// tile shape is chosen at plan time by timing the candidates (autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "msm.h"
#include "plan.hpp"
#include "plan_state.hpp"
#include "stencil_fold.hpp"

namespace msm {

constexpr int kPairThreads = 128;  // brute-force pair kernel of the batch path

struct ConvTask {
  long long goff;     // output: offset of the system's level grid (n^3)
  long long goff_in;  // input: the same grid, or its omega'-filtered extension
  int n;              // cubic output grid size
  int n_in;           // cubic input grid size: n, or n + 2M
  int shift;          // input index of output index 0: 0, or M
  int x0, y0, z;      // output tile origin
};

struct BatchConv {
  int level;
  int top;       // 1: dense top kernel of the systems whose top level is `level`
  double scale;  // multiplies the stencil (K^l = K^1 / 2^((l-1) nu))
  int off, len;  // cubic stencil box: offsets off .. off+len-1 per axis
  int fold = 0;  // z-planes j and len-1-j share coefficients
  int cfg = 0;   // tile shape (kTiles), chosen per convolution by the autotuner
  int fact = 0;  // 1: K is the ball S^l, read from the omega'-filtered extension
  int group = 0;  // candidates of one group (a level's direct and factored forms): one is kept
  void* K = nullptr;
  int2* rowext = nullptr;
  ConvTask* tasks = nullptr;
  int ntasks = 0;
};

struct BatchState {
  int n_sys = 0, Lmax = 0, p = 0, M = 0, precision = 0, max_total_n = 0;
  int nu = 1;  // the kernel r^-nu (1: Coulomb, 6: dispersion)
  double h = 0, a = 0, self_const = 0;
  double gcoef[kMaxOrder] = {};
  double J[kMaxOrder + 1] = {};
  std::vector<double> omega, box;
  std::vector<int> L;
  std::vector<int> n[kMaxLevels];
  std::vector<long long> goff[kMaxLevels];
  long long Gtot[kMaxLevels] = {};
  int* d_n[kMaxLevels] = {};
  long long* d_goff[kMaxLevels] = {};
  void* qcat[kMaxLevels] = {};
  void* ecat[kMaxLevels] = {};
  void* d_box = nullptr;
  int* sys_of = nullptr;
  void* phi0 = nullptr;
  void* F0 = nullptr;
  int* flag = nullptr;
  std::vector<BatchConv> convs;
  // factored intermediate levels: per level, each system's offset in the
  // extended buffers (n + 2M)^3 (zero size where the system does not take
  // part) and, per omega' pass, the first workgroup of each system
  std::vector<long long> goffe[kMaxLevels];
  long long* d_goffe[kMaxLevels] = {};
  int* d_bfirst[kMaxLevels][3] = {};  // first workgroup of each system, per pass
  int pass_blocks[kMaxLevels][3] = {};
  void* xbuf = nullptr;  // omega' pass buffers, max over levels of sum (n + 2M)^3
  void* ybuf = nullptr;
  int tile_cfg = 0;
  std::string tuning;
  // graph cache
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  const void* key[7] = {};
};

void destroy_batch(BatchState* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
}

// tile shapes the autotuner chooses from: (R outputs per thread, threads in x, in y)
struct TileCfg {
  int R, TXT, TYT;
};
static const TileCfg kTiles[] = {{4, 4, 16}, {4, 8, 16}, {2, 8, 8}, {8, 4, 16}};
constexpr int kNumTiles = 4;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_batch_sysid(int n_sys, const int* __restrict__ off, int max_n,
                              int* __restrict__ sys_of, int* __restrict__ flag) {
  const int s = blockIdx.x;
  const int b = off[s], e = off[s + 1];
  if (threadIdx.x == 0 && (b < 0 || e < b || e > max_n || (s == 0 && b != 0)))
    atomicOr(flag, kFlagOffsets);
  const int lo = max(b, 0), hi = min(e, max_n);
  for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) sys_of[i] = s;
}

template <typename T>
__device__ inline void load_clamped(const T* pos, int i, T box, T& x, T& y, T& z, int& bad) {
  T v[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (!isfinite(v[k])) {
      bad |= kFlagNonfinite;
      v[k] = T(0);
    }
    if (v[k] < T(0) || v[k] > box) {
      bad |= kFlagDomain;
      v[k] = v[k] < T(0) ? T(0) : box;
    }
  }
  x = v[0];
  y = v[1];
  z = v[2];
}

template <typename T, int P, int NU>
__global__ void __launch_bounds__(kPairThreads)
    k_batch_pair(const int* __restrict__ off, int max_n, const T* __restrict__ pos,
                 const T* __restrict__ q, const T* __restrict__ boxes, PairParams<T> pp,
                 double* __restrict__ phi0, T* __restrict__ F0, int* __restrict__ flag) {
  __shared__ vec4_t<T> tile[kPairThreads];
  const int s = blockIdx.x;
  const int b = max(off[s], 0), e = min(off[s + 1], max_n);
  const T box = boxes[s];
  int bad = 0;
  for (int ib = b; ib < e; ib += kPairThreads) {
    const int i = ib + (int)threadIdx.x;
    const bool active = i < e;
    T xi = 0, yi = 0, zi = 0, qi = 0;
    if (active) {
      load_clamped(pos, i, box, xi, yi, zi, bad);
      qi = q[i];
      if (!isfinite(qi)) {
        bad |= kFlagNonfinite;
        qi = T(0);
      }
    }
    double ph = 0.0;
    T fx = 0, fy = 0, fz = 0;
    for (int jb = b; jb < e; jb += kPairThreads) {
      __syncthreads();
      const int j = jb + (int)threadIdx.x;
      if (j < e) {
        vec4_t<T> t;
        int dummy = 0;
        load_clamped(pos, j, box, t.x, t.y, t.z, dummy);
        T qj = q[j];
        t.w = isfinite(qj) ? qj : T(0);
        tile[threadIdx.x] = t;
      }
      __syncthreads();
      const int cnt = min(kPairThreads, e - jb);
      for (int jj = 0; jj < cnt; ++jj) {
        const vec4_t<T> pj = tile[jj];
        const T dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < pp.a2 && jb + jj != i) {
          const T rinv = rsqrt_t(r2);
          T fs;
          if constexpr (NU == 1) {  // the softener in t = r^2 / a^2
            const T t = r2 * pp.inv_a2;
            T Pt = pp.c[P - 1], dP = pp.dc[P - 2];
#pragma unroll
            for (int k = P - 2; k >= 0; --k) Pt = Pt * t + pp.c[k];
#pragma unroll
            for (int k = P - 3; k >= 0; --k) dP = dP * t + pp.dc[k];
            ph += (double)(pj.w * (rinv - Pt * pp.inv_a));
            fs = pj.w * (rinv * rinv * rinv + T(2) * dP * pp.inv_a3);
          } else {
            // r^-NU: the softener in r^2 with pre-scaled coefficients,
            // gamma(r/a)/a^NU = sum er[k] r^2k, 2 gamma'(t)/a^(NU+2) = sum fr[k] r^2k
            T pe = pp.er[P - 1], pf = pp.fr[P - 2];
#pragma unroll
            for (int k = P - 2; k >= 0; --k) pe = pe * r2 + pp.er[k];
#pragma unroll
            for (int k = P - 3; k >= 0; --k) pf = pf * r2 + pp.fr[k];
            const T rinv2 = rinv * rinv;
            const T kr = rinv2 * rinv2 * rinv2;
            ph += (double)(pj.w * (kr - pe));
            fs = pj.w * (T(NU) * kr * rinv2 + pf);
          }
          fx += fs * dx;
          fy += fs * dy;
          fz += fs * dz;
        }
      }
    }
    if (active) {
      phi0[i] = ph;
      F0[3 * i] = qi * fx;
      F0[3 * i + 1] = qi * fy;
      F0[3 * i + 2] = qi * fz;
    }
  }
  if (bad) atomicOr(flag, bad);
}

template <typename T, int P>
__global__ void k_batch_anterp(const int* __restrict__ off, int n_sys, int max_n,
                               const T* __restrict__ pos, const T* __restrict__ q,
                               const int* __restrict__ sys_of, const T* __restrict__ boxes,
                               const int* __restrict__ n1, const long long* __restrict__ goff1,
                               double h, T* __restrict__ grid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = min(max(off[n_sys], 0), max_n);
  if (i >= total) return;
  const int s = sys_of[i];
  if (s < 0 || s >= n_sys) return;
  T xt[3];
  int bad = 0;
  load_clamped(pos, i, boxes[s], xt[0], xt[1], xt[2], bad);
  T qt = q[i];
  if (!isfinite(qt)) qt = T(0);
  const double qi = (double)qt;
  const int n = n1[s], lo = -P / 2 + 1;
  double w[3][P];
  int idx[3][P];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double f;
    const int base = grid_coord<double>((double)xt[k], h, f);
    bspline_weights<P, double>(f, w[k], nullptr, nullptr);
#pragma unroll
    for (int j = 0; j < P; ++j) idx[k][j] = axis_index(base - P / 2 + 1 + j, n, lo, 0);
  }
  T* g = grid + goff1[s];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    if (idx[2][c] < 0) continue;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      if (idx[1][b] < 0) continue;
      const double wyz = qi * w[2][c] * w[1][b];
      const long long row = ((long long)idx[2][c] * n + idx[1][b]) * n;
#pragma unroll
      for (int a = 0; a < P; ++a)
        if (idx[0][a] >= 0) atomicAdd(&g[row + idx[0][a]], (T)(wyz * w[0][a]));
    }
  }
}

// system owning flat grid point gid (goff: n_sys+1 prefix offsets)
__device__ inline int find_system(const long long* goff, int n_sys, long long gid) {
  int lo = 0, hi = n_sys;  // goff[lo] <= gid < goff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= gid) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, int P>
__global__ void k_batch_restrict(int n_sys, long long Gc, const long long* __restrict__ goff_c,
                                 const int* __restrict__ n_c, const long long* __restrict__ goff_f,
                                 const int* __restrict__ n_f, JTapsB<T> jt,
                                 const T* __restrict__ qf, T* __restrict__ qc) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Gc) return;
  const int s = find_system(goff_c, n_sys, gid);
  const int nc = n_c[s], nf = n_f[s];
  const long long loc = gid - goff_c[s];
  const int ic[3] = {(int)(loc % nc), (int)((loc / nc) % nc), (int)(loc / ((long long)nc * nc))};
  const int lo = -P / 2 + 1;
  int idx[3][P + 1];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int t = 0; t <= P; ++t) idx[k][t] = axis_index(2 * (ic[k] + lo) + t - P / 2, nf, lo, 0);
  const T* f = qf + goff_f[s];
  T sum = 0;
#pragma unroll
  for (int tz = 0; tz <= P; ++tz) {
    if (idx[2][tz] < 0) continue;
    T sy = 0;
#pragma unroll
    for (int ty = 0; ty <= P; ++ty) {
      if (idx[1][ty] < 0) continue;
      const T* row = f + ((long long)idx[2][tz] * nf + idx[1][ty]) * nf;
      T sx = 0;
#pragma unroll
      for (int tx = 0; tx <= P; ++tx)
        if (idx[0][tx] >= 0) sx += jt.J[tx] * row[idx[0][tx]];
      sy += jt.J[ty] * sx;
    }
    sum += jt.J[tz] * sy;
  }
  qc[gid] = sum;
}

template <typename T, int P>
__global__ void k_batch_prolong(int n_sys, long long Gf, const long long* __restrict__ goff_f,
                                const int* __restrict__ n_f, const long long* __restrict__ goff_c,
                                const int* __restrict__ n_c, JTapsB<T> jt,
                                const T* __restrict__ ec, T* __restrict__ ef) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Gf) return;
  const int s = find_system(goff_f, n_sys, gid);
  const int nf = n_f[s], nc = n_c[s];
  if (nc == 0) return;  // this system's top level is the fine level
  const long long loc = gid - goff_f[s];
  const int im[3] = {(int)(loc % nf), (int)((loc / nf) % nf), (int)(loc / ((long long)nf * nf))};
  const int lo = -P / 2 + 1;
  constexpr int NC = P / 2 + 1;
  int idx[3][NC];
  T wt[3][NC];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int m = im[k] + lo;
    const int v = -(m - P / 2);
    const int n_lo = -(v >= 0 ? v / 2 : -((-v + 1) / 2));  // ceil((m - P/2)/2)
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int nn = n_lo + t;
      const int kk = m - 2 * nn;
      if (kk >= -P / 2 && kk <= P / 2) {
        idx[k][t] = axis_index(nn, nc, lo, 0);
        wt[k][t] = jt.J[kk + P / 2];
      } else {
        idx[k][t] = -1;
        wt[k][t] = 0;
      }
    }
  }
  const T* c = ec + goff_c[s];
  T sum = 0;
#pragma unroll
  for (int tz = 0; tz < NC; ++tz) {
    if (idx[2][tz] < 0) continue;
    T sy = 0;
#pragma unroll
    for (int ty = 0; ty < NC; ++ty) {
      if (idx[1][ty] < 0) continue;
      const T* row = c + ((long long)idx[2][tz] * nc + idx[1][ty]) * nc;
      T sx = 0;
#pragma unroll
      for (int tx = 0; tx < NC; ++tx)
        if (idx[0][tx] >= 0) sx += wt[0][tx] * row[idx[0][tx]];
      sy += wt[1][ty] * sx;
    }
    sum += wt[2][tz] * sy;
  }
  ef[gid] += sum;
}

constexpr int kBConvCH = 8;

// omega' taps w_0..w_M (w_-k = w_k), M <= 24
struct OmegaTaps {
  double w[25];
  int M;
};

// One omega' pass of a factored level over every taking-part system: along
// axis AX, out[c] = sum_{|k| <= M} w_|k| in[c - M - k] over input indices
// 0..n-1 (zero outside), c = 0..n+2M-1; the axes before AX are already
// extended to n + 2M, the axes after it not yet.  Each thread computes OPT
// consecutive outputs along AX from one register window of OPT + 2M inputs
// (MT = M at compile time; MT = 0 takes M from w, one output per thread);
// kOmegaBlock threads per workgroup; bfirst[s] = first workgroup of system s
// (systems that do not take part have none, so the last s with bfirst[s] <=
// blockIdx.x owns the workgroup: a search uniform over it).  FP64 sums,
// stored in the grid precision.
constexpr int kOmegaBlock = 256;
constexpr int kOmegaOut = 4;  // outputs per thread when M is 4, 6 or 8
template <typename T, int AX, int OPT, int MT>
__global__ void __launch_bounds__(kOmegaBlock)
    k_batch_omega(int n_sys, const int* __restrict__ bfirst, const int* __restrict__ nn,
                  const long long* __restrict__ goff_in, const long long* __restrict__ goff_out,
                  OmegaTaps w, const T* __restrict__ in, T* __restrict__ out) {
  const int b = blockIdx.x;
  int lo = 0, hi = n_sys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bfirst[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int s = lo, n = nn[s], M = MT > 0 ? MT : w.M, ne = n + 2 * M;
  // extents (within one system every index fits 32 bits: n <= 512, M <= 24)
  const int o0 = ne, o1 = AX >= 1 ? ne : n, o2 = AX >= 2 ? ne : n;  // output
  const int i0 = AX > 0 ? ne : n, i1 = AX > 1 ? ne : n;              // input (x, y)
  const int na = (ne + OPT - 1) / OPT;  // thread positions along AX
  const int t0 = AX == 0 ? na : o0, t1 = AX == 1 ? na : o1, t2 = AX == 2 ? na : o2;
  const int t = (b - bfirst[s]) * kOmegaBlock + (int)threadIdx.x;
  if (t >= t0 * t1 * t2) return;
  const int x = t % t0, y = (t / t0) % t1, z = t / (t0 * t1);
  const int ca = (AX == 0 ? x : (AX == 1 ? y : z)) * OPT;  // first output along AX
  // input offset of the line (AX coordinate 0) and its stride along AX
  const int sa = AX == 0 ? 1 : (AX == 1 ? i0 : i0 * i1);
  const int line_in = AX == 0 ? (y + z * i1) * i0 : (AX == 1 ? x + z * i0 * i1 : x + y * i0);
  // output offset of the line and its stride along AX
  const int so = AX == 0 ? 1 : (AX == 1 ? o0 : o0 * o1);
  const int line_out = AX == 0 ? (y + z * o1) * o0 : (AX == 1 ? x + z * o0 * o1 : x + y * o0);
  const T* src = in + goff_in[s] + line_in;
  T* dst = out + goff_out[s] + line_out;
  if constexpr (MT > 0) {
    double win[OPT + 2 * MT];
#pragma unroll
    for (int j = 0; j < OPT + 2 * MT; ++j) {
      const int i = ca - 2 * MT + j;
      win[j] = (i >= 0 && i < n) ? (double)src[i * sa] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < OPT; ++o) {
      if (ca + o >= ne) break;
      double acc = 0.0;
#pragma unroll
      for (int k = -MT; k <= MT; ++k) acc += w.w[k < 0 ? -k : k] * win[o + MT - k];
      dst[(ca + o) * so] = (T)acc;
    }
  } else {
    double acc = 0.0;
    for (int k = -M; k <= M; ++k) {
      const int i = ca - M - k;
      if (i >= 0 && i < n) acc += w.w[k < 0 ? -k : k] * (double)src[i * sa];
    }
    dst[ca * so] = (T)acc;
  }
}

// outputs per thread of k_batch_omega for a given M (its compile-time cases)
inline int omega_outputs_per_thread(int M) {
  return (M == 4 || M == 6 || M == 8) ? kOmegaOut : 1;
}

// Stencil convolution over a task list: each workgroup computes one output
// tile (one z plane) of one system's grid, all stencil planes; free axes.
// With fold, plane jz and its mirror len-1-jz hold the same coefficients:
// their two input planes are added while staging and walked once.
template <typename T, int R, int TXT, int TYT>
__global__ void __launch_bounds__(TXT * TYT)
    k_batch_conv(const ConvTask* __restrict__ tasks, int off, int len, int fold, int lds_w,
                 double scale, const double* __restrict__ K, const int2* __restrict__ rowext,
                 const T* __restrict__ qcat, T* __restrict__ ecat) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const ConvTask tk = tasks[blockIdx.x];
  const int n = tk.n, ni = tk.n_in, sh = tk.shift;
  const int tx = threadIdx.x % TXT, ty = threadIdx.x / TXT;
  const int LW = lds_w, LH = TYT + len - 1;
  // input index of output m at stencil offset d: m + sh - d
  const int xs = tk.x0 + sh - (off + len - 1), ys = tk.y0 + sh - (off + len - 1);
  const T* q = qcat + tk.goff_in;
  double total[R];  // FP64 accumulation (long sums with cancellation)
#pragma unroll
  for (int r = 0; r < R; ++r) total[r] = 0;
  const int nplanes = fold ? (len + 1) / 2 : len;
  for (int jz = 0; jz < nplanes; ++jz) {
    const int za = tk.z + sh - (off + jz), jm = len - 1 - jz;
    const int zb = (fold && jm != jz) ? tk.z + sh - (off + jm) : -1;
    const bool va = za >= 0 && za < ni, vb = zb >= 0 && zb < ni;
    if (!va && !vb) continue;  // uniform over the workgroup
    __syncthreads();
    const T* qa = q + (long long)(va ? za : zb) * ni * ni;
    const T* qb = q + (long long)(vb ? zb : 0) * ni * ni;
    const bool two = va && vb;
    for (int idx = threadIdx.x; idx < LW * LH; idx += TXT * TYT) {
      const int ry = idx / LW, rx = idx - ry * LW;
      const int yi = ys + ry, xi = xs + rx;
      T v = T(0);
      if (yi >= 0 && yi < ni && xi >= 0 && xi < ni) {
        const long long o = (long long)yi * ni + xi;
        v = two ? qa[o] + qb[o] : qa[o];
      }
      lds[idx] = v;
    }
    __syncthreads();
    const double* Kz = K + (long long)jz * len * len;
    const int2* ext_z = rowext + jz * len;
    // rows whose input y lies inside the grid for some output row of the tile
    const int jy_lo = max(0, tk.y0 + sh - off - (ni - 1));
    const int jy_hi = min(len - 1, tk.y0 + TYT - 1 + sh - off);
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    for (int jy = jy_lo; jy <= jy_hi; ++jy) {
      int2 ext = ext_z[jy];
      // x offsets whose inputs can lie inside the grid for this tile
      ext.x = max(ext.x, tk.x0 + sh - off - (ni - 1));
      ext.y = min(ext.y, tk.x0 + TXT * R - 1 + sh - off);
      if (ext.x > ext.y) continue;
      const T* lrow = lds + (ty - jy + len - 1) * LW + tx * R;
      const double* Krow = Kz + jy * len;
      int jx = ext.x;
      for (; jx + kBConvCH - 1 <= ext.y; jx += kBConvCH) {
        double win[kBConvCH + R - 1];
        const T* wp = lrow + (len - jx - kBConvCH);
#pragma unroll
        for (int u = 0; u < kBConvCH + R - 1; ++u) win[u] = (double)wp[u];
#pragma unroll
        for (int c = 0; c < kBConvCH; ++c) {
          const double kv = Krow[jx + c];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = fma(kv, win[kBConvCH - 1 - c + r], acc[r]);
        }
      }
      for (; jx <= ext.y; ++jx) {
        const double kv = Krow[jx];
        const T* wp = lrow + (len - 1 - jx);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(kv, (double)wp[r], acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) total[r] += acc[r];
  }
  const int y = tk.y0 + ty;
  if (y < n) {
    T* erow = ecat + tk.goff + ((long long)tk.z * n + y) * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = tk.x0 + tx * R + r;
      if (x < n) erow[x] = (T)(scale * total[r]);
    }
  }
}

template <typename T, int P>
__global__ void __launch_bounds__(256)
    k_batch_interp(const int* __restrict__ off, int n_sys, int max_n, const T* __restrict__ pos,
                   const T* __restrict__ q, const int* __restrict__ sys_of,
                   const T* __restrict__ boxes, const int* __restrict__ n1,
                   const long long* __restrict__ goff1, double h, double inv_h,
                   const T* __restrict__ ecat1, const double* __restrict__ phi0,
                   const T* __restrict__ F0, double self_const, T* __restrict__ dEdq,
                   T* __restrict__ F, double* __restrict__ energies) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = min(max(off[n_sys], 0), max_n);
  if (i >= total) return;
  const int s = sys_of[i];
  if (s < 0 || s >= n_sys) return;
  T xt[3];
  int bad = 0;
  load_clamped(pos, i, boxes[s], xt[0], xt[1], xt[2], bad);
  T qt = q[i];
  if (!isfinite(qt)) qt = T(0);
  const double qi = (double)qt;
  const int n = n1[s], lo = -P / 2 + 1;
  double w[3][P], dw[3][P];
  int idx[3][P];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double f;
    const int base = grid_coord<double>((double)xt[k], h, f);
    bspline_weights<P, double>(f, w[k], dw[k], nullptr);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      idx[k][j] = axis_index(base - P / 2 + 1 + j, n, lo, 0);
      dw[k][j] *= inv_h;
    }
  }
  const T* e1 = ecat1 + goff1[s];
  double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    if (idx[2][c] < 0) continue;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      if (idx[1][b] < 0) continue;
      const long long row = ((long long)idx[2][c] * n + idx[1][b]) * n;
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
  const double phid = phi0[i] + v - qi * self_const;
  if (dEdq) dEdq[i] = (T)phid;
  if (F) {
    F[3 * i] = (T)((double)F0[3 * i] - qi * gx);
    F[3 * i + 1] = (T)((double)F0[3 * i + 1] - qi * gy);
    F[3 * i + 2] = (T)((double)F0[3 * i + 2] - qi * gz);
  }
  atomicAdd(&energies[s], 0.5 * qi * phid);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T>
static void launch_batch_conv(const BatchConv& bc, int cfg, const T* qcat, T* ecat,
                              hipStream_t s) {
  if (bc.ntasks <= 0) return;
  const TileCfg tc = kTiles[cfg];
  int lds_w = tc.TXT * tc.R + bc.len - 1;
  if (sizeof(T) == 4) lds_w |= 1;
  const size_t lds = (size_t)lds_w * (tc.TYT + bc.len - 1) * sizeof(T);
  const double scale = bc.scale;
  const double* K = (const double*)bc.K;
  switch (cfg) {
    case 0: hipLaunchKernelGGL((k_batch_conv<T, 4, 4, 16>), dim3(bc.ntasks), dim3(64), lds, s, bc.tasks, bc.off, bc.len, bc.fold, lds_w, scale, K, bc.rowext, qcat, ecat); break;
    case 1: hipLaunchKernelGGL((k_batch_conv<T, 4, 8, 16>), dim3(bc.ntasks), dim3(128), lds, s, bc.tasks, bc.off, bc.len, bc.fold, lds_w, scale, K, bc.rowext, qcat, ecat); break;
    case 2: hipLaunchKernelGGL((k_batch_conv<T, 2, 8, 8>), dim3(bc.ntasks), dim3(64), lds, s, bc.tasks, bc.off, bc.len, bc.fold, lds_w, scale, K, bc.rowext, qcat, ecat); break;
    default: hipLaunchKernelGGL((k_batch_conv<T, 8, 4, 16>), dim3(bc.ntasks), dim3(64), lds, s, bc.tasks, bc.off, bc.len, bc.fold, lds_w, scale, K, bc.rowext, qcat, ecat); break;
  }
}

static std::vector<ConvTask> build_tasks(const BatchState& B, const BatchConv& bc, int cfg) {
  std::vector<ConvTask> t;
  const int level = bc.level;
  const int TXo = kTiles[cfg].TXT * kTiles[cfg].R, TY = kTiles[cfg].TYT;
  for (int s = 0; s < B.n_sys; ++s) {
    if (level > B.L[s]) continue;
    if ((B.L[s] == level) != (bc.top != 0)) continue;
    const int n = B.n[level - 1][s];
    const long long go = B.goff[level - 1][s];
    const long long gi = bc.fact ? B.goffe[level - 1][s] : go;
    const int ni = bc.fact ? n + 2 * B.M : n, sh = bc.fact ? B.M : 0;
    for (int z = 0; z < n; ++z)
      for (int y0 = 0; y0 < n; y0 += TY)
        for (int x0 = 0; x0 < n; x0 += TXo) t.push_back({go, gi, n, ni, sh, x0, y0, z});
  }
  return t;
}

// The three omega' passes of factored level l: level grid -> ybuf (x
// extended) -> xbuf (x, y) -> ybuf (all three), which the ball convolution
// reads.
template <typename T>
static void launch_omega_passes(const BatchState& B, int l, hipStream_t s) {
  OmegaTaps w{};
  w.M = B.M;
  for (int k = 0; k <= B.M; ++k) w.w[k] = B.omega[k];
  const long long* gin[3] = {B.d_goff[l - 1], B.d_goffe[l - 1], B.d_goffe[l - 1]};
  const T* in[3] = {(const T*)B.qcat[l - 1], (const T*)B.ybuf, (const T*)B.xbuf};
  T* out[3] = {(T*)B.ybuf, (T*)B.xbuf, (T*)B.ybuf};
  for (int ax = 0; ax < 3; ++ax) {
    const int g = B.pass_blocks[l - 1][ax];
    if (g <= 0) continue;
    const dim3 grid(g), block(kOmegaBlock);
    const int* bf = B.d_bfirst[l - 1][ax];
    const int* nn = B.d_n[l - 1];
    const long long* go = B.d_goffe[l - 1];
#define MSM_OMEGA_LAUNCH(AXV)                                                                   \
  switch (B.M) {                                                                                \
    case 4: hipLaunchKernelGGL((k_batch_omega<T, AXV, kOmegaOut, 4>), grid, block, 0, s, B.n_sys, bf, nn, gin[ax], go, w, in[ax], out[ax]); break; \
    case 6: hipLaunchKernelGGL((k_batch_omega<T, AXV, kOmegaOut, 6>), grid, block, 0, s, B.n_sys, bf, nn, gin[ax], go, w, in[ax], out[ax]); break; \
    case 8: hipLaunchKernelGGL((k_batch_omega<T, AXV, kOmegaOut, 8>), grid, block, 0, s, B.n_sys, bf, nn, gin[ax], go, w, in[ax], out[ax]); break; \
    default: hipLaunchKernelGGL((k_batch_omega<T, AXV, 1, 0>), grid, block, 0, s, B.n_sys, bf, nn, gin[ax], go, w, in[ax], out[ax]); break; \
  }
    if (ax == 0) {
      MSM_OMEGA_LAUNCH(0)
    } else if (ax == 1) {
      MSM_OMEGA_LAUNCH(1)
    } else {
      MSM_OMEGA_LAUNCH(2)
    }
#undef MSM_OMEGA_LAUNCH
  }
}

// A cubic stencil [len]^3 to the device; *fold says whether its z-planes
// mirror (make_planes_mirror, which may average the mirrored pairs first).
template <typename T>
static msm_status upload_stencil(msm_plan P, const std::vector<double>& K0, int len, void** dK,
                                 int2** dext, int* fold) {
  std::vector<double> K = K0;
  *fold = fold_allowed() && make_planes_mirror(K, len, len, len);
  std::vector<T> kt(K.size());
  for (size_t i = 0; i < K.size(); ++i) kt[i] = (T)K[i];
  std::vector<int2> ext((size_t)len * len);
  for (int z = 0; z < len; ++z)
    for (int y = 0; y < len; ++y) {
      int first = len, last = -1;
      for (int x = 0; x < len; ++x)
        if (kt[((size_t)z * len + y) * len + x] != T(0)) {
          first = std::min(first, x);
          last = x;
        }
      ext[(size_t)z * len + y] = make_int2(first, last);
    }
  msm_status st;
  if ((st = hip_alloc(P, dK, kt.size() * sizeof(T)))) return st;
  if ((st = hip_alloc(P, (void**)dext, ext.size() * sizeof(int2)))) return st;
  if (hipMemcpy(*dK, kt.data(), kt.size() * sizeof(T), hipMemcpyHostToDevice) ||
      hipMemcpy(*dext, ext.data(), ext.size() * sizeof(int2), hipMemcpyHostToDevice))
    return MSM_ERR_HIP;
  return MSM_OK;
}

template <typename T>
static msm_status enqueue_batch(msm_plan P, const int* off, const T* pos, const T* q,
                                double* energies, T* F, T* dEdq, hipStream_t s) {
  BatchState& B = *P->bs;
  const int p = B.p, NS = B.n_sys, maxn = B.max_total_n;
  launch_fill<int>(B.sys_of, std::max(maxn, 1), -1, s);
  launch_fill<T>((T*)B.qcat[0], B.Gtot[0], T(0), s);
  launch_fill<double>(energies, NS, 0.0, s);
  hipLaunchKernelGGL(k_batch_sysid, dim3(NS), dim3(256), 0, s, NS, off, maxn, B.sys_of, B.flag);
  PairParams<T> pp{};
  const double a = B.a;
  pp.a2 = (T)(a * a);
  pp.inv_a2 = (T)(1.0 / (a * a));
  pp.inv_a = (T)(1.0 / a);
  pp.inv_a3 = (T)(1.0 / (a * a * a));
  pp.inv_a5 = (T)(1.0 / (a * a * a * a * a));
  pp.nu = B.nu;
  for (int k = 0; k < 8; ++k) {
    pp.c[k] = k < p ? (T)B.gcoef[k] : T(0);
    pp.dc[k] = (k + 1 < p) ? (T)((k + 1) * B.gcoef[k + 1]) : T(0);
    pp.d2c[k] = 0;
    // t^k = r^2k / a^2k, scaled in FP64 before the cast
    const double a2k = std::pow(a, 2 * k), anu = std::pow(a, B.nu);
    pp.er[k] = k < p ? (T)(B.gcoef[k] / (a2k * anu)) : T(0);
    pp.fr[k] = (k + 1 < p) ? (T)(2.0 * (k + 1) * B.gcoef[k + 1] / (a2k * anu * a * a)) : T(0);
    pp.gr[k] = 0;
  }
  for (int k = 0; k < 3; ++k) {
    pp.box[k] = pp.inv_box[k] = 0;
    pp.per[k] = 0;
    pp.nc[k] = 1;
    pp.cs[k] = 0;
  }
  pp.tri = 0;
  for (int k = 0; k < 9; ++k) pp.H[k] = 0;
  const T* boxes = (const T*)B.d_box;
  int ev = P->prof.begin("batch_pair", s);
  if (B.nu == 6) {
    switch (p) {
      case 4: hipLaunchKernelGGL((k_batch_pair<T, 4, 6>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
      case 6: hipLaunchKernelGGL((k_batch_pair<T, 6, 6>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
      default: hipLaunchKernelGGL((k_batch_pair<T, 8, 6>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
    }
  } else {
    switch (p) {
      case 4: hipLaunchKernelGGL((k_batch_pair<T, 4, 1>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
      case 6: hipLaunchKernelGGL((k_batch_pair<T, 6, 1>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
      default: hipLaunchKernelGGL((k_batch_pair<T, 8, 1>), dim3(NS), dim3(kPairThreads), 0, s, off, maxn, pos, q, boxes, pp, (double*)B.phi0, (T*)B.F0, B.flag); break;
    }
  }
  P->prof.end(ev, s);
  const int nb = (std::max(maxn, 1) + 255) / 256;
  const double h = B.h;
  ev = P->prof.begin("batch_anterp", s);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_batch_anterp<T, 4>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, (T*)B.qcat[0]); break;
    case 6: hipLaunchKernelGGL((k_batch_anterp<T, 6>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, (T*)B.qcat[0]); break;
    default: hipLaunchKernelGGL((k_batch_anterp<T, 8>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, (T*)B.qcat[0]); break;
  }
  P->prof.end(ev, s);
  JTapsB<T> jt;
  for (int k = 0; k < 9; ++k) jt.J[k] = k <= p ? (T)B.J[k] : T(0);
  ev = P->prof.begin("batch_restrict", s);
  for (int l = 1; l < B.Lmax; ++l) {
    const long long Gc = B.Gtot[l];
    if (Gc <= 0) continue;
    const unsigned g = (unsigned)((Gc + 255) / 256);
    switch (p) {
      case 4: hipLaunchKernelGGL((k_batch_restrict<T, 4>), dim3(g), dim3(256), 0, s, NS, Gc, B.d_goff[l], B.d_n[l], B.d_goff[l - 1], B.d_n[l - 1], jt, (const T*)B.qcat[l - 1], (T*)B.qcat[l]); break;
      case 6: hipLaunchKernelGGL((k_batch_restrict<T, 6>), dim3(g), dim3(256), 0, s, NS, Gc, B.d_goff[l], B.d_n[l], B.d_goff[l - 1], B.d_n[l - 1], jt, (const T*)B.qcat[l - 1], (T*)B.qcat[l]); break;
      default: hipLaunchKernelGGL((k_batch_restrict<T, 8>), dim3(g), dim3(256), 0, s, NS, Gc, B.d_goff[l], B.d_n[l], B.d_goff[l - 1], B.d_n[l - 1], jt, (const T*)B.qcat[l - 1], (T*)B.qcat[l]); break;
    }
  }
  P->prof.end(ev, s);
  for (const BatchConv& bc : B.convs) {
    ev = P->prof.begin(bc.level == 1 ? "batch_conv_l1" : (bc.top ? "batch_conv_top" : "batch_conv_l2+"), s);
    if (bc.fact) launch_omega_passes<T>(B, bc.level, s);
    launch_batch_conv<T>(bc, bc.cfg, bc.fact ? (const T*)B.ybuf : (const T*)B.qcat[bc.level - 1],
                         (T*)B.ecat[bc.level - 1], s);
    P->prof.end(ev, s);
  }
  ev = P->prof.begin("batch_prolong", s);
  for (int l = B.Lmax - 1; l >= 1; --l) {
    const long long Gf = B.Gtot[l - 1];
    if (Gf <= 0) continue;
    const unsigned g = (unsigned)((Gf + 255) / 256);
    switch (p) {
      case 4: hipLaunchKernelGGL((k_batch_prolong<T, 4>), dim3(g), dim3(256), 0, s, NS, Gf, B.d_goff[l - 1], B.d_n[l - 1], B.d_goff[l], B.d_n[l], jt, (const T*)B.ecat[l], (T*)B.ecat[l - 1]); break;
      case 6: hipLaunchKernelGGL((k_batch_prolong<T, 6>), dim3(g), dim3(256), 0, s, NS, Gf, B.d_goff[l - 1], B.d_n[l - 1], B.d_goff[l], B.d_n[l], jt, (const T*)B.ecat[l], (T*)B.ecat[l - 1]); break;
      default: hipLaunchKernelGGL((k_batch_prolong<T, 8>), dim3(g), dim3(256), 0, s, NS, Gf, B.d_goff[l - 1], B.d_n[l - 1], B.d_goff[l], B.d_n[l], jt, (const T*)B.ecat[l], (T*)B.ecat[l - 1]); break;
    }
  }
  P->prof.end(ev, s);
  const double sc = B.self_const;
  const double ih = 1.0 / B.h;
  ev = P->prof.begin("batch_interp", s);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_batch_interp<T, 4>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, ih, (const T*)B.ecat[0], (const double*)B.phi0, (const T*)B.F0, sc, dEdq, F, energies); break;
    case 6: hipLaunchKernelGGL((k_batch_interp<T, 6>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, ih, (const T*)B.ecat[0], (const double*)B.phi0, (const T*)B.F0, sc, dEdq, F, energies); break;
    default: hipLaunchKernelGGL((k_batch_interp<T, 8>), dim3(nb), dim3(256), 0, s, off, NS, maxn, pos, q, B.sys_of, boxes, B.d_n[0], B.d_goff[0], h, ih, (const T*)B.ecat[0], (const double*)B.phi0, (const T*)B.F0, sc, dEdq, F, energies); break;
  }
  P->prof.end(ev, s);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

// Times every candidate convolution of the plan (each level's intermediate
// forms and top kernels: their grids differ in size) for every tile shape on
// the plan's (zero) grids, a factored form with its three omega' passes;
// keeps the fastest shape per candidate and the fastest candidate per group
// (a level's direct and factored forms).  MSM_BATCH_TILE=c (0 .. 3) pins
// shape c; the forms are still timed against each other.
template <typename T>
static msm_status autotune(msm_plan P) {
  BatchState& B = *P->bs;
  const char* pin = std::getenv("MSM_BATCH_TILE");
  const bool pinned = pin && pin[0] >= '0' && pin[0] < '0' + kNumTiles && pin[1] == 0;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  ConvTask* dt = nullptr;
  // every exit releases the events and the trial task list
  auto done = [&](msm_status st) {
    if (dt) (void)hipFree(dt);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return st;
  };
  if (hipEventCreate(&a) || hipEventCreate(&b)) return done(MSM_ERR_HIP);
  std::ostringstream log;
  std::vector<float> best(B.convs.size(), 1e30f);
  for (size_t ci = 0; ci < B.convs.size(); ++ci) {
    BatchConv& bc = B.convs[ci];
    int best_cfg = pinned ? pin[0] - '0' : 0;
    log << (ci ? "," : "") << "{\"level\":" << bc.level << ",\"top\":" << bc.top
        << ",\"factored\":" << bc.fact << ",\"ms\":[";
    for (int cfg = pinned ? best_cfg : 0; cfg < (pinned ? best_cfg + 1 : kNumTiles); ++cfg) {
      std::vector<ConvTask> t = build_tasks(B, bc, cfg);
      if (hipMalloc((void**)&dt, std::max<size_t>(t.size(), 1) * sizeof(ConvTask))) {
        dt = nullptr;
        (void)hipGetLastError();
        return done(MSM_ERR_OOM);
      }
      if (!t.empty() &&
          hipMemcpy(dt, t.data(), t.size() * sizeof(ConvTask), hipMemcpyHostToDevice))
        return done(MSM_ERR_HIP);
      BatchConv trial = bc;
      trial.tasks = dt;
      trial.ntasks = (int)t.size();
      const T* q = bc.fact ? (const T*)B.ybuf : (const T*)B.qcat[bc.level - 1];
      T* e = (T*)B.ecat[bc.level - 1];
      auto run = [&]() {
        if (bc.fact) launch_omega_passes<T>(B, bc.level, s);
        launch_batch_conv<T>(trial, cfg, q, e, s);
      };
      run();  // warm-up
      (void)hipEventRecord(a, s);
      for (int r = 0; r < 3; ++r) run();
      (void)hipEventRecord(b, s);
      if (hipEventSynchronize(b)) return done(MSM_ERR_HIP);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      (void)hipFree(dt);
      dt = nullptr;
      log << (cfg > (pinned ? best_cfg : 0) ? "," : "") << ms / 3;
      if (ms < best[ci]) {
        best[ci] = ms;
        best_cfg = cfg;
      }
    }
    bc.cfg = best_cfg;
    log << "],\"cfg\":" << best_cfg << "}";
  }
  if (hipGetLastError() != hipSuccess) return done(MSM_ERR_HIP);
  // one candidate per group: the fastest
  std::vector<BatchConv> kept;
  for (size_t ci = 0; ci < B.convs.size(); ++ci) {
    bool keep = true;
    for (size_t cj = 0; cj < B.convs.size(); ++cj)
      if (cj != ci && B.convs[cj].group == B.convs[ci].group &&
          (best[cj] < best[ci] || (best[cj] == best[ci] && cj < ci)))
        keep = false;
    if (keep) kept.push_back(B.convs[ci]);
  }
  B.convs.swap(kept);
  B.tile_cfg = B.convs.empty() ? 0 : B.convs[0].cfg;
  B.tuning = "[" + log.str() + "]";
  return done(MSM_OK);
}

template <typename T>
static msm_status upload_batch(msm_plan P, const std::vector<double>& K1, int W1,
                               const std::vector<double>& S1, int R1,
                               const std::vector<std::vector<double>>& tops,
                               const std::vector<int>& top_len) {
  BatchState& B = *P->bs;
  msm_status st;
  for (int l = 1; l <= B.Lmax; ++l) {
    const size_t g = (size_t)std::max<long long>(B.Gtot[l - 1], 1);
    if ((st = hip_alloc(P, &B.qcat[l - 1], g * sizeof(T)))) return st;
    if ((st = hip_alloc(P, &B.ecat[l - 1], g * sizeof(T)))) return st;
    if ((st = hip_alloc(P, (void**)&B.d_n[l - 1], B.n_sys * sizeof(int)))) return st;
    if ((st = hip_alloc(P, (void**)&B.d_goff[l - 1], (B.n_sys + 1) * sizeof(long long))))
      return st;
    if (hipMemcpy(B.d_n[l - 1], B.n[l - 1].data(), B.n_sys * sizeof(int), hipMemcpyHostToDevice) ||
        hipMemcpy(B.d_goff[l - 1], B.goff[l - 1].data(), (B.n_sys + 1) * sizeof(long long),
                  hipMemcpyHostToDevice))
      return MSM_ERR_HIP;
    launch_fill<T>((T*)B.qcat[l - 1], (long long)g, T(0), nullptr);
    launch_fill<T>((T*)B.ecat[l - 1], (long long)g, T(0), nullptr);
  }
  std::vector<T> bx(B.n_sys);
  for (int s = 0; s < B.n_sys; ++s) bx[s] = (T)B.box[s];
  if ((st = hip_alloc(P, &B.d_box, B.n_sys * sizeof(T)))) return st;
  if (hipMemcpy(B.d_box, bx.data(), B.n_sys * sizeof(T), hipMemcpyHostToDevice)) return MSM_ERR_HIP;
  const size_t nmax = (size_t)std::max(B.max_total_n, 1);
  if ((st = hip_alloc(P, (void**)&B.sys_of, nmax * sizeof(int)))) return st;
  if ((st = hip_alloc(P, &B.phi0, nmax * sizeof(double)))) return st;
  if ((st = hip_alloc(P, &B.F0, nmax * 3 * sizeof(T)))) return st;
  if ((st = hip_alloc(P, (void**)&B.flag, sizeof(int)))) return st;
  if (hipMemset(B.flag, 0, sizeof(int))) return MSM_ERR_HIP;
  P->flag = B.flag;
  // stencils: K^1 (intermediate levels, scaled per level) and the top tables
  void* dK1 = nullptr;
  int2* dK1ext = nullptr;
  int fold1 = 0;
  if ((st = upload_stencil<double>(P, K1, 2 * W1 + 1, &dK1, &dK1ext, &fold1))) return st;
  // factored intermediate levels: both forms of each intermediate level are
  // candidates and the autotuner keeps the faster (on small grids the direct
  // stencil, cropped at the grid, can win); MSM_FACTORED=0 keeps only the
  // direct form, MSM_FACTORED=1 only the factored one
  void* dS1 = nullptr;
  int2* dS1ext = nullptr;
  int foldS = 0;
  const char* fenv = std::getenv("MSM_FACTORED");
  const bool want_direct = !(fenv && fenv[0] == '1');
  const bool want_fact = !(fenv && fenv[0] == '0');
  bool fact[kMaxLevels] = {};
  {
    long long ext_max = 0;
    for (int l = 1; l < B.Lmax && want_fact; ++l) {
      bool any = false;
      for (int s = 0; s < B.n_sys; ++s) any |= B.L[s] > l;
      fact[l - 1] = any;
      if (!any) continue;
      B.goffe[l - 1].assign(B.n_sys + 1, 0);
      std::vector<int> bfirst[3];
      for (int ax = 0; ax < 3; ++ax) bfirst[ax].assign(B.n_sys, 0);
      long long acc = 0, pa[3] = {0, 0, 0};
      for (int s = 0; s < B.n_sys; ++s) {
        B.goffe[l - 1][s] = acc;
        for (int ax = 0; ax < 3; ++ax) bfirst[ax][s] = (int)pa[ax];
        if (B.L[s] <= l) continue;
        const long long n = B.n[l - 1][s], ne = n + 2 * B.M;
        acc += ne * ne * ne;
        // threads per pass: OPT outputs each along the pass's axis
        const int opt = omega_outputs_per_thread(B.M);
        const long long na = (ne + opt - 1) / opt;
        const long long cnt[3] = {na * n * n, ne * na * n, ne * ne * na};
        for (int ax = 0; ax < 3; ++ax) pa[ax] += (cnt[ax] + kOmegaBlock - 1) / kOmegaBlock;
      }
      if (pa[2] > (1LL << 31) - 1) return MSM_ERR_GRID;
      B.goffe[l - 1][B.n_sys] = acc;
      ext_max = std::max(ext_max, acc);
      if ((st = hip_alloc(P, (void**)&B.d_goffe[l - 1], (B.n_sys + 1) * sizeof(long long))))
        return st;
      if (hipMemcpy(B.d_goffe[l - 1], B.goffe[l - 1].data(), (B.n_sys + 1) * sizeof(long long),
                    hipMemcpyHostToDevice))
        return MSM_ERR_HIP;
      for (int ax = 0; ax < 3; ++ax) {
        B.pass_blocks[l - 1][ax] = (int)pa[ax];
        if ((st = hip_alloc(P, (void**)&B.d_bfirst[l - 1][ax], B.n_sys * sizeof(int))))
          return st;
        if (hipMemcpy(B.d_bfirst[l - 1][ax], bfirst[ax].data(), B.n_sys * sizeof(int),
                      hipMemcpyHostToDevice))
          return MSM_ERR_HIP;
      }
    }
    if (ext_max > 0) {
      if ((st = upload_stencil<double>(P, S1, 2 * R1 + 1, &dS1, &dS1ext, &foldS))) return st;
      if ((st = hip_alloc(P, &B.xbuf, (size_t)ext_max * sizeof(T)))) return st;
      if ((st = hip_alloc(P, &B.ybuf, (size_t)ext_max * sizeof(T)))) return st;
      launch_fill<T>((T*)B.xbuf, ext_max, T(0), nullptr);
      launch_fill<T>((T*)B.ybuf, ext_max, T(0), nullptr);
    }
  }
  int group = 0;
  for (int l = 1; l <= B.Lmax; ++l) {
    BatchConv inter;
    inter.level = l;
    inter.top = 0;
    inter.scale = std::ldexp(1.0, -(l - 1) * B.nu);
    inter.group = group++;
    inter.off = -W1;
    inter.len = 2 * W1 + 1;
    inter.K = dK1;
    inter.rowext = dK1ext;
    inter.fold = fold1;
    BatchConv interf = inter;
    const bool has_fact = l < B.Lmax && fact[l - 1];
    if (has_fact) {
      interf.fact = 1;
      interf.off = -R1;
      interf.len = 2 * R1 + 1;
      interf.K = dS1;
      interf.rowext = dS1ext;
      interf.fold = foldS;
    }
    BatchConv top;
    top.level = l;
    top.top = 1;
    top.scale = 1.0;
    top.group = group++;
    top.len = top_len[l];
    top.off = -(top_len[l] - 1) / 2;
    if (top_len[l] > 0) {
      if ((st = upload_stencil<double>(P, tops[l], top_len[l], &top.K, &top.rowext, &top.fold)))
        return st;
    }
    for (BatchConv* bc : {&inter, &interf, &top}) {
      if (bc->top && top_len[l] == 0) continue;
      if (bc == &interf && !has_fact) continue;
      if (bc == &inter && has_fact && !want_direct) continue;
      bool any = false;
      for (int s = 0; s < B.n_sys; ++s)
        if (l <= B.L[s] && ((B.L[s] == l) == (bc->top != 0))) any = true;
      if (!any) continue;
      int lw = kTiles[0].TXT * kTiles[0].R + bc->len - 1;
      for (int c = 0; c < kNumTiles; ++c) {
        int w = kTiles[c].TXT * kTiles[c].R + bc->len - 1;
        if ((size_t)(w | 1) * (kTiles[c].TYT + bc->len - 1) * sizeof(T) > 160 * 1024)
          return MSM_ERR_GRID;
        (void)lw;
      }
      B.convs.push_back(*bc);
    }
  }
  if (hipDeviceSynchronize()) return MSM_ERR_HIP;
  // autotune the tile shape of each convolution, then build the task lists
  if ((st = autotune<T>(P))) return st;
  bool any_fact = false;
  for (const BatchConv& bc : B.convs) any_fact |= bc.fact != 0;
  if (!any_fact)  // the pass buffers are not needed
    for (void** buf : {&B.xbuf, &B.ybuf}) {
      for (size_t k = 0; k < P->allocs.size(); ++k)
        if (P->allocs[k] == *buf) {
          (void)hipFree(*buf);
          P->allocs.erase(P->allocs.begin() + k);
          break;
        }
      *buf = nullptr;
    }
  for (BatchConv& bc : B.convs) {
    std::vector<ConvTask> t = build_tasks(B, bc, bc.cfg);
    if ((st = hip_alloc(P, (void**)&bc.tasks, std::max<size_t>(t.size(), 1) * sizeof(ConvTask))))
      return st;
    if (!t.empty() &&
        hipMemcpy(bc.tasks, t.data(), t.size() * sizeof(ConvTask), hipMemcpyHostToDevice))
      return MSM_ERR_HIP;
    bc.ntasks = (int)t.size();
  }
  if (hipStreamCreateWithFlags(&B.gstream, hipStreamNonBlocking) ||
      hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming) ||
      hipEventCreateWithFlags(&B.ev_join, hipEventDisableTiming))
    return MSM_ERR_HIP;
  return MSM_OK;
}

}  // namespace msm

using namespace msm;

extern "C" msm_status msm_batch_plan_create_kernel(msm_plan* out, int kernel, int n_sys,
                                                   const double* boxes, const int* levels,
                                                   unsigned periodic_mask, int order, double h,
                                                   double cutoff_a, int precision,
                                                   int max_total_n, int quasi_degree_M) {
  if (!out) return MSM_ERR_INVALID_ARG;
  *out = nullptr;
  if (kernel != MSM_KERNEL_COULOMB && kernel != MSM_KERNEL_DISPERSION) return MSM_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_sys < 1 || !boxes || !levels || !(h > 0) || !(cutoff_a > 0) || max_total_n < 0)
    return MSM_ERR_INVALID_ARG;
  // the batched kernels take free-space systems in cubic boxes
  if (periodic_mask != 0) return MSM_ERR_UNSUPPORTED;
  for (int s = 0; s < n_sys; ++s) {
    const double* b = boxes + 3 * (size_t)s;
    if (!(b[0] > 0) || !std::isfinite(b[0])) return MSM_ERR_INVALID_ARG;
    if (std::fabs(b[1] - b[0]) > 1e-12 * b[0] || std::fabs(b[2] - b[0]) > 1e-12 * b[0])
      return MSM_ERR_UNSUPPORTED;
  }
  if (precision != MSM_FP32 && precision != MSM_FP64) return MSM_ERR_INVALID_ARG;
  if (order != 4 && order != 6 && order != 8) return MSM_ERR_UNSUPPORTED;
  const int M = quasi_degree_M < 0 ? order : quasi_degree_M;
  if (M > 24) return MSM_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return MSM_ERR_HIP;
  }
  msm_plan P = new (std::nothrow) msm_plan_s;
  if (!P) return MSM_ERR_OOM;
  P->batch = true;
  P->device = true;
  P->bs = new (std::nothrow) BatchState;
  if (!P->bs) {
    delete P;
    return MSM_ERR_OOM;
  }
  BatchState& B = *P->bs;
  msm_status st = MSM_OK;
  try {
    B.n_sys = n_sys;
    B.p = order;
    B.M = M;
    B.h = h;
    B.a = cutoff_a;
    B.precision = precision;
    B.nu = kernel;
    B.max_total_n = max_total_n;
    B.box.resize(n_sys);
    for (int s = 0; s < n_sys; ++s) B.box[s] = boxes[3 * (size_t)s];
    B.L.assign(levels, levels + n_sys);
    for (int s = 0; s < n_sys; ++s) {
      if (!(B.box[s] > 0) || !std::isfinite(B.box[s]) || B.L[s] < 1 || B.L[s] > kMaxLevels)
        st = MSM_ERR_INVALID_ARG;
      B.Lmax = std::max(B.Lmax, B.L[s]);
    }
    if (st == MSM_OK) {
      softener_coefficients(order, B.gcoef, B.nu);
      B.self_const = B.gcoef[0] / std::pow(cutoff_a, B.nu);
      B.omega = quasi_sequence(order, M);
      for (int k = 0; k <= order; ++k) {
        double c = 1.0;
        for (int i = 1; i <= k; ++i) c = c * (order - k + i) / i;
        B.J[k] = std::ldexp(c, 1 - order);
      }
      for (int l = 1; l <= B.Lmax; ++l) {
        B.n[l - 1].assign(n_sys, 0);
        B.goff[l - 1].assign(n_sys + 1, 0);
        long long acc = 0;
        for (int s = 0; s < n_sys; ++s) {
          B.goff[l - 1][s] = acc;
          if (l <= B.L[s]) {
            const double hl = std::ldexp(h, l - 1);
            const int nn = (int)std::ceil(B.box[s] / hl - 1e-9) + order - 1;
            if (nn > 512) st = MSM_ERR_GRID;
            B.n[l - 1][s] = nn;
            acc += (long long)nn * nn * nn;
          }
        }
        B.goff[l - 1][n_sys] = acc;
        B.Gtot[l - 1] = acc;
      }
    }
    std::vector<double> K1, S1;
    int W[3] = {0, 0, 0};
    std::vector<std::vector<double>> tops(kMaxLevels + 1);
    std::vector<int> top_len(kMaxLevels + 1, 0);
    if (st == MSM_OK) {
      const double h3[3] = {h, h, h};
      level1_stencil(order, M, cutoff_a, h3, W, K1, B.gcoef, nullptr, B.nu);
      const int R1[3] = {W[0] - M, W[1] - M, W[2] - M};
      level1_samples(order, cutoff_a, h3, R1, B.gcoef, S1, B.nu);
      for (int l = 1; l <= B.Lmax; ++l) {
        int nmax = 0;
        for (int s = 0; s < n_sys; ++s)
          if (B.L[s] == l) nmax = std::max(nmax, B.n[l - 1][s]);
        if (!nmax) continue;
        const double hl = std::ldexp(h, l - 1);
        const double hl3[3] = {hl, hl, hl};
        const int n3[3] = {nmax, nmax, nmax};
        free_top_kernel(order, M, cutoff_a, l, hl3, n3, B.omega, B.gcoef, tops[l], B.nu);
        top_len[l] = 2 * nmax - 1;
      }
      st = precision == MSM_FP64 ? upload_batch<double>(P, K1, W[0], S1, W[0] - M, tops, top_len)
                                 : upload_batch<float>(P, K1, W[0], S1, W[0] - M, tops, top_len);
    }
  } catch (...) {
    st = MSM_ERR_OOM;
  }
  if (st != MSM_OK) {
    msm_plan_destroy(P);
    return st;
  }
  *out = P;
  return MSM_OK;
}

extern "C" msm_status msm_batch_energy_forces(msm_plan plan, const int* offsets, const void* pos,
                                              const void* q, void* ws, double* energies,
                                              void* forces, void* dEdq, void* stream) {
  if (!plan || !plan->batch || !plan->bs) return MSM_ERR_INVALID_ARG;
  if (!offsets || !pos || !q || !energies) return MSM_ERR_INVALID_ARG;
  if (ws) return MSM_ERR_UNSUPPORTED;  // there is no batched backward to save state for
  BatchState& B = *plan->bs;
  hipStream_t s = (hipStream_t)stream;
  const void* key[7] = {offsets, pos, q, energies, forces, dEdq, (const void*)s};
  const char* env = std::getenv("MSM_BATCH_GRAPH");
  const bool use_graph = !(env && env[0] == '0') && !plan->prof.on;
  auto enqueue = [&](hipStream_t st) {
    return B.precision == MSM_FP64
               ? enqueue_batch<double>(plan, offsets, (const double*)pos, (const double*)q,
                                       energies, (double*)forces, (double*)dEdq, st)
               : enqueue_batch<float>(plan, offsets, (const float*)pos, (const float*)q,
                                      energies, (float*)forces, (float*)dEdq, st);
  };
  if (!use_graph) return enqueue(s);
  if (!B.exec || std::memcmp(key, B.key, sizeof(key)) != 0) {
    if (B.exec) {
      (void)hipGraphExecDestroy(B.exec);
      B.exec = nullptr;
    }
    if (B.graph) {
      (void)hipGraphDestroy(B.graph);
      B.graph = nullptr;
    }
    if (hipStreamBeginCapture(B.gstream, hipStreamCaptureModeThreadLocal)) return MSM_ERR_HIP;
    msm_status st = enqueue(B.gstream);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(B.gstream, &g) || st != MSM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st != MSM_OK ? st : MSM_ERR_HIP;
    }
    B.graph = g;
    if (hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0)) {
      B.exec = nullptr;
      return MSM_ERR_HIP;
    }
    std::memcpy(B.key, key, sizeof(key));
  }
  if (hipEventRecord(B.ev_fork, s) || hipStreamWaitEvent(B.gstream, B.ev_fork, 0) ||
      hipGraphLaunch(B.exec, B.gstream) || hipEventRecord(B.ev_join, B.gstream) ||
      hipStreamWaitEvent(s, B.ev_join, 0))
    return MSM_ERR_HIP;
  return MSM_OK;
}

extern "C" msm_status msm_batch_plan_create(msm_plan* out, int n_sys, const double* boxes,
                                            const int* levels, unsigned periodic_mask, int order,
                                            double h, double cutoff_a, int precision,
                                            int max_total_n, int quasi_degree_M) {
  return msm_batch_plan_create_kernel(out, MSM_KERNEL_COULOMB, n_sys, boxes, levels,
                                      periodic_mask, order, h, cutoff_a, precision, max_total_n,
                                      quasi_degree_M);
}

// JSON of the batch plan (systems, grids, autotuner result) for describe.
std::string describe_batch(const msm::BatchState& B) {
  std::ostringstream o;
  o.precision(17);
  long long G1 = B.Gtot[0];
  o << "{\"batch\":true,\"n_sys\":" << B.n_sys << ",\"order\":" << B.p << ",\"M\":" << B.M
    << ",\"h\":" << B.h << ",\"cutoff\":" << B.a << ",\"kernel_power\":" << B.nu
    << ",\"max_levels\":" << B.Lmax
    << ",\"precision\":\"" << (B.precision ? "fp64" : "fp32") << "\",\"grid1_points\":" << G1
    << ",\"tile_cfg\":" << B.tile_cfg << ",\"autotune\":" << (B.tuning.empty() ? "[]" : B.tuning)
    << ",\"convs\":[";
  for (size_t i = 0; i < B.convs.size(); ++i)
    o << (i ? "," : "") << "{\"level\":" << B.convs[i].level << ",\"top\":" << B.convs[i].top
      << ",\"len\":" << B.convs[i].len << ",\"factored\":" << B.convs[i].fact
      << ",\"tasks\":" << B.convs[i].ntasks
      << ",\"tile_cfg\":" << B.convs[i].cfg << "}";
  o << "]}";
  return o.str();
}
