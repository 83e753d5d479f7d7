// api.hip -- the C ABI of libmsm (include/msm.h): plan lifetime, the forward
// pass a1..a9 and its orchestration on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "msm.h"
#include "plan.hpp"
#include "plan_state.hpp"
#include "stencil_fold.hpp"

using namespace msm;

namespace msm {
msm_status hip_alloc(msm_plan P, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return MSM_ERR_OOM;
  }
  P->allocs.push_back(*ptr);
  return MSM_OK;
}
}  // namespace msm

namespace {

template <typename T>
GridDev<T> grid_dev(const HostPlan& hp, int level) {
  const LevelGeom& g = hp.lev[level - 1];
  GridDev<T> d;
  for (int k = 0; k < 3; ++k) {
    d.n[k] = g.n[k];
    d.lo[k] = g.lo[k];
    d.per[k] = hp.periodic[k];
    d.h[k] = (T)g.h[k];
    d.inv_h[k] = (T)(1.0 / g.h[k]);
    d.hd[k] = g.h[k];
  }
  d.tri = hp.tri;
  for (int k = 0; k < 9; ++k) d.Hi[k] = hp.tri ? hp.Hinv[k] : 0.0;
  return d;
}

// Binning parameters: the cell list in the box, or in the unit cube of a
// triclinic cell.
template <typename T>
BinParams<T> bin_params(const HostPlan& hp) {
  BinParams<T> bp;
  for (int k = 0; k < 3; ++k) {
    bp.box[k] = (T)hp.box[k];
    bp.cs[k] = (T)hp.cs[k];
    bp.nc[k] = hp.nc[k];
    bp.per[k] = hp.periodic[k];
  }
  bp.tri = hp.tri;
  for (int k = 0; k < 9; ++k) {
    bp.H[k] = hp.tri ? hp.H[k] : 0.0;
    bp.Hi[k] = hp.tri ? hp.Hinv[k] : 0.0;
  }
  return bp;
}

size_t tsize(const HostPlan& hp) { return hp.precision == MSM_FP64 ? 8 : 4; }

// Saved forward state inside the caller's workspace.
struct WsLayout {
  size_t sorted, perm, start, phi, F, e1, total;
};

WsLayout ws_layout(const msm_plan P, int n) {
  const size_t ts = tsize(P->hp);
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  WsLayout w;
  size_t o = 0;
  w.sorted = o;
  o += al(4 * ts * (size_t)std::max(n, 1));
  w.perm = o;
  o += al(sizeof(int) * (size_t)std::max(n, 1));
  w.start = o;
  o += al(sizeof(int) * (size_t)(P->ncell + 1));
  w.phi = o;
  o += al(ts * (size_t)std::max(n, 1));
  w.F = o;
  o += al(3 * ts * (size_t)std::max(n, 1));
  w.e1 = o;
  o += al(ts * (size_t)P->hp.lev[0].G);
  w.total = o;
  return w;
}

// The stencil of a level as uploaded: radial kernels sampled on offsets
// symmetric about 0 have mirrored z-planes, and the convolution then adds
// the two input planes of a mirrored pair before one pass over the shared
// coefficients (make_planes_mirror).  A periodic table over all n residues
// (n even, offsets -n/2..n/2-1) first gets its plane -n/2 split in two
// halves at -n/2 and +n/2 (the same input plane mod n; halving is exact).
static ConvGeom mirror_stencil(const std::vector<double>& A, const int off[3], const int len[3],
                               bool per_z, int nz, std::vector<double>& B) {
  ConvGeom g;
  for (int k = 0; k < 3; ++k) {
    g.off[k] = off[k];
    g.len[k] = len[k];
  }
  g.fold = 0;
  B = A;
  if (!fold_allowed() || len[2] < 2) return g;
  const size_t plane = (size_t)len[0] * len[1];
  std::vector<double> C;
  int lz = len[2];
  if (per_z && len[2] == nz && nz % 2 == 0 && off[2] == -(nz / 2)) {
    lz = nz + 1;
    C.resize(plane * lz);
    for (size_t i = 0; i < plane; ++i) C[i] = C[plane * nz + i] = 0.5 * A[i];
    std::copy(A.begin() + plane, A.begin() + plane * nz, C.begin() + plane);
  } else {
    C = A;
  }
  if (!make_planes_mirror(C, len[0], len[1], lz)) return g;
  B.swap(C);
  g.len[2] = lz;
  g.fold = 1;
  return g;
}

// Convolution parameters of level l: its direct stencil K, or on a factored
// level its samples S (output on the extended grid), as uploaded.
template <typename T>
static ConvParams level_conv(const msm_plan P, int l, bool samples) {
  const HostPlan& hp = P->hp;
  const LevelGeom& g = hp.lev[l - 1];
  const int zero3[3] = {0, 0, 0};
  const ConvGeom& c = samples ? P->sgeom[l - 1] : P->kgeom[l - 1];
  return samples ? make_conv_params(g.n, g.next, g.shift, hp.periodic, c.off, c.len, sizeof(T),
                                    c.fold)
                 : make_conv_params(g.n, g.n, zero3, hp.periodic, c.off, c.len, sizeof(T), c.fold);
}

// The working memory of calls with up to n particles, carved from base in
// 256-byte aligned pieces (base = null: sizes only); returns its bytes, or 0
// when the cluster slots would not be addressable with 32-bit byte offsets.
template <typename T>
size_t work_layout(const msm_plan P, int n, char* base, WorkBufs* wb) {
  const HostPlan& hp = P->hp;
  const size_t nn = (size_t)std::max(n, 1), nc = (size_t)P->ncell;
  const size_t ncl = (size_t)cluster_capacity((int)nn, P->ncell);
  // cluster slots plus the null j-group, addressed with 32-bit byte offsets
  const size_t slots = ncl * 8 + kGroupSize;
  if (slots * 4 * sizeof(T) >= (size_t(1) << 32)) return 0;
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + o : nullptr;
    o += (std::max(bytes, size_t(16)) + 255) & ~size_t(255);
    return p;
  };
  WorkBufs w;
  for (int l = 1; l <= hp.L; ++l) {
    const LevelGeom& g = hp.lev[l - 1];
    w.qg[l - 1] = take((size_t)g.G * sizeof(T));
    w.eg[l - 1] = take((size_t)g.G * sizeof(T));
    // FP64 accumulation buffer of the level's convolution
    const long long gbuf = std::max(g.G, g.factored ? g.Gext : 0LL);
    w.ug[l - 1] = (double*)take((size_t)gbuf * sizeof(double));
    if (g.factored) w.ut[l - 1] = (double*)take((size_t)g.Gext * sizeof(double));
  }
  w.cell_of = (int*)take(nn * sizeof(int));
  w.rank = (int*)take(nn * sizeof(int));
  w.counts = (int*)take(nc * kCountCopies * sizeof(int));
  w.start = (int*)take((nc + 1) * sizeof(int));
  w.scan_tmp = (int*)take((size_t)scan_tmp_ints(P->ncell) * sizeof(int));
  w.perm = (int*)take(nn * sizeof(int));
  w.wrapped = take(nn * 4 * sizeof(T));
  w.sorted = take(nn * 4 * sizeof(T));
  w.cl_start = (int*)take((nc + 1) * sizeof(int));
  w.cpos = take(slots * 4 * sizeof(T));
  w.cv = take(slots * 4 * sizeof(T));
  w.cbox = take(ncl * 2 * 2 * 4 * sizeof(T));
  w.cinfo = (int4*)take(ncl * sizeof(int4));
  w.phi0 = take(nn * sizeof(double));
  w.F0 = take(nn * 3 * sizeof(T));
  w.null_h = (int)(2 * ncl);
  if (wb) *wb = w;
  return o;
}

// The null j-group (far-away zero charges, zero vectors) and zero cell
// counters: what a call expects of its working memory on entry.
template <typename T>
__global__ void k_prepare_work(vec4_t<T>* cpos_null, vec4_t<T>* cv_null, int* counts,
                               long long ncount) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kGroupSize) {
    vec4_t<T> far, zero;
    far.x = far.y = far.z = T(1e15);
    far.w = T(0);
    zero.x = zero.y = zero.z = zero.w = T(0);
    cpos_null[i] = far;
    cv_null[i] = zero;
  }
  for (long long k = i; k < ncount; k += (long long)gridDim.x * blockDim.x) counts[k] = 0;
}

template <typename T>
msm_status prepare_work(const msm_plan P, const WorkBufs& w, hipStream_t s) {
  const long long ncount = (long long)P->ncell * kCountCopies;
  const int blocks = (int)std::min<long long>(1024, (ncount + 255) / 256 + 1);
  const size_t null_slot = (size_t)w.null_h * kGroupSize;
  hipLaunchKernelGGL(k_prepare_work<T>, dim3(blocks), dim3(256), 0, s,
                     (vec4_t<T>*)w.cpos + null_slot, (vec4_t<T>*)w.cv + null_slot, w.counts,
                     ncount);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

// Uploads every level's stencil (and the k-samples of factored levels) in the
// padded form the convolution reads; fails when a stencil exceeds the
// convolution's LDS window.
// An FP64 stencil [len2][len1][len0] as the convolution reads it: rows
// padded with zeros to conv_row_stride(len0), kConvRowPad zero rows before
// and after every plane, plus the [first, last] non-zero x range of every
// (unpadded) row; mirrored z-planes folded when they are mirrored.
static msm_status upload_padded(msm_plan P, const std::vector<double>& A0, const int off[3],
                                const int len0[3], int nz, double** dA, int2** dext,
                                ConvGeom* cg) {
  const HostPlan& hp = P->hp;
  {
    std::vector<double> A;
    *cg = mirror_stencil(A0, off, len0, hp.periodic[2] != 0, nz, A);
    const int* len = cg->len;
    const int lxp = conv_row_stride(len[0]);
    const int lyp = len[1] + 2 * kConvRowPad;
    const size_t rows = (size_t)len[1] * len[2];
    std::vector<double> pad((size_t)len[2] * lyp * lxp, 0.0);
    std::vector<int2> ext(rows);
    for (int z = 0; z < len[2]; ++z)
      for (int y = 0; y < len[1]; ++y) {
        const size_t r = (size_t)z * len[1] + y;
        const size_t rp = (size_t)z * lyp + y + kConvRowPad;
        int first = len[0], last = -1;
        for (int x = 0; x < len[0]; ++x) {
          const double v = A[r * len[0] + x];
          pad[rp * lxp + x] = v;
          if (v != 0.0) {
            first = std::min(first, x);
            last = x;
          }
        }
        ext[r] = make_int2(first, last);
      }
    msm_status s2;
    if ((s2 = hip_alloc(P, (void**)dA, pad.size() * sizeof(double)))) return s2;
    if ((s2 = hip_alloc(P, (void**)dext, ext.size() * sizeof(int2)))) return s2;
    if (hipMemcpy(*dA, pad.data(), pad.size() * sizeof(double), hipMemcpyHostToDevice) ||
        hipMemcpy(*dext, ext.data(), ext.size() * sizeof(int2), hipMemcpyHostToDevice))
      return MSM_ERR_HIP;
    return MSM_OK;
  }
}

template <typename T>
msm_status upload_stencils(msm_plan P) {
  HostPlan& hp = P->hp;
  msm_status st;
  auto upload_stencil = [&](const std::vector<double>& A0, const int off[3], const int len0[3],
                            int nz, double** dA, int2** dext, ConvGeom* cg) -> msm_status {
    return upload_padded(P, A0, off, len0, nz, dA, dext, cg);
  };
  for (int l = 1; l <= hp.L; ++l) {
    LevelGeom& g = hp.lev[l - 1];
    if ((st = upload_stencil(g.K, g.off, g.len, g.n[2], &P->K64[l - 1], &P->rowext64[l - 1],
                             &P->kgeom[l - 1]))) return st;
    ConvParams cp = level_conv<T>(P, l, false);
    if (conv_lds_bytes(cp, sizeof(T)) > 64 * 1024 || cp.lds_w > kConvMaxLW) return MSM_ERR_GRID;
    if (g.factored) {
      if ((st = upload_stencil(g.S, g.s_off, g.s_len, g.n[2], &P->S[l - 1], &P->srowext[l - 1],
                               &P->sgeom[l - 1]))) return st;
      ConvParams cs = level_conv<T>(P, l, true);
      if (conv_lds_bytes(cs, sizeof(T)) > 64 * 1024 || cs.lds_w > kConvMaxLW) return MSM_ERR_GRID;
    }
  }
  return MSM_OK;
}

template <typename T>
msm_status upload_plan(msm_plan P) {
  HostPlan& hp = P->hp;
  msm_status st;
  if (hipGetDevice(&P->device_id) != hipSuccess) return MSM_ERR_HIP;
  if ((st = upload_stencils<T>(P))) return st;
  T J[9] = {};
  for (int k = 0; k <= hp.p; ++k) J[k] = (T)hp.J[k];
  if ((st = hip_alloc(P, &P->Jd, sizeof(J)))) return st;
  if (hipMemcpy(P->Jd, J, sizeof(J), hipMemcpyHostToDevice)) return MSM_ERR_HIP;
  P->ncell = hp.nc[0] * hp.nc[1] * hp.nc[2];
  for (int k = 0; k < 3; ++k) P->nc_cap[k] = hp.nc[k];
  if ((long long)P->ncell * kCountCopies > (1LL << 30)) return MSM_ERR_GRID;
  {
    const size_t bytes = work_layout<T>(P, std::max(hp.max_n, 1), nullptr, nullptr);
    if (bytes == 0) return MSM_ERR_CAPACITY;
    void* base = nullptr;
    if ((st = hip_alloc(P, &base, bytes))) return st;
    work_layout<T>(P, std::max(hp.max_n, 1), (char*)base, &P->own);
    if ((st = prepare_work<T>(P, P->own, nullptr))) return st;
  }
  if ((st = hip_alloc(P, (void**)&P->flag, sizeof(int)))) return st;
  if (hipMemset(P->flag, 0, sizeof(int))) return MSM_ERR_HIP;
  if (hipStreamCreateWithFlags(&P->sb, hipStreamNonBlocking) ||
      hipStreamCreateWithFlags(&P->sc, hipStreamNonBlocking) ||
      hipStreamCreateWithFlags(&P->sd, hipStreamNonBlocking))
    return MSM_ERR_HIP;
  for (auto& e : P->ev)
    // fork/join events between this plan's streams on one GPU: no timing and
    // no system-scope fence (nothing on the host or another device waits on
    // them; the streams share the device's caches)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence))
      return MSM_ERR_HIP;
  if (hipDeviceSynchronize()) return MSM_ERR_HIP;
  return MSM_OK;
}

void free_plan(msm_plan P) {
  if (!P) return;
  if (P->device) (void)hipDeviceSynchronize();
  if (P->bs) destroy_batch(P->bs);
  for (auto& e : P->ev)
    if (e) (void)hipEventDestroy(e);
  if (P->sb) (void)hipStreamDestroy(P->sb);
  if (P->sc) (void)hipStreamDestroy(P->sc);
  if (P->sd) (void)hipStreamDestroy(P->sd);
  for (void* p : P->allocs) (void)hipFree(p);
  delete P;
}

template <typename T>
PairParams<T> pair_params(const HostPlan& hp) {
  PairParams<T> pp{};
  const int p = hp.p;
  for (int k = 0; k < 3; ++k) {
    pp.box[k] = (T)hp.box[k];
    pp.inv_box[k] = (T)(1.0 / hp.box[k]);
    pp.cs[k] = (T)hp.cs[k];
    pp.per[k] = hp.periodic[k];
    pp.nc[k] = hp.nc[k];
  }
  pp.ncell = hp.nc[0] * hp.nc[1] * hp.nc[2];
  pp.margin = (T)(0.5 * hp.skin);
  pp.nu = hp.nu;
  const double a = hp.a;
  pp.a2 = (T)(a * a);
  pp.inv_a2 = (T)(1.0 / (a * a));
  pp.inv_a = (T)(1.0 / a);
  pp.inv_a3 = (T)(1.0 / (a * a * a));
  pp.inv_a5 = (T)(1.0 / (a * a * a * a * a));
  for (int k = 0; k < 8; ++k) {
    const double c = k < p ? hp.gcoef[k] : 0.0;
    const double dc = (k + 1 < p) ? (k + 1) * hp.gcoef[k + 1] : 0.0;
    const double d2c = (k + 2 < p) ? (k + 2) * (k + 1) * hp.gcoef[k + 2] : 0.0;
    pp.c[k] = (T)c;
    pp.dc[k] = (T)dc;
    pp.d2c[k] = (T)d2c;
    // t^k = r^2k / a^2k, scaled in FP64 before the cast; the kernel r^-nu
    // softens as gamma(r/a)/a^nu
    const double a2k = std::pow(a, 2 * k), anu = std::pow(a, hp.nu);
    pp.er[k] = (T)(c / (a2k * anu));
    pp.fr[k] = (T)(2.0 * dc / (a2k * anu * a * a));
    pp.gr[k] = (T)(4.0 * d2c / (a2k * anu * a * a * a * a));
  }
  pp.tri = hp.tri;
  for (int k = 0; k < 9; ++k) pp.H[k] = hp.tri ? (T)hp.H[k] : T(0);
  return pp;
}

// Accumulators a grid pass adds into atomically (the FP64 convolution
// buffers of levels whose stencil planes are split across workgroups); they
// must be zero when grid_pass starts.
template <typename T>
void grid_zero_jobs(msm_plan P, ZeroJobs& z) {
  const HostPlan& hp = P->hp;
  for (int l = 1; l <= hp.L; ++l) {
    const LevelGeom& g = hp.lev[l - 1];
    const ConvParams cp = level_conv<T>(P, l, g.factored);
    if (cp.nsplit > 1 && z.n < kZeroJobs) {
      z.ptr[z.n] = P->w->ug[l - 1];
      z.words[z.n] = 2 * (g.factored ? g.Gext : g.G);
      z.n += 1;
    }
  }
}

// One level of eq. (u_oneplus_nested_eval): e^l = K^l q~^l, into eg[l-1]
// for a factored level (omega' writes the grid precision) and into the FP64
// buffer ug[l-1] for a direct one (the prolongation that finalises the level
// reads it there).
template <typename T>
void conv_level(msm_plan P, int l, hipStream_t s) {
  const HostPlan& hp = P->hp;
  StageProfiler& pf = P->prof;
  static const char* conv_names[kMaxLevels] = {
      "conv_l1", "conv_l2", "conv_l3", "conv_l4", "conv_l5", "conv_l6", "conv_l7", "conv_l8",
      "conv_l9", "conv_l10", "conv_l11", "conv_l12", "conv_l13", "conv_l14", "conv_l15", "conv_l16"};
  static const char* omega_names[kMaxLevels] = {
      "omega_l1", "omega_l2", "omega_l3", "omega_l4", "omega_l5", "omega_l6",
      "omega_l7", "omega_l8", "omega_l9", "omega_l10", "omega_l11", "omega_l12",
      "omega_l13", "omega_l14", "omega_l15", "omega_l16"};
  const LevelGeom& g = hp.lev[l - 1];
  const char* cname = l == hp.L ? "conv_top" : conv_names[l - 1];
  if (g.factored) {
    // K^l q = omega' * (S^l * q): FP64 sample convolution, then omega' per axis
    ConvParams cs = level_conv<T>(P, l, true);
    int ev = pf.begin(cname, s);
    launch_conv<T, double>(cs, P->S[l - 1], P->srowext[l - 1], (const T*)P->w->qg[l - 1],
                           P->w->ug[l - 1], s);
    pf.end(ev, s);
    OmegaParams op;
    for (int k = 0; k < 3; ++k) {
      op.n[k] = g.n[k];
      op.next[k] = g.next[k];
      op.per[k] = hp.periodic[k];
    }
    op.M = hp.M;
    for (int k = 0; k < 25; ++k) op.omega[k] = k <= hp.M ? hp.omega[k] : 0.0;
    ev = pf.begin(omega_names[l - 1], s);
    launch_omega<T>(op, P->w->ug[l - 1], P->w->ut[l - 1], (T*)P->w->eg[l - 1], s);
    pf.end(ev, s);
  } else {
    // direct stencil, accumulated in FP64 (sums of thousands of terms with
    // cancellation)
    ConvParams cp = level_conv<T>(P, l, false);
    int ev = pf.begin(cname, s);
    launch_conv<T, double>(cp, P->K64[l - 1], P->rowext64[l - 1], (const T*)P->w->qg[l - 1],
                           P->w->ug[l - 1], s);
    pf.end(ev, s);
  }
}

// Nested grid pass of eq. (u_oneplus_nested_eval): from the level-1 grid in
// qg[0] to e^{1+} in eg[0].  Level 1 runs on sa; the coarse branch on sb:
// restriction to level 2, level 2's convolution, then (after the join
// below) prolongation down to level 2.  Below level 2 the restrictions and
// convolutions run on sd beside level 2's convolution (they need only q~^2),
// and join sb before its prolongations.  The branches join sa before the
// last prolongation.  sb == sa (or sd == sb) runs the parts in order.
// Prolongation finalises each level: e^l = (its own convolution output) +
// I e^{l+1}, reading a direct level's output from its FP64 buffer.
template <typename T>
void grid_pass(msm_plan P, hipStream_t sa, hipStream_t sb, hipStream_t sd) {
  const HostPlan& hp = P->hp;
  const int L = hp.L, p = hp.p;
  StageProfiler& pf = P->prof;
  const bool fork = sb != sa && L > 1;
  if (fork) {
    (void)hipEventRecord(P->ev[2], sa);
    (void)hipStreamWaitEvent(sb, P->ev[2], 0);
  }
  // level 1 first: the host enqueues it before the coarse branch's launches,
  // so it starts as soon as anterpolation ends
  conv_level<T>(P, 1, sa);
  hipStream_t sc = fork ? sb : sa;
  if (L > 1) {
    int ev = pf.begin("restrict", sc);
    launch_restrict<T>(p, grid_dev<T>(hp, 1), grid_dev<T>(hp, 2), hp.J, (const T*)P->w->qg[0],
                       (T*)P->w->qg[1], sc);
    pf.end(ev, sc);
  }
  const bool fork2 = fork && sd != sc && L > 2;
  hipStream_t se = fork2 ? sd : sc;
  if (fork2) {
    (void)hipEventRecord(P->ev[4], sc);
    (void)hipStreamWaitEvent(sd, P->ev[4], 0);
  }
  if (L > 1) conv_level<T>(P, 2, sc);
  if (L > 2) {
    int ev = pf.begin("restrict", se);
    for (int l = 2; l < L; ++l)
      launch_restrict<T>(p, grid_dev<T>(hp, l), grid_dev<T>(hp, l + 1), hp.J,
                         (const T*)P->w->qg[l - 1], (T*)P->w->qg[l], se);
    pf.end(ev, se);
  }
  for (int l = 3; l <= L; ++l) conv_level<T>(P, l, se);
  if (fork2) {
    (void)hipEventRecord(P->ev[5], sd);
    (void)hipStreamWaitEvent(sc, P->ev[5], 0);
  }
  // 0-based level l of the output e^l: grid precision in eg[l] for a factored
  // level, FP64 in ug[l] for a direct one (until its prolongation)
  auto coarse_src64 = [&](int l) -> const double* {
    return (l == L - 1 && !hp.lev[l].factored) ? P->w->ug[l] : nullptr;
  };
  auto fine_src64 = [&](int l) -> const double* {
    return hp.lev[l].factored ? nullptr : P->w->ug[l];
  };
  int ev = pf.begin("prolong", sc);
  for (int l = L - 2; l >= 1; --l)
    launch_prolong<T>(p, grid_dev<T>(hp, l + 1), grid_dev<T>(hp, l + 2), hp.J,
                      (const T*)P->w->eg[l + 1], coarse_src64(l + 1), (T*)P->w->eg[l],
                      fine_src64(l), sc);
  pf.end(ev, sc);
  if (fork) {
    (void)hipEventRecord(P->ev[3], sb);
    (void)hipStreamWaitEvent(sa, P->ev[3], 0);
  }
  if (L > 1) {
    ev = pf.begin("prolong", sa);
    launch_prolong<T>(p, grid_dev<T>(hp, 1), grid_dev<T>(hp, 2), hp.J, (const T*)P->w->eg[1],
                      coarse_src64(1), (T*)P->w->eg[0], fine_src64(0), sa);
    pf.end(ev, sa);
  } else if (!hp.lev[0].factored) {
    int e2 = pf.begin("grid_cast", sa);
    launch_cast<T>(P->w->ug[0], (T*)P->w->eg[0], hp.lev[0].G, sa);
    pf.end(e2, sa);
  }
}

// Whether a call runs as a DAG over four streams (MSM_STREAMS=0: one; read
// on every call).  A call recorded into a graph (the caller's stream is
// capturing) stays on the caller's stream: a capture of the four-stream
// fork and join ended in a crash inside the runtime's end of capture, so
// graphs hold the one-stream sequence.
static bool use_streams(hipStream_t s) {
  const char* e = getenv("MSM_STREAMS");
  if (e && atoi(e) == 0) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusNone;
}

template <typename T>
msm_status forward(msm_plan P, int n, const T* pos, const T* q, void* ws, double* energy, T* F,
                   T* dEdq, hipStream_t s) {
  const HostPlan& hp = P->hp;
  const int L = hp.L, p = hp.p;
  // where the cell list goes: the caller's workspace if given (saved state)
  vec4_t<T>* sorted = (vec4_t<T>*)P->w->sorted;
  int* perm = P->w->perm;
  int* start = P->w->start;
  T* save_phi = nullptr;
  T* save_F = nullptr;
  T* save_e1 = nullptr;
  if (ws) {
    WsLayout w = ws_layout(P, n);
    char* b = (char*)ws;
    sorted = (vec4_t<T>*)(b + w.sorted);
    perm = (int*)(b + w.perm);
    start = (int*)(b + w.start);
    save_phi = (T*)(b + w.phi);
    save_F = (T*)(b + w.F);
    save_e1 = (T*)(b + w.e1);
  }
  StageProfiler& pf = P->prof;
  // accumulators of the pass, cleared by the binning's scatter (a kernel,
  // not a memset: graph-safe); the cell counters are zero on entry
  const GridDev<T> g1 = grid_dev<T>(hp, 1);
  CellGrid cg;
  for (int k = 0; k < 3; ++k) {
    cg.nc[k] = hp.nc[k];
    cg.cs[k] = hp.cs[k];
  }
  cg.margin = 0.5 * hp.skin;
  ZeroJobs z;
  z.n = 0;
  if (!anterp_tiled(p, n, cg, g1.n, g1.per, g1.hd)) {  // (tiles write every value)
    z.ptr[z.n] = P->w->qg[0];
    z.words[z.n++] = hp.lev[0].G * (long long)(sizeof(T) / 4);
  }
  z.ptr[z.n] = energy;
  z.words[z.n++] = 2;
  grid_zero_jobs<T>(P, z);

  // a1 binning (cell counts, scans of cell starts and cluster offsets,
  // scatter), then Morton order inside cells and the 8-particle clusters
  const BinParams<T> bp = bin_params<T>(hp);
  // Verlet skin: the device decides whether this call rebuilds the cell
  // list; a new n or a call that keeps its list in a workspace always does,
  // and the call after one with a workspace too
  SkinDev<T> sk{};
  int force = 0;
  if (hp.skin > 0 && P->skin_state) {
    sk.state = P->skin_state;
    sk.ref = (vec4_t<T>*)P->skin_ref;
    sk.shift = (vec4_t<T>*)P->skin_shift;
    sk.half2 = (T)(0.25 * hp.skin * hp.skin);
    sk.keep_force = ws ? 1 : 0;
    force = (n != P->skin_n || ws) ? 1 : 0;
    P->skin_n = n;
  }
  int ev = pf.begin("bin", s);
  launch_binning<T>(n, pos, q, bp, P->ncell, P->w->cell_of, P->w->rank, P->w->counts,
                    (vec4_t<T>*)P->w->wrapped, start, P->w->cl_start, sorted, perm, P->flag,
                    P->w->scan_tmp, z, sk, force, s);
  pf.end(ev, s);
  ev = pf.begin("cluster", s);
  launch_cluster_layout<T>(1, 0, P->ncell, start, P->w->cl_start, bp, (const vec4_t<T>*)P->w->wrapped,
                           sorted, perm, (vec4_t<T>*)P->w->cpos, (vec4_t<T>*)P->w->cbox, P->w->cinfo,
                           P->w->counts, sk.state, n, s);
  pf.end(ev, s);

  // a2 short-range pairs (i-clusters against culled j particles), on its
  // own stream: it only needs the cluster layout, and interpolation waits
  // for it
  const bool dag = use_streams(s);
  hipStream_t sp = dag ? P->sc : s;
  if (dag) {
    (void)hipEventRecord(P->ev[0], s);
    (void)hipStreamWaitEvent(sp, P->ev[0], 0);
  }
  const PairParams<T> pp = pair_params<T>(hp);
  ev = pf.begin("pair", sp);
  launch_pair_cl<T>(p, n, P->ncell, P->w->cl_start, (const vec4_t<T>*)P->w->cpos,
                    (const vec4_t<T>*)P->w->cbox, P->w->cinfo, pp, (double*)P->w->phi0, (T*)P->w->F0, sp);
  pf.end(ev, sp);
  if (dag) (void)hipEventRecord(P->ev[1], sp);

  // a3 anterpolation onto level 1
  ev = pf.begin("anterp", s);
  launch_anterp<T>(p, n, P->ncell, start, cg, sorted, g1, (T*)P->w->qg[0], s);
  pf.end(ev, s);
  // a4 restriction, a5 per-level stencils, a6 top level, a7 prolongation
  grid_pass<T>(P, s, dag ? P->sb : s, dag ? P->sd : s);
  if (dag) (void)hipStreamWaitEvent(s, P->ev[1], 0);
  // a8 + a9 interpolation, combination, energy
  ev = pf.begin("interp", s);
  launch_interp<T>(p, n, sorted, perm, g1, (const T*)P->w->eg[0], (const double*)P->w->phi0,
                   (const T*)P->w->F0, hp.self_const, dEdq, F, save_phi, save_F, energy, s);
  pf.end(ev, s);
  if (save_e1)
    if (hipMemcpyAsync(save_e1, P->w->eg[0], sizeof(T) * hp.lev[0].G, hipMemcpyDeviceToDevice, s))
      return MSM_ERR_HIP;
  if (hipGetLastError() != hipSuccess) return MSM_ERR_HIP;
  return MSM_OK;
}

template <typename T>
msm_status backward(msm_plan P, int n, const void* ws, const double* gE, const T* gF,
                    const T* gphi, T* grad_pos, T* grad_q, hipStream_t s) {
  const HostPlan& hp = P->hp;
  const int p = hp.p;
  WsLayout w = ws_layout(P, n);
  const char* b = (const char*)ws;
  const vec4_t<T>* sorted = (const vec4_t<T>*)(b + w.sorted);
  const int* perm = (const int*)(b + w.perm);
  const int* start = (const int*)(b + w.start);
  const T* save_phi = (const T*)(b + w.phi);
  const T* save_F = (const T*)(b + w.F);
  const T* save_e1 = (const T*)(b + w.e1);
  StageProfiler& pf = P->prof;
  if (!gF && !gphi) {
    int ev = pf.begin("bwd_energy_only", s);
    launch_grad_energy_only<T>(n, perm, save_phi, save_F, gE, grad_q, grad_pos, s);
    pf.end(ev, s);
    return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
  }
  vec4_t<T>* v = (vec4_t<T>*)P->w->wrapped;  // cotangent in cell order
  T* gq_sr = (T*)P->w->phi0;
  T* gr_sr = (T*)P->w->F0;
  int ev = pf.begin("bwd_layout", s);
  launch_gather_v<T>(n, perm, gF, gphi, grid_dev<T>(hp, 1), v, s);
  {
    // cluster layout of the saved (already Morton-ordered) cell list
    const BinParams<T> bp = bin_params<T>(hp);
    launch_cluster_layout<T>(0, 1, P->ncell, start, P->w->cl_start, bp, nullptr,
                             const_cast<vec4_t<T>*>(sorted), const_cast<int*>(perm),
                             (vec4_t<T>*)P->w->cpos, (vec4_t<T>*)P->w->cbox, P->w->cinfo, nullptr,
                             nullptr, n, s);
  }
  pf.end(ev, s);
  // the pair-sum VJP beside the grid part (as in the forward)
  const bool dag = use_streams(s);
  hipStream_t sp = dag ? P->sc : s;
  if (dag) {
    (void)hipEventRecord(P->ev[0], s);
    (void)hipStreamWaitEvent(sp, P->ev[0], 0);
  }
  ev = pf.begin("bwd_pair", sp);
  launch_pair_vjp_cl<T>(p, n, P->ncell, P->w->cl_start, P->w->cinfo, perm, gF, gphi,
                        (const vec4_t<T>*)P->w->cpos, (vec4_t<T>*)P->w->cv, (const vec4_t<T>*)P->w->cbox,
                        pair_params<T>(hp), P->w->null_h, gq_sr, gr_sr, sp);
  pf.end(ev, sp);
  if (dag) (void)hipEventRecord(P->ev[1], sp);
  const GridDev<T> g1 = grid_dev<T>(hp, 1);
  ev = pf.begin("bwd_anterp", s);
  {
    ZeroJobs z;
    z.n = 0;
    z.ptr[z.n] = P->w->qg[0];
    z.words[z.n++] = hp.lev[0].G * (long long)(sizeof(T) / 4);
    grid_zero_jobs<T>(P, z);
    launch_zero_multi(z, s);
  }
  {
    CellGrid cg;
    for (int k = 0; k < 3; ++k) {
      cg.nc[k] = hp.nc[k];
      cg.cs[k] = hp.cs[k];
    }
    cg.margin = 0.5 * hp.skin;
    launch_anterp_dipole<T>(p, n, P->ncell, start, cg, sorted, v, g1, (T*)P->w->qg[0], s);
  }
  pf.end(ev, s);
  grid_pass<T>(P, s, dag ? P->sb : s, dag ? P->sd : s);  // eg[0] = (A D)^{1+}
  if (dag) (void)hipStreamWaitEvent(s, P->ev[1], 0);
  ev = pf.begin("bwd_interp", s);
  launch_interp_vjp<T>(p, n, sorted, v, perm, g1, save_e1, (const T*)P->w->eg[0], save_phi, save_F,
                       gq_sr, gr_sr, gE, hp.self_const, grad_q, grad_pos, s);
  pf.end(ev, s);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

msm_status create_common(msm_plan* out, const double box[3], unsigned mask, int order, double h,
                         double a, int levels, int precision, int max_n, int M, bool device,
                         const double* cell = nullptr, int nu = 1) {
  if (!out) return MSM_ERR_INVALID_ARG;
  *out = nullptr;
  msm_plan P = new (std::nothrow) msm_plan_s;
  if (!P) return MSM_ERR_OOM;
  int rc;
  try {
    rc = build_host_plan(P->hp, box, mask, order, h, a, levels, precision, max_n, M, cell,
                         nullptr, 0.0, nu);
  } catch (...) {
    rc = MSM_ERR_OOM;
  }
  if (rc != MSM_OK) {
    delete P;
    return (msm_status)rc;
  }
  if (device) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      delete P;
      return MSM_ERR_HIP;
    }
    P->device = true;
    msm_status st;
    try {
      st = precision == MSM_FP64 ? upload_plan<double>(P) : upload_plan<float>(P);
    } catch (...) {
      st = MSM_ERR_OOM;
    }
    if (st != MSM_OK) {
      free_plan(P);
      return st;
    }
  }
  *out = P;
  return MSM_OK;
}

// Frees one device buffer of the plan (and forgets it).
void free_plan_buffer(msm_plan P, void* ptr) {
  if (!ptr) return;
  for (size_t k = 0; k < P->allocs.size(); ++k)
    if (P->allocs[k] == ptr) {
      (void)hipFree(ptr);
      P->allocs.erase(P->allocs.begin() + k);
      return;
    }
}

// A new cell for a triclinic plan: the grids keep their point counts (so the
// spacings follow the cell) and the cell list its size (fewer cells per axis
// if the new cell is thinner); stencils and the top-level table are rebuilt
// from the new cell on the host and uploaded again.
template <typename T>
msm_status set_cell(msm_plan P, const double cell[9]) {
  const HostPlan& old = P->hp;
  int ntop[3];
  for (int k = 0; k < 3; ++k) ntop[k] = old.lev[old.L - 1].n[k];
  HostPlan hp;
  int rc;
  try {
    rc = build_host_plan(hp, nullptr, 7, old.p, old.h_req, old.a, old.L, old.precision, old.max_n,
                         old.M, cell, ntop, old.skin, old.nu);
  } catch (...) {
    rc = MSM_ERR_OOM;
  }
  if (rc != MSM_OK) return (msm_status)rc;
  for (int k = 0; k < 3; ++k) {  // the cell list never grows past its buffers
    if (hp.nc[k] > P->nc_cap[k]) hp.nc[k] = P->nc_cap[k];
    hp.cs[k] = hp.box[k] / hp.nc[k];
  }
  if (P->skin_state) {  // the next call rebuilds the cell list
    const int one = 1;
    if (hipDeviceSynchronize() ||
        hipMemcpy(P->skin_state + kSkinForce, &one, sizeof(int), hipMemcpyHostToDevice))
      return MSM_ERR_HIP;
  }
  for (int l = 1; l <= hp.L; ++l) hp.lev[l - 1].factored = old.lev[l - 1].factored;
  if (hipDeviceSynchronize() != hipSuccess) return MSM_ERR_HIP;
  for (int l = 0; l < old.L; ++l) {
    free_plan_buffer(P, P->K64[l]);
    free_plan_buffer(P, P->rowext64[l]);
    free_plan_buffer(P, P->S[l]);
    free_plan_buffer(P, P->srowext[l]);
    P->K64[l] = nullptr;
    P->rowext64[l] = nullptr;
    P->S[l] = nullptr;
    P->srowext[l] = nullptr;
  }
  // the cell-derivative stencils follow the cell (rebuilt at the next such call)
  for (int l = 0; l < kMaxLevels; ++l)
    for (int k = 0; k < 6; ++k) {
      free_plan_buffer(P, P->TS[l][k]);
      free_plan_buffer(P, P->TSext[l][k]);
      P->TS[l][k] = nullptr;
      P->TSext[l][k] = nullptr;
    }
  for (int k = 0; k < 9; ++k) {
    free_plan_buffer(P, P->dKd[k]);
    free_plan_buffer(P, P->dKext[k]);
    P->dKd[k] = nullptr;
    P->dKext[k] = nullptr;
  }
  P->stress_ready = false;
  P->hp = hp;
  P->ncell = hp.nc[0] * hp.nc[1] * hp.nc[2];
  return upload_stencils<T>(P);
}

// Cell derivative of a triclinic plan, dE/dH at fixed Cartesian positions
// (H with the lattice vectors as columns): at fixed fractional coordinates s
// the grid charges do not move and
//   dE/dH|_s = (V0 + sum_{l<L} V_l) H^{-T} + dE_L/dH,
// V0 = -1/2 sum_i q_i sum_j q_j f(r) d d^T (the short-range virial),
// V_l = 1/2 sum_m q~_m (T^l * w)_m with w = omega' * q~^l (the level's
// derivative stencils), dE_L/dH = 1/2 sum_m q~^L_m (dK^L * q~^L)_m; then
// dE/dH|_r = dE/dH|_s + sum_i F_i s_i^T.  The stencils are built and uploaded
// on the first call after a cell change.
template <typename T>
msm_status stress_setup(msm_plan P) {
  if (P->stress_ready) return MSM_OK;
  const HostPlan& hp = P->hp;
  const int zero3[3] = {0, 0, 0};
  msm_status st;
  auto check = [&](const LevelGeom& g, const ConvGeom& c) -> msm_status {
    ConvParams cp = make_conv_params(g.n, g.n, zero3, hp.periodic, c.off, c.len, sizeof(T), c.fold);
    if (conv_lds_bytes(cp, sizeof(T)) > 64 * 1024 || cp.lds_w > kConvMaxLW) return MSM_ERR_GRID;
    return MSM_OK;
  };
  try {
    for (int l = 1; l < hp.L; ++l) {
      const LevelGeom& g = hp.lev[l - 1];
      std::vector<double> Tv[6];
      cell_stress_stencils(hp, l, Tv);
      for (int k = 0; k < 6; ++k) {
        if ((st = upload_padded(P, Tv[k], g.s_off, g.s_len, g.n[2], &P->TS[l - 1][k],
                                &P->TSext[l - 1][k], &P->tsgeom[l - 1][k])))
          return st;
        if ((st = check(g, P->tsgeom[l - 1][k]))) return st;
      }
    }
    std::vector<double> dK[9];
    const int rc = top_cell_derivative(hp, dK);
    if (rc != MSM_OK) return (msm_status)rc;
    const LevelGeom& gL = hp.lev[hp.L - 1];
    for (int k = 0; k < 9; ++k) {
      if ((st = upload_padded(P, dK[k], gL.off, gL.len, gL.n[2], &P->dKd[k], &P->dKext[k],
                              &P->dkgeom[k])))
        return st;
      if ((st = check(gL, P->dkgeom[k]))) return st;
    }
  } catch (...) {
    return MSM_ERR_OOM;
  }
  if (!P->sgrid) {  // u, t, y (FP64) and w (plan precision) of level 1's size, then 30 sums
    const size_t G1 = (size_t)hp.lev[0].G;
    if ((st = hip_alloc(P, (void**)&P->sgrid, sizeof(double) * (4 * G1 + 32)))) return st;
    if ((st = hip_alloc(P, (void**)&P->cellm, 9 * sizeof(double)))) return st;
  }
  if (hipMemcpy(P->cellm, hp.Hinv, 9 * sizeof(double), hipMemcpyHostToDevice)) return MSM_ERR_HIP;
  P->stress_ready = true;
  return MSM_OK;
}

template <typename T>
msm_status cell_gradient(msm_plan P, int n, const T* pos, const T* q, double* energy, T* F,
                         T* dEdq, double* dEdH, hipStream_t s) {
  msm_status st = stress_setup<T>(P);
  if (st != MSM_OK) return st;
  if ((st = forward<T>(P, n, pos, q, nullptr, energy, F, dEdq, s))) return st;
  const HostPlan& hp = P->hp;
  const int zero3[3] = {0, 0, 0};
  const long long G1 = hp.lev[0].G;
  double* u = P->sgrid;
  double* t = u + G1;
  double* y = t + G1;
  T* w = reinterpret_cast<T*>(y + G1);
  double* acc = u + 4 * G1;
  launch_fill<double>(acc, 30, 0.0, s);
  // short-range virial (the forward's cluster layout)
  launch_pair_virial<T>(hp.p, n, P->ncell, P->w->cl_start, (const vec4_t<T>*)P->w->cpos,
                        (const vec4_t<T>*)P->w->cbox, P->w->cinfo, pair_params<T>(hp), acc, s);
  // levels 1..L-1: w = omega' * q~, then six derivative stencils on w
  for (int l = 1; l < hp.L; ++l) {
    const LevelGeom& g = hp.lev[l - 1];
    const T* qg = (const T*)P->w->qg[l - 1];
    launch_to_double<T>(qg, u, g.G, s);
    OmegaParams op;
    for (int k = 0; k < 3; ++k) {
      op.n[k] = g.n[k];
      op.next[k] = g.n[k];
      op.per[k] = 1;
    }
    op.M = hp.M;
    for (int k = 0; k < 25; ++k) op.omega[k] = k <= hp.M ? hp.omega[k] : 0.0;
    launch_omega<T>(op, u, t, w, s);
    for (int k = 0; k < 6; ++k) {
      const ConvGeom& c = P->tsgeom[l - 1][k];
      ConvParams cp = make_conv_params(g.n, g.n, zero3, hp.periodic, c.off, c.len, sizeof(T), c.fold);
      if (cp.nsplit > 1) launch_fill<double>(y, g.G, 0.0, s);
      launch_conv<T, double>(cp, P->TS[l - 1][k], P->TSext[l - 1][k], w, y, s);
      launch_dot<T>(qg, y, g.G, acc + 6 + k, s);
    }
  }
  // top level: dK^L/dH_rc on q~^L
  {
    const LevelGeom& g = hp.lev[hp.L - 1];
    const T* qg = (const T*)P->w->qg[hp.L - 1];
    for (int k = 0; k < 9; ++k) {
      const ConvGeom& c = P->dkgeom[k];
      ConvParams cp = make_conv_params(g.n, g.n, zero3, hp.periodic, c.off, c.len, sizeof(T), c.fold);
      if (cp.nsplit > 1) launch_fill<double>(y, g.G, 0.0, s);
      launch_conv<T, double>(cp, P->dKd[k], P->dKext[k], qg, y, s);
      launch_dot<T>(qg, y, g.G, acc + 12 + k, s);
    }
  }
  // the particles' term, then the combination
  launch_cell_fs<T>(n, pos, F, P->cellm, acc + 21, s);
  launch_cell_combine(acc, P->cellm, dEdH, s);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

// Working memory of msm_energy_forces_noalloc: one array per GPU, held from
// the library's load until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex scratch_mutex;
void* scratch_ptr[kScratchDevices] = {};

msm_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kScratchDevices) return MSM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MSM_ERR_HIP;
    }
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return MSM_OK;
}

template <typename T>
msm_status forward_noalloc(msm_plan P, int n, const T* pos, const T* q, void* ws,
                           double* energy, T* F, T* dEdq, hipStream_t s) {
  if (P->hp.skin > 0) return MSM_ERR_UNSUPPORTED;  // (its cell list lives in the plan)
  const size_t need = work_layout<T>(P, n, nullptr, nullptr);
  if (need == 0 || need > kScratchBytes) return MSM_ERR_CAPACITY;
  void* base = nullptr;
  msm_status st = scratch_address(P->device_id, &base);
  if (st != MSM_OK) return st;
  WorkBufs w;
  work_layout<T>(P, n, (char*)base, &w);
  if ((st = prepare_work<T>(P, w, s))) return st;
  // no stage events either (their creation would allocate)
  const bool prof = P->prof.on;
  P->prof.on = false;
  P->w = &w;
  st = forward<T>(P, n, pos, q, ws, energy, F, dEdq, s);
  P->w = &P->own;
  P->prof.on = prof;
  return st;
}

}  // namespace

extern "C" {

msm_status msm_plan_create(msm_plan* out, const double box[3], unsigned periodic_mask, int order,
                           double h, double cutoff_a, int levels, int precision, int max_n,
                           int quasi_degree_M) {
  return create_common(out, box, periodic_mask, order, h, cutoff_a, levels, precision, max_n,
                       quasi_degree_M, true);
}

msm_status msm_plan_create_kernel(msm_plan* out, int kernel, const double box[3],
                                  unsigned periodic_mask, int order, double h, double cutoff_a,
                                  int levels, int precision, int max_n, int quasi_degree_M) {
  if (kernel != MSM_KERNEL_COULOMB && kernel != MSM_KERNEL_DISPERSION) {
    if (out) *out = nullptr;
    return MSM_ERR_INVALID_ARG;
  }
  return create_common(out, box, periodic_mask, order, h, cutoff_a, levels, precision, max_n,
                       quasi_degree_M, true, nullptr, kernel);
}

msm_status msm_plan_create_cell(msm_plan* out, const double cell[9], unsigned periodic_mask,
                                int order, double h, double cutoff_a, int levels, int precision,
                                int max_n, int quasi_degree_M) {
  if (!cell) return MSM_ERR_INVALID_ARG;
  return create_common(out, nullptr, periodic_mask, order, h, cutoff_a, levels, precision, max_n,
                       quasi_degree_M, true, cell);
}

msm_status msm_plan_create_cell_kernel(msm_plan* out, int kernel, const double cell[9],
                                       unsigned periodic_mask, int order, double h,
                                       double cutoff_a, int levels, int precision, int max_n,
                                       int quasi_degree_M) {
  if (kernel != MSM_KERNEL_COULOMB && kernel != MSM_KERNEL_DISPERSION) {
    if (out) *out = nullptr;
    return MSM_ERR_INVALID_ARG;
  }
  if (!cell) return MSM_ERR_INVALID_ARG;
  return create_common(out, nullptr, periodic_mask, order, h, cutoff_a, levels, precision, max_n,
                       quasi_degree_M, true, cell, kernel);
}

msm_status msm_plan_set_cell(msm_plan plan, const double cell[9]) {
  if (!plan || plan->batch || !cell || !plan->hp.tri) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  return plan->hp.precision == MSM_FP64 ? set_cell<double>(plan, cell) : set_cell<float>(plan, cell);
}

msm_status msm_energy_forces_cell_gradient(msm_plan plan, int n, const void* pos, const void* q,
                                           double* energy, void* forces, void* dEdq,
                                           double* dEdH, void* stream) {
  if (!plan || plan->batch) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  if (!plan->hp.tri) return MSM_ERR_UNSUPPORTED;
  if (n < 0 || !energy || !forces || !dEdH || (n > 0 && (!pos || !q))) return MSM_ERR_INVALID_ARG;
  if (n > plan->hp.max_n) return MSM_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  if (plan->hp.precision == MSM_FP64)
    return cell_gradient<double>(plan, n, (const double*)pos, (const double*)q, energy,
                                 (double*)forces, (double*)dEdq, dEdH, s);
  return cell_gradient<float>(plan, n, (const float*)pos, (const float*)q, energy, (float*)forces,
                              (float*)dEdq, dEdH, s);
}

msm_status msm_plan_set_skin(msm_plan plan, double skin) {
  if (!plan || plan->batch || !(skin >= 0) || !std::isfinite(skin)) return MSM_ERR_INVALID_ARG;
  HostPlan& hp = plan->hp;
  if (!plan->device) {  // a host plan: the cell-list geometry only
    hp.skin = skin;
    cell_list_geometry(hp);
    return MSM_OK;
  }
  const size_t vec = (size_t)std::max(hp.max_n, 1) * 4 *
                     (hp.precision == MSM_FP64 ? sizeof(double) : sizeof(float));
  if (skin > 0 && !plan->skin_state) {
    msm_status st;
    if ((st = hip_alloc(plan, (void**)&plan->skin_state, 4 * sizeof(int))) ||
        (st = hip_alloc(plan, &plan->skin_ref, vec)) ||
        (st = hip_alloc(plan, &plan->skin_shift, vec)))
      return st;
  }
  if (hipDeviceSynchronize() != hipSuccess) return MSM_ERR_HIP;
  hp.skin = skin;
  cell_list_geometry(hp);
  for (int k = 0; k < 3; ++k) {  // the cell list never grows past its buffers
    if (hp.nc[k] > plan->nc_cap[k]) hp.nc[k] = plan->nc_cap[k];
    hp.cs[k] = hp.box[k] / hp.nc[k];
  }
  plan->ncell = hp.nc[0] * hp.nc[1] * hp.nc[2];
  if (plan->skin_state) {
    const int init[4] = {1, 1, 0, 0};  // force a rebuild; no calls yet
    if (hipMemcpy(plan->skin_state, init, sizeof(init), hipMemcpyHostToDevice))
      return MSM_ERR_HIP;
  }
  return MSM_OK;
}

msm_status msm_plan_skin_stats(msm_plan plan, long long* calls, long long* rebuilds,
                               void* stream) {
  if (!plan || plan->batch || !calls || !rebuilds) return MSM_ERR_INVALID_ARG;
  *calls = *rebuilds = 0;
  if (!plan->skin_state) return MSM_OK;
  int st[4];
  if (hipStreamSynchronize((hipStream_t)stream) ||
      hipMemcpy(st, plan->skin_state, sizeof(st), hipMemcpyDeviceToHost))
    return MSM_ERR_HIP;
  *calls = (unsigned)st[kSkinCalls];
  *rebuilds = (unsigned)st[kSkinRebuilds];
  return MSM_OK;
}

msm_status msm_plan_create_host(msm_plan* out, const double box[3], unsigned periodic_mask,
                                int order, double h, double cutoff_a, int levels, int precision,
                                int max_n, int quasi_degree_M) {
  return create_common(out, box, periodic_mask, order, h, cutoff_a, levels, precision, max_n,
                       quasi_degree_M, false);
}

msm_status msm_plan_destroy(msm_plan plan) {
  if (!plan) return MSM_ERR_INVALID_ARG;
  free_plan(plan);
  return MSM_OK;
}

msm_status msm_plan_describe(msm_plan plan, char* json, size_t cap) {
  if (!plan || !json || cap == 0) return MSM_ERR_INVALID_ARG;
  std::string s;
  try {
    s = plan->batch ? describe_batch(*plan->bs) : describe_json(plan->hp);
  } catch (...) {
    return MSM_ERR_OOM;
  }
  if (s.size() + 1 > cap) {
    json[0] = 0;
    return MSM_ERR_INVALID_ARG;
  }
  std::memcpy(json, s.c_str(), s.size() + 1);
  return MSM_OK;
}

msm_status msm_plan_get_stencil(msm_plan plan, int level, int dims_off[6], double* K, size_t cap) {
  if (!plan || !dims_off || level < 1 || level > plan->hp.L || plan->batch)
    return MSM_ERR_INVALID_ARG;
  const LevelGeom& g = plan->hp.lev[level - 1];
  for (int k = 0; k < 3; ++k) {
    dims_off[k] = g.len[k];
    dims_off[3 + k] = g.off[k];
  }
  if (K) {
    if (cap < g.K.size()) return MSM_ERR_INVALID_ARG;
    std::memcpy(K, g.K.data(), g.K.size() * sizeof(double));
  }
  return MSM_OK;
}

msm_status msm_plan_grid_dims(msm_plan plan, int level, int n[3]) {
  if (!plan || !n || level < 1 || level > plan->hp.L || plan->batch) return MSM_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k) n[k] = plan->hp.lev[level - 1].n[k];
  return MSM_OK;
}

size_t msm_workspace_bytes(msm_plan plan, int n, int flags) {
  if (!plan || n < 0 || plan->batch || flags != 0) return 0;
  return ws_layout(plan, n).total;
}

msm_status msm_energy_forces(msm_plan plan, int n, const void* pos, const void* q, void* ws,
                             double* energy, void* forces, void* dEdq, void* stream) {
  if (!plan || plan->batch) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  if (n < 0 || !energy || (n > 0 && (!pos || !q))) return MSM_ERR_INVALID_ARG;
  if (n > plan->hp.max_n) return MSM_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  if (plan->hp.precision == MSM_FP64)
    return forward<double>(plan, n, (const double*)pos, (const double*)q, ws, energy,
                           (double*)forces, (double*)dEdq, s);
  return forward<float>(plan, n, (const float*)pos, (const float*)q, ws, energy, (float*)forces,
                        (float*)dEdq, s);
}

msm_status msm_energy_forces_noalloc(msm_plan plan, int n, const void* pos, const void* q,
                                     void* ws, double* energy, void* forces, void* dEdq,
                                     void* stream) {
  if (!plan || plan->batch) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  if (n < 0 || !energy || (n > 0 && (!pos || !q))) return MSM_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device_id) return MSM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (plan->hp.precision == MSM_FP64)
    return forward_noalloc<double>(plan, n, (const double*)pos, (const double*)q, ws, energy,
                                   (double*)forces, (double*)dEdq, s);
  return forward_noalloc<float>(plan, n, (const float*)pos, (const float*)q, ws, energy,
                                (float*)forces, (float*)dEdq, s);
}

msm_status msm_backward_full(msm_plan plan, int n, const void* pos, const void* q,
                             const void* ws, const double* gE, const void* gF, const void* gdEdq,
                             void* grad_pos, void* grad_q, void* stream) {
  (void)pos;
  (void)q;
  if (!plan || plan->batch) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  if (n < 0 || !ws) return MSM_ERR_INVALID_ARG;
  if (n > plan->hp.max_n) return MSM_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  if (plan->hp.precision == MSM_FP64)
    return backward<double>(plan, n, ws, gE, (const double*)gF, (const double*)gdEdq,
                            (double*)grad_pos, (double*)grad_q, s);
  return backward<float>(plan, n, ws, gE, (const float*)gF, (const float*)gdEdq,
                         (float*)grad_pos, (float*)grad_q, s);
}

msm_status msm_backward(msm_plan plan, int n, const void* pos, const void* q, const void* ws,
                        const double* gE, const void* gF, void* grad_pos, void* grad_q,
                        void* stream) {
  return msm_backward_full(plan, n, pos, q, ws, gE, gF, nullptr, grad_pos, grad_q, stream);
}

msm_status msm_plan_status(msm_plan plan, void* stream) {
  if (!plan) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  hipStream_t s = (hipStream_t)stream;
  int f = 0;
  if (hipStreamSynchronize(s) != hipSuccess) return MSM_ERR_HIP;
  if (hipMemcpy(&f, plan->flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return MSM_ERR_HIP;
  if (f) {
    if (hipMemset(plan->flag, 0, sizeof(int)) != hipSuccess) return MSM_ERR_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return MSM_ERR_HIP;
  }
  if (f & kFlagOffsets) return MSM_ERR_INVALID_ARG;
  if (f & kFlagNonfinite) return MSM_ERR_NONFINITE;
  if (f & kFlagDomain) return MSM_ERR_OUT_OF_DOMAIN;
  return MSM_OK;
}

msm_status msm_plan_get_grid(msm_plan plan, int level, int which, void* dst, void* stream) {
  if (!plan || plan->batch || !dst || level < 1 || level > plan->hp.L || (which != 0 && which != 1))
    return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  const HostPlan& hp = plan->hp;
  const long long G = hp.lev[level - 1].G;
  if (which == 1 && level == hp.L && hp.L > 1 && !hp.lev[level - 1].factored) {
    // the top level's potential lives in its FP64 buffer (prolongation reads
    // it there); hand it out in the grid precision
    if (hp.precision == MSM_FP64) launch_cast<double>(plan->w->ug[level - 1], (double*)dst, G, (hipStream_t)stream);
    else launch_cast<float>(plan->w->ug[level - 1], (float*)dst, G, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
  }
  const void* src = which == 0 ? plan->w->qg[level - 1] : plan->w->eg[level - 1];
  if (hipMemcpyAsync(dst, src, tsize(hp) * G, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
      hipSuccess)
    return MSM_ERR_HIP;
  return MSM_OK;
}

msm_status msm_plan_set_profiling(msm_plan plan, int enable) {
  if (!plan) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  plan->prof.on = enable != 0;
  return MSM_OK;
}

msm_status msm_plan_set_profile_stages(msm_plan plan, const char* stages) {
  if (!plan) return MSM_ERR_INVALID_ARG;
  try {
    plan->prof.only.clear();
    if (stages) {
      std::string cur;
      for (const char* c = stages;; ++c) {
        if (*c == ',' || *c == 0) {
          if (!cur.empty()) plan->prof.only.push_back(cur);
          cur.clear();
          if (*c == 0) break;
        } else if (*c != ' ') {
          cur.push_back(*c);
        }
      }
    }
  } catch (...) {
    return MSM_ERR_OOM;
  }
  return MSM_OK;
}

msm_status msm_plan_get_profile(msm_plan plan, char* json, size_t cap, int reset) {
  if (!plan || !json || cap == 0) return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  std::string out;
  try {
    plan->prof.collect();
    std::ostringstream o;
    o.precision(9);
    o << "{";
    bool first = true;
    for (auto& kv : plan->prof.total) {
      o << (first ? "" : ",") << "\"" << kv.first << "\":{\"ms\":" << kv.second.first
        << ",\"launches\":" << kv.second.second;
      auto it = plan->prof.offsets.find(kv.first);
      if (it != plan->prof.offsets.end())
        o << ",\"start_ms\":" << it->second.first << ",\"end_ms\":" << it->second.second;
      o << "}";
      first = false;
    }
    o << "}";
    out = o.str();
    if (reset) {
      plan->prof.total.clear();
      plan->prof.offsets.clear();
    }
  } catch (...) {
    return MSM_ERR_OOM;
  }
  if (out.size() + 1 > cap) return MSM_ERR_INVALID_ARG;
  std::memcpy(json, out.c_str(), out.size() + 1);
  return MSM_OK;
}

const char* msm_status_string(msm_status st) {
  switch (st) {
    case MSM_OK: return "ok";
    case MSM_ERR_INVALID_ARG: return "invalid argument";
    case MSM_ERR_UNSUPPORTED: return "unsupported order or periodicity";
    case MSM_ERR_CUTOFF_TOO_LARGE: return "cutoff exceeds half of a periodic box edge";
    case MSM_ERR_GRID: return "grid or stencil exceeds the plan limits";
    case MSM_ERR_OUT_OF_DOMAIN: return "position outside the non-periodic box";
    case MSM_ERR_NONFINITE: return "non-finite position or charge";
    case MSM_ERR_CAPACITY: return "particle count exceeds max_n";
    case MSM_ERR_HIP: return "HIP runtime error";
    case MSM_ERR_OOM: return "out of device memory";
    case MSM_ERR_NO_DEVICE: return "plan has no device state";
  }
  return "unknown status";
}

}  // extern "C"
