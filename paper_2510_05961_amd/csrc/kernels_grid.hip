// kernels_grid.hip -- grid-side kernels of the MSM: restriction, prolongation
// and the per-level stencil convolution (also used for the dense top level).
#include "kernels.hpp"

namespace msm {

template <typename T>
struct JTaps {
  T J[9];  // J_{-p/2..p/2}
};

__device__ inline int floor_div2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

// ---------------------------------------------------------------------------
// a4: restriction (eq. restriction_prolongation_explicit_formulas, first line)
//   q~^{l+1}_m = sum_n J_{n-2m} q~^l_n,  J_n = J_nx J_ny J_nz,
// applied as three 1-D tap sets of p+1 taps per coarse point.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ void k_restrict(GridDev<T> f, GridDev<T> c, JTaps<T> jt, const T* __restrict__ qf,
                           T* __restrict__ qc) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long G = (long long)c.n[0] * c.n[1] * c.n[2];
  if (gid >= G) return;
  const int ic[3] = {(int)(gid % c.n[0]), (int)((gid / c.n[0]) % c.n[1]),
                     (int)(gid / ((long long)c.n[0] * c.n[1]))};
  int idx[3][P + 1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int m = ic[k] + c.lo[k];
#pragma unroll
    for (int t = 0; t <= P; ++t) idx[k][t] = axis_index(2 * m + t - P / 2, f.n[k], f.lo[k], f.per[k]);
  }
  T s = T(0);
#pragma unroll
  for (int tz = 0; tz <= P; ++tz) {
    if (idx[2][tz] < 0) continue;
    T sy = T(0);
#pragma unroll
    for (int ty = 0; ty <= P; ++ty) {
      if (idx[1][ty] < 0) continue;
      const T* row = qf + ((long long)idx[2][tz] * f.n[1] + idx[1][ty]) * f.n[0];
      T sx = T(0);
#pragma unroll
      for (int tx = 0; tx <= P; ++tx)
        if (idx[0][tx] >= 0) sx += jt.J[tx] * row[idx[0][tx]];
      sy += jt.J[ty] * sx;
    }
    s += jt.J[tz] * sy;
  }
  qc[gid] = s;
}

// ---------------------------------------------------------------------------
// a7: prolongation, the transpose of restriction (paper's corrected form)
//   e^l_m += sum_n J_{m-2n} e^{l+1}_n,
// gathered per fine point over the at most p/2+1 coarse points per axis.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ void k_prolong(GridDev<T> f, GridDev<T> c, JTaps<T> jt, const T* __restrict__ ec,
                          T* __restrict__ ef) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long G = (long long)f.n[0] * f.n[1] * f.n[2];
  if (gid >= G) return;
  const int im[3] = {(int)(gid % f.n[0]), (int)((gid / f.n[0]) % f.n[1]),
                     (int)(gid / ((long long)f.n[0] * f.n[1]))};
  constexpr int NC = P / 2 + 1;
  int idx[3][NC];
  T wt[3][NC];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int m = im[k] + f.lo[k];
    const int n_lo = -floor_div2(-(m - P / 2));  // ceil((m - P/2)/2)
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int n = n_lo + t;
      const int kk = m - 2 * n;  // tap index, in [-P/2, P/2] when valid
      if (kk >= -P / 2 && kk <= P / 2) {
        idx[k][t] = axis_index(n, c.n[k], c.lo[k], c.per[k]);
        wt[k][t] = jt.J[kk + P / 2];
      } else {
        idx[k][t] = -1;
        wt[k][t] = T(0);
      }
    }
  }
  T s = T(0);
#pragma unroll
  for (int tz = 0; tz < NC; ++tz) {
    if (idx[2][tz] < 0) continue;
    T sy = T(0);
#pragma unroll
    for (int ty = 0; ty < NC; ++ty) {
      if (idx[1][ty] < 0) continue;
      const T* row = ec + ((long long)idx[2][tz] * c.n[1] + idx[1][ty]) * c.n[0];
      T sx = T(0);
#pragma unroll
      for (int tx = 0; tx < NC; ++tx)
        if (idx[0][tx] >= 0) sx += wt[0][tx] * row[idx[0][tx]];
      sy += wt[1][ty] * sx;
    }
    s += wt[2][tz] * sy;
  }
  ef[gid] += s;
}

// ---------------------------------------------------------------------------
// a5 / a6: stencil convolution e_o = sum_d K_d q_{o+shift-d} (eq.
// action_of_K_as_convolution).  A workgroup owns a TX x TY tile of output
// points of one z-plane and a contiguous range of stencil z-planes; for each
// plane it stages the input window (with periodic wrap or zero padding)
// through LDS, and every thread keeps R consecutive x outputs in registers.
// The stencil coefficients are uniform across the workgroup (scalar loads);
// per stencil row only the non-zero x range is visited.  TI is the grid type
// (what LDS holds), TA the stencil / accumulation / output type: the factored
// levels accumulate the k-sample convolution in FP64.
// ---------------------------------------------------------------------------
constexpr int kConvCH = 8;

template <typename TI, typename TA, int R, int TXT, int TYT>
__global__ void __launch_bounds__(TXT * TYT)
    k_conv(ConvParams cp, const TA* __restrict__ K, const int2* __restrict__ rowext,
           const TI* __restrict__ q, TA* __restrict__ e) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TI* lds = reinterpret_cast<TI*>(smem_raw);
  const int tx = threadIdx.x % TXT, ty = threadIdx.x / TXT;
  const int n0 = cp.n[0], n1 = cp.n[1], n2 = cp.n[2];
  const int o0 = cp.nout[0], o1 = cp.nout[1], o2 = cp.nout[2];
  const int lx = cp.len[0], ly = cp.len[1];
  const int x0 = blockIdx.x * (TXT * R), y0 = blockIdx.y * TYT;
  const int z = blockIdx.z % o2, split = blockIdx.z / o2;
  const int jz0 = split * cp.dz_per_split;
  const int jz1 = min(cp.len[2], jz0 + cp.dz_per_split);
  const int LW = cp.lds_w, LH = cp.lds_h;
  const int xs = x0 + cp.shift[0] - (cp.off[0] + lx - 1);
  const int ys = y0 + cp.shift[1] - (cp.off[1] + ly - 1);
  TA total[R];
#pragma unroll
  for (int r = 0; r < R; ++r) total[r] = TA(0);
  for (int jz = jz0; jz < jz1; ++jz) {
    int zi = z + cp.shift[2] - (cp.off[2] + jz);
    if (cp.per[2]) zi = wrap_index(zi, n2);
    else if (zi < 0 || zi >= n2) continue;  // uniform over the workgroup
    __syncthreads();
    const TI* qz = q + (long long)zi * n1 * n0;
    for (int idx = threadIdx.x; idx < LW * LH; idx += TXT * TYT) {
      const int ry = idx / LW, rx = idx - ry * LW;
      int yi = ys + ry, xi = xs + rx;
      bool ok = true;
      if (cp.per[1]) yi = wrap_index(yi, n1);
      else ok = (yi >= 0 && yi < n1);
      if (cp.per[0]) xi = wrap_index(xi, n0);
      else ok = ok && (xi >= 0 && xi < n0);
      lds[idx] = ok ? qz[(long long)yi * n0 + xi] : TI(0);
    }
    __syncthreads();
    TA acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = TA(0);
    const TA* Kz = K + (long long)jz * ly * lx;
    const int2* ext_z = rowext + jz * ly;
    for (int jy = 0; jy < ly; ++jy) {
      const int2 ext = ext_z[jy];
      if (ext.x > ext.y) continue;
      const TI* lrow = lds + (ty - jy + ly - 1) * LW + tx * R;
      const TA* Krow = Kz + jy * lx;
      int jx = ext.x;
      for (; jx + kConvCH - 1 <= ext.y; jx += kConvCH) {
        TA win[kConvCH + R - 1];
        const TI* wp = lrow + (lx - jx - kConvCH);
#pragma unroll
        for (int u = 0; u < kConvCH + R - 1; ++u) win[u] = (TA)wp[u];
#pragma unroll
        for (int c = 0; c < kConvCH; ++c) {
          const TA kv = Krow[jx + c];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = fma(kv, win[kConvCH - 1 - c + r], acc[r]);
        }
      }
      for (; jx <= ext.y; ++jx) {
        const TA kv = Krow[jx];
        const TI* wp = lrow + (lx - 1 - jx);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(kv, (TA)wp[r], acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) total[r] += acc[r];
  }
  const int y = y0 + ty;
  if (y < o1) {
    TA* erow = e + ((long long)z * o1 + y) * o0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = x0 + tx * R + r;
      if (x < o0) {
        if (cp.nsplit > 1) atomicAdd(&erow[x], total[r]);
        else erow[x] = total[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Second half of the factored stencil: e_m = sum_k omega'_kx omega'_ky
// omega'_kz u_{m-k}, applied one axis at a time inside LDS on a T^3 output
// tile (u lives on the extended domain of the free axes).
// ---------------------------------------------------------------------------
template <typename TO, int T>
__global__ void __launch_bounds__(256)
    k_omega(OmegaParams op, const double* __restrict__ u, TO* __restrict__ e) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* buf = reinterpret_cast<double*>(smem_raw);
  const int M = op.M, W = T + 2 * M;
  double* reg0 = buf;                 // [W][W][W]   u window
  double* reg1 = reg0 + W * W * W;    // [W][W][T]   after the x pass
  double* reg2 = reg1 + W * W * T;    // [W][T][T]   after the y pass
  const int m0[3] = {(int)blockIdx.x * T, (int)blockIdx.y * T, (int)blockIdx.z * T};
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < W * W * W; idx += nt) {
    const int rx = idx % W, ry = (idx / W) % W, rz = idx / (W * W);
    const int r3[3] = {rx, ry, rz};
    long long off = 0, stride = 1;
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      int m = m0[k] - M + r3[k];  // grid index of u needed
      int ui;
      if (op.per[k]) {
        ui = wrap_index(m, op.n[k]);
      } else {
        ui = m + M;  // extended index
        ok = ok && (ui >= 0 && ui < op.next[k]);
      }
      off += (long long)ui * stride;
      stride *= op.next[k];
    }
    reg0[idx] = ok ? u[off] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < W * W * T; idx += nt) {
    const int x = idx % T, ry = (idx / T) % W, rz = idx / (T * W);
    const double* row = reg0 + (rz * W + ry) * W;
    double s = 0.0;
    for (int k = -M; k <= M; ++k) s += op.omega[k < 0 ? -k : k] * row[x + M - k];
    reg1[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < W * T * T; idx += nt) {
    const int x = idx % T, y = (idx / T) % T, rz = idx / (T * T);
    double s = 0.0;
    for (int k = -M; k <= M; ++k)
      s += op.omega[k < 0 ? -k : k] * reg1[(rz * W + (y + M - k)) * T + x];
    reg2[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < T * T * T; idx += nt) {
    const int x = idx % T, y = (idx / T) % T, z = idx / (T * T);
    const int mx = m0[0] + x, my = m0[1] + y, mz = m0[2] + z;
    if (mx >= op.n[0] || my >= op.n[1] || mz >= op.n[2]) continue;
    double s = 0.0;
    for (int k = -M; k <= M; ++k)
      s += op.omega[k < 0 ? -k : k] * reg2[((z + M - k) * T + y) * T + x];
    e[((long long)mz * op.n[1] + my) * op.n[0] + mx] = (TO)s;
  }
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

template <typename T>
void launch_restrict(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                     const T* qf, T* qc, hipStream_t s) {
  const long long G = (long long)coarse.n[0] * coarse.n[1] * coarse.n[2];
  const int nb = (int)((G + 255) / 256);
  JTaps<T> jt = make_taps<T>(J, p);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_restrict<T, 4>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
    case 6: hipLaunchKernelGGL((k_restrict<T, 6>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
    case 8: hipLaunchKernelGGL((k_restrict<T, 8>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, qf, qc); break;
  }
}

template <typename T>
void launch_prolong(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                    const T* ec, T* ef, hipStream_t s) {
  const long long G = (long long)fine.n[0] * fine.n[1] * fine.n[2];
  const int nb = (int)((G + 255) / 256);
  JTaps<T> jt = make_taps<T>(J, p);
  switch (p) {
    case 4: hipLaunchKernelGGL((k_prolong<T, 4>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, ec, ef); break;
    case 6: hipLaunchKernelGGL((k_prolong<T, 6>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, ec, ef); break;
    case 8: hipLaunchKernelGGL((k_prolong<T, 8>), dim3(nb), dim3(256), 0, s, fine, coarse, jt, ec, ef); break;
  }
}

// big tiles (64 x 32 outputs, 256 threads) for wide grids, small tiles
// (16 x 16 outputs, 64 threads) for grids narrower than 48 points
static bool conv_small(const int nout[3]) { return nout[0] < 48; }

ConvParams make_conv_params(const int n[3], const int nout[3], const int shift[3],
                            const int per[3], const int off[3], const int len[3], int tsize) {
  ConvParams cp;
  for (int k = 0; k < 3; ++k) {
    cp.n[k] = n[k];
    cp.nout[k] = nout[k];
    cp.shift[k] = shift[k];
    cp.per[k] = per[k];
    cp.off[k] = off[k];
    cp.len[k] = len[k];
  }
  const bool small = conv_small(nout);
  const int TXo = small ? 16 : 64, TY = small ? 16 : 32;
  cp.lds_w = TXo + len[0] - 1;
  if (tsize == 4) cp.lds_w |= 1;  // odd row stride spreads rows over LDS banks
  cp.lds_h = TY + len[1] - 1;
  const long long tiles =
      (long long)((nout[0] + TXo - 1) / TXo) * ((nout[1] + TY - 1) / TY) * nout[2];
  long long want = (2048 + tiles - 1) / tiles;
  if (want < 1) want = 1;
  if (want > len[2]) want = len[2];
  cp.dz_per_split = (int)((len[2] + want - 1) / want);
  cp.nsplit = (len[2] + cp.dz_per_split - 1) / cp.dz_per_split;
  cp.small = small;
  return cp;
}

size_t conv_lds_bytes(const ConvParams& cp, int tsize) {
  return (size_t)cp.lds_w * cp.lds_h * tsize;
}

template <typename TI, typename TA>
void launch_conv(const ConvParams& cp, const TA* K, const int2* rowext, const TI* q, TA* e,
                 hipStream_t s) {
  const size_t lds = (size_t)cp.lds_w * cp.lds_h * sizeof(TI);
  if (cp.small) {
    dim3 grid((cp.nout[0] + 15) / 16, (cp.nout[1] + 15) / 16, cp.nout[2] * cp.nsplit);
    hipLaunchKernelGGL((k_conv<TI, TA, 4, 4, 16>), grid, dim3(64), lds, s, cp, K, rowext, q, e);
  } else {
    dim3 grid((cp.nout[0] + 63) / 64, (cp.nout[1] + 31) / 32, cp.nout[2] * cp.nsplit);
    hipLaunchKernelGGL((k_conv<TI, TA, 8, 8, 32>), grid, dim3(256), lds, s, cp, K, rowext, q, e);
  }
}

size_t omega_lds_bytes(int M) {
  const int T = M <= 6 ? 8 : 4, W = T + 2 * M;
  return sizeof(double) * ((size_t)W * W * W + (size_t)W * W * T + (size_t)W * T * T);
}

template <typename TO>
void launch_omega(const OmegaParams& op, const double* u, TO* e, hipStream_t s) {
  const int T = op.M <= 6 ? 8 : 4;
  dim3 grid((op.n[0] + T - 1) / T, (op.n[1] + T - 1) / T, (op.n[2] + T - 1) / T);
  const size_t lds = omega_lds_bytes(op.M);
  if (T == 8) hipLaunchKernelGGL((k_omega<TO, 8>), grid, dim3(256), lds, s, op, u, e);
  else hipLaunchKernelGGL((k_omega<TO, 4>), grid, dim3(256), lds, s, op, u, e);
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
                                  const T*, T*, hipStream_t);                                     \
  template void launch_conv<T, T>(const ConvParams&, const T*, const int2*, const T*, T*,         \
                                  hipStream_t);                                                   \
  template void launch_omega<T>(const OmegaParams&, const double*, T*, hipStream_t);              \
  template void launch_fill<T>(T*, long long, T, hipStream_t);                                    \
  template void launch_cast<T>(const double*, T*, long long, hipStream_t);
MSM_INST_GRID(float)
MSM_INST_GRID(double)
template void launch_fill<int>(int*, long long, int, hipStream_t);
template void launch_conv<float, double>(const ConvParams&, const double*, const int2*,
                                         const float*, double*, hipStream_t);

}  // namespace msm
