// stress.hip -- helper kernels of the cell derivative dE/dH (triclinic
// plans): grid copies and dot products for the level terms, the particles'
// term sum_i F_i s_i^T, and the final 3 x 3 combination.
#include <algorithm>

#include "kernels.hpp"

namespace msm {

template <typename T>
__global__ void k_to_double(const T* __restrict__ a, double* __restrict__ b, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}

// acc += sum_i a_i b_i (FP64; one atomic per workgroup)
template <typename T>
__global__ void __launch_bounds__(256)
    k_dot(const T* __restrict__ a, const double* __restrict__ b, long long count,
          double* __restrict__ acc) {
  __shared__ double part[4];
  double t = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    t += (double)a[i] * b[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(acc, part[0] + part[1] + part[2] + part[3]);
}

// acc9[3 a + b] += sum_i F_i,a s_i,b with s_i = Hinv r_i (FP64)
template <typename T>
__global__ void __launch_bounds__(256)
    k_cell_fs(int n, const T* __restrict__ pos, const T* __restrict__ F,
              const double* __restrict__ Hinv, double* __restrict__ acc9) {
  __shared__ double part[4][9];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double f[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
  if (i < n) {
    const double r[3] = {(double)pos[3 * i], (double)pos[3 * i + 1], (double)pos[3 * i + 2]};
    for (int k = 0; k < 3; ++k) {
      f[k] = (double)F[3 * i + k];
      sv[k] = Hinv[3 * k] * r[0] + Hinv[3 * k + 1] * r[1] + Hinv[3 * k + 2] * r[2];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double t = f[a] * sv[b];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
      if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][3 * a + b] = t;
    }
  __syncthreads();
  if (threadIdx.x < 9)
    atomicAdd(&acc9[threadIdx.x], part[0][threadIdx.x] + part[1][threadIdx.x] +
                                      part[2][threadIdx.x] + part[3][threadIdx.x]);
}

__global__ void k_cell_combine(const double* __restrict__ acc, const double* __restrict__ Hinv,
                               double* __restrict__ dEdH) {
  if (threadIdx.x != 0) return;
  // symmetric V = -A0/2 + Vg/2 from (xx, yy, zz, xy, xz, yz)
  double V[9];
  const int sym[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
  for (int k = 0; k < 9; ++k) V[k] = -0.5 * acc[sym[k]] + 0.5 * acc[6 + sym[k]];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      // (V H^{-T})_{rc} = sum_k V_rk Hinv_ck
      double t = 0.0;
      for (int k = 0; k < 3; ++k) t += V[3 * r + k] * Hinv[3 * c + k];
      dEdH[3 * r + c] = t + 0.5 * acc[12 + 3 * r + c] + acc[21 + 3 * r + c];
    }
}

template <typename T>
void launch_to_double(const T* a, double* b, long long count, hipStream_t s) {
  if (count <= 0) return;
  const long long nb = std::min<long long>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(k_to_double<T>, dim3((unsigned)nb), dim3(256), 0, s, a, b, count);
}

template <typename T>
void launch_dot(const T* a, const double* b, long long count, double* acc, hipStream_t s) {
  if (count <= 0) return;
  const long long nb = std::min<long long>(1024, (count + 255) / 256);
  hipLaunchKernelGGL(k_dot<T>, dim3((unsigned)nb), dim3(256), 0, s, a, b, count, acc);
}

template <typename T>
void launch_cell_fs(int n, const T* pos, const T* F, const double* Hinv, double* acc9,
                    hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cell_fs<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, F, Hinv, acc9);
}

void launch_cell_combine(const double* acc, const double* Hinv, double* dEdH, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_combine, dim3(1), dim3(64), 0, s, acc, Hinv, dEdH);
}

#define MSM_INST_STRESS(T)                                                                    \
  template void launch_to_double<T>(const T*, double*, long long, hipStream_t);               \
  template void launch_dot<T>(const T*, const double*, long long, double*, hipStream_t);      \
  template void launch_cell_fs<T>(int, const T*, const T*, const double*, double*, hipStream_t);
MSM_INST_STRESS(float)
MSM_INST_STRESS(double)

}  // namespace msm
