// kernels.hpp -- kernel parameter blocks and launch helpers of libmsm.
#pragma once

#include "device.hpp"

namespace msm {

constexpr int kPairThreads = 128;

template <typename T>
struct BinParams {
  T box[3];
  T cs[3];     // cell edge
  int nc[3];   // cells per axis
  int per[3];
};

template <typename T>
struct PairParams {
  T box[3], inv_box[3];
  int per[3];
  int nc[3];
  T a2, inv_a2, inv_a, inv_a3;
  T c[8];   // softening polynomial in t = (r/a)^2
  T dc[8];  // its t-derivative: dc[k] = (k+1) c[k+1]
};

// One stencil convolution e = K q on a level grid (a5, a6).
template <typename T>
struct ConvParams {
  int n[3];
  int per[3];
  int off[3], len[3];   // stencil offsets d_k = off_k .. off_k + len_k - 1
  int dz_per_split;     // stencil z-planes handled by one workgroup
  int nsplit;
  int lds_w, lds_h;     // staged input tile
};

template <typename T>
void launch_binning(int n, const T* pos, const T* q, const BinParams<T>& bp, int ncell,
                    int* cell_of, int* rank, int* counts, vec4_t<T>* wrapped, int* start,
                    vec4_t<T>* sorted, int* perm, int* flag, hipStream_t s);
template <typename T>
void launch_pair(int p, int ncell, const vec4_t<T>* sorted, const int* start,
                 const PairParams<T>& pp, T* phi0, T* F0, hipStream_t s);
template <typename T>
void launch_anterp(int p, int n, const vec4_t<T>* sorted, const GridDev<T>& g, T* grid,
                   hipStream_t s);
template <typename T>
void launch_interp(int p, int n, const vec4_t<T>* sorted, const int* perm, const GridDev<T>& g,
                   const T* e1, const T* phi0, const T* F0, T self_const, T* dEdq, T* F,
                   T* save_phi, T* save_F, double* energy, hipStream_t s);

// J is a HOST array of the p+1 restriction taps (passed by value to the kernel).
template <typename T>
void launch_restrict(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                     const T* qf, T* qc, hipStream_t s);
template <typename T>
void launch_prolong(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                    const T* ec, T* ef, hipStream_t s);
// Returns the dynamic LDS bytes the conv kernel needs for this stencil.
template <typename T>
size_t conv_lds_bytes(const int len[3], bool small);
template <typename T>
void launch_conv(const ConvParams<T>& cp, const T* K, const int2* rowext, const T* q, T* e,
                 hipStream_t s);
template <typename T>
ConvParams<T> make_conv_params(const int n[3], const int per[3], const int off[3],
                               const int len[3]);

template <typename T>
void launch_fill(T* p, long long count, T value, hipStream_t s);

}  // namespace msm
