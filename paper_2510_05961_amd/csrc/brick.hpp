// brick.hpp -- the cells whose charges one anterpolation brick gathers
// (a3, and the dipole anterpolation of the backward pass).
#pragma once

#include "kernels.hpp"

namespace msm {

// Run r holds the sorted particles beg[r] .. beg[r] + off[r+1] - off[r] - 1.
struct BrickRuns {
  int beg[kBrickMaxCells * kBrickMaxCells];
  int off[kBrickMaxCells * kBrickMaxCells + 1];
};

// Cell range [c0, c1) per axis of super-cell sc, split into runs of cells
// consecutive along x (one per (y, z) row: consecutive in the sorted order).
// Sets nruns and returns the super-cell's particle count; every thread of
// the workgroup (blockDim.x >= kBrickMaxCells^2) must call it.
__device__ inline int brick_runs(int sc, const int* __restrict__ start, const CellGrid& cg,
                                 const BrickGeom& bg, int c0[3], int c1[3], BrickRuns& R,
                                 int& nruns) {
  const int s3[3] = {sc % bg.nsc[0], (sc / bg.nsc[0]) % bg.nsc[1],
                     sc / (bg.nsc[0] * bg.nsc[1])};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c0[k] = s3[k] * bg.kc;
    c1[k] = min(cg.nc[k], c0[k] + bg.kc);
  }
  const int ny = c1[1] - c0[1];
  nruns = ny * (c1[2] - c0[2]);
  const int t = threadIdx.x;
  if (t < nruns) {
    const int cy = c0[1] + t % ny, cz = c0[2] + t / ny;
    const int row = (cz * cg.nc[1] + cy) * cg.nc[0];
    const int b = start[row + c0[0]];
    R.beg[t] = b;
    R.off[t + 1] = start[row + c1[0]] - b;  // run length, scanned below
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    R.off[0] = 0;
    for (int r = 0; r < nruns; ++r) {
      acc += R.off[r + 1];
      R.off[r + 1] = acc;
    }
  }
  __syncthreads();
  return R.off[nruns];
}

// Sorted index of the brick's j-th particle (0 <= j < count).
__device__ inline int brick_particle(const BrickRuns& R, int nruns, int j) {
  int r = 0;  // last run with off[r] <= j (it is non-empty)
#pragma unroll
  for (int step = kBrickMaxCells * kBrickMaxCells / 2; step > 0; step >>= 1)
    if (r + step < nruns && R.off[r + step] <= j) r += step;
  return R.beg[r] + (j - R.off[r]);
}

// Grid index range of the brick: every point the super-cell's charges can
// touch, one point of margin each side for the rounding of the binning.
template <int P>
__device__ inline int brick_box(const int c0[3], const int c1[3], const CellGrid& cg,
                                const double hd[3], int lo[3], int ext[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = (int)floor(c0[k] * cg.cs[k] / hd[k]) - P / 2 - 1;
    const int hi = (int)floor(c1[k] * cg.cs[k] / hd[k]) + P / 2 + 1;
    ext[k] = hi - lo[k] + 1;
  }
  return ext[0] * ext[1] * ext[2];
}

}  // namespace msm
