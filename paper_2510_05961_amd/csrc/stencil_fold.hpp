// stencil_fold.hpp -- host-side check that a stencil's z-planes mirror, so
// the convolution can add the two input planes of a mirrored pair before one
// pass over their shared coefficients (radial kernels sampled on offsets
// symmetric about 0 give mirrored planes).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

namespace msm {

// 1 when every z-plane j of A ([len2][len1][len0]) agrees with plane
// len2-1-j to 1e-12 of A's largest entry; the pairs are then replaced by
// their mean, so they match bit for bit.  0 leaves A as it is.
inline int make_planes_mirror(std::vector<double>& A, int len0, int len1, int len2) {
  const size_t plane = (size_t)len0 * len1;
  if (len2 < 2 || A.size() != plane * len2) return 0;
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  const double tol = 1e-12 * amax;
  for (int j = 0; j < len2 / 2; ++j)
    for (size_t i = 0; i < plane; ++i)
      if (!(std::fabs(A[plane * j + i] - A[plane * (len2 - 1 - j) + i]) <= tol)) return 0;
  for (int j = 0; j < len2 / 2; ++j)
    for (size_t i = 0; i < plane; ++i) {
      double& u = A[plane * j + i];
      double& w = A[plane * (len2 - 1 - j) + i];
      u = w = 0.5 * (u + w);
    }
  return 1;
}

// MSM_FOLD=0 (read when a plan is created) keeps every stencil unfolded.
inline bool fold_allowed() {
  const char* env = std::getenv("MSM_FOLD");
  return !(env && env[0] == '0');
}

}  // namespace msm
