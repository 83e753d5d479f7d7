// conv_tile.hpp -- the inner loop of the stencil convolution (eq.
// action_of_K_as_convolution) over one stencil plane.
#pragma once

#include "kernels.hpp"

namespace msm {

// Adds one stencil plane to a thread's Q x R outputs (Q consecutive rows, R
// consecutive x) from the staged input window `lds` (row stride LW; window
// column lx - 1 - jx + tx R + r holds the input of tap jx for output r).
// Kz points at stencil row 0 of the plane (rows of stride lxp, zero-padded
// to lx + kConvCH - 1, kConvRowPad zero rows before and after the plane);
// ext_z holds each row's [first, last] non-zero tap.  The thread walks the
// window rows v: row v serves output row a through stencil row
// a + ly - 1 - v, so every LDS value, converted once to TA, feeds up to
// Q R kConvCH multiply-adds.  Taps run in chunks of kConvCH over the union
// of the Q rows' ranges, clipped to [jlo, jhi]; rows v outside [vlo, vhi]
// are skipped (both clips are for inputs that are known to be zero), and
// only every vstep-th row from vlo is walked (the rows of one plane can be
// shared out among the waves of a workgroup).
template <typename TI, typename TA, int R, int Q>
__device__ inline void conv_plane(const TI* __restrict__ lds, int LW, int tx, int ty,
                                  const TA* __restrict__ Kz, const int2* __restrict__ ext_z,
                                  int lx, int ly, int lxp, int jlo, int jhi, int vlo, int vhi,
                                  TA (&acc)[Q][R], int vstep = 1) {
  constexpr int CH = kConvCH;
  for (int v = vlo; v <= vhi; v += vstep) {
    // output row a of the thread uses stencil row jy = a + ly - 1 - v
    const int alo = max(0, v - ly + 1), ahi = min(Q - 1, v);
    int first = lx, last = -1;
    for (int a = alo; a <= ahi; ++a) {
      const int2 ex = ext_z[a + ly - 1 - v];
      first = min(first, ex.x);
      last = max(last, ex.y);
    }
    first = max(first, jlo);
    last = min(last, jhi);
    const TI* lrow = lds + (ty * Q + v) * LW + tx * R + (lx - 1);
    for (int j0 = first; j0 <= last; j0 += CH) {
      TA win[CH + R - 1];
      const TI* wp = lrow - j0;
#pragma unroll
      for (int u = 0; u < CH + R - 1; ++u) win[u] = (TA)wp[u];
      // rows outside the stencil (a < alo or a > ahi) are zero padding;
      // all Q CH coefficients are loaded first, then the multiply-adds go
      // tap by tap across all Q R accumulators (independent chains)
      TA kv[Q][CH];
#pragma unroll
      for (int a = 0; a < Q; ++a)
#pragma unroll
        for (int c = 0; c < CH; ++c) kv[a][c] = Kz[(long long)(a + ly - 1 - v) * lxp + j0 + c];
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int a = 0; a < Q; ++a)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[a][r] = fma(kv[a][c], win[CH - 1 - c + r], acc[a][r]);
    }
  }
}

}  // namespace msm
