// plan.hpp -- host-side MSM plan: geometry, constants and FP64 stencils.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

namespace msm {

constexpr int kMaxLevels = 16;
constexpr int kMaxOrder = 8;

struct LevelGeom {
  int n[3];        // grid points per axis
  int lo[3];       // grid index of array element 0 (free axis: -p/2+1, periodic: 0)
  double h[3];     // spacing
  long long G;     // n0 n1 n2
  // stencil (levels < L) or top-level kernel (level L) in FP64
  int off[3];      // first offset per axis
  int len[3];      // number of offsets per axis
  std::vector<double> K;  // [len2][len1][len0]
  // Factored form K^l = (omega' x omega' x omega') * S^l (eq.
  // kernel_stencil_by_conv_with_universal_coeff), used when cheaper: the
  // samples S^l(d) = k_l(|h_l o d|) are convolved first, on an output domain
  // extended by M on free axes, then omega' is applied axis by axis.
  bool factored = false;
  int s_off[3], s_len[3];  // sample box offsets (folded on periodic axes)
  std::vector<double> S;   // [s_len2][s_len1][s_len0]
  int next[3];             // extended output dims: n + 2M on free axes, n on periodic
  int shift[3];            // grid index of extended element 0 (-M free, 0 periodic)
  long long Gext;
};

struct HostPlan {
  double box[3];   // edge lengths; (1, 1, 1) in a triclinic cell (grids in the unit cube)
  int periodic[3];
  // triclinic cell (all axes periodic): H has the lattice vectors as columns
  // (H[3*row + col]); positions map to the unit cube, s = H^{-1} r
  int tri = 0;
  double H[9], Hinv[9];
  int p, L, M;
  double h_req, a;
  int nu = 1;      // the kernel r^-nu (1: Coulomb, 6: dispersion)
  int precision;   // 0 fp32, 1 fp64
  int max_n;
  // softener gamma(rho) = sum_k gcoef[k] t^k, t = rho^2, rho < 1
  double gcoef[kMaxOrder];
  double gamma0;        // gamma(0)
  double self_const;    // sum_{l>=1} k_l(0) = gamma(0)/a
  std::vector<double> omega;  // omega'_0..omega'_M
  double J[kMaxOrder + 1];    // restriction taps J_{-p/2..p/2}
  LevelGeom lev[kMaxLevels];
  int W1[3];            // unfolded level-1 stencil half-widths (R + M)
  // cell list for the short-range part: cells of edge >= a + skin (a
  // Verlet skin keeps the list between calls), width = the box's (or the
  // cell's) width across each axis
  double skin = 0.0;
  double width[3];
  int nc[3];
  double cs[3];
};

// nc and cs from width, a and skin (at most 1024 cells per axis)
void cell_list_geometry(HostPlan& P);

// Builds geometry and every stencil; returns 0 or an msm_status code.
// cell (optional, 9 doubles: rows a, b, c) makes a triclinic plan (box is
// then ignored and periodic_mask must be 7); ntop (optional) fixes the
// top-grid point counts (a cell that changes keeps its grids).
int build_host_plan(HostPlan& P, const double box[3], unsigned periodic_mask, int order,
                    double h, double a, int levels, int precision, int max_n, int M,
                    const double* cell = nullptr, const int* ntop = nullptr,
                    double skin = 0.0, int nu = 1);

std::string describe_json(const HostPlan& P);

// Cell-derivative stencils of a triclinic plan: T^l_ab(d) = k_l'(r)/r x_a x_b
// (ab = xx, yy, zz, xy, xz, yz) in level l's sample layout (s_off, s_len),
// 1 <= l < L; and the top level's dK^L/dH_rc (K^L's layout) by central
// differences of plans for H +- eps e_rc.
void cell_stress_stencils(const HostPlan& P, int l, std::vector<double> T[6]);
int top_cell_derivative(const HostPlan& P, std::vector<double> dK[9]);

// Softener pieces used by the batch planner as well.
void softener_coefficients(int p, double* c, int nu = 1);
std::vector<double> quasi_sequence(int p, int M);
// Unfolded level-1 stencil of a free-space system with spacing h (all axes).
// A (optional): the Cartesian step of one grid point along each axis as the
// columns of a 3x3 matrix (a triclinic grid); else the steps are h_k along
// the Cartesian axes.
void level1_stencil(int p, int M, double a, const double h[3], int W[3], std::vector<double>& K,
                    const double* gcoef, const double* A = nullptr, int nu = 1);
// The ball of the factored level-1 stencil, S^1(d) = k_1(|h o d|) on
// |d_k| <= R_k (orthorhombic grid), [2R_2+1][2R_1+1][2R_0+1].
void level1_samples(int p, double a, const double h[3], const int R[3], const double* gcoef,
                    std::vector<double>& S, int nu = 1);
// Dense top-level kernel of a free-space system: offsets |d_k| <= n_k - 1.
void free_top_kernel(int p, int M, double a, int L, const double hL[3], const int n[3],
                     const std::vector<double>& omega, const double* gcoef,
                     std::vector<double>& K, int nu = 1);

}  // namespace msm
