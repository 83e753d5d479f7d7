// kernels.hpp -- kernel parameter blocks and launch helpers of libmsm.
#pragma once

#include "device.hpp"

namespace msm {

template <typename T>
struct BinParams {
  T box[3];
  T cs[3];     // cell edge
  int nc[3];   // cells per axis
  int per[3];
  // triclinic cell: cells live in the unit cube of s = H^{-1} r (box 1);
  // positions are wrapped by whole lattice vectors and stay Cartesian
  // (row-major matrices, lattice vectors as the columns of H)
  int tri;
  double H[9], Hi[9];
};

template <typename T>
struct PairParams {
  T box[3], inv_box[3];
  T cs[3];     // cell edge
  int per[3];
  int nc[3];
  int ncell;
  T a2, inv_a2, inv_a, inv_a3, inv_a5;
  T c[8];    // softening polynomial in t = (r/a)^2
  T dc[8];   // its t-derivative: dc[k] = (k+1) c[k+1]
  T d2c[8];  // second t-derivative: d2c[k] = (k+2)(k+1) c[k+2]
  // the same in r^2: gamma(r/a)/a = sum er[k] r^2k, 2 gamma'(t)/a^3 =
  // sum fr[k] r^2k, 4 gamma''(t)/a^5 = sum gr[k] r^2k
  T er[8], fr[8], gr[8];
  // triclinic cell: cells in fractional coordinates, the image shift of a
  // neighbour cell is H (shx, shy, shz) (H row-major, lattice vectors as
  // columns)
  int tri;
  T H[9];
  // how far a charge may lie outside its cell (half the Verlet skin)
  T margin;
  int nu;  // the kernel r^-nu (1: Coulomb, 6: dispersion)
};

// One stencil convolution e_o = sum_d K_d q_{o+shift-d} (a5, a6).
struct ConvParams {
  int n[3];             // input grid
  int nout[3];          // output grid (extended on free axes for the factored form)
  int shift[3];         // input grid index of output element 0
  int per[3];
  int off[3], len[3];   // stencil offsets d_k = off_k .. off_k + len_k - 1
  int dz_per_split;     // stencil z-planes handled by one workgroup
  int nsplit;
  int lxp;              // row stride of the stencil (len[0] + kConvCH - 1, zero padded)
  int lds_w, lds_h;     // staged input tile
  int shape;            // tile shape (kernels_grid.hip)
  int fold;             // plane j and plane len2-1-j share coefficients
  int nplanes;          // stencil planes the kernel walks: len2, or (len2+1)/2 folded
};
// A stencil as the convolution walks it: offsets and lengths per axis and
// whether z-plane j and z-plane len2-1-j hold the same coefficients.
struct ConvGeom {
  int off[3], len[3];
  int fold;
};
constexpr int kConvCH = 4;      // taps per register window of the convolution
constexpr int kConvMaxLW = 512; // widest staged window row
constexpr int kConvRowPad = 3;  // zero rows around each stencil plane (Q - 1 for Q <= 4)
int conv_row_stride(int len0);

// restriction taps J_{-p/2..p/2} passed by value
template <typename T>
struct JTapsB {
  T J[9];
};

// omega' applied axis by axis (second half of the factored stencil).
struct OmegaParams {
  int n[3];      // output grid
  int next[3];   // input (extended) grid
  int per[3];
  int M;
  double omega[25];
};

// One axis pass of omega': dims of its input and output (they differ only
// along the pass's axis), whether that axis is periodic, the taps.
struct OmegaPass {
  int in[3], out[3];
  int per, M;
  double omega[25];
};

// Zero several buffers (sizes in 4-byte words) with one launch.
constexpr int kZeroJobs = 24;
struct ZeroJobs {
  void* ptr[kZeroJobs];
  long long words[kZeroJobs];
  int n;
};
void launch_zero_multi(const ZeroJobs& jobs, hipStream_t s);

// Binning: counts (kCountCopies counters per cell, ncell * kCountCopies
// ints, zero on entry), the scans of cell starts and cluster offsets
// (cl_start), and the scatter into cell order, which also clears the
// buffers in `zero`.  The counts are left holding slot bases; the cluster
// layout's kernel sets them back to zero for the next binning.  scan_tmp
// (scan_tmp_ints(ncell) ints, or null: one-workgroup scan) lets many cells
// be scanned by many workgroups.
constexpr int kCountCopies = 8;
int scan_tmp_ints(int ncell);
// Verlet-skin state of a plan (device): ints [force, rebuild, calls,
// rebuilds], each charge's position at the last rebuild and its wrap
// (position minus wrapped position) in the caller's order; half2 = (skin/2)^2.
// state == null: no skin, every call rebuilds.
constexpr int kSkinForce = 0, kSkinRebuild = 1, kSkinCalls = 2, kSkinRebuilds = 3;
template <typename T>
struct SkinDev {
  int* state;
  vec4_t<T>* ref;
  vec4_t<T>* shift;
  T half2;
  int keep_force;  // this call's rebuild leaves force set (its list goes to a workspace)
};
// With a skin the binning first decides (on the device) whether this call
// rebuilds: force != 0, a pending forced rebuild, or a charge that moved
// more than skin/2; without a rebuild the binning kernels return at once
// and the cell-ordered list is refreshed instead.
template <typename T>
void launch_binning(int n, const T* pos, const T* q, const BinParams<T>& bp, int ncell,
                    int* cell_of, int* rank, int* counts, vec4_t<T>* wrapped, int* start,
                    int* cl_start, vec4_t<T>* sorted, int* perm, int* flag, int* scan_tmp,
                    const ZeroJobs& zero, const SkinDev<T>& sk, int force, hipStream_t s);
// Cluster layout of the cell-sorted particles (sort != 0: also reorders each
// cell along a Morton curve, in place) and the short-range pair sum (an
// i-cluster against the j particles within the cutoff of its box).  Buffers hold
// cluster_capacity(n, ncell) clusters: 8 slots each in cpos and cv, two
// boxes (lo, hi per j-group) in cbox; cpos and cv hold one more j-group, the
// null group (far-away zero charges, zero vectors) at index null_h, set once
// by the caller.
int cluster_capacity(int n, int ncell);
constexpr int kGroupSize = 4;  // particles per j-group
// scan != 0: compute cl_start from start here (else it is already there)
// skin != null (a SkinState): on a call without rebuild only the cluster
// slots and j-group boxes are refreshed from the cell-ordered list
template <typename T>
void launch_cluster_layout(int sort, int scan, int ncell, const int* start, int* cl_start,
                           const BinParams<T>& bp, const vec4_t<T>* wrapped, vec4_t<T>* sorted,
                           int* perm, vec4_t<T>* cpos, vec4_t<T>* cbox, int4* cinfo,
                           int* counts, const int* skin, int n, hipStream_t s);
template <typename T>
void launch_pair_cl(int p, int n, int ncell, const int* cl_start, const vec4_t<T>* cpos,
                    const vec4_t<T>* cbox, const int4* cinfo, const PairParams<T>& pp,
                    double* phi0, T* F0, hipStream_t s);
// sum_i q_i sum_j q_j f(r) d d^T of the short-range pairs (cell derivative),
// added to acc[0..5] (xx, yy, zz, xy, xz, yz), FP64, Coulomb kernel
template <typename T>
void launch_pair_virial(int p, int n, int ncell, const int* cl_start, const vec4_t<T>* cpos,
                        const vec4_t<T>* cbox, const int4* cinfo, const PairParams<T>& pp,
                        double* acc, hipStream_t s);
// Cell-derivative helpers (csrc/stress.hip): FP64 copy of a grid; acc[k] +=
// sum_m a_m b_m; acc9 += sum_i F_i (Hinv r_i)^T; and the final combination
// dEdH = (-A0/2 + Vg/2) H^{-T} + D/2 + FS (A0, Vg symmetric 6-vectors; D,
// FS 3 x 3 row-major) from acc = [A0 6, Vg 6, D 9, FS 9].
template <typename T>
void launch_to_double(const T* a, double* b, long long count, hipStream_t s);
template <typename T>
void launch_dot(const T* a, const double* b, long long count, double* acc, hipStream_t s);
template <typename T>
void launch_cell_fs(int n, const T* pos, const T* F, const double* Hinv, double* acc9,
                    hipStream_t s);
void launch_cell_combine(const double* acc, const double* Hinv, double* dEdH, hipStream_t s);
// cell list geometry in FP64 (bricks of the staged anterpolation)
struct CellGrid {
  int nc[3];
  double cs[3];
  // how far a charge may lie outside its cell (half a Verlet skin: the
  // tiled anterpolation, which finds charges by their cells, is then off)
  double margin = 0.0;
};
// Cells of one anterpolation brick: kc^3 cells of the cell list (a
// super-cell), nsc super-cells per axis.  Sparse cells share a brick so
// that the brick's clearing and flushing stay below the work of its charges.
struct BrickGeom {
  int kc;
  int nsc[3];
  int split;  // workgroups per brick, each over a share of its charges
};
constexpr int kBrickMaxCells = 8;  // kc limit (kc^2 runs of cells per brick)
// kc for a call with n charges: BrickGeom of the cell grid (MSM_BRICK_CELLS=k
// forces k, as far as the brick still fits).
BrickGeom brick_geom(int p, int n, int ncell, const CellGrid& cg, const double hd[3]);
// LDS elements of the bricks of this geometry (at most kBrickMax)
int brick_lds_cap(int p, const BrickGeom& bg, const CellGrid& cg, const double hd[3]);
constexpr int kBrickMax = 8192;  // largest brick in LDS (64 KB)
// Whether launch_anterp sums level 1 in tiles that write every grid value
// (large grids); then the grid need not be cleared before it.
bool anterp_tiled(int p, int n, const CellGrid& cg, const int gn[3], const int gper[3],
                  const double hd[3]);
template <typename T>
void launch_anterp(int p, int n, int ncell, const int* start, const CellGrid& cg,
                   const vec4_t<T>* sorted, const GridDev<T>& g, T* grid, hipStream_t s);
template <typename T>
void launch_interp(int p, int n, const vec4_t<T>* sorted, const int* perm, const GridDev<T>& g,
                   const T* e1, const double* phi0, const T* F0, double self_const, T* dEdq,
                   T* F, T* save_phi, T* save_F, double* energy, hipStream_t s);

// J is a HOST array of the p+1 restriction taps (passed by value to the kernel).
template <typename T>
void launch_restrict(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                     const T* qf, T* qc, hipStream_t s);
// Coarse grid from ecT or ec64 (one of them null); ef64 != null: ef =
// (T) ef64 + prolongation, else ef += prolongation.
template <typename T>
void launch_prolong(int p, const GridDev<T>& fine, const GridDev<T>& coarse, const double* J,
                    const T* ecT, const double* ec64, T* ef, const double* ef64,
                    hipStream_t s);


ConvParams make_conv_params(const int n[3], const int nout[3], const int shift[3],
                            const int per[3], const int off[3], const int len[3], int tsize,
                            int fold);
// LDS bytes of the conv kernel for these parameters, staged window plus its
// static arrays (tsize = grid type size)
size_t conv_lds_bytes(const ConvParams& cp, int tsize);
template <typename TI, typename TA>
void launch_conv(const ConvParams& cp, const TA* K, const int2* rowext, const TI* q, TA* e,
                 hipStream_t s);
// Three passes; u (extended grid) is overwritten by the y pass, t holds the
// x pass (both at least next0 next1 next2 doubles).
template <typename TO>
void launch_omega(const OmegaParams& op, double* u, double* t, TO* e, hipStream_t s);

template <typename T>
void launch_fill(T* p, long long count, T value, hipStream_t s);
template <typename T>
void launch_cast(const double* src, T* dst, long long count, hipStream_t s);

// backward (vector-Jacobian product)
// (g.tri: the cotangent in the grid frame, H^{-1} v)
template <typename T>
void launch_gather_v(int n, const int* perm, const T* gF, const T* gphi, const GridDev<T>& g,
                     vec4_t<T>* v, hipStream_t s);
template <typename T>
void launch_pair_vjp_cl(int p, int n, int ncell, const int* cl_start, const int4* cinfo,
                        const int* perm, const T* gF, const T* gphi, const vec4_t<T>* cpos,
                        vec4_t<T>* cv,
                        const vec4_t<T>* cbox, const PairParams<T>& pp, int null_h, T* gq,
                        T* gr, hipStream_t s);
template <typename T>
void launch_anterp_dipole(int p, int n, int ncell, const int* start, const CellGrid& cg,
                          const vec4_t<T>* sorted, const vec4_t<T>* v, const GridDev<T>& g,
                          T* grid, hipStream_t s);
template <typename T>
void launch_interp_vjp(int p, int n, const vec4_t<T>* sorted, const vec4_t<T>* v, const int* perm,
                       const GridDev<T>& g, const T* psi, const T* psiD, const T* save_phi,
                       const T* save_F, const T* gq_sr, const T* gr_sr, const double* gE,
                       double self_const, T* grad_q, T* grad_pos, hipStream_t s);
template <typename T>
void launch_grad_energy_only(int n, const int* perm, const T* save_phi, const T* save_F,
                             const double* gE, T* grad_q, T* grad_pos, hipStream_t s);

}  // namespace msm
