/*
 * msm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference for the multilevel summation method (MSM)
 * with B-spline interpolation (arXiv 2510.05961).  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code with the HIP library: every formula here is written out again from the
 * paper (or from the textbook definition it cites), in the plainest form.
 *
 * Conventions: positions are [n][3] row-major doubles, charges [n] doubles,
 * grids are [nz][ny][nx] with x fastest.  A level-l grid axis is described by
 * its point count n, its first grid index lo (grid point m sits at m*h) and
 * its spacing h; periodic axes have lo = 0 and wrap indices modulo n.
 */
#ifndef MSM_ORACLE_H
#define MSM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXL 16

typedef struct {
  int p;                  /* B-spline order (even)                          */
  int L;                  /* number of grid levels, l = 1..L                */
  int M;                  /* half-width of the quasi-interpolation sequence */
  double a;               /* level-zero cutoff                              */
  double box[3];
  int periodic[3];
  int n[ORC_MAXL][3];     /* level l stored at index l-1                    */
  int lo[ORC_MAXL][3];
  double h[ORC_MAXL][3];
  double omega[32];       /* omega'_0 .. omega'_M (symmetric sequence)      */
  /* Triclinic cell (tri = 1, all axes periodic): the grids live in the unit
   * cube of fractional coordinates s = H^{-1} r (box = 1, h = 1/n), H the
   * cell matrix whose columns are the lattice vectors (H[3*row + col]). */
  int tri;
  double H[9];
  double Hinv[9];
  /* the kernel k(r) = r^-nu (1 or 0: Coulomb; 6: dispersion; free space
   * only for nu != 1) */
  int nu;
} orc_geom;

int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Softening function and its rho-derivatives (Sec. Coulomb splitting). */
double orc_gamma(int p, double rho);
double orc_gamma_d1(int p, double rho);
double orc_gamma_d2(int p, double rho);
/* Partial kernel k_l(r), l = 0..L (eq. coulomb_splitting_with_softener). */
double orc_kernel(int l, int L, double a, int p, double r);
/* First and second r-derivatives of k_0. */
double orc_k0_d1(double a, int p, double r);
double orc_k0_d2(double a, int p, double r);
/* The same for k(r) = r^-nu: softener (deriv 0..2 in rho), partial kernels
 * k_l, and k_0' (deriv 1) / k_0'' (deriv 2). */
double orc_gamma_nu(int nu, int p, double rho, int deriv);
double orc_kernel_nu(int nu, int l, int L, double a, int p, double r);
double orc_k0_nu(int nu, double a, int p, double r, int deriv);
/* Centred cardinal B-spline of order p and its first two derivatives. */
double orc_bspline(int p, double t);
double orc_bspline_d1(int p, double t);
double orc_bspline_d2(int p, double t);

/* Grid charge q~^l by direct anterpolation (eq. grid_charge). */
int orc_anterpolate(const orc_geom* g, int level, int n, const double* pos,
                    const double* q, double* grid);
/* "Dipole" anterpolation D^l_m = sum_i q_i v_i . grad phi^l_m(r_i). */
int orc_anterpolate_dipole(const orc_geom* g, int level, int n, const double* pos,
                           const double* q, const double* v, double* grid);
/* Stencil K^l over the box |d_k| <= W[k] (eq. kernel_stencil_by_conv...). */
void orc_stencil(const orc_geom* g, int level, const int W[3], double* K);
/* e = K q on a level grid, K given over |d_k| <= W[k]; periodic axes wrap the
 * input index, non-periodic axes drop out-of-grid inputs.  If npts >= 0 only
 * the listed flat grid indices are computed (others untouched). */
void orc_conv(const orc_geom* g, int level, const int W[3], const double* K,
              const double* qgrid, double* egrid, int npts, const int* pts);
/* phi_i += sum_m e_m phi_m(r_i);  F_i += -q_i sum_m e_m grad phi_m(r_i). */
int orc_interpolate(const orc_geom* g, int level, int n, const double* pos,
                    const double* q, const double* egrid, double* phi, double* F);
/* Adjoint of interpolation for the force VJP (see msm_backward). */
int orc_interpolate_vjp(const orc_geom* g, int level, int n, const double* pos,
                        const double* q, const double* v, const double* psi,
                        const double* psiD, double* gq, double* gr);

/* Short-range part: phi0_i = sum_{j != i, r < a} q_j k0(r) (min image), and
 * F0_i = -q_i sum_j q_j k0'(r) rhat.  Brute force over all pairs for the
 * listed particles (nsel < 0: all). */
void orc_short_range(const orc_geom* g, int n, const double* pos, const double* q,
                     int nsel, const int* sel, double* phi, double* F);
/* Same sum through a plain cell list, for the listed particles (nsel < 0:
 * all; outputs indexed like sel). */
void orc_short_range_cells(const orc_geom* g, int n, const double* pos,
                           const double* q, int nsel, const int* sel, double* phi, double* F);
/* VJP of the short-range forces against cotangent v: adds d(sum_k v_k.F0_k)/dq_i
 * and /dr_i.  Brute force over all pairs for the listed particles (nsel < 0:
 * all; output row s belongs to particle sel[s]). */
void orc_short_range_vjp(const orc_geom* g, int n, const double* pos, const double* q,
                         const double* v, int nsel, const int* sel, double* gq, double* gr);
/* Same VJP through the plain cell list (all particles). */
void orc_short_range_vjp_cells(const orc_geom* g, int n, const double* pos,
                               const double* q, const double* v, double* gq, double* gr);

/* Exact non-periodic Coulomb sums: phi_i = sum_{j!=i} q_j / r, F_i. */
void orc_direct_coulomb(int n, const double* pos, const double* q, double* phi,
                        double* F);
/* phi_i = sum_{j!=i} q_j r^-nu, F_i = -q_i grad_i phi_i. */
void orc_direct_nu(int nu, int n, const double* pos, const double* q, double* phi, double* F);

/* Ewald potential of a unit charge plus its periodic images, tin-foil
 * boundary and neutralising background; 3-D (all axes periodic) and 2-D
 * slab (x, y periodic, z free); the 1-D sum below.  reg = 1 returns
 * lim (psi - 1/|x|) at x = 0. */
double orc_ewald3d(const double box[3], double alpha, const double x[3], int reg);
/* The 3-D Ewald potential for the lattice spanned by the columns of H. */
double orc_ewald3d_cell(const double H[9], double alpha, const double x[3], int reg);
double orc_ewald2d(const double box[3], double alpha, const double x[3], int reg);
/* 1-D sum: axis periodic (length box[axis]), the other two free; the
 * constant is the one for which psi -> -(2/L) ln(rho/L) far from the axis. */
double orc_ewald1d(const double box[3], int axis, double alpha, const double x[3], int reg);
/* The lattice sum of r^-6 over a 3-D periodic box, sum_n |x + n|^-6, by the
 * Ewald method (absolutely convergent: no boundary term); reg = 1 at x = 0
 * leaves out the n = 0 term. */
double orc_ewald3d_r6(const double box[3], double alpha, const double x[3], int reg);
/* The same lattice sum of r^-6 over two periodic axes (free axis f) or one
 * (axis), and for any mask 1..7. */
double orc_ewald2d_r6(const double box[3], int f, double alpha, const double x[3], int reg);
double orc_ewald1d_r6(const double box[3], int axis, double alpha, const double x[3], int reg);
double orc_ewald_r6(const double box[3], unsigned mask, double alpha, const double x[3],
                    int reg);
/* ... and over the lattice spanned by the columns of H. */
double orc_ewald3d_cell_r6(const double H[9], double alpha, const double x[3], int reg);
/* psi for the periodic axes of mask (bit k = axis k): 7, any two, any one. */
double orc_ewald_psi(const double box[3], unsigned mask, double alpha, const double x[3],
                     int reg);
/* phi_i = sum_j q_j psi(r_i - r_j), with psi_reg(0) for j = i. */
void orc_ewald_potentials_mask(const double box[3], unsigned mask, double alpha, int n,
                               const double* pos, const double* q, double* phi);
void orc_ewald_potentials(const double box[3], int slab, double alpha, int n,
                          const double* pos, const double* q, double* phi);
void orc_ewald_potentials_cell(const double H[9], double alpha, int n, const double* pos,
                               const double* q, double* phi);
/* The same potentials for a 3-D periodic box, and the forces, through the
 * structure factor (O(N K) reciprocal space instead of a lattice sum per pair). */
void orc_ewald3d_system(const double box[3], double alpha, int n, const double* pos,
                        const double* q, double* phi, double* F);

#ifdef __cplusplus
}
#endif
#endif
