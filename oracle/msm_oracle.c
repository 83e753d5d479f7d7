/*
 * msm_oracle.c -- TEST INFRASTRUCTURE ONLY (see msm_oracle.h).
 *
 * Plain FP64 reference of the multilevel summation method with B-spline
 * interpolation.  Each routine follows one passage of the paper and is
 * written for the reader, not for speed: no blocking, no fusion, no
 * reordering beyond what the quoted definition states.  OpenMP only
 * distributes independent outer iterations.
 */
#include "msm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops of this file run on. */
int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets that number (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Softening function (Sec. "Splitting for Coulomb kernels"): gamma(rho) is
 * 1/rho for rho >= 1 and, below 1, the Taylor polynomial of s^(-1/2) about
 * s = 1 up to degree p-1 in s, evaluated at s = rho^2.  The same
 * construction splits k(r) = r^-nu for other powers (the paper's splitting
 * applies to any such kernel; nu = 6 is the dispersion kernel): gamma_nu is
 * rho^-nu for rho >= 1 and the Taylor polynomial of s^(-nu/2) below.
 * ---------------------------------------------------------------------- */
static double binom_gen(double x, int k) /* binomial coefficient C(x, k) */
{
  double c = 1.0;
  for (int j = 0; j < k; ++j) c *= (x - j) / (double)(j + 1);
  return c;
}

/* g(s) = sum_{k<p} C(-nu/2,k) (s-1)^k and its s-derivatives */
static double taylor_g(int nu, int p, double s, int deriv)
{
  double sum = 0.0;
  for (int k = deriv; k < p; ++k) {
    double fall = 1.0; /* k (k-1) ... (k-deriv+1) */
    for (int j = 0; j < deriv; ++j) fall *= (double)(k - j);
    sum += binom_gen(-0.5 * nu, k) * fall * pow(s - 1.0, k - deriv);
  }
  return sum;
}

/* gamma_nu(rho) (deriv = 0) and its first two rho-derivatives */
double orc_gamma_nu(int nu, int p, double rho, int deriv)
{
  if (rho >= 1.0) {
    if (deriv == 0) return pow(rho, -nu);
    if (deriv == 1) return -nu * pow(rho, -nu - 1);
    return nu * (nu + 1.0) * pow(rho, -nu - 2);
  }
  double s = rho * rho;
  if (deriv == 0) return taylor_g(nu, p, s, 0);
  if (deriv == 1) return 2.0 * rho * taylor_g(nu, p, s, 1);
  return 2.0 * taylor_g(nu, p, s, 1) + 4.0 * s * taylor_g(nu, p, s, 2);
}

double orc_gamma(int p, double rho) { return orc_gamma_nu(1, p, rho, 0); }
double orc_gamma_d1(int p, double rho) { return orc_gamma_nu(1, p, rho, 1); }
double orc_gamma_d2(int p, double rho) { return orc_gamma_nu(1, p, rho, 2); }

/* Partial kernels of r^-nu (eq. coulomb_splitting_with_softener):
 * k_0 = r^-nu - gamma(r/a)/a^nu, k_l = gamma(r/a_l)/a_l^nu -
 * gamma(r/a_{l+1})/a_{l+1}^nu, k_L = gamma(r/a_L)/a_L^nu, a_l = 2^(l-1) a. */
double orc_kernel_nu(int nu, int l, int L, double a, int p, double r)
{
  if (l == 0) return pow(r, -nu) - orc_gamma_nu(nu, p, r / a, 0) / pow(a, nu);
  double s0 = ldexp(a, l - 1); /* 2^(l-1) a */
  if (l == L) return orc_gamma_nu(nu, p, r / s0, 0) / pow(s0, nu);
  double s1 = ldexp(a, l); /* 2^l a */
  return orc_gamma_nu(nu, p, r / s0, 0) / pow(s0, nu) -
         orc_gamma_nu(nu, p, r / s1, 0) / pow(s1, nu);
}

double orc_kernel(int l, int L, double a, int p, double r)
{
  return orc_kernel_nu(1, l, L, a, p, r);
}

/* First (deriv = 1) and second r-derivatives of k_0 */
double orc_k0_nu(int nu, double a, int p, double r, int deriv)
{
  if (deriv == 1)
    return -nu * pow(r, -nu - 1) - orc_gamma_nu(nu, p, r / a, 1) / pow(a, nu + 1);
  return nu * (nu + 1.0) * pow(r, -nu - 2) - orc_gamma_nu(nu, p, r / a, 2) / pow(a, nu + 2);
}

double orc_k0_d1(double a, int p, double r) { return orc_k0_nu(1, a, p, r, 1); }
double orc_k0_d2(double a, int p, double r) { return orc_k0_nu(1, a, p, r, 2); }

/* the power of the geometry's kernel (0 stands for Coulomb, nu = 1) */
static int geom_nu(const orc_geom* g) { return g->nu > 0 ? g->nu : 1; }

/* ------------------------------------------------------------------------
 * Cardinal B-splines (Sec. "B-spline interpolation"): M_1 is the indicator
 * of [0,1) and M_k(t) = [t M_{k-1}(t) + (k-t) M_{k-1}(t-1)] / (k-1) (de Boor
 * recursion).  The basis function centred on a grid point is
 * Phi_p(t) = M_p(t + p/2).  M_k' = M_{k-1}(t) - M_{k-1}(t-1).
 * cardinal_M evaluates M_k(t - j) for j = 0..k-1 bottom-up through the same
 * recursion and returns M_k(t).
 * ---------------------------------------------------------------------- */
static double cardinal_M(int k, double t)
{
  if (k <= 0) return 0.0;
  double B[32];
  /* order 1: B[j] = M_1(t - j) */
  for (int j = 0; j < k; ++j) {
    double tj = t - j;
    B[j] = (tj >= 0.0 && tj < 1.0) ? 1.0 : 0.0;
  }
  for (int ord = 2; ord <= k; ++ord) {
    /* B[j] <- M_ord(t - j) for j = 0..k-ord */
    for (int j = 0; j + ord <= k; ++j) {
      double tj = t - j;
      B[j] = (tj * B[j] + (ord - tj) * B[j + 1]) / (double)(ord - 1);
    }
  }
  return B[0];
}

double orc_bspline(int p, double t) { return cardinal_M(p, t + 0.5 * p); }

double orc_bspline_d1(int p, double t)
{
  double u = t + 0.5 * p;
  return cardinal_M(p - 1, u) - cardinal_M(p - 1, u - 1.0);
}

double orc_bspline_d2(int p, double t)
{
  double u = t + 0.5 * p;
  return cardinal_M(p - 2, u) - 2.0 * cardinal_M(p - 2, u - 1.0) +
         cardinal_M(p - 2, u - 2.0);
}

/* ------------------------------------------------------------------------
 * Basis functions of one level along one axis.  For a particle coordinate x
 * the non-zero basis functions are the p grid points m = floor(x/h) - p/2 + 1
 * ... floor(x/h) + p/2 (index set M_i of the paper).  Periodic axes use the
 * periodic basis sum_j Phi(x/h - m - j n), i.e. the index is taken mod n.
 * Returns -1 if a non-zero weight falls outside a non-periodic grid.
 * ---------------------------------------------------------------------- */
typedef struct {
  int idx[32];    /* array index (0..n-1) */
  double w[32];   /* Phi */
  double dw[32];  /* d Phi / dx */
  double d2w[32]; /* d^2 Phi / dx^2 */
} axis_basis;

static int basis_axis(const orc_geom* g, int level, int ax, double x, axis_basis* b)
{
  const int p = g->p;
  const double h = g->h[level - 1][ax];
  const int n = g->n[level - 1][ax];
  const int lo = g->lo[level - 1][ax];
  if (g->periodic[ax]) {
    double Lb = g->box[ax];
    x = x - Lb * floor(x / Lb);
  }
  double u = x / h;
  int base = (int)floor(u);
  for (int k = 0; k < p; ++k) {
    int m = base - p / 2 + 1 + k;
    double t = u - m;
    b->w[k] = orc_bspline(p, t);
    b->dw[k] = orc_bspline_d1(p, t) / h;
    b->d2w[k] = orc_bspline_d2(p, t) / (h * h);
    int ai;
    if (g->periodic[ax]) {
      ai = ((m % n) + n) % n;
    } else {
      ai = m - lo;
      if (ai < 0 || ai >= n) {
        if (b->w[k] != 0.0 || b->dw[k] != 0.0) return -1;
        ai = -1; /* zero weight, skipped */
      }
    }
    b->idx[k] = ai;
  }
  return 0;
}

/* Grid coordinates of a position: r itself in an orthorhombic box; in a
 * triclinic cell the fractional coordinates s = H^{-1} r, in which the grids
 * are rectangular (the unit-cube transform, Sec. MSM core algorithm). */
static void grid_position(const orc_geom* g, const double* r, double s[3])
{
  for (int k = 0; k < 3; ++k)
    s[k] = g->tri ? g->Hinv[3 * k] * r[0] + g->Hinv[3 * k + 1] * r[1] + g->Hinv[3 * k + 2] * r[2]
                  : r[k];
}

/* A vector v in grid coordinates: H^{-1} v in a triclinic cell (so that
 * v . grad_r f = (H^{-1} v) . grad_s f), v itself otherwise. */
static void grid_vector(const orc_geom* g, const double* v, double vs[3])
{
  grid_position(g, v, vs);
}

/* A gradient taken in grid coordinates, made Cartesian: grad_r = H^{-T} grad_s. */
static void cart_gradient(const orc_geom* g, const double gs[3], double gr[3])
{
  for (int j = 0; j < 3; ++j)
    gr[j] = g->tri ? g->Hinv[j] * gs[0] + g->Hinv[3 + j] * gs[1] + g->Hinv[6 + j] * gs[2]
                   : gs[j];
}

static long flat(const orc_geom* g, int level, int ix, int iy, int iz)
{
  const int* n = g->n[level - 1];
  return ((long)iz * n[1] + iy) * n[0] + ix;
}

int orc_anterpolate(const orc_geom* g, int level, int n, const double* pos,
                    const double* q, double* grid)
{
  /* Alg. anterpolation_double_loop: outer loop over particles, inner loop
   * over the index set of each particle. */
  const int p = g->p;
  for (int i = 0; i < n; ++i) {
    axis_basis bx, by, bz;
    double x[3];
    grid_position(g, pos + 3 * i, x);
    if (basis_axis(g, level, 0, x[0], &bx) || basis_axis(g, level, 1, x[1], &by) ||
        basis_axis(g, level, 2, x[2], &bz))
      return -1;
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) {
          if (bx.idx[a] < 0 || by.idx[b] < 0 || bz.idx[c] < 0) continue;
          grid[flat(g, level, bx.idx[a], by.idx[b], bz.idx[c])] +=
              q[i] * bx.w[a] * by.w[b] * bz.w[c];
        }
  }
  return 0;
}

int orc_anterpolate_dipole(const orc_geom* g, int level, int n, const double* pos,
                           const double* q, const double* v, double* grid)
{
  const int p = g->p;
  for (int i = 0; i < n; ++i) {
    axis_basis bx, by, bz;
    double x[3], vs[3];
    grid_position(g, pos + 3 * i, x);
    grid_vector(g, v + 3 * i, vs);
    if (basis_axis(g, level, 0, x[0], &bx) || basis_axis(g, level, 1, x[1], &by) ||
        basis_axis(g, level, 2, x[2], &bz))
      return -1;
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) {
          if (bx.idx[a] < 0 || by.idx[b] < 0 || bz.idx[c] < 0) continue;
          double gx = bx.dw[a] * by.w[b] * bz.w[c];
          double gy = bx.w[a] * by.dw[b] * bz.w[c];
          double gz = bx.w[a] * by.w[b] * bz.dw[c];
          grid[flat(g, level, bx.idx[a], by.idx[b], bz.idx[c])] +=
              q[i] * (vs[0] * gx + vs[1] * gy + vs[2] * gz);
        }
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Stencil (eq. kernel_stencil_by_conv_with_universal_coeff):
 *   K^l_m = sum_n omega'_{mx-nx} omega'_{my-ny} omega'_{mz-nz} k_l(|h_l o n|)
 * written as the plain triple sum over the omega' support.  The samples of
 * k_l are tabulated first on the box |n_k| <= W_k + M.  In a triclinic cell
 * the grid offset n is the Cartesian vector H (h_l o n) (fractional spacing
 * h_l = 1/n_l along each lattice vector).
 * ---------------------------------------------------------------------- */
static double omega_at(const orc_geom* g, int j)
{
  j = j < 0 ? -j : j;
  return j <= g->M ? g->omega[j] : 0.0;
}

void orc_stencil(const orc_geom* g, int level, const int W[3], double* K)
{
  const int M = g->M;
  const double* h = g->h[level - 1];
  int S[3], ns[3];
  for (int k = 0; k < 3; ++k) {
    S[k] = W[k] + M;
    ns[k] = 2 * S[k] + 1;
  }
  double* samp = (double*)malloc(sizeof(double) * ns[0] * ns[1] * ns[2]);
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = -S[2]; z <= S[2]; ++z)
    for (int y = -S[1]; y <= S[1]; ++y)
      for (int x = -S[0]; x <= S[0]; ++x) {
        double u[3] = {x * h[0], y * h[1], z * h[2]}, d[3];
        for (int k = 0; k < 3; ++k)
          d[k] = g->tri ? g->H[3 * k] * u[0] + g->H[3 * k + 1] * u[1] + g->H[3 * k + 2] * u[2]
                        : u[k];
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        samp[((long)(z + S[2]) * ns[1] + (y + S[1])) * ns[0] + (x + S[0])] =
            orc_kernel_nu(geom_nu(g), level, g->L, g->a, g->p, r);
      }
  int nk[3] = {2 * W[0] + 1, 2 * W[1] + 1, 2 * W[2] + 1};
#pragma omp parallel for collapse(2) schedule(static)
  for (int mz = -W[2]; mz <= W[2]; ++mz)
    for (int my = -W[1]; my <= W[1]; ++my)
      for (int mx = -W[0]; mx <= W[0]; ++mx) {
        double sum = 0.0;
        for (int kz = -M; kz <= M; ++kz)
          for (int ky = -M; ky <= M; ++ky)
            for (int kx = -M; kx <= M; ++kx) {
              /* n = m - k */
              int nx = mx - kx, ny = my - ky, nz = mz - kz;
              double s = samp[((long)(nz + S[2]) * ns[1] + (ny + S[1])) * ns[0] +
                              (nx + S[0])];
              sum += omega_at(g, kx) * omega_at(g, ky) * omega_at(g, kz) * s;
            }
        K[((long)(mz + W[2]) * nk[1] + (my + W[1])) * nk[0] + (mx + W[0])] = sum;
      }
  free(samp);
}

/* ------------------------------------------------------------------------
 * Grid potential (eq. action_of_K_as_convolution): e_m = sum_n K_{m-n} q_n.
 * Written as a sum over stencil offsets d = m - n.
 * ---------------------------------------------------------------------- */
static void conv_point(const orc_geom* g, int level, const int W[3], const double* K,
                       const double* qgrid, double* egrid, long m)
{
  const int* n = g->n[level - 1];
  int nk[3] = {2 * W[0] + 1, 2 * W[1] + 1, 2 * W[2] + 1};
  int mx = (int)(m % n[0]);
  int my = (int)((m / n[0]) % n[1]);
  int mz = (int)(m / ((long)n[0] * n[1]));
  double sum = 0.0;
  for (int dz = -W[2]; dz <= W[2]; ++dz) {
    int iz = mz - dz;
    if (g->periodic[2]) iz = ((iz % n[2]) + n[2]) % n[2];
    else if (iz < 0 || iz >= n[2]) continue;
    for (int dy = -W[1]; dy <= W[1]; ++dy) {
      int iy = my - dy;
      if (g->periodic[1]) iy = ((iy % n[1]) + n[1]) % n[1];
      else if (iy < 0 || iy >= n[1]) continue;
      for (int dx = -W[0]; dx <= W[0]; ++dx) {
        int ix = mx - dx;
        if (g->periodic[0]) ix = ((ix % n[0]) + n[0]) % n[0];
        else if (ix < 0 || ix >= n[0]) continue;
        double kv = K[((long)(dz + W[2]) * nk[1] + (dy + W[1])) * nk[0] + (dx + W[0])];
        sum += kv * qgrid[((long)iz * n[1] + iy) * n[0] + ix];
      }
    }
  }
  egrid[m] = sum;
}

void orc_conv(const orc_geom* g, int level, const int W[3], const double* K,
              const double* qgrid, double* egrid, int npts, const int* pts)
{
  const int* n = g->n[level - 1];
  if (npts < 0) {
    long G = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (long m = 0; m < G; ++m) conv_point(g, level, W, K, qgrid, egrid, m);
  } else {
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < npts; ++i) conv_point(g, level, W, K, qgrid, egrid, pts[i]);
  }
}

/* ------------------------------------------------------------------------
 * Interpolation (eqs. uoneplus_interpolation_with_index_set,
 * analytic_uoneplus_position_grad, analytic_uoneplus_charge_grad).
 * ---------------------------------------------------------------------- */
int orc_interpolate(const orc_geom* g, int level, int n, const double* pos,
                    const double* q, const double* egrid, double* phi, double* F)
{
  const int p = g->p;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    axis_basis bx, by, bz;
    double x[3];
    grid_position(g, pos + 3 * i, x);
    if (basis_axis(g, level, 0, x[0], &bx) || basis_axis(g, level, 1, x[1], &by) ||
        basis_axis(g, level, 2, x[2], &bz)) {
      bad = 1;
      continue;
    }
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) {
          if (bx.idx[a] < 0 || by.idx[b] < 0 || bz.idx[c] < 0) continue;
          double e = egrid[flat(g, level, bx.idx[a], by.idx[b], bz.idx[c])];
          v += e * bx.w[a] * by.w[b] * bz.w[c];
          gx += e * bx.dw[a] * by.w[b] * bz.w[c];
          gy += e * bx.w[a] * by.dw[b] * bz.w[c];
          gz += e * bx.w[a] * by.w[b] * bz.dw[c];
        }
    if (phi) phi[i] += v;
    if (F) {
      double gs[3] = {gx, gy, gz}, gr[3];
      cart_gradient(g, gs, gr);
      F[3 * i + 0] -= q[i] * gr[0];
      F[3 * i + 1] -= q[i] * gr[1];
      F[3 * i + 2] -= q[i] * gr[2];
    }
  }
  return bad ? -1 : 0;
}

/* For L = sum_i v_i . F_i with F_i = -q_i sum_m psi_m grad phi_m(r_i) and
 * psi = K q~ (K symmetric), the cotangents are
 *   dL/dq_i = -sum_m [psiD_m phi_m(r_i) + psi_m v_i . grad phi_m(r_i)]
 *   dL/dr_i = -q_i sum_m [psiD_m grad phi_m(r_i) + psi_m (Hess phi_m(r_i)) v_i]
 * with psiD = K D and D the dipole anterpolation of q_i v_i. */
int orc_interpolate_vjp(const orc_geom* g, int level, int n, const double* pos,
                        const double* q, const double* v, const double* psi,
                        const double* psiD, double* gq, double* gr)
{
  const int p = g->p;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    axis_basis bx, by, bz;
    double x[3], vs[3];
    grid_position(g, pos + 3 * i, x);
    grid_vector(g, v + 3 * i, vs); /* grid-coordinate cotangent */
    if (basis_axis(g, level, 0, x[0], &bx) || basis_axis(g, level, 1, x[1], &by) ||
        basis_axis(g, level, 2, x[2], &bz)) {
      bad = 1;
      continue;
    }
    const double vx = vs[0], vy = vs[1], vz = vs[2];
    double sq = 0.0, sr[3] = {0, 0, 0};
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) {
          if (bx.idx[a] < 0 || by.idx[b] < 0 || bz.idx[c] < 0) continue;
          long f = flat(g, level, bx.idx[a], by.idx[b], bz.idx[c]);
          double w = bx.w[a] * by.w[b] * bz.w[c];
          double grad[3] = {bx.dw[a] * by.w[b] * bz.w[c], bx.w[a] * by.dw[b] * bz.w[c],
                            bx.w[a] * by.w[b] * bz.dw[c]};
          double H[3][3];
          H[0][0] = bx.d2w[a] * by.w[b] * bz.w[c];
          H[1][1] = bx.w[a] * by.d2w[b] * bz.w[c];
          H[2][2] = bx.w[a] * by.w[b] * bz.d2w[c];
          H[0][1] = H[1][0] = bx.dw[a] * by.dw[b] * bz.w[c];
          H[0][2] = H[2][0] = bx.dw[a] * by.w[b] * bz.dw[c];
          H[1][2] = H[2][1] = bx.w[a] * by.dw[b] * bz.dw[c];
          double vg = vx * grad[0] + vy * grad[1] + vz * grad[2];
          sq += psiD[f] * w + psi[f] * vg;
          for (int k = 0; k < 3; ++k)
            sr[k] += psiD[f] * grad[k] +
                     psi[f] * (H[k][0] * vx + H[k][1] * vy + H[k][2] * vz);
        }
    gq[i] -= sq;
    double srr[3];
    cart_gradient(g, sr, srr); /* grad_r = H^{-T} grad_s, Hess_r v = H^{-T} Hess_s H^{-1} v */
    for (int k = 0; k < 3; ++k) gr[3 * i + k] -= q[i] * srr[k];
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * Short-range part (eq. U_zero): pairs closer than a, minimum image on the
 * periodic axes (valid for a <= L/2, Sec. Madelung constants).
 * ---------------------------------------------------------------------- */
static void min_image(const orc_geom* g, double d[3])
{
  if (!g->tri) {
    for (int k = 0; k < 3; ++k)
      if (g->periodic[k]) d[k] -= g->box[k] * round(d[k] / g->box[k]);
    return;
  }
  /* triclinic: round the fractional difference, then take the shortest of
   * that image and its 26 neighbours (rounding alone can miss the nearest
   * image of a skewed cell) */
  double ds[3];
  grid_position(g, d, ds);
  for (int k = 0; k < 3; ++k) ds[k] -= round(ds[k]);
  double best[3] = {0, 0, 0}, b2 = INFINITY;
  for (int jz = -1; jz <= 1; ++jz)
    for (int jy = -1; jy <= 1; ++jy)
      for (int jx = -1; jx <= 1; ++jx) {
        double u[3] = {ds[0] + jx, ds[1] + jy, ds[2] + jz}, c[3];
        for (int k = 0; k < 3; ++k)
          c[k] = g->H[3 * k] * u[0] + g->H[3 * k + 1] * u[1] + g->H[3 * k + 2] * u[2];
        double r2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (r2 < b2) {
          b2 = r2;
          best[0] = c[0];
          best[1] = c[1];
          best[2] = c[2];
        }
      }
  d[0] = best[0];
  d[1] = best[1];
  d[2] = best[2];
}

void orc_short_range(const orc_geom* g, int n, const double* pos, const double* q,
                     int nsel, const int* sel, double* phi, double* F)
{
  const int cnt = nsel < 0 ? n : nsel;
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < cnt; ++s) {
    int i = nsel < 0 ? s : sel[s];
    double ph = 0.0, f[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                     pos[3 * i + 2] - pos[3 * j + 2]};
      min_image(g, d);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(r < g->a)) continue;
      ph += q[j] * orc_kernel_nu(geom_nu(g), 0, g->L, g->a, g->p, r);
      double c = -q[i] * q[j] * orc_k0_nu(geom_nu(g), g->a, g->p, r, 1) / r;
      for (int k = 0; k < 3; ++k) f[k] += c * d[k];
    }
    if (phi) phi[s] += ph;
    if (F)
      for (int k = 0; k < 3; ++k) F[3 * s + k] += f[k];
  }
}

/* Plain cell list: cells of edge >= a, so every partner within a lies in the
 * -1..1 neighbour cells of a particle's own cell (distinct cells only: an axis
 * with fewer than 3 cells lists each cell once). */
typedef struct {
  int nc[3];
  double cs[3];
  int* cell;
  int* head;
  int* next;
} cell_list;

static void cell_list_build(const orc_geom* g, int n, const double* pos, cell_list* cl)
{
  /* (triclinic: cells in fractional coordinates, as many per axis as the
   * cell's width across that axis, V / |face|, holds whole cutoffs) */
  for (int k = 0; k < 3; ++k) {
    double w = g->box[k];
    if (g->tri) {
      const double* b = g->Hinv + 3 * k;
      w = 1.0 / sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    }
    cl->nc[k] = (int)floor(w / g->a);
    if (cl->nc[k] < 1) cl->nc[k] = 1;
    cl->cs[k] = g->box[k] / cl->nc[k];
  }
  long ncell = (long)cl->nc[0] * cl->nc[1] * cl->nc[2];
  cl->cell = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  cl->head = (int*)malloc(sizeof(int) * ncell);
  cl->next = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  for (long c = 0; c < ncell; ++c) cl->head[c] = -1;
  for (int i = n - 1; i >= 0; --i) {
    int ci[3];
    double xs[3];
    grid_position(g, pos + 3 * i, xs);
    for (int k = 0; k < 3; ++k) {
      double x = xs[k];
      if (g->periodic[k]) x -= g->box[k] * floor(x / g->box[k]);
      int c = (int)floor(x / cl->cs[k]);
      if (c < 0) c = 0;
      if (c >= cl->nc[k]) c = cl->nc[k] - 1;
      ci[k] = c;
    }
    long c = ((long)ci[2] * cl->nc[1] + ci[1]) * cl->nc[0] + ci[0];
    cl->cell[i] = (int)c;
    cl->next[i] = cl->head[c];
    cl->head[c] = i;
  }
}

static void cell_list_free(cell_list* cl)
{
  free(cl->cell);
  free(cl->head);
  free(cl->next);
}

/* The distinct neighbour cells of particle i: out[] receives up to 27 cell
 * indices, the count is returned. */
static int cell_list_neighbours(const orc_geom* g, const cell_list* cl, int i, long out[27])
{
  const int* nc = cl->nc;
  int c = cl->cell[i];
  int ci[3] = {c % nc[0], (c / nc[0]) % nc[1], c / (nc[0] * nc[1])};
  int list[3][3], cntk[3];
  for (int k = 0; k < 3; ++k) {
    cntk[k] = 0;
    for (int o = -1; o <= 1; ++o) {
      int cc = ci[k] + o;
      if (g->periodic[k]) cc = ((cc % nc[k]) + nc[k]) % nc[k];
      else if (cc < 0 || cc >= nc[k]) continue;
      int dup = 0;
      for (int u = 0; u < cntk[k]; ++u) dup |= (list[k][u] == cc);
      if (!dup) list[k][cntk[k]++] = cc;
    }
  }
  int m = 0;
  for (int uz = 0; uz < cntk[2]; ++uz)
    for (int uy = 0; uy < cntk[1]; ++uy)
      for (int ux = 0; ux < cntk[0]; ++ux)
        out[m++] = ((long)list[2][uz] * nc[1] + list[1][uy]) * nc[0] + list[0][ux];
  return m;
}

/* Pair (i, j) of the short-range sum: d = r_i - r_j (minimum image); returns 0
 * when r >= a, else adds q_j k0(r) to *ph and -q_i q_j k0'(r)/r d to f. */
static int sr_pair(const orc_geom* g, const double* pos, const double* q, int i, int j,
                   double* ph, double f[3])
{
  double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                 pos[3 * i + 2] - pos[3 * j + 2]};
  min_image(g, d);
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (!(r < g->a)) return 0;
  *ph += q[j] * orc_kernel_nu(geom_nu(g), 0, g->L, g->a, g->p, r);
  double c = -q[i] * q[j] * orc_k0_nu(geom_nu(g), g->a, g->p, r, 1) / r;
  for (int k = 0; k < 3; ++k) f[k] += c * d[k];
  return 1;
}

void orc_short_range_cells(const orc_geom* g, int n, const double* pos,
                           const double* q, int nsel, const int* sel, double* phi, double* F)
{
  cell_list cl;
  cell_list_build(g, n, pos, &cl);
  const int cnt = nsel < 0 ? n : nsel;
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < cnt; ++s) {
    int i = nsel < 0 ? s : sel[s];
    long nb[27];
    int m = cell_list_neighbours(g, &cl, i, nb);
    double ph = 0.0, f[3] = {0, 0, 0};
    for (int u = 0; u < m; ++u)
      for (int j = cl.head[nb[u]]; j >= 0; j = cl.next[j])
        if (j != i) sr_pair(g, pos, q, i, j, &ph, f);
    if (phi) phi[s] += ph;
    if (F)
      for (int k = 0; k < 3; ++k) F[3 * s + k] += f[k];
  }
  cell_list_free(&cl);
}

/* With f(r) = -k0'(r)/r the short-range force is F0_i = q_i sum_j q_j f d_ij,
 * d_ij = r_i - r_j.  For L0 = sum_i v_i . F0_i the pair (i, j) adds
 *   dL0/dq_i = q_j f (v_i - v_j) . d_ij
 *   dL0/dr_i = q_i q_j [ f (v_i - v_j) + (f'/r) ((v_i - v_j) . d_ij) d_ij ]
 * with f'(r) = -k0''(r)/r + k0'(r)/r^2. */
static void vjp_pair(const orc_geom* g, const double* pos, const double* q, const double* v,
                     int i, int j, double* sq, double sr[3])
{
  double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                 pos[3 * i + 2] - pos[3 * j + 2]};
  min_image(g, d);
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (!(r < g->a)) return;
  double k1 = orc_k0_nu(geom_nu(g), g->a, g->p, r, 1), k2 = orc_k0_nu(geom_nu(g), g->a, g->p, r, 2);
  double f = -k1 / r;
  double fp = -k2 / r + k1 / (r * r);
  double dv[3] = {v[3 * i] - v[3 * j], v[3 * i + 1] - v[3 * j + 1],
                  v[3 * i + 2] - v[3 * j + 2]};
  double dvd = dv[0] * d[0] + dv[1] * d[1] + dv[2] * d[2];
  *sq += q[j] * f * dvd;
  for (int k = 0; k < 3; ++k)
    sr[k] += q[i] * q[j] * (f * dv[k] + (fp / r) * dvd * d[k]);
}

void orc_short_range_vjp(const orc_geom* g, int n, const double* pos, const double* q,
                         const double* v, int nsel, const int* sel, double* gq, double* gr)
{
  const int cnt = nsel < 0 ? n : nsel;
#pragma omp parallel for schedule(dynamic, 16)
  for (int s = 0; s < cnt; ++s) {
    int i = nsel < 0 ? s : sel[s];
    double sq = 0.0, sr[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j)
      if (j != i) vjp_pair(g, pos, q, v, i, j, &sq, sr);
    gq[s] += sq;
    for (int k = 0; k < 3; ++k) gr[3 * s + k] += sr[k];
  }
}

void orc_short_range_vjp_cells(const orc_geom* g, int n, const double* pos,
                               const double* q, const double* v, double* gq, double* gr)
{
  cell_list cl;
  cell_list_build(g, n, pos, &cl);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    long nb[27];
    int m = cell_list_neighbours(g, &cl, i, nb);
    double sq = 0.0, sr[3] = {0, 0, 0};
    for (int u = 0; u < m; ++u)
      for (int j = cl.head[nb[u]]; j >= 0; j = cl.next[j])
        if (j != i) vjp_pair(g, pos, q, v, i, j, &sq, sr);
    gq[i] += sq;
    for (int k = 0; k < 3; ++k) gr[3 * i + k] += sr[k];
  }
  cell_list_free(&cl);
}

void orc_direct_coulomb(int n, const double* pos, const double* q, double* phi,
                        double* F)
{
  orc_direct_nu(1, n, pos, q, phi, F);
}

void orc_direct_nu(int nu, int n, const double* pos, const double* q, double* phi, double* F)
{
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    double ph = 0.0, f[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                     pos[3 * i + 2] - pos[3 * j + 2]};
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      ph += q[j] * pow(r, -nu);
      double c = nu * q[i] * q[j] * pow(r, -nu - 2);
      for (int k = 0; k < 3; ++k) f[k] += c * d[k];
    }
    if (phi) phi[i] = ph;
    if (F)
      for (int k = 0; k < 3; ++k) F[3 * i + k] = f[k];
  }
}

/* ------------------------------------------------------------------------
 * Ewald sums (Ewald 1921; slab form of Parry 1975 / Heyes, Barber and
 * Clarke 1977).  Potential of a unit charge at the origin plus its images,
 * tin-foil boundary; the 3-D form includes the neutralising background
 * -pi/(alpha^2 V).  Cut-offs keep every dropped term below ~1e-19.
 * ---------------------------------------------------------------------- */
#define ORC_EWALD_X 6.6 /* erfc(6.6) ~ 1e-20 */

double orc_ewald3d(const double box[3], double alpha, const double x[3], int reg)
{
  const double V = box[0] * box[1] * box[2];
  const double rc = ORC_EWALD_X / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  double real = 0.0;
  int nr[3];
  for (int k = 0; k < 3; ++k) nr[k] = (int)ceil(rc / box[k]) + 1;
  for (int jz = -nr[2]; jz <= nr[2]; ++jz)
    for (int jy = -nr[1]; jy <= nr[1]; ++jy)
      for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
        double dx = x[0] + jx * box[0], dy = x[1] + jy * box[1], dz = x[2] + jz * box[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) {
          if (!reg) return INFINITY;
          real -= 2.0 * alpha / sqrt(M_PI); /* lim erfc(ar)/r - 1/r */
          continue;
        }
        if (r > rc) continue;
        real += erfc(alpha * r) / r;
      }
  double recip = 0.0;
  int nk[3];
  for (int k = 0; k < 3; ++k) nk[k] = (int)ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  for (int kz = -nk[2]; kz <= nk[2]; ++kz)
    for (int ky = -nk[1]; ky <= nk[1]; ++ky)
      for (int kx = -nk[0]; kx <= nk[0]; ++kx) {
        if (kx == 0 && ky == 0 && kz == 0) continue;
        double gx = 2.0 * M_PI * kx / box[0], gy = 2.0 * M_PI * ky / box[1],
               gz = 2.0 * M_PI * kz / box[2];
        double k2 = gx * gx + gy * gy + gz * gz;
        if (k2 > kc * kc) continue;
        recip += exp(-k2 / (4.0 * alpha * alpha)) * cos(gx * x[0] + gy * x[1] + gz * x[2]) / k2;
      }
  recip *= 4.0 * M_PI / V;
  return real + recip - M_PI / (alpha * alpha * V);
}

double orc_ewald2d(const double box[3], double alpha, const double x[3], int reg)
{
  const double A = box[0] * box[1];
  const double rc = ORC_EWALD_X / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  const double z = x[2];
  double real = 0.0;
  int nr[2];
  for (int k = 0; k < 2; ++k) nr[k] = (int)ceil(rc / box[k]) + 1;
  for (int jy = -nr[1]; jy <= nr[1]; ++jy)
    for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
      double dx = x[0] + jx * box[0], dy = x[1] + jy * box[1];
      double r = sqrt(dx * dx + dy * dy + z * z);
      if (r == 0.0) {
        if (!reg) return INFINITY;
        real -= 2.0 * alpha / sqrt(M_PI);
        continue;
      }
      if (r > rc) continue;
      real += erfc(alpha * r) / r;
    }
  double recip = 0.0;
  int nk[2];
  for (int k = 0; k < 2; ++k) nk[k] = (int)ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  for (int ky = -nk[1]; ky <= nk[1]; ++ky)
    for (int kx = -nk[0]; kx <= nk[0]; ++kx) {
      if (kx == 0 && ky == 0) continue;
      double gx = 2.0 * M_PI * kx / box[0], gy = 2.0 * M_PI * ky / box[1];
      double k = sqrt(gx * gx + gy * gy);
      if (k > kc) continue;
      double t1 = 0.0, t2;
      double u1 = k / (2.0 * alpha) + alpha * z;
      if (k * z < 700.0) t1 = exp(k * z) * erfc(u1);
      t2 = (-k * z < 700.0) ? exp(-k * z) * erfc(k / (2.0 * alpha) - alpha * z) : 0.0;
      recip += cos(gx * x[0] + gy * x[1]) / k * (t1 + t2);
    }
  recip *= M_PI / A;
  double k0 = -(2.0 * M_PI / A) *
              (z * erf(alpha * z) + exp(-alpha * alpha * z * z) / (alpha * sqrt(M_PI)));
  return real + recip + k0;
}

/* ------------------------------------------------------------------------
 * 1-D Ewald sum: one periodic axis of length L, the other two free.  With
 * rho the distance from the periodic axis and z the coordinate along it,
 * Poisson summation of the smooth part erf(alpha r)/r along the axis gives
 *   psi(x) = sum_n erfc(alpha r_n)/r_n
 *          + (1/L) [gamma_E + 2 ln(alpha L) - Ein(alpha^2 rho^2)]
 *          + (2/L) sum_{m >= 1} cos(k_m z) F(k_m, rho),     k_m = 2 pi m / L,
 *   F(k, rho) = int_{k^2/(4 alpha^2)}^inf exp(-s - rho^2 k^2/(4 s)) ds / s
 *             = int_0^inf exp(-b e^t - alpha^2 rho^2 e^-t) dt,  b = k^2/(4 alpha^2),
 * (the incomplete Bessel function; 2 K0(k rho) as alpha -> inf).  The k = 0
 * term diverges logarithmically; the constant kept is the one for which
 * psi -> -(2/L) ln(rho/L) far from the axis, the same for every alpha, so
 * non-neutral systems get that convention and neutral ones are free of it.
 * Ein(x) = int_0^x (1 - e^-v)/v dv = gamma_E + ln x + E1(x).
 * ---------------------------------------------------------------------- */
#define ORC_EULER_GAMMA 0.57721566490153286061

/* Ein by its power series (Abramowitz and Stegun 5.1.11) for x <= 2, else
 * through E1 by its continued fraction (A&S 5.1.22, evaluated from the tail
 * with a fixed depth that is ample for x > 2). */
static double orc_ein(double x)
{
  if (x <= 2.0) {
    double term = x, sum = x;
    for (int k = 2; k < 200 && fabs(term) > 1e-20 * fabs(sum); ++k) {
      term *= -x * (k - 1) / ((double)k * k);
      sum += term;
    }
    return sum;
  }
  /* E1(x) = e^-x / (x + 1 - 1^2/(x + 3 - 2^2/(x + 5 - ...))) */
  double f = x + 2.0 * 400 + 1.0;
  for (int k = 400; k >= 1; --k) f = x + 2.0 * k - 1.0 - (double)k * k / f;
  const double e1 = exp(-x) / f;
  return e1 + ORC_EULER_GAMMA + log(x);
}

/* 16-point Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on
 * P_16 from the Chebyshev-like first guess). */
static void orc_gauss16(double xg[16], double wg[16])
{
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    xg[i] = x;
    wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

/* int_0^inf e^{-w t} exp(-b e^t - c e^-t) dt (w >= 0, b > 0) over the t-range
 * where the exponent b e^t + c e^-t stays below 45 (outside it the integrand
 * is below e^-45 and the tails add less than 1e-18), in panels of width
 * <= 1/8 with 16 Gauss points each.  w = 0 is F(k, rho) above. */
static double orc_exp_integral(double wexp, double b, double c, const double xg[16],
                               const double wg[16])
{
  const double E = 45.0, D = E * E - 4.0 * b * c;
  if (D <= 0.0) return 0.0;
  const double t1 = log((E + sqrt(D)) / (2.0 * b));
  if (t1 <= 0.0) return 0.0;
  double t0 = log((E - sqrt(D)) / (2.0 * b));
  if (t0 < 0.0) t0 = 0.0;
  const int np = (int)ceil((t1 - t0) * 8.0);
  const double w = (t1 - t0) / np;
  double sum = 0.0;
  for (int j = 0; j < np; ++j) {
    const double mid = t0 + (j + 0.5) * w;
    for (int i = 0; i < 16; ++i) {
      const double t = mid + 0.5 * w * xg[i];
      sum += 0.5 * w * wg[i] * exp(-wexp * t - b * exp(t) - c * exp(-t));
    }
  }
  return sum;
}

static double orc_incomplete_bessel(double b, double c, const double xg[16],
                                    const double wg[16])
{
  return orc_exp_integral(0.0, b, c, xg, wg);
}

double orc_ewald1d(const double box[3], int axis, double alpha, const double x[3], int reg)
{
  const double L = box[axis], z = x[axis];
  double rho2 = 0.0;
  for (int k = 0; k < 3; ++k)
    if (k != axis) rho2 += x[k] * x[k];
  const double rc = ORC_EWALD_X / alpha;
  const int nr = (int)ceil((rc + fabs(z)) / L) + 1;
  double real = 0.0;
  for (int j = -nr; j <= nr; ++j) {
    const double dz = z + j * L;
    const double r = sqrt(rho2 + dz * dz);
    if (r == 0.0) {
      if (!reg) return INFINITY;
      real -= 2.0 * alpha / sqrt(M_PI);
      continue;
    }
    if (r > rc) continue;
    real += erfc(alpha * r) / r;
  }
  const double c = alpha * alpha * rho2;
  const double k0 = (ORC_EULER_GAMMA + 2.0 * log(alpha * L) - orc_ein(c)) / L;
  double xg[16], wg[16];
  orc_gauss16(xg, wg);
  double recip = 0.0;
  for (int m = 1;; ++m) {
    const double k = 2.0 * M_PI * m / L, b = k * k / (4.0 * alpha * alpha);
    if (b > 45.0) break; /* F <= E1(b) < 1e-21 from here on */
    recip += cos(k * z) * orc_incomplete_bessel(b, c, xg, wg);
  }
  return real + k0 + 2.0 * recip / L;
}

/* ------------------------------------------------------------------------
 * 3-D lattice sum of the dispersion kernel r^-6 by the Ewald method.
 * From r^-6 = (1/2) int_0^inf t^2 e^{-r^2 t} dt split at t = alpha^2:
 *   real space   (1/2) int_{alpha^2}^inf t^2 e^{-r^2 t} dt
 *                = e^{-a^2} (1 + a^2 + a^4/2) / r^6,   a = alpha r;
 *   Fourier space (Poisson summation of the rest over the lattice)
 *                (pi^{3/2} alpha^3 / (3V)) sum_k [(1 - 2b^2) e^{-b^2}
 *                + 2 sqrt(pi) b^3 erfc(b)] cos(k.x),    b = |k| / (2 alpha),
 *   the k = 0 term included (pi^{3/2} alpha^3 / (3V)).
 * The sum converges absolutely, so no boundary term arises.  At a lattice
 * point the regular part replaces the real-space term of r = 0 by its limit
 * minus r^-6: -alpha^6 / 6.
 * ---------------------------------------------------------------------- */
double orc_ewald3d_r6(const double box[3], double alpha, const double x[3], int reg)
{
  const double V = box[0] * box[1] * box[2];
  /* e^{-a^2}(1 + a^2 + a^4/2) < 1e-18 from a = 7 on; b = 6.6 as in the
   * Coulomb sums bounds the dropped Fourier terms */
  const double rc = 7.0 / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  double real = 0.0;
  int nr[3];
  for (int k = 0; k < 3; ++k) nr[k] = (int)ceil((rc + fabs(x[k])) / box[k]) + 1;
  for (int jz = -nr[2]; jz <= nr[2]; ++jz)
    for (int jy = -nr[1]; jy <= nr[1]; ++jy)
      for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
        double dx = x[0] + jx * box[0], dy = x[1] + jy * box[1], dz = x[2] + jz * box[2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0) {
          if (!reg) return INFINITY;
          real -= pow(alpha, 6) / 6.0;
          continue;
        }
        if (r2 > rc * rc) continue;
        double a2 = alpha * alpha * r2;
        real += exp(-a2) * (1.0 + a2 + 0.5 * a2 * a2) / (r2 * r2 * r2);
      }
  double recip = 0.0;
  int nk[3];
  for (int k = 0; k < 3; ++k) nk[k] = (int)ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  for (int kz = -nk[2]; kz <= nk[2]; ++kz)
    for (int ky = -nk[1]; ky <= nk[1]; ++ky)
      for (int kx = -nk[0]; kx <= nk[0]; ++kx) {
        double gx = 2.0 * M_PI * kx / box[0], gy = 2.0 * M_PI * ky / box[1],
               gz = 2.0 * M_PI * kz / box[2];
        double k = sqrt(gx * gx + gy * gy + gz * gz);
        if (k > kc) continue;
        double b = k / (2.0 * alpha);
        double f = (1.0 - 2.0 * b * b) * exp(-b * b) + 2.0 * sqrt(M_PI) * b * b * b * erfc(b);
        recip += f * cos(gx * x[0] + gy * x[1] + gz * x[2]);
      }
  return real + pow(M_PI, 1.5) * alpha * alpha * alpha / (3.0 * V) * recip;
}

/* ------------------------------------------------------------------------
 * Lattice sums of r^-6 over two periodic axes (slab) or one (line), by the
 * same split as the 3-D sum: real space e^{-y}(1 + y + y^2/2)/r^6 over the
 * images, y = alpha^2 r^2; the rest, f(r) = (1/2) int_0^{alpha^2} t^2
 * e^{-r^2 t} dt, by Poisson summation over the periodic axes only.
 *   slab (cell area A, z the free coordinate, k over the 2-D reciprocal
 *   lattice): (1/A) sum_k cos(k.x) (pi/2) int_0^{alpha^2} t e^{-t z^2 - k^2/(4t)} dt;
 *   line (period L, rho the distance from the axis, k = 2 pi m / L):
 *   (1/L) sum_m cos(k z) (sqrt(pi)/2) int_0^{alpha^2} t^{3/2} e^{-t rho^2 - k^2/(4t)} dt.
 * With t = alpha^2 e^{-u} the k != 0 integrals become alpha^4 (slab), alpha^5
 * (line) times int_0^inf e^{-w u} exp(-b e^u - c e^-u) du, w = 2 or 5/2,
 * b = k^2/(4 alpha^2), c = alpha^2 z^2 or alpha^2 rho^2; the k = 0 ones are
 * elementary.  Both sums converge absolutely (no boundary term).
 * ---------------------------------------------------------------------- */
/* int_0^{alpha^2} t e^{-t z^2} dt */
static double orc_r6_slab_k0(double alpha, double z)
{
  const double a2 = alpha * alpha, y = a2 * z * z;
  if (y < 1.0) { /* series: alpha^4 sum_j (-y)^j / (j! (j + 2)) */
    double term = 1.0, sum = 0.5;
    for (int j = 1; j < 60; ++j) {
      term *= -y / j;
      sum += term / (j + 2);
    }
    return a2 * a2 * sum;
  }
  const double z4 = z * z * z * z;
  return (1.0 - exp(-y) * (1.0 + y)) / z4;
}

/* int_0^{alpha^2} t^{3/2} e^{-t rho^2} dt */
static double orc_r6_line_k0(double alpha, double rho)
{
  const double a2 = alpha * alpha, x = a2 * rho * rho;
  if (x < 1.0) { /* series: alpha^5 sum_j (-x)^j / (j! (j + 5/2)) */
    double term = 1.0, sum = 0.4;
    for (int j = 1; j < 60; ++j) {
      term *= -x / j;
      sum += term / (j + 2.5);
    }
    return a2 * a2 * alpha * sum;
  }
  /* lower incomplete gamma: gamma(5/2, x) / rho^5, with
   * Gamma(1/2, x) = sqrt(pi) erfc(sqrt x), Gamma(s+1, x) = s Gamma(s, x) + x^s e^-x */
  const double g12 = sqrt(M_PI) * erfc(sqrt(x));
  const double g32 = 0.5 * g12 + sqrt(x) * exp(-x);
  const double g52 = 1.5 * g32 + x * sqrt(x) * exp(-x);
  const double lower = 0.75 * sqrt(M_PI) - g52;
  const double r5 = rho * rho * rho * rho * rho;
  return lower / r5;
}

static double orc_r6_real(double alpha, double r2)
{
  const double y = alpha * alpha * r2;
  return exp(-y) * (1.0 + y + 0.5 * y * y) / (r2 * r2 * r2);
}

/* slab: free axis f, the other two periodic */
double orc_ewald2d_r6(const double box[3], int f, double alpha, const double x[3], int reg)
{
  const int a0 = f == 0 ? 1 : 0, a1 = f == 2 ? 1 : 2;
  const double La = box[a0], Lb = box[a1], A = La * Lb, z = x[f];
  const double rc = 7.0 / alpha;
  const int na = (int)ceil((rc + fabs(x[a0])) / La) + 1, nb = (int)ceil((rc + fabs(x[a1])) / Lb) + 1;
  double real = 0.0;
  for (int j = -nb; j <= nb; ++j)
    for (int i = -na; i <= na; ++i) {
      const double da = x[a0] + i * La, db = x[a1] + j * Lb;
      const double r2 = da * da + db * db + z * z;
      if (r2 == 0.0) {
        if (!reg) return INFINITY;
        real -= pow(alpha, 6) / 6.0;
        continue;
      }
      if (r2 > rc * rc) continue;
      real += orc_r6_real(alpha, r2);
    }
  double xg[16], wg[16];
  orc_gauss16(xg, wg);
  const double c = alpha * alpha * z * z, a4 = pow(alpha, 4);
  /* b <= 45 bounds the Fourier terms kept */
  const double kc = 2.0 * alpha * sqrt(45.0);
  const int ma = (int)ceil(kc * La / (2.0 * M_PI)) + 1, mb = (int)ceil(kc * Lb / (2.0 * M_PI)) + 1;
  double recip = orc_r6_slab_k0(alpha, z);
  for (int j = -mb; j <= mb; ++j)
    for (int i = -ma; i <= ma; ++i) {
      if (i == 0 && j == 0) continue;
      const double ka = 2.0 * M_PI * i / La, kb = 2.0 * M_PI * j / Lb;
      const double b = (ka * ka + kb * kb) / (4.0 * alpha * alpha);
      if (b > 45.0) continue;
      recip += a4 * cos(ka * x[a0] + kb * x[a1]) * orc_exp_integral(2.0, b, c, xg, wg);
    }
  return real + 0.5 * M_PI / A * recip;
}

/* line: axis periodic, the other two free */
double orc_ewald1d_r6(const double box[3], int axis, double alpha, const double x[3], int reg)
{
  const double L = box[axis], z = x[axis];
  double rho2 = 0.0;
  for (int k = 0; k < 3; ++k)
    if (k != axis) rho2 += x[k] * x[k];
  const double rc = 7.0 / alpha;
  const int nr = (int)ceil((rc + fabs(z)) / L) + 1;
  double real = 0.0;
  for (int j = -nr; j <= nr; ++j) {
    const double dz = z + j * L, r2 = rho2 + dz * dz;
    if (r2 == 0.0) {
      if (!reg) return INFINITY;
      real -= pow(alpha, 6) / 6.0;
      continue;
    }
    if (r2 > rc * rc) continue;
    real += orc_r6_real(alpha, r2);
  }
  double xg[16], wg[16];
  orc_gauss16(xg, wg);
  const double c = alpha * alpha * rho2, a5 = pow(alpha, 5);
  double recip = 0.0;
  for (int m = 1;; ++m) {
    const double k = 2.0 * M_PI * m / L, b = k * k / (4.0 * alpha * alpha);
    if (b > 45.0) break;
    recip += 2.0 * a5 * cos(k * z) * orc_exp_integral(2.5, b, c, xg, wg);
  }
  recip += orc_r6_line_k0(alpha, sqrt(rho2));
  return real + 0.5 * sqrt(M_PI) / L * recip;
}

/* sum_n |x + n|^-6 over the lattice of the periodic axes of mask (1..7) */
double orc_ewald_r6(const double box[3], unsigned mask, double alpha, const double x[3],
                    int reg)
{
  if (mask == 7) return orc_ewald3d_r6(box, alpha, x, reg);
  int np = 0, axis = 0, freeax = 0;
  for (int k = 0; k < 3; ++k) {
    if ((mask >> k) & 1) {
      ++np;
      axis = k;
    } else {
      freeax = k;
    }
  }
  if (np == 2) return orc_ewald2d_r6(box, freeax, alpha, x, reg);
  if (np == 1) return orc_ewald1d_r6(box, axis, alpha, x, reg);
  return NAN;
}

/* psi for any set of periodic axes (bit k of mask = axis k periodic): the
 * 3-D sum, the slab sum with the free axis moved to z, or the 1-D sum. */
double orc_ewald_psi(const double box[3], unsigned mask, double alpha, const double x[3],
                     int reg)
{
  if (mask == 7) return orc_ewald3d(box, alpha, x, reg);
  int np = 0, axis = 0, freeax = 0;
  for (int k = 0; k < 3; ++k) {
    if ((mask >> k) & 1) {
      ++np;
      axis = k;
    } else {
      freeax = k;
    }
  }
  if (np == 1) return orc_ewald1d(box, axis, alpha, x, reg);
  if (np != 2) return NAN;
  double b2[3], x2[3];
  int o = 0;
  for (int k = 0; k < 3; ++k)
    if (k != freeax) {
      b2[o] = box[k];
      x2[o++] = x[k];
    }
  b2[2] = box[freeax];
  x2[2] = x[freeax];
  return orc_ewald2d(b2, alpha, x2, reg);
}

static double det3(const double A[9])
{
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* The same sums for the lattice L = {H n}: real space over lattice vectors,
 * reciprocal space over k = 2 pi H^{-T} m, V = |det H|. */
double orc_ewald3d_cell(const double H[9], double alpha, const double x[3], int reg)
{
  const double det = det3(H), V = fabs(det);
  double Hi[9]; /* H^{-1} by cofactors */
  Hi[0] = (H[4] * H[8] - H[5] * H[7]) / det;
  Hi[1] = (H[2] * H[7] - H[1] * H[8]) / det;
  Hi[2] = (H[1] * H[5] - H[2] * H[4]) / det;
  Hi[3] = (H[5] * H[6] - H[3] * H[8]) / det;
  Hi[4] = (H[0] * H[8] - H[2] * H[6]) / det;
  Hi[5] = (H[2] * H[3] - H[0] * H[5]) / det;
  Hi[6] = (H[3] * H[7] - H[4] * H[6]) / det;
  Hi[7] = (H[1] * H[6] - H[0] * H[7]) / det;
  Hi[8] = (H[0] * H[4] - H[1] * H[3]) / det;
  const double rc = ORC_EWALD_X / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  /* image range: |n_k| covers |s_k(x)| + rc |row k of H^{-1}| */
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    double bk = sqrt(Hi[3 * k] * Hi[3 * k] + Hi[3 * k + 1] * Hi[3 * k + 1] +
                     Hi[3 * k + 2] * Hi[3 * k + 2]);
    double sk = Hi[3 * k] * x[0] + Hi[3 * k + 1] * x[1] + Hi[3 * k + 2] * x[2];
    nr[k] = (int)ceil(rc * bk + fabs(sk)) + 1;
    double ak = sqrt(H[k] * H[k] + H[3 + k] * H[3 + k] + H[6 + k] * H[6 + k]);
    nk[k] = (int)ceil(kc * ak / (2.0 * M_PI)) + 1;
  }
  double real = 0.0;
  for (int jz = -nr[2]; jz <= nr[2]; ++jz)
    for (int jy = -nr[1]; jy <= nr[1]; ++jy)
      for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = x[k] + H[3 * k] * jx + H[3 * k + 1] * jy + H[3 * k + 2] * jz;
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r == 0.0) {
          if (!reg) return INFINITY;
          real -= 2.0 * alpha / sqrt(M_PI);
          continue;
        }
        if (r > rc) continue;
        real += erfc(alpha * r) / r;
      }
  double recip = 0.0;
  for (int mz = -nk[2]; mz <= nk[2]; ++mz)
    for (int my = -nk[1]; my <= nk[1]; ++my)
      for (int mx = -nk[0]; mx <= nk[0]; ++mx) {
        if (mx == 0 && my == 0 && mz == 0) continue;
        double gk[3];
        for (int j = 0; j < 3; ++j)
          gk[j] = 2.0 * M_PI * (Hi[j] * mx + Hi[3 + j] * my + Hi[6 + j] * mz);
        double k2 = gk[0] * gk[0] + gk[1] * gk[1] + gk[2] * gk[2];
        if (k2 > kc * kc) continue;
        recip += exp(-k2 / (4.0 * alpha * alpha)) * cos(gk[0] * x[0] + gk[1] * x[1] + gk[2] * x[2]) / k2;
      }
  recip *= 4.0 * M_PI / V;
  return real + recip - M_PI / (alpha * alpha * V);
}

/* The lattice sum of r^-6 over the lattice spanned by the columns of H: the
 * 3-D r^-6 Ewald sum above with images H n and wave vectors 2 pi H^{-T} m. */
double orc_ewald3d_cell_r6(const double H[9], double alpha, const double x[3], int reg)
{
  const double det = det3(H), V = fabs(det);
  double Hi[9]; /* H^{-1} by cofactors */
  Hi[0] = (H[4] * H[8] - H[5] * H[7]) / det;
  Hi[1] = (H[2] * H[7] - H[1] * H[8]) / det;
  Hi[2] = (H[1] * H[5] - H[2] * H[4]) / det;
  Hi[3] = (H[5] * H[6] - H[3] * H[8]) / det;
  Hi[4] = (H[0] * H[8] - H[2] * H[6]) / det;
  Hi[5] = (H[2] * H[3] - H[0] * H[5]) / det;
  Hi[6] = (H[3] * H[7] - H[4] * H[6]) / det;
  Hi[7] = (H[1] * H[6] - H[0] * H[7]) / det;
  Hi[8] = (H[0] * H[4] - H[1] * H[3]) / det;
  const double rc = 7.0 / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    double bk = sqrt(Hi[3 * k] * Hi[3 * k] + Hi[3 * k + 1] * Hi[3 * k + 1] +
                     Hi[3 * k + 2] * Hi[3 * k + 2]);
    double sk = Hi[3 * k] * x[0] + Hi[3 * k + 1] * x[1] + Hi[3 * k + 2] * x[2];
    nr[k] = (int)ceil(rc * bk + fabs(sk)) + 1;
    double ak = sqrt(H[k] * H[k] + H[3 + k] * H[3 + k] + H[6 + k] * H[6 + k]);
    nk[k] = (int)ceil(kc * ak / (2.0 * M_PI)) + 1;
  }
  double real = 0.0;
  for (int jz = -nr[2]; jz <= nr[2]; ++jz)
    for (int jy = -nr[1]; jy <= nr[1]; ++jy)
      for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = x[k] + H[3 * k] * jx + H[3 * k + 1] * jy + H[3 * k + 2] * jz;
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) {
          if (!reg) return INFINITY;
          real -= pow(alpha, 6) / 6.0;
          continue;
        }
        if (r2 > rc * rc) continue;
        real += orc_r6_real(alpha, r2);
      }
  double recip = 0.0;
  for (int mz = -nk[2]; mz <= nk[2]; ++mz)
    for (int my = -nk[1]; my <= nk[1]; ++my)
      for (int mx = -nk[0]; mx <= nk[0]; ++mx) {
        double gk[3];
        for (int j = 0; j < 3; ++j)
          gk[j] = 2.0 * M_PI * (Hi[j] * mx + Hi[3 + j] * my + Hi[6 + j] * mz);
        const double k = sqrt(gk[0] * gk[0] + gk[1] * gk[1] + gk[2] * gk[2]);
        if (k > kc) continue;
        const double b = k / (2.0 * alpha);
        const double f = (1.0 - 2.0 * b * b) * exp(-b * b) + 2.0 * sqrt(M_PI) * b * b * b * erfc(b);
        recip += f * cos(gk[0] * x[0] + gk[1] * x[1] + gk[2] * x[2]);
      }
  return real + pow(M_PI, 1.5) * alpha * alpha * alpha / (3.0 * V) * recip;
}

void orc_ewald_potentials_cell(const double H[9], double alpha, int n, const double* pos,
                               const double* q, double* phi)
{
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                     pos[3 * i + 2] - pos[3 * j + 2]};
      s += q[j] * orc_ewald3d_cell(H, alpha, d, j == i);
    }
    phi[i] = s;
  }
}

void orc_ewald_potentials_mask(const double box[3], unsigned mask, double alpha, int n,
                               const double* pos, const double* q, double* phi)
{
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                     pos[3 * i + 2] - pos[3 * j + 2]};
      s += q[j] * orc_ewald_psi(box, mask, alpha, d, j == i);
    }
    phi[i] = s;
  }
}

void orc_ewald_potentials(const double box[3], int slab, double alpha, int n,
                          const double* pos, const double* q, double* phi)
{
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                     pos[3 * i + 2] - pos[3 * j + 2]};
      int reg = (j == i);
      s += q[j] * (slab ? orc_ewald2d(box, alpha, d, reg) : orc_ewald3d(box, alpha, d, reg));
    }
    phi[i] = s;
  }
}

/* ------------------------------------------------------------------------
 * The same 3-D Ewald sum for a whole system at once, with forces: the
 * reciprocal part through the structure factor S(k) = sum_j q_j e^{i k.r_j}
 * (Ewald 1921, in the textbook form of e.g. Frenkel and Smit,
 * "Understanding Molecular Simulation", ch. 12), so that N = 10^4 takes
 * seconds instead of N^2 lattice sums.  phi_i is the potential of
 * orc_ewald_potentials (self term regular, neutralising background), and
 * F_i = -q_i grad_i phi_i with the self term held fixed:
 *   real space   F_i += q_i q_j (erfc(a r)/r + 2a/sqrt(pi) e^{-a^2 r^2}) d/r^2
 *                over images d = r_i - r_j - j L with 0 < |d| < rc,
 *   reciprocal   phi_i += (4 pi / V) sum_{k != 0} e^{-k^2/4a^2}/k^2 Re[e^{i k.r_i} S*(k)],
 *                F_i += q_i (4 pi / V) sum_k e^{-k^2/4a^2}/k^2 k Im[e^{i k.r_i} S*(k)],
 *   constants    phi_i += -2 a/sqrt(pi) q_i - pi/(a^2 V) sum_j q_j.
 * alpha <= 0 picks the splitting whose real-space cutoff is half the shortest
 * edge (one image per pair, the fewest k vectors).
 * ------------------------------------------------------------------------ */
void orc_ewald3d_system(const double box[3], double alpha, int n, const double* pos,
                        const double* q, double* phi, double* F)
{
  const double V = box[0] * box[1] * box[2];
  const double minbox = fmin(box[0], fmin(box[1], box[2]));
  if (!(alpha > 0.0)) alpha = ORC_EWALD_X / (0.5 * minbox); /* rc = half the shortest edge */
  const double rc = ORC_EWALD_X / alpha, kc = 2.0 * alpha * ORC_EWALD_X;
  /* real space, over the images of the minimum-image difference: with rc at
   * most half the shortest edge only the minimum image itself can lie within
   * rc, otherwise every image within rc + half an edge per axis is visited */
  int nr[3], nk[3];
  for (int k = 0; k < 3; ++k) {
    nr[k] = rc <= 0.5 * minbox ? 0 : (int)ceil(rc / box[k]) + 1;
    nk[k] = (int)ceil(kc * box[k] / (2.0 * M_PI)) + 1;
  }
  double qsum = 0.0;
  for (int j = 0; j < n; ++j) qsum += q[j];

#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < n; ++i) {
    double ph = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
      double m[3];
      for (int k = 0; k < 3; ++k) {
        m[k] = pos[3 * i + k] - pos[3 * j + k];
        m[k] -= box[k] * nearbyint(m[k] / box[k]);
      }
      for (int jz = -nr[2]; jz <= nr[2]; ++jz)
        for (int jy = -nr[1]; jy <= nr[1]; ++jy)
          for (int jx = -nr[0]; jx <= nr[0]; ++jx) {
            double d[3] = {m[0] + jx * box[0], m[1] + jy * box[1], m[2] + jz * box[2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0 || r2 >= rc * rc) continue;
            double r = sqrt(r2), e = erfc(alpha * r) / r;
            ph += q[j] * e;
            double c = q[j] * (e + 2.0 * alpha / sqrt(M_PI) * exp(-alpha * alpha * r2)) / r2;
            for (int k = 0; k < 3; ++k) f[k] += c * d[k];
          }
    }
    phi[i] = ph - 2.0 * alpha / sqrt(M_PI) * q[i] - M_PI / (alpha * alpha * V) * qsum;
    for (int k = 0; k < 3; ++k) F[3 * i + k] = q[i] * f[k];
  }

  /* reciprocal space: every k = 2 pi (mx/Lx, my/Ly, mz/Lz), m != 0, |k| <= kc */
  int nvec = 0;
  const int mx = 2 * nk[0] + 1, my = 2 * nk[1] + 1, mz = 2 * nk[2] + 1;
  double* kv = (double*)malloc(sizeof(double) * 4 * (size_t)mx * my * mz);
  for (int a = -nk[0]; a <= nk[0]; ++a)
    for (int b = -nk[1]; b <= nk[1]; ++b)
      for (int c = -nk[2]; c <= nk[2]; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        double g[3] = {2.0 * M_PI * a / box[0], 2.0 * M_PI * b / box[1], 2.0 * M_PI * c / box[2]};
        double k2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (k2 > kc * kc) continue;
        kv[4 * nvec] = g[0];
        kv[4 * nvec + 1] = g[1];
        kv[4 * nvec + 2] = g[2];
        kv[4 * nvec + 3] = 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
        ++nvec;
      }
  double* S = (double*)malloc(sizeof(double) * 2 * (size_t)(nvec > 0 ? nvec : 1));
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < nvec; ++v) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < n; ++j) {
      double t = kv[4 * v] * pos[3 * j] + kv[4 * v + 1] * pos[3 * j + 1] + kv[4 * v + 2] * pos[3 * j + 2];
      re += q[j] * cos(t);
      im += q[j] * sin(t);
    }
    S[2 * v] = re;
    S[2 * v + 1] = im;
  }
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < n; ++i) {
    double ph = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < nvec; ++v) {
      double t = kv[4 * v] * pos[3 * i] + kv[4 * v + 1] * pos[3 * i + 1] + kv[4 * v + 2] * pos[3 * i + 2];
      double c = cos(t), s = sin(t);
      /* e^{i t} S* = (c + i s)(Sr - i Si) */
      double re = c * S[2 * v] + s * S[2 * v + 1];
      double im = s * S[2 * v] - c * S[2 * v + 1];
      ph += kv[4 * v + 3] * re;
      for (int k = 0; k < 3; ++k) f[k] += kv[4 * v + 3] * kv[4 * v + k] * im;
    }
    phi[i] += ph;
    for (int k = 0; k < 3; ++k) F[3 * i + k] += q[i] * f[k];
  }
  free(S);
  free(kv);
}
