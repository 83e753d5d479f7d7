/*
 * msm.h -- C ABI of libmsm: multilevel summation method (MSM) electrostatics
 * with B-spline interpolation (arXiv 2510.05961) on AMD Instinct MI355X.
 *
 * What is computed (Sec. "Fundamentals of the multilevel summation method"):
 *
 *   U = 1/2 sum_i sum_{j != i} q_i q_j k(r_ij),   k(r) = 1/r      (eq. generic_pair_potential_sum)
 *
 * approximated by splitting k into partial kernels k_0..k_L (eq. kernel_splitting,
 * eq. coulomb_splitting_with_softener), summing k_0 directly over a cell list
 * (eq. U_zero) and interpolating k_1..k_L from grids of spacing h_l = 2^(l-1) h
 * (eqs. kernel_interpolation, grid_charge, u_oneplus_nested_eval,
 * uoneplus_interpolation).  Outputs: the energy U (FP64), the forces
 * F_i = -dU/dr_i (eq. analytic_uoneplus_position_grad) and the charge gradient
 * dU/dq_i (eq. analytic_uoneplus_charge_grad).  No units are assumed (Sec. Units).
 *
 * Conventions for every entry point:
 *  - Device pointers are HIP device memory owned by the caller, contiguous,
 *    in the plan's precision (float for MSM_FP32, double for MSM_FP64), except
 *    energies, which are always double.  Positions are [n][3] row-major,
 *    charges [n], forces [n][3], dE/dq [n].
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; the hot-path calls neither allocate nor synchronise.
 *  - Errors found on the host are returned synchronously; errors that depend on
 *    the data (non-finite input, a position outside a non-periodic box) set a
 *    sticky device flag that msm_plan_status reports; the outputs of such a
 *    call are then undefined (but every kernel stays within its buffers).
 *  - A plan may be used from one stream at a time; concurrent calls on one
 *    plan race on its internal grids.
 *  - No C++ exception crosses this boundary.
 */
#ifndef LIBMSM_H
#define LIBMSM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msm_plan_s* msm_plan;

typedef enum {
  MSM_OK = 0,
  MSM_ERR_INVALID_ARG = 1,       /* bad parameter, NULL pointer, wrong plan kind */
  MSM_ERR_UNSUPPORTED = 2,       /* unsupported order, kernel or periodicity for the call */
  MSM_ERR_CUTOFF_TOO_LARGE = 3,  /* a > box/2 on a periodic axis (minimum image) */
  MSM_ERR_GRID = 4,              /* grid or stencil too large for the plan limits */
  MSM_ERR_OUT_OF_DOMAIN = 5,     /* device flag: coordinate outside [0, box] on a free axis */
  MSM_ERR_NONFINITE = 6,         /* device flag: NaN/Inf position or charge */
  MSM_ERR_CAPACITY = 7,          /* n > max_n */
  MSM_ERR_HIP = 8,               /* a HIP runtime call failed */
  MSM_ERR_OOM = 9,               /* device allocation failed */
  MSM_ERR_NO_DEVICE = 10         /* plan was created host-only */
} msm_status;

enum { MSM_FP32 = 0, MSM_FP64 = 1 };

/*
 * msm_plan_create -- set up the MSM for one orthorhombic box (Sec. "High-level
 * interface": cell, pbc, level_one_spacings, level_zero_cutoff, p).
 *   box[3]          host, box edge lengths (> 0).
 *   periodic_mask   bit k set = axis k periodic (0..7, any combination; 8 or
 *                   more: MSM_ERR_INVALID_ARG).  The top level sums the
 *                   periodic images with the Ewald method of the periodic
 *                   axes: 3-D (tin-foil boundary, neutralising background),
 *                   2-D (alpha = 3 / the shorter periodic edge, which fixes
 *                   the constant of a non-neutral slab) or 1-D (the constant
 *                   of a non-neutral line is the one for which a unit charge's
 *                   potential tends to -(2/L) ln(rho/L) far from the axis,
 *                   L its period, rho the distance to the axis).  Neutral
 *                   systems depend on neither convention.
 *   order           B-spline order p (Sec. "B-spline interpolation"): 4, 6 or 8.
 *   h               requested level-1 spacing.  Free axes use h exactly; a
 *                   periodic axis uses box/N_1 with N_1 = N_top 2^(L-1),
 *                   N_top = max(1, floor(box/(h 2^(L-1)) + 1/2)).
 *   cutoff_a        level-zero cutoff a (r_cut^(0) of eq. kernel_splitting).
 *   levels          number of grid levels L >= 1 (kernels k_0..k_L).
 *   precision       MSM_FP32 or MSM_FP64 for particle and grid arithmetic;
 *                   stencils are built in FP64 and the energy is summed in FP64.
 *   max_n           largest particle count a call may pass (the particle
 *                   buffers must stay below 4 GiB: max_n up to about 2^26
 *                   in FP32 and 2^25 in FP64, else MSM_ERR_CAPACITY).
 *   quasi_degree_M  half-width M of the quasi-interpolation sequence omega'
 *                   (eq. kernel_stencil_by_conv_with_universal_coeff); -1 = p.
 * On success *out owns device memory for stencils, grids and cell lists.
 */
msm_status msm_plan_create(msm_plan* out, const double box[3], unsigned periodic_mask, int order,
                           double h, double cutoff_a, int levels, int precision, int max_n,
                           int quasi_degree_M);

/*
 * msm_energy_forces_cell_gradient -- msm_energy_forces plus the derivative
 * of the energy with respect to the cell, for plans made by
 * msm_plan_create_cell (Sec. "MSM core algorithm", long-range part: the
 * stencils follow the current cell; their derivative gives the stress):
 *   dEdH     device double[9], dE/dH[3 r + c] with H the matrix whose
 *            columns are the lattice vectors (H[r][c] = component r of
 *            vector c), taken at fixed Cartesian positions.
 * The derivative is that of the MSM energy with the grid counts held: the
 * short-range pairs' virial, each level's derivative stencils
 * k_l'(r)/r x x^T applied to omega'-filtered grid charges, and the top
 * level's table differentiated in H (central differences on the host,
 * relative step 1e-5, built on the first call after each cell change);
 * with the particles' term sum_i F_i (H^{-1} r_i)^T.  The stress tensor is
 * -(1/V) dE/dH H^T.  forces is required; energy, dEdq and the stream as for
 * msm_energy_forces.  One stream; allocates on its first call per cell
 * (stencils) and per plan (three FP64 level-1 grids).  The cutoff must stay
 * below half the cell's smallest width under a relative change of 1e-5 of
 * the cell (the top derivative builds such plans).  r^-6 cell plans
 * (msm_plan_create_cell_kernel) take the same call with their own kernel
 * in every term (degree -6 homogeneity in place of -1).  Errors: as
 * msm_energy_forces, MSM_ERR_UNSUPPORTED for non-triclinic plans,
 * MSM_ERR_GRID when a derivative stencil exceeds the convolution's window.
 */
msm_status msm_energy_forces_cell_gradient(msm_plan plan, int n, const void* pos, const void* q,
                                           double* energy, void* forces, void* dEdq,
                                           double* dEdH, void* stream);

/*
 * msm_plan_create_kernel -- msm_plan_create for the kernel k(r) = r^-nu,
 * nu = kernel: MSM_KERNEL_COULOMB (1, the same plan as msm_plan_create) or
 * MSM_KERNEL_DISPERSION (6).  The paper's splitting carries over unchanged
 * (Sec. "Splitting for Coulomb kernels"; the package's core is meant to take
 * other kernels): k_0 = r^-nu - gamma(r/a)/a^nu, k_l = gamma(r/a_l)/a_l^nu -
 * gamma(r/a_{l+1})/a_{l+1}^nu (a_l = 2^(l-1) a), k_L = gamma(r/a_L)/a_L^nu,
 * with gamma the degree-(p-1) Taylor polynomial of s^(-nu/2) about s = 1 at
 * s = (r/a)^2 below 1 and r^-nu above; the intermediate stencils are
 * K^1 / 2^((l-1) nu).  For nu = 6 "charges" are per-particle coefficients c_i
 * (E = 1/2 sum_{i != j} c_i c_j r^-6, geometric mixing; negate the result
 * for an attractive dispersion energy).  nu = 6 takes every periodic_mask:
 * with periodic axes the top level sums k_L over the lattice of those axes
 * with the Ewald method for r^-6 (3-D, slab or line form), which converges
 * absolutely (no boundary term; E = 1/2 sum_{i,j} c_i c_j sum_n' |r_i - r_j
 * + n|^-6, the n = 0 term left out for i = j).  a/h of about 8 or more is
 * needed before the higher orders pay (the softened r^-6 is stiff).
 * Every compute call, the backward included, works as for Coulomb plans;
 * batched plans take r^-6 through msm_batch_plan_create_kernel.
 */
#define MSM_KERNEL_COULOMB 1
#define MSM_KERNEL_DISPERSION 6
msm_status msm_plan_create_kernel(msm_plan* out, int kernel, const double box[3],
                                  unsigned periodic_mask, int order, double h, double cutoff_a,
                                  int levels, int precision, int max_n, int quasi_degree_M);

/*
 * msm_plan_create_cell_kernel -- msm_plan_create_cell for the kernel
 * k(r) = r^-nu, nu = kernel (MSM_KERNEL_COULOMB or MSM_KERNEL_DISPERSION;
 * other values: MSM_ERR_INVALID_ARG), with the splitting described at
 * msm_plan_create_kernel and the triclinic geometry of msm_plan_create_cell
 * (Sec. "MSM core algorithm", long-range part).  For r^-6 the top level sums
 * k_L over the lattice H n with the Ewald method for r^-6 (real space over
 * H n, reciprocal space over 2 pi H^{-T} m; no boundary term).  Every
 * compute call, msm_plan_set_cell and msm_energy_forces_cell_gradient work
 * as for a Coulomb cell plan.
 */
msm_status msm_plan_create_cell_kernel(msm_plan* out, int kernel, const double cell[9],
                                       unsigned periodic_mask, int order, double h,
                                       double cutoff_a, int levels, int precision, int max_n,
                                       int quasi_degree_M);

/*
 * msm_plan_create_cell -- msm_plan_create for a triclinic cell (Sec. "MSM core
 * algorithm", long-range part: positions are mapped to the unit cube,
 * s = [a b c]^{-1} r, and the grids are set up there).
 *   cell[9]         host, the lattice vectors a, b, c as consecutive rows
 *                   (cell[0..2] = a, ...), any orientation, non-singular.
 *   periodic_mask   must be 7 (all axes periodic; else MSM_ERR_UNSUPPORTED).
 * Each grid has N_l points along each lattice vector, chosen from the
 * vector's length as for a periodic box edge; stencils sample k_l at the
 * Cartesian grid offsets H (n / N_l) and the top level sums k_L's tail over
 * the lattice with a triclinic Ewald sum.  The cutoff must not exceed half
 * the cell's smallest width V / |face| (minimum image, else
 * MSM_ERR_CUTOFF_TOO_LARGE).  Positions may take any finite value (they are
 * wrapped into the cell); forces and dE/dq are Cartesian.  All other
 * arguments and every compute call are as for msm_plan_create; a diagonal
 * cell gives the orthorhombic plan's results up to rounding.
 */
msm_status msm_plan_create_cell(msm_plan* out, const double cell[9], unsigned periodic_mask,
                                int order, double h, double cutoff_a, int levels, int precision,
                                int max_n, int quasi_degree_M);

/*
 * msm_plan_set_cell -- a new cell for a plan made by msm_plan_create_cell
 * (a cell that changes between calls, as under constant pressure): the
 * grids keep their point counts, so their spacings follow the cell, and the
 * stencils and the top-level table are rebuilt from the new cell on the
 * host and uploaded again (Sec. "MSM core algorithm": stencils computed from
 * the current cell).  Synchronises the device; not for the hot path.  The
 * cell list keeps at most its number of cells per axis (a thinner cell gets
 * fewer).  MSM_ERR_INVALID_ARG for other plans; MSM_ERR_CUTOFF_TOO_LARGE if
 * the new cell is too thin for the cutoff; MSM_ERR_GRID if a stencil outgrows
 * the convolution's limits (create a new plan then).  On an error the plan's
 * stencils are undefined.  The stencils move to new device buffers: a graph
 * captured from this plan's calls before must be captured again.
 */
msm_status msm_plan_set_cell(msm_plan plan, const double cell[9]);

/* Same as msm_plan_create but touches no GPU: only the host-side plan
 * (geometry, softener, omega', J, stencils) is built, for inspection with
 * msm_plan_describe / msm_plan_get_stencil.  Compute calls return
 * MSM_ERR_NO_DEVICE. */
msm_status msm_plan_create_host(msm_plan* out, const double box[3], unsigned periodic_mask,
                                int order, double h, double cutoff_a, int levels, int precision,
                                int max_n, int quasi_degree_M);

/* Frees the plan and its device memory (synchronises the device first). */
msm_status msm_plan_destroy(msm_plan plan);

/* Writes a NUL-terminated JSON description (parameters, actual spacings, grid
 * sizes, stencil boxes, gamma/omega'/J coefficients) into json[cap]. */
msm_status msm_plan_describe(msm_plan plan, char* json, size_t cap);

/* Host copy of the FP64 stencil of grid level `level` (1..L; level L is the
 * dense top-level kernel).  dims_off[6] receives (len_x, len_y, len_z,
 * off_x, off_y, off_z): the stencil covers offsets d_k = off_k .. off_k+len_k-1
 * and K is stored [len_z][len_y][len_x].  Periodic axes are folded onto the
 * grid (each residue once); free axes are cropped to |d| < grid size.
 * K may be NULL to query dims only; otherwise cap is its length in doubles. */
msm_status msm_plan_get_stencil(msm_plan plan, int level, int dims_off[6], double* K,
                                size_t cap);

/* Grid sizes of level `level`: n[3] points per axis (x, y, z). */
msm_status msm_plan_grid_dims(msm_plan plan, int level, int n[3]);

/* Bytes of caller workspace that msm_energy_forces writes and msm_backward
 * reads for a call with n particles (saved forward state: the cell-ordered
 * particles and their permutation, the cell starts, phi, F and e^{1+}).
 * flags: 0 (the one layout; other values are reserved and return 0).
 * Returns 0 for a NULL or batch plan or n < 0. */
size_t msm_workspace_bytes(msm_plan plan, int n, int flags);

/*
 * msm_energy_forces -- one forward evaluation on the device.
 *   n          particle count, 0 <= n <= max_n.
 *   pos, q     device, inputs ([n][3], [n]) in the plan's precision.  Periodic
 *              coordinates may take any finite value (they are wrapped); free
 *              coordinates must lie in [0, box].
 *   ws         device workspace of msm_workspace_bytes(plan, n) bytes, or NULL
 *              when no msm_backward call will follow.
 *   energy     device, 1 double: U.
 *   forces     device [n][3] or NULL: F_i = -dU/dr_i.
 *   dEdq       device [n] or NULL: dU/dq_i (the potential phi_i at particle i).
 */
msm_status msm_energy_forces(msm_plan plan, int n, const void* pos, const void* q, void* ws,
                             double* energy, void* forces, void* dEdq, void* stream);

/*
 * msm_energy_forces_noalloc -- msm_energy_forces for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the call allocates nothing.  Its working
 * memory (grids, cell list, cluster layout, short-range sums) is a static
 * array of the library, 64 MiB per GPU, held from the library's load until
 * the process ends, instead of the plan's own working buffers; the plan's
 * stencils and streams are used as they are.  Arguments as for
 * msm_energy_forces, except that n is bounded by that array instead of
 * max_n: MSM_ERR_CAPACITY when the call's working memory (plan grids plus
 * about 200 bytes per particle in FP32) would exceed 64 MiB.  The plan's
 * GPU must be the current device (else MSM_ERR_INVALID_ARG).  ws, if given,
 * receives the saved state as in msm_energy_forces, for msm_backward.
 * Every such call on one GPU uses the same array: calls that overlap on one
 * GPU (several streams or host threads) race, and msm_plan_get_grid keeps
 * reporting the plan's own grids.  Stage profiling is not recorded.
 */
msm_status msm_energy_forces_noalloc(msm_plan plan, int n, const void* pos, const void* q,
                                     void* ws, double* energy, void* forces, void* dEdq,
                                     void* stream);

/*
 * msm_backward -- vector-Jacobian product of the forward outputs.
 * For the scalar L = gE * U + sum_i gF_i . F_i it writes
 *   grad_q[i]   = dL/dq_i   = gE dU/dq_i + d(sum gF.F)/dq_i
 *   grad_pos[i] = dL/dr_i   = -gE F_i    + d(sum gF.F)/dr_i
 * The force part differentiates eqs. (analytic_uoneplus_position_grad) and
 * the short-range forces once more (B-spline Hessians, k_0'').
 *   pos, q     the same device inputs as the forward call that filled ws.
 *   ws         the workspace that forward call wrote.
 *   gE         device, 1 double (may be NULL = 0).
 *   gF         device [n][3] cotangent on the forces, or NULL (= 0).
 *   grad_pos   device [n][3] or NULL;  grad_q  device [n] or NULL.
 */
msm_status msm_backward(msm_plan plan, int n, const void* pos, const void* q, const void* ws,
                        const double* gE, const void* gF, void* grad_pos, void* grad_q,
                        void* stream);

/*
 * msm_backward_full -- the same product with a cotangent on the third output,
 * the charge gradient dE/dq = phi (Sec. Fundamentals; losses on the
 * potentials, as in charge equilibration).  For
 *   L = gE * U + sum_i gF_i . F_i + sum_i gdEdq_i phi_i
 * it writes grad_q = dL/dq and grad_pos = dL/dr.  U = q^T G q / 2 with G
 * symmetric, so the last term is w^T G q (w = gdEdq): its q-gradient is the
 * potential of charges w, G w, and its r-gradient is
 * w_i grad phi^q(r_i) + q_i grad phi^w(r_i) (both fields taken at r_i, the
 * short-range pairs and every level included).
 *   gdEdq      device [n] (plan precision), or NULL (= 0; the call is then
 *              msm_backward).
 * The other arguments, the errors and the stream are those of msm_backward.
 */
msm_status msm_backward_full(msm_plan plan, int n, const void* pos, const void* q,
                             const void* ws, const double* gE, const void* gF, const void* gdEdq,
                             void* grad_pos, void* grad_q, void* stream);

/*
 * msm_plan_set_skin -- Verlet skin for the short-range cell list (molecular
 * dynamics: the neighbour structure kept over steps while no charge has
 * moved far; Sec. MD simulation of charged Lennard-Jonesium uses a
 * neighbour list refreshed this way).  With skin > 0 the cells have edge
 * >= cutoff_a + skin, and a call rebuilds the cell list only when some
 * charge moved more than skin/2 (Euclidean, in the caller's coordinates)
 * since the last rebuild; otherwise it reuses the cell assignment and the
 * cluster layout with the new positions and charges.  The decision is made
 * on the device, so a captured graph of msm_energy_forces stays valid over
 * steps.  Results equal those of a rebuilt list up to the summation order.
 * A call with a different n, a call with a workspace (msm_backward's saved
 * state) and the call after it, and the first call after msm_plan_set_skin or
 * msm_plan_set_cell always rebuild.  skin = 0 (the default) rebuilds on every
 * call.  The cell count changes, so msm_workspace_bytes may too; the cell
 * list never has more cells per axis than at plan creation.
 * msm_energy_forces_noalloc returns MSM_ERR_UNSUPPORTED on a plan with a
 * skin.  Errors: MSM_ERR_INVALID_ARG (skin < 0 or not finite), MSM_ERR_OOM.
 */
msm_status msm_plan_set_skin(msm_plan plan, double skin);
/* Calls of msm_energy_forces since msm_plan_set_skin and how many of them
 * rebuilt the cell list (synchronises `stream`; both 0 without a skin). */
msm_status msm_plan_skin_stats(msm_plan plan, long long* calls, long long* rebuilds,
                               void* stream);

/* Synchronises `stream`, returns the sticky device error of the plan
 * (MSM_OK, MSM_ERR_OUT_OF_DOMAIN or MSM_ERR_NONFINITE) and clears it. */
msm_status msm_plan_status(msm_plan plan, void* stream);

/* Copies the device grid of level `level` (1..L) into dst (device, grid size
 * elements of the plan precision): which = 0 grid charge q~^l as left by the
 * last forward call, which = 1 accumulated potential e^{l+} (eq.
 * u_oneplus_nested_eval; e^{1+} for level 1). */
msm_status msm_plan_get_grid(msm_plan plan, int level, int which, void* dst, void* stream);

/*
 * Batched evaluation of many independent non-periodic systems in one launch
 * sequence (Sec. "Madelung constants", batching by vmap, done here without
 * padding).  All systems share order, h, cutoff_a and precision; system s has
 * its own box and level count.
 *   boxes[n_sys][3]  host, edge lengths of each system's box; the batched
 *                    kernels take cubic boxes (the three edges equal, else
 *                    MSM_ERR_UNSUPPORTED).
 *   levels[n_sys]    host, grid levels L of each system.
 *   periodic_mask    must be 0 (free space; otherwise MSM_ERR_UNSUPPORTED).
 * The other arguments are those of msm_plan_create (max_total_n bounds the
 * summed particle count of a call).
 */
msm_status msm_batch_plan_create(msm_plan* out, int n_sys, const double* boxes,
                                 const int* levels, unsigned periodic_mask, int order, double h,
                                 double cutoff_a, int precision, int max_total_n,
                                 int quasi_degree_M);
/*
 * msm_batch_plan_create_kernel -- msm_batch_plan_create for the kernel
 * k(r) = r^-nu, nu = kernel (MSM_KERNEL_COULOMB or MSM_KERNEL_DISPERSION;
 * other values: MSM_ERR_INVALID_ARG), with the splitting described at
 * msm_plan_create_kernel (Sec. "Splitting for Coulomb kernels": the softened
 * pair part, K^1 and its k-sample ball, K^l = K^1 / 2^((l-1) nu) and each
 * system's dense top table, all from the same softener of r^-nu).  Every
 * system of the plan uses that kernel; msm_batch_energy_forces works as for
 * a Coulomb batch.
 */
msm_status msm_batch_plan_create_kernel(msm_plan* out, int kernel, int n_sys,
                                        const double* boxes, const int* levels,
                                        unsigned periodic_mask, int order, double h,
                                        double cutoff_a, int precision, int max_total_n,
                                        int quasi_degree_M);
/* offsets: device int32 [n_sys+1] CSR ranges into pos/q/forces/dEdq, with
 * offsets[0] = 0, non-decreasing, offsets[n_sys] <= max_total_n (checked on the
 * device: malformed offsets set the sticky flag, msm_plan_status then returns
 * MSM_ERR_INVALID_ARG); energies: device double [n_sys].  Positions of system s
 * must lie in [0, boxes[s]]^3.  The launch sequence is captured in a hipGraph
 * on the first call and replayed while the pointers and stream stay the same
 * (MSM_BATCH_GRAPH=0 launches directly).  The conv tile shape is chosen at
 * plan creation by timing the candidates (MSM_BATCH_TILE=0|1|2 pins one);
 * msm_plan_describe reports it.  ws must be NULL: there is no batched
 * backward whose saved state it would hold (non-NULL: MSM_ERR_UNSUPPORTED). */
msm_status msm_batch_energy_forces(msm_plan plan, const int* offsets, const void* pos,
                                   const void* q, void* ws, double* energies, void* forces,
                                   void* dEdq, void* stream);

/*
 * Stage timing with HIP events (benchmarks, MSM_PROFILE-style breakdowns).
 * msm_plan_set_profiling(plan, 1) makes every later msm_energy_forces /
 * msm_backward call record an event pair around each stage, on the stream
 * the stage runs on (the forward runs the pair sum and the coarse levels on
 * three plan-owned streams beside the caller's; MSM_STREAMS=0 keeps everything
 * on the caller's stream)
 * (binning, pair, anterpolation, restriction, conv per level, prolongation,
 * interpolation, backward passes); 0 stops recording.  Recording adds no
 * synchronisation.  msm_plan_get_profile synchronises on the recorded events,
 * writes {"stage": {"ms": total, "launches": calls, "start_ms": s,
 * "end_ms": e}, ...} into json[cap] and, if reset != 0, clears the totals;
 * s and e sum the stage's start and end times after the first stage of its
 * call ("bin" for the forward, "bwd_layout" for the backward), so s/calls
 * and e/calls place the stage on the call's timeline across streams.
 */
msm_status msm_plan_set_profiling(msm_plan plan, int enable);
msm_status msm_plan_get_profile(msm_plan plan, char* json, size_t cap, int reset);
/*
 * Restrict the recording to the stages named in stages (comma separated,
 * e.g. "conv_l1,pair"; NULL or "" records every stage).  Fewer event pairs
 * keep the timing of a multi-stream forward close to an unprofiled one.
 * The string is copied.  MSM_ERR_INVALID_ARG for a NULL plan.
 */
msm_status msm_plan_set_profile_stages(msm_plan plan, const char* stages);

const char* msm_status_string(msm_status status);

/*
 * Molecular dynamics around the forward (Sec. "MD simulation of charged
 * Lennard-Jonesium"): n charged Lennard-Jones particles in the plan's box,
 * integrated with velocity Verlet,
 *   v += dt/2 F/m;  x += dt v;  F = F_MSM(x) + F_LJ(x);  v += dt/2 F/m,
 * where F_MSM comes from msm_energy_forces on `plan` and
 *   u_LJ(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] S(r)
 * with the smooth switch S = 1 - 10 x^3 + 15 x^4 - 6 x^5,
 * x = (r - switch_on)/(cutoff - switch_on) between switch_on and cutoff
 * (S = 1 below, 0 beyond), minimum images on periodic axes.  The driver owns
 * its state (device, plan precision) and a stream; the plan (orthorhombic,
 * max_n >= n) stays the caller's and must outlive the driver.  Set a Verlet
 * skin on the plan (msm_plan_set_skin) to keep its cell list over steps.
 *   log_steps   steps whose energies are kept (msm_md_energies).
 * Errors: MSM_ERR_INVALID_ARG, MSM_ERR_UNSUPPORTED (triclinic plan),
 * MSM_ERR_CAPACITY (n > max_n), MSM_ERR_CUTOFF_TOO_LARGE (cutoff above half a
 * periodic edge), MSM_ERR_OOM.
 */
typedef struct msm_md_s* msm_md;
msm_status msm_md_create(msm_md* out, msm_plan plan, int n, double dt, double lj_epsilon,
                         double lj_sigma, double lj_cutoff, double lj_switch_on, int log_steps);
msm_status msm_md_destroy(msm_md md);
/* Copies the state in (device pos [n][3], vel [n][3], q [n], mass [n]),
 * evaluates the forces of pos and clears the energy log; ordered after
 * `stream`, and `stream` after it. */
msm_status msm_md_set_state(msm_md md, const void* pos, const void* vel, const void* q,
                            const void* mass, void* stream);
/* nsteps velocity-Verlet steps.  use_graph != 0: the first such call
 * captures one step in a HIP graph and every step replays it (the plan must
 * then not be used with another n, or re-celled, while the driver lives). */
msm_status msm_md_run(msm_md md, int nsteps, int use_graph, void* stream);
/* Copies positions, velocities and total forces out (device; NULL skips). */
msm_status msm_md_get_state(msm_md md, void* pos, void* vel, void* forces, void* stream);
/* Host copy of the energies after each step since msm_md_set_state:
 * host[3 k + 0..2] = kinetic, Lennard-Jones, MSM energy of step k, for
 * k < min(steps, log_steps, max_steps); *steps = steps run (synchronises). */
msm_status msm_md_energies(msm_md md, double* host, int max_steps, int* steps);

#ifdef __cplusplus
}
#endif
#endif
