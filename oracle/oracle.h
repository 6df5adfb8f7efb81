/*
 * FP64 CPU oracle of the gliding-assay micro-step.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no source with the HIP path: its own trig tables, its own
 * loops, its own sums.  Every array is a host, C-contiguous double array:
 *   psi [nx][ny][nth], M [nx][ny][nth][ns], m0/m1 [nx][ny][nth],
 *   u [2][nx][ny], gradu [4][nx][ny] = (dux/dx, dux/dy, duy/dx, duy/dy),
 *   stress [3][nx][ny] = (xx, xy, yy), mom [7][nx][ny] = (c, nx, ny, Dxx, Dxy, Dyy, B).
 *
 * Model: Cook & Shinar, Sec. 2 (Eqs. (1)-(6) of the model-summary table) and Alg. 2.
 */
#ifndef MMK_ORACLE_H
#define MMK_ORACLE_H

typedef struct {
    int nx, ny, nth, ns;
    double lx, ly, L;
    double k_on, k_off, v0;
    double F, sigma_f;
    int limiter;              /* 0: superbee MUSCL, 1: first-order upwind (sigma = 0) */
    double m_total;           /* total motor density per unit area; 0: free pool taken as 1 */
    double motor_cfl;         /* > 0: motor sub-cycling (local dt*), see oracle_motor_substeps */
    double rc;                /* > 0: capture radius of the anchor-resolved model (oracle_r0.c) */
} oracle_params;

/* superbee slope of the two one-sided differences a (left) and b (right) */
double oracle_superbee(double a, double b);

/* right-hand side of the motor walk + attach/detach equation on one column of ns cells */
void oracle_motor_rhs(const oracle_params *p, const double *z, double *R);
/* the same with the attachment source `src` (k_on times the free-motor density) */
void oracle_motor_rhs_src(const oracle_params *p, const double *z, double src, double *R);

/* the same on a run of n consecutive cells of width L/ns: minus-end rules at the run's
 * first cell, plus-end rules at its last (n = ns: a whole column) */
void oracle_run_rhs(const oracle_params *p, int n, const double *z, double src, double *R);

/* one explicit-midpoint step of one column: Mout = M + dt R(M + dt/2 R(M)) */
void oracle_column_step(const oracle_params *p, double dt, const double *M, double *Mout);
void oracle_column_step_src(const oracle_params *p, double dt, const double *M, double src, double *Mout);
void oracle_run_step(const oracle_params *p, int n, double dt, const double *M, double src, double *Mout);

/* coarse bound-motor density B [nx][ny] = sum_th psi m0 dth (Eq. (5), anchor-marginal) */
void oracle_coarse_bound(const oracle_params *p, const double *psi, const double *m0, double *B);

/* free-motor pool of Eq. (6) with the over-binding clamp of Alg. 2, per (x, y):
 * scale = M_total / B where B > M_total (else 1), src = k_on (M_total - min(B, M_total)). */
void oracle_depletion(const oracle_params *p, const double *B, double *scale, double *src);

/* zeroth and first arclength moments of one column */
void oracle_column_moments(const oracle_params *p, const double *M, double *m0, double *m1);

/* all columns: Mout, m0, m1 (m1 may be NULL) */
/* Motor sub-steps of one micro-step of length dt (Alg. 2: the inner step dt* is limited by
 * the motor's walking speed and detachment, a rate v0/ds + k_off that is the same at every
 * point): 1 when motor_cfl <= 0, else the least n >= 1 with dt/n * rate <= motor_cfl, i.e.
 * ceil(dt rate / motor_cfl).  With depletion (oracle_run) each sub-step starts with the coarse
 * density, the clamp and the free pool of the current sub-state. */
int oracle_motor_substeps(const oracle_params *p, double dt);

/* n explicit-midpoint steps of dt/n of every column (n from oracle_motor_substeps), then
 * the s-moments of the result (either moment pointer may be NULL). */
void oracle_motor_substepped(const oracle_params *p, double dt, const double *M, double *Mout,
                             double *m0, double *m1);

void oracle_motor_step(const oracle_params *p, double dt, const double *M, double *Mout,
                       double *m0, double *m1);

/* conservative donor-cell update of psi with velocities built from m0, u, gradu */
void oracle_psi_step(const oracle_params *p, double dt, const double *psi, const double *m0,
                     const double *u, const double *gradu, double *psi_out);

/* theta-moments and extra stress of (psi, m0, m1) */
void oracle_moments(const oracle_params *p, const double *psi, const double *m0,
                    const double *m1, double *stress, double *mom);

/* compensated FP64 totals: mass = sum psi dx dy dth, sum_sigma[c] = sum sigma_c dx dy */
void oracle_global_sums(const oracle_params *p, const double *psi, const double *stress,
                        double *mass, double *sum_sigma);

/* Motor force density F2 [2][nx][ny] of the state (psi, M), Eq. (10): the bound motors of cell l
 * of a filament centred at (x_i, y_j) with orientation p_k push with F p_k psi M_l ds dth; each
 * acts at the motor head x_h = (x_i, y_j) + (s_l - L/2) p_k and is spread onto the grid with the
 * two-point hat (bilinear) kernel, periodic in x and y.  Sequential loops (scatter). */
void oracle_motor_force(const oracle_params *p, const double *psi, const double *M, double *force);

/* nsteps micro-steps with one fluid field; psi and M are updated in place.
 * m0/m1 receive the moments of the final M (either may be NULL).  With m_total > 0 each
 * micro-step (every motor sub-step, with motor_cfl > 0) starts with the depletion of
 * oracle_depletion on the current state. */
void oracle_run(const oracle_params *p, double dt, int nsteps, double *psi, double *M,
                const double *u, const double *gradu, double *m0, double *m1);

/* ---- anchor-resolved bound motors M_b(r0, x, th, s) with capture radius rc (oracle_r0.c) ----
 * Anchors r0 sit on the cell centres.  A tracked cell is (a, b, k, l): the filament centred at
 * x = r0 + (a dx, b dy) with angle th_k, arclength cell l, whose point x + (s_l - L/2) p_k lies
 * within rc of r0.  Cells are listed in lexicographic order of (a, b, k, l); cells[4 c + 0..3]
 * = (a, b, k, l).  M_b is stored [cell][i][j] with (i, j) the filament's cell x (the anchor is
 * x - (a, b), periodic).  coarse, src, scale are per anchor [nx][ny]. */

/* number of tracked cells (cells may be NULL); -1 when rc <= 0 or rc + L/2 >= lx/2 or ly/2 */
long oracle_r0_cells(const oracle_params *p, int *cells);

/* Eq. (5) at every anchor: coarse = sum over its tracked cells of M_b psi ds dx dy dth */
void oracle_r0_coarse(const oracle_params *p, const int *cells, long ncell, const double *psi,
                      const double *Mb, double *coarse);

/* one motor step of every run of consecutive tracked cells (same a, b, k) as its own column;
 * the anchor's scale (NULL: 1) multiplies the run first, its src (NULL: k_on) is the source */
void oracle_r0_motor_step(const oracle_params *p, double dt, const int *cells, long ncell,
                          const double *Mb, double *Mout, const double *scale, const double *src);

/* anchor marginals of Eq. (10)'s r0 integral: m0[x][k] = sum over anchors and s of M_b ds dx dy,
 * m1 the same with the lever arm (s_l - L/2) (either may be NULL) */
void oracle_r0_marginal(const oracle_params *p, const int *cells, long ncell, const double *Mb,
                        double *m0, double *m1);

/* the anchor-marginal bound motors M[x][k][l] = sum over anchors of M_b dx dy (the r0 integral
 * of Eq. (10)); the motor force of the anchor-resolved state is oracle_motor_force of (psi, M) */
void oracle_r0_marginal_field(const oracle_params *p, const int *cells, long ncell, const double *Mb,
                              double *M);

/* nsteps micro-steps of the anchor-resolved model; psi and Mb in place.  Each micro-step: n
 * motor sub-steps of dt/n (n from oracle_motor_substeps), each preceded, with m_total > 0, by
 * the coarse density of the current sub-state (psi of the step's start), the clamp and the
 * free pool of oracle_depletion per anchor; then psi driven by the marginal m0.  m0, m1, coarse
 * (each may be NULL) receive the marginals and the coarse density of the final state. */
void oracle_r0_run(const oracle_params *p, double dt, int nsteps, const int *cells, long ncell,
                   double *psi, double *Mb, const double *u, const double *gradu, double *m0,
                   double *m1, double *coarse);

int oracle_max_threads(void);
void oracle_set_threads(int n);

#endif
