/*
 * FP64 CPU oracle of the gliding-assay micro-step.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg, never by
 * the product path.  Plain loops in the order the scheme is stated; no blocking, no
 * fusion.  OpenMP only splits independent outer loops (x rows) across threads; every
 * cell's arithmetic is the same as with one thread.  Build: -O2 -ffp-contract=off.
 *
 * Source of the method: S. Cook and T. Shinar, "Enabling Simulation of High-Dimensional
 * Micro-Macro Biophysical Models through Hybrid CPU and Multi-GPU Parallelism".
 *   - Sec. 2, Eq. (4): bound motors walk along s and attach/detach.  Reading used here:
 *     the anchor-marginal density M(x, th, s) with walking speed v0 in +s, linear
 *     attachment at rate k_on (free-motor pool taken as 1) and detachment k_off M.
 *   - Sec. 2: the s-flux uses a superbee limiter; Sec. 3.1 "Numerical Integration Scheme"
 *     and Alg. 2: a two-stage Runge-Kutta step (state at t + dt/2, then at t + dt).
 *   - Sec. 2, Eqs. (1)-(3): conservative transport of Psi(x, th) with translational
 *     velocity (motor gliding along -p plus the fluid velocity) and the rotational
 *     velocity p_perp . grad(u) . p.  Discretised here as first-order upwind (donor-cell)
 *     fluxes, forward Euler, periodic in x, y and th.
 *   - Sec. 2, Eq. (5) and the extra-stress step of Alg. 1: moments of Psi.
 *   - Optional depletion (m_total > 0): Eqs. (5)-(6) and the over-binding clamp of Alg. 2,
 *     applied at the start of each micro-step from the current state.
 *   - Optional motor sub-cycling (motor_cfl > 0): the inner loop of Alg. 2, n steps of dt/n
 *     with n from the motor's stability limit; with depletion the clamp and the free pool are
 *     taken again before every sub-step.
 * Where the paper leaves the discretisation open, the reading is written next to the code.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Superbee slope: zero when the one-sided differences a (left) and b (right) do not
 * have the same strict sign; otherwise sgn(b) max(min(2|a|,|b|), min(|a|,2|b|)), which is
 * Roe's superbee phi(r) = max(0, min(2r, 1), min(r, 2)) times b with r = a/b, written
 * without the division.  Ties: min keeps its first argument on <=, max on >=. */
double oracle_superbee(double a, double b) {
    if (a * b <= 0.0) return 0.0;
    double aa = fabs(a), ab = fabs(b);
    double p = (2.0 * aa <= ab) ? 2.0 * aa : ab;
    double q = (aa <= 2.0 * ab) ? aa : 2.0 * ab;
    double r = (p >= q) ? p : q;
    return (b > 0.0) ? r : -r;
}

/* R(z)_l = -(Phi_{l+1/2} - Phi_{l-1/2}) / ds + k_on - k_off z_l  on one column.
 * Fluxes (readings of the s boundaries, which the paper does not state):
 *   Phi_{-1/2} = 0                      no walking influx at the minus end s = 0
 *   Phi_{l+1/2} = v0 (z_l + sigma_l/2)  MUSCL face value, upwind for v0 >= 0
 *   Phi_{ns-1/2} = v0 z_{ns-1}          first-order free outflow at the plus end s = L
 * sigma_l = superbee(z_l - z_{l-1}, z_{l+1} - z_l) with ghosts z_{-1} = 0, z_{ns} = z_{ns-1}. */
void oracle_motor_rhs(const oracle_params *p, const double *z, double *R) {
    oracle_motor_rhs_src(p, z, p->k_on, R);
}

void oracle_motor_rhs_src(const oracle_params *p, const double *z, double src, double *R) {
    oracle_run_rhs(p, p->ns, z, src, R);
}

/* The same right-hand side on a run of n consecutive arclength cells (cell width ds = L/ns):
 * the run's first cell takes the minus-end rules (no influx, ghost 0) and its last cell the
 * plus-end rules (first-order outflow, ghost = itself).  n = ns is the whole column. */
void oracle_run_rhs(const oracle_params *p, int n, const double *z, double src, double *R) {
    const double ds = p->L / p->ns;
    double phi[n + 1]; /* phi[l] = Phi_{l-1/2} */
    phi[0] = 0.0;
    for (int l = 0; l < n; ++l) {
        double zl = z[l];
        double zm = (l == 0) ? 0.0 : z[l - 1];
        double zp = (l == n - 1) ? z[n - 1] : z[l + 1];
        double sig = (p->limiter == 0) ? oracle_superbee(zl - zm, zp - zl) : 0.0;
        if (l == n - 1)
            phi[l + 1] = p->v0 * zl;
        else
            phi[l + 1] = p->v0 * (zl + 0.5 * sig);
    }
    for (int l = 0; l < n; ++l)
        R[l] = -(phi[l + 1] - phi[l]) / ds + src - p->k_off * z[l];
}

/* Explicit midpoint: M* = M + (dt/2) R(M), Mout = M + dt R(M*). */
void oracle_column_step(const oracle_params *p, double dt, const double *M, double *Mout) {
    oracle_column_step_src(p, dt, M, p->k_on, Mout);
}

void oracle_column_step_src(const oracle_params *p, double dt, const double *M, double src, double *Mout) {
    oracle_run_step(p, p->ns, dt, M, src, Mout);
}

void oracle_run_step(const oracle_params *p, int n, double dt, const double *M, double src, double *Mout) {
    if (n <= 0) return;
    double R[n], Ms[n];
    for (int l = 0; l < n; ++l) Ms[l] = 0.0;
    oracle_run_rhs(p, n, M, src, R);
    for (int l = 0; l < n; ++l) Ms[l] = M[l] + 0.5 * dt * R[l];
    oracle_run_rhs(p, n, Ms, src, R);
    for (int l = 0; l < n; ++l) Mout[l] = M[l] + dt * R[l];
}

/* m0 = sum_l M_l ds (bound motors per filament, the gliding force magnitude up to F);
 * m1 = sum_l (s_l - L/2) M_l ds with s_l = (l + 1/2) ds (lever arm about the centre). */
void oracle_column_moments(const oracle_params *p, const double *M, double *m0, double *m1) {
    const int ns = p->ns;
    const double ds = p->L / ns;
    double a = 0.0, b = 0.0;
    for (int l = 0; l < ns; ++l) {
        double s = (l + 0.5) * ds;
        a += M[l] * ds;
        b += (s - 0.5 * p->L) * M[l] * ds;
    }
    *m0 = a;
    *m1 = b;
}

void oracle_motor_step(const oracle_params *p, double dt, const double *M, double *Mout,
                       double *m0, double *m1) {
    const long ncol_x = (long)p->ny * p->nth;
    const int ns = p->ns;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < p->nx; ++i) {
        for (long c = 0; c < ncol_x; ++c) {
            long col = (long)i * ncol_x + c;
            const double *src = M + col * ns;
            double *dst = Mout + col * ns;
            oracle_column_step(p, dt, src, dst);
            double a, b;
            oracle_column_moments(p, dst, &a, &b);
            if (m0) m0[col] = a;
            if (m1) m1[col] = b;
        }
    }
}

int oracle_motor_substeps(const oracle_params *p, double dt) {
    if (!(p->motor_cfl > 0.0)) return 1;
    const double rate = p->v0 / (p->L / p->ns) + p->k_off;
    const double n = ceil(dt * rate / p->motor_cfl);
    return n < 1.0 ? 1 : (int)n;
}

void oracle_motor_substepped(const oracle_params *p, double dt, const double *M, double *Mout,
                             double *m0, double *m1) {
    const int n = oracle_motor_substeps(p, dt), ns = p->ns;
    const double h = dt / n;
    const long ncol = (long)p->nx * p->ny * p->nth;
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * (size_t)ns);
#pragma omp for schedule(static)
        for (long col = 0; col < ncol; ++col) {
            double *dst = Mout + col * ns;
            memcpy(dst, M + col * ns, sizeof(double) * (size_t)ns);
            for (int q = 0; q < n; ++q) {
                oracle_column_step(p, h, dst, tmp);
                memcpy(dst, tmp, sizeof(double) * (size_t)ns);
            }
            double a, b;
            oracle_column_moments(p, dst, &a, &b);
            if (m0) m0[col] = a;
            if (m1) m1[col] = b;
        }
        free(tmp);
    }
}

/* donor-cell face flux: upwind value of psi times the face velocity; A = 0 takes the
 * left branch (both branches give 0 there). */
static double donor(double A, double left, double right) {
    return (A >= 0.0) ? A * left : A * right;
}

/* rotational velocity of a thin rod at angle th in the velocity gradient G:
 * p_perp . G . p with p = (cos th, sin th), p_perp = (-sin th, cos th) (Jeffery term). */
static double jeffery(const double G[4], double c, double s) {
    return -s * (G[0] * c + G[1] * s) + c * (G[2] * c + G[3] * s);
}

#define IDX3(i, j, k) (((long)(i) * ny + (j)) * nth + (k))
#define IDX2(i, j) ((long)(i) * ny + (j))

void oracle_psi_step(const oracle_params *p, double dt, const double *psi, const double *m0,
                     const double *u, const double *gradu, double *psi_out) {
    const int nx = p->nx, ny = p->ny, nth = p->nth;
    const long npsi = (long)nx * ny * nth, nxy = (long)nx * ny;
    const double dx = p->lx / nx, dy = p->ly / ny, dth = TWO_PI / nth;
    double *cs = (double *)malloc(sizeof(double) * (size_t)nth);
    double *sn = (double *)malloc(sizeof(double) * (size_t)nth);
    double *ch = (double *)malloc(sizeof(double) * (size_t)nth); /* at faces th_{k+1/2} */
    double *sh = (double *)malloc(sizeof(double) * (size_t)nth);
    for (int k = 0; k < nth; ++k) {
        cs[k] = cos(k * dth);
        sn[k] = sin(k * dth);
        ch[k] = cos((k + 0.5) * dth);
        sh[k] = sin((k + 0.5) * dth);
    }
    /* fx[i,j,k]: flux through the face between cells i and i+1; likewise fy in j and
     * fth between k and k+1 (all periodic). */
    double *fx = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *fy = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *ft = (double *)malloc(sizeof(double) * (size_t)npsi);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        int ip = (i + 1) % nx;
        for (int j = 0; j < ny; ++j) {
            int jp = (j + 1) % ny;
            double G[4] = {gradu[0 * nxy + IDX2(i, j)], gradu[1 * nxy + IDX2(i, j)],
                           gradu[2 * nxy + IDX2(i, j)], gradu[3 * nxy + IDX2(i, j)]};
            for (int k = 0; k < nth; ++k) {
                int kp = (k + 1) % nth;
                /* cell velocity: fluid velocity minus gliding F m0 p (reading of V_sp) */
                double ax_c = u[0 * nxy + IDX2(i, j)] - p->F * m0[IDX3(i, j, k)] * cs[k];
                double ax_r = u[0 * nxy + IDX2(ip, j)] - p->F * m0[IDX3(ip, j, k)] * cs[k];
                double ay_c = u[1 * nxy + IDX2(i, j)] - p->F * m0[IDX3(i, j, k)] * sn[k];
                double ay_r = u[1 * nxy + IDX2(i, jp)] - p->F * m0[IDX3(i, jp, k)] * sn[k];
                double Ax = 0.5 * (ax_c + ax_r);
                double Ay = 0.5 * (ay_c + ay_r);
                double At = jeffery(G, ch[k], sh[k]);
                fx[IDX3(i, j, k)] = donor(Ax, psi[IDX3(i, j, k)], psi[IDX3(ip, j, k)]);
                fy[IDX3(i, j, k)] = donor(Ay, psi[IDX3(i, j, k)], psi[IDX3(i, jp, k)]);
                ft[IDX3(i, j, k)] = donor(At, psi[IDX3(i, j, k)], psi[IDX3(i, j, kp)]);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        int im = (i + nx - 1) % nx;
        for (int j = 0; j < ny; ++j) {
            int jm = (j + ny - 1) % ny;
            for (int k = 0; k < nth; ++k) {
                int km = (k + nth - 1) % nth;
                double div = (fx[IDX3(i, j, k)] - fx[IDX3(im, j, k)]) / dx
                           + (fy[IDX3(i, j, k)] - fy[IDX3(i, jm, k)]) / dy
                           + (ft[IDX3(i, j, k)] - ft[IDX3(i, j, km)]) / dth;
                psi_out[IDX3(i, j, k)] = psi[IDX3(i, j, k)] - dt * div;
            }
        }
    }
    free(fx);
    free(fy);
    free(ft);
    free(cs);
    free(sn);
    free(ch);
    free(sh);
}

/* c = sum psi dth, n = sum psi p dth, D = sum psi p p dth, B = sum psi m0 dth,
 * sigma = sigma_f (D - c I / 2) + F sum psi m1 p p dth, with D - c I/2 formed per angle
 * as (cos 2th / 2, sin 2th / 2, -cos 2th / 2). */
void oracle_moments(const oracle_params *p, const double *psi, const double *m0,
                    const double *m1, double *stress, double *mom) {
    const int nx = p->nx, ny = p->ny, nth = p->nth;
    const long nxy = (long)nx * ny;
    const double dth = TWO_PI / nth;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < ny; ++j) {
            double c = 0, n1 = 0, n2 = 0, dxx = 0, dxy = 0, dyy = 0, B = 0;
            double sxx = 0, sxy = 0, syy = 0;
            for (int k = 0; k < nth; ++k) {
                double th = k * dth;
                double co = cos(th), si = sin(th);
                double h1 = 0.5 * cos(2.0 * th), h2 = 0.5 * sin(2.0 * th);
                double ps = psi[IDX3(i, j, k)];
                double mm1 = m1[IDX3(i, j, k)];
                c += ps;
                n1 += ps * co;
                n2 += ps * si;
                dxx += ps * co * co;
                dxy += ps * co * si;
                dyy += ps * si * si;
                B += ps * m0[IDX3(i, j, k)];
                sxx += ps * (p->sigma_f * h1 + p->F * mm1 * co * co);
                sxy += ps * (p->sigma_f * h2 + p->F * mm1 * co * si);
                syy += ps * (-p->sigma_f * h1 + p->F * mm1 * si * si);
            }
            long o = IDX2(i, j);
            mom[0 * nxy + o] = c * dth;
            mom[1 * nxy + o] = n1 * dth;
            mom[2 * nxy + o] = n2 * dth;
            mom[3 * nxy + o] = dxx * dth;
            mom[4 * nxy + o] = dxy * dth;
            mom[5 * nxy + o] = dyy * dth;
            mom[6 * nxy + o] = B * dth;
            stress[0 * nxy + o] = sxx * dth;
            stress[1 * nxy + o] = sxy * dth;
            stress[2 * nxy + o] = syy * dth;
        }
    }
}

/* Neumaier's compensated summation, sequential in index order. */
static double neumaier(const double *x, long n) {
    double s = 0.0, c = 0.0;
    for (long i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i]))
            c += (s - t) + x[i];
        else
            c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

void oracle_global_sums(const oracle_params *p, const double *psi, const double *stress,
                        double *mass, double *sum_sigma) {
    const long nxy = (long)p->nx * p->ny, npsi = nxy * p->nth;
    const double dx = p->lx / p->nx, dy = p->ly / p->ny, dth = TWO_PI / p->nth;
    if (mass) *mass = neumaier(psi, npsi) * (dx * dy * dth);
    if (sum_sigma && stress)
        for (int c = 0; c < 3; ++c) sum_sigma[c] = neumaier(stress + c * nxy, nxy) * (dx * dy);
}

/* Eq. (10) with the delta function of the immersed-boundary spreading taken as the two-point
 * hat in each direction: a point force at x_h lands on the four cell centres around it with
 * the bilinear weights (1 - a)(1 - b), a(1 - b), (1 - a)b, ab.  The y-integral's dx dy cancels
 * the hat's 1/(dx dy), so each motor cell adds F p psi M ds dth times its weights. */
void oracle_motor_force(const oracle_params *p, const double *psi, const double *M, double *force) {
    const long nx = p->nx, ny = p->ny, nth = p->nth;
    const int ns = p->ns;
    const long nxy = nx * ny;
    const double dx = p->lx / nx, dy = p->ly / ny, dth = TWO_PI / nth, ds = p->L / ns;
    for (long o = 0; o < 2 * nxy; ++o) force[o] = 0.0;
    for (long i = 0; i < nx; ++i)
        for (long j = 0; j < ny; ++j)
            for (long k = 0; k < nth; ++k) {
                const double th = k * dth, co = cos(th), si = sin(th);
                const double ps = psi[IDX3(i, j, k)];
                for (int l = 0; l < ns; ++l) {
                    const double lever = (l + 0.5) * ds - 0.5 * p->L;
                    const double hx = (i + 0.5) * dx + lever * co, hy = (j + 0.5) * dy + lever * si;
                    /* fractional cell-centre index of the head, its lower neighbour and weight */
                    const double fx = hx / dx - 0.5, fy = hy / dy - 0.5;
                    const double ix = floor(fx), iy = floor(fy);
                    const double ax = fx - ix, ay = fy - iy;
                    const long i0 = (((long)ix % nx) + nx) % nx, j0 = (((long)iy % ny) + ny) % ny;
                    const long i1 = (i0 + 1) % nx, j1 = (j0 + 1) % ny;
                    const double v = p->F * ps * M[IDX3(i, j, k) * ns + l] * ds * dth;
                    const double w[4] = {(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay};
                    const long cell[4] = {IDX2(i0, j0), IDX2(i1, j0), IDX2(i0, j1), IDX2(i1, j1)};
                    for (int q = 0; q < 4; ++q) {
                        force[cell[q]] += v * co * w[q];
                        force[nxy + cell[q]] += v * si * w[q];
                    }
                }
            }
}

/* Coarse bound-motor density: Eq. (5) integrates the bound motors of every filament over
 * s, x and th at an anchor r0; in the anchor-marginal reading the bound motors per unit area
 * at (x, y) are sum over th of psi times the motors per filament m0. */
void oracle_coarse_bound(const oracle_params *p, const double *psi, const double *m0, double *B) {
    const long nx = p->nx, ny = p->ny, nth = p->nth;
    const double dth = TWO_PI / nth;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double b = 0.0;
            for (int k = 0; k < nth; ++k) b += psi[IDX3(i, j, k)] * m0[IDX3(i, j, k)];
            B[IDX2(i, j)] = b * dth;
        }
}

/* Eq. (6): free motors M_f = M_total - B.  Alg. 2: where the bound motors exceed the total,
 * every bound-motor column at that point is scaled down to the total (then M_f = 0). */
void oracle_depletion(const oracle_params *p, const double *B, double *scale, double *src) {
    const long nxy = (long)p->nx * p->ny;
    for (long o = 0; o < nxy; ++o) {
        if (B[o] > p->m_total) {
            scale[o] = p->m_total / B[o];
            src[o] = 0.0;
        } else {
            scale[o] = 1.0;
            src[o] = p->k_on * (p->m_total - B[o]);
        }
    }
}

/* One motor step with depletion: each column of (x, y) is first scaled by scale[x, y],
 * then stepped with the attachment source src[x, y] held over the step. */
static void motor_step_depleted(const oracle_params *p, double dt, const double *M, double *Mout, double *m0,
                                const double *scale, const double *src) {
    const int ns = p->ns;
    const long ny = p->ny, nth = p->nth;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < p->nx; ++i) {
        double Mc[ns];
        for (int j = 0; j < ny; ++j) {
            const long o = IDX2(i, j);
            for (int k = 0; k < nth; ++k) {
                const long col = IDX3(i, j, k);
                for (int l = 0; l < ns; ++l) Mc[l] = scale[o] * M[col * ns + l];
                oracle_column_step_src(p, dt, Mc, src[o], Mout + col * ns);
                double a, b;
                oracle_column_moments(p, Mout + col * ns, &a, &b);
                m0[col] = a;
            }
        }
    }
}

void oracle_run(const oracle_params *p, double dt, int nsteps, double *psi, double *M,
                const double *u, const double *gradu, double *m0_out, double *m1_out) {
    const long npsi = (long)p->nx * p->ny * p->nth, nm = npsi * p->ns, nxy = (long)p->nx * p->ny;
    const int depl = p->m_total > 0.0;
    double *M2 = (double *)malloc(sizeof(double) * (size_t)nm);
    double *psi2 = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *m0 = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *B = depl ? (double *)malloc(sizeof(double) * (size_t)(3 * nxy)) : NULL;
    double *Ma = M, *Mb = M2, *pa = psi, *pb = psi2;
    if (depl) /* m0 of the current state, for its coarse bound density */
        for (long c = 0; c < npsi; ++c) {
            double a, b;
            oracle_column_moments(p, M + c * p->ns, &a, &b);
            m0[c] = a;
        }
    for (int n = 0; n < nsteps; ++n) {
        /* order within a micro-step: [depletion of the current state,] motors, then psi
         * driven by the new m0 */
        if (depl) {
            /* Alg. 2's inner loop with depletion: before each of the n sub-steps of dt/n, the
             * coarse density of the current sub-state (psi held at its start-of-step value),
             * the clamp and the pool (n = 1 without sub-cycling) */
            double *scale = B + nxy, *src = B + 2 * nxy;
            const int nsub = oracle_motor_substeps(p, dt);
            for (int q = 0; q < nsub; ++q) {
                oracle_coarse_bound(p, pa, m0, B);
                oracle_depletion(p, B, scale, src);
                motor_step_depleted(p, dt / nsub, Ma, Mb, m0, scale, src);
                if (q + 1 < nsub) {
                    double *t = Ma; Ma = Mb; Mb = t;
                }
            }
        } else if (p->motor_cfl > 0.0) {
            oracle_motor_substepped(p, dt, Ma, Mb, m0, NULL);
        } else {
            oracle_motor_step(p, dt, Ma, Mb, m0, NULL);
        }
        oracle_psi_step(p, dt, pa, m0, u, gradu, pb);
        double *t = Ma; Ma = Mb; Mb = t;
        t = pa; pa = pb; pb = t;
    }
    if (Ma != M) memcpy(M, Ma, sizeof(double) * (size_t)nm);
    if (pa != psi) memcpy(psi, pa, sizeof(double) * (size_t)npsi);
    if (m0_out || m1_out) {
        const long ncol = npsi;
#pragma omp parallel for schedule(static)
        for (long c = 0; c < ncol; ++c) {
            double a, b;
            oracle_column_moments(p, M + c * p->ns, &a, &b);
            if (m0_out) m0_out[c] = a;
            if (m1_out) m1_out[c] = b;
        }
    }
    free(M2);
    free(psi2);
    free(m0);
    free(B);
}
