/*
 * FP64 CPU oracle of the anchor-resolved bound-motor step.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg, never by the
 * product path.  Plain loops in the order the model is stated.
 *
 * Source: Cook & Shinar, Sec. 2 (the density M_b(r0, x, p, s) of motors anchored at r0, the
 * capture ball B_rc(r0) of the configurations whose motor point x + s p lies within rc of r0,
 * Eqs. (4)-(6)) and Alg. 2 (per anchor: the motor update of every configuration in B_rc(r0),
 * the coarse integral of Eq. (5), the over-binding clamp, the free pool of Eq. (6)).
 * Readings, where the paper leaves the discretisation open:
 *   - anchors sit on the cell centres of the x grid, so an anchor and a filament cell differ
 *     by a whole-cell offset (a, b); the motor point of arclength cell l is
 *     x + (s_l - L/2) p_k (the arclength is measured from the filament centre);
 *   - configurations outside B_rc(r0) are not tracked (zero): along a filament the tracked
 *     cells form runs, and each run is a column of its own.  A motor walking out of the ball
 *     leaves (first-order free outflow at the run's plus end), none walks in at the run's
 *     minus end; inside the run the flux and the RK2 step are those of the full column;
 *   - the attachment indicator of Eq. (4) is 1 on every tracked cell;
 *   - the clamp and the free pool are taken at the start of each micro-step from the current
 *     (psi, M_b), as in the anchor-marginal depletion; with motor sub-cycling (motor_cfl > 0)
 *     at the start of each motor sub-step, from the current sub-state and psi of the step's
 *     start (Alg. 2 clamps inside its inner loop);
 *   - psi is driven by the anchor marginal m0 = sum over anchors and s of M_b ds dx dy (the r0
 *     integral of Eq. (10) taken as a sum over the anchor lattice with area dx dy).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925286766559

/* The motor point of cell (a, b, k, l) relative to its anchor is (a dx, b dy) + t p_k with
 * t = s_l - L/2; tracked when its squared length is at most rc^2. */
static int tracked(const oracle_params *p, int a, int b, int k, int l) {
    const double dx = p->lx / p->nx, dy = p->ly / p->ny, dth = TWO_PI / p->nth, ds = p->L / p->ns;
    const double t = (l + 0.5) * ds - 0.5 * p->L;
    const double th = k * dth;
    const double hx = a * dx + t * cos(th);
    const double hy = b * dy + t * sin(th);
    return hx * hx + hy * hy <= p->rc * p->rc;
}

long oracle_r0_cells(const oracle_params *p, int *cells) {
    if (!(p->rc > 0.0) || !(p->rc + 0.5 * p->L < 0.5 * p->lx) || !(p->rc + 0.5 * p->L < 0.5 * p->ly)) return -1;
    /* every tracked point lies within rc + L/2 of the anchor: this window holds them all */
    const int A = (int)ceil((p->rc + 0.5 * p->L) / (p->lx / p->nx)) + 1;
    const int B = (int)ceil((p->rc + 0.5 * p->L) / (p->ly / p->ny)) + 1;
    long n = 0;
    for (int a = -A; a <= A; ++a)
        for (int b = -B; b <= B; ++b)
            for (int k = 0; k < p->nth; ++k)
                for (int l = 0; l < p->ns; ++l)
                    if (tracked(p, a, b, k, l)) {
                        if (cells) {
                            cells[4 * n + 0] = a;
                            cells[4 * n + 1] = b;
                            cells[4 * n + 2] = k;
                            cells[4 * n + 3] = l;
                        }
                        ++n;
                    }
    return n;
}

static long wrap(long v, long n) { return ((v % n) + n) % n; }

void oracle_r0_coarse(const oracle_params *p, const int *cells, long ncell, const double *psi,
                      const double *Mb, double *coarse) {
    const long nx = p->nx, ny = p->ny, nth = p->nth, nxy = nx * ny;
    const double dx = p->lx / nx, dy = p->ly / ny, dth = TWO_PI / nth, ds = p->L / p->ns;
#pragma omp parallel for schedule(static)
    for (long i0 = 0; i0 < nx; ++i0)
        for (long j0 = 0; j0 < ny; ++j0) {
            double sum = 0.0;
            for (long c = 0; c < ncell; ++c) {
                const long i = wrap(i0 + cells[4 * c + 0], nx), j = wrap(j0 + cells[4 * c + 1], ny);
                sum += Mb[c * nxy + i * ny + j] * psi[(i * ny + j) * nth + cells[4 * c + 2]];
            }
            coarse[i0 * ny + j0] = sum * ds * dx * dy * dth;
        }
}

void oracle_r0_motor_step(const oracle_params *p, double dt, const int *cells, long ncell,
                          const double *Mb, double *Mout, const double *scale, const double *src) {
    const long nx = p->nx, ny = p->ny, nxy = nx * ny;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nx; ++i) {
        double run[p->ns], out[p->ns];
        for (long j = 0; j < ny; ++j) {
            const long x = i * ny + j;
            long c0 = 0;
            while (c0 < ncell) {
                /* the run starting at c0: same (a, b, k), consecutive l */
                long c1 = c0 + 1;
                while (c1 < ncell && cells[4 * c1 + 0] == cells[4 * c0 + 0] && cells[4 * c1 + 1] == cells[4 * c0 + 1] &&
                       cells[4 * c1 + 2] == cells[4 * c0 + 2] && cells[4 * c1 + 3] == cells[4 * (c1 - 1) + 3] + 1)
                    ++c1;
                const long r0 = wrap(i - cells[4 * c0 + 0], nx) * ny + wrap(j - cells[4 * c0 + 1], ny);
                const int n = (int)(c1 - c0);
                for (int t = 0; t < n; ++t) run[t] = (scale ? scale[r0] : 1.0) * Mb[(c0 + t) * nxy + x];
                oracle_run_step(p, n, dt, run, src ? src[r0] : p->k_on, out);
                for (int t = 0; t < n; ++t) Mout[(c0 + t) * nxy + x] = out[t];
                c0 = c1;
            }
        }
    }
}

void oracle_r0_marginal(const oracle_params *p, const int *cells, long ncell, const double *Mb,
                        double *m0, double *m1) {
    const long nx = p->nx, ny = p->ny, nth = p->nth, nxy = nx * ny;
    const double dx = p->lx / nx, dy = p->ly / ny, ds = p->L / p->ns;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < nxy; ++x) {
        for (long k = 0; k < nth; ++k) {
            if (m0) m0[x * nth + k] = 0.0;
            if (m1) m1[x * nth + k] = 0.0;
        }
        for (long c = 0; c < ncell; ++c) {
            const long k = cells[4 * c + 2];
            const double s = (cells[4 * c + 3] + 0.5) * ds;
            const double v = Mb[c * nxy + x];
            if (m0) m0[x * nth + k] += v * ds * dx * dy;
            if (m1) m1[x * nth + k] += (s - 0.5 * p->L) * v * ds * dx * dy;
        }
    }
}

void oracle_r0_marginal_field(const oracle_params *p, const int *cells, long ncell, const double *Mb,
                              double *M) {
    const long nx = p->nx, ny = p->ny, nth = p->nth, ns = p->ns, nxy = nx * ny;
    const double dx = p->lx / nx, dy = p->ly / ny;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < nxy; ++x) {
        for (long q = 0; q < nth * ns; ++q) M[x * nth * ns + q] = 0.0;
        for (long c = 0; c < ncell; ++c)
            M[(x * nth + cells[4 * c + 2]) * ns + cells[4 * c + 3]] += Mb[c * nxy + x] * dx * dy;
    }
}

void oracle_r0_run(const oracle_params *p, double dt, int nsteps, const int *cells, long ncell,
                   double *psi, double *Mb, const double *u, const double *gradu, double *m0_out,
                   double *m1_out, double *coarse_out) {
    const long nxy = (long)p->nx * p->ny, npsi = nxy * p->nth, nm = ncell * nxy;
    const int depl = p->m_total > 0.0;
    double *M2 = (double *)malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1));
    double *psi2 = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *m0 = (double *)malloc(sizeof(double) * (size_t)npsi);
    double *B = (double *)malloc(sizeof(double) * (size_t)(3 * nxy));
    double *Ma = Mb, *Mn = M2, *pa = psi, *pb = psi2;
    /* motor sub-cycling (the local dt* of Alg. 2): nsub steps of dt/nsub, nsub = 1 when
     * motor_cfl is 0; the rate bound is the same for every anchor, so one count serves all */
    const int nsub = oracle_motor_substeps(p, dt);
    for (int n = 0; n < nsteps; ++n) {
        /* order: for each motor sub-step [the clamp and the pool of every anchor from the
         * current sub-state, psi held at its start-of-step value,] the run step; then psi
         * driven by the new m0 */
        for (int q = 0; q < nsub; ++q) {
            double *scale = NULL, *src = NULL;
            if (depl) {
                scale = B + nxy;
                src = B + 2 * nxy;
                oracle_r0_coarse(p, cells, ncell, pa, Ma, B);
                oracle_depletion(p, B, scale, src);
            }
            oracle_r0_motor_step(p, dt / nsub, cells, ncell, Ma, Mn, scale, src);
            if (q + 1 < nsub) {
                double *t = Ma; Ma = Mn; Mn = t;
            }
        }
        oracle_r0_marginal(p, cells, ncell, Mn, m0, NULL);
        oracle_psi_step(p, dt, pa, m0, u, gradu, pb);
        double *t = Ma; Ma = Mn; Mn = t;
        t = pa; pa = pb; pb = t;
    }
    if (Ma != Mb) memcpy(Mb, Ma, sizeof(double) * (size_t)nm);
    if (pa != psi) memcpy(psi, pa, sizeof(double) * (size_t)npsi);
    if (m0_out || m1_out) oracle_r0_marginal(p, cells, ncell, Mb, m0_out, m1_out);
    if (coarse_out) oracle_r0_coarse(p, cells, ncell, psi, Mb, coarse_out);
    free(M2);
    free(psi2);
    free(m0);
    free(B);
}
