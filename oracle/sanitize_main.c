/*
 * Driver of the FP64 oracle for an AddressSanitizer + UndefinedBehaviorSanitizer build (test
 * infrastructure, CPU only): runs every entry point of oracle.h on small grids with ragged
 * sizes, both limiters, depletion, motor sub-cycling and the anchor-resolved model, so that an
 * out-of-bounds access, a use of an uninitialised allocation or undefined arithmetic in the
 * oracle's loops is reported by the sanitizers.  Prints "ok" and the finite-ness of the results.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

static double *fill(size_t n, unsigned *seed, double lo, double hi) {
    double *a = malloc(n * sizeof *a);
    for (size_t i = 0; i < n; ++i) {
        *seed = *seed * 1103515245u + 12345u;
        a[i] = lo + (hi - lo) * (double)((*seed >> 8) & 0xffffff) / 16777216.0;
    }
    return a;
}

static int finite_all(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run_case(int nx, int ny, int nth, int ns, int limiter, double m_total, double motor_cfl, unsigned seed) {
    oracle_params p = {nx, ny, nth, ns, 6.283185307179586, 5.0, 1.0, 1.0, 0.5, 1.5, 0.8, 1.0,
                       limiter, m_total, motor_cfl, 0.0};
    const size_t npsi = (size_t)nx * ny * nth, nm = npsi * ns, nxy = (size_t)nx * ny;
    double *psi = fill(npsi, &seed, 0.5, 1.5), *M = fill(nm, &seed, 0.0, 2.0);
    double *u = fill(2 * nxy, &seed, -0.1, 0.1), *g = fill(4 * nxy, &seed, -0.1, 0.1);
    double *Mo = malloc(nm * sizeof *Mo), *m0 = malloc(npsi * sizeof *m0), *m1 = malloc(npsi * sizeof *m1);
    double *po = malloc(npsi * sizeof *po), *st = malloc(3 * nxy * sizeof *st), *mo = malloc(7 * nxy * sizeof *mo);
    double *B = malloc(nxy * sizeof *B), *sc = malloc(nxy * sizeof *sc), *src = malloc(nxy * sizeof *src);
    double *f = malloc(2 * nxy * sizeof *f), *R = malloc(ns * sizeof *R);
    double mass, ss[3], a0, a1;
    const double dt = 2e-3;
    oracle_motor_rhs(&p, M, R);
    oracle_motor_rhs_src(&p, M, 0.7, R);
    oracle_run_rhs(&p, ns, M, 0.7, R);
    oracle_column_step(&p, dt, M, Mo);
    oracle_column_step_src(&p, dt, M, 0.7, Mo);
    oracle_run_step(&p, ns > 2 ? ns - 1 : ns, dt, M, 0.7, Mo);
    oracle_column_moments(&p, M, &a0, &a1);
    oracle_motor_step(&p, dt, M, Mo, m0, m1);
    (void)oracle_motor_substeps(&p, dt);
    oracle_motor_substepped(&p, dt, M, Mo, m0, NULL);
    oracle_coarse_bound(&p, psi, m0, B);
    oracle_depletion(&p, B, sc, src);
    oracle_psi_step(&p, dt, psi, m0, u, g, po);
    oracle_moments(&p, po, m0, m1, st, mo);
    oracle_global_sums(&p, po, st, &mass, ss);
    oracle_motor_force(&p, po, Mo, f);
    oracle_run(&p, dt, 3, psi, M, u, g, m0, m1);
    int ok = finite_all(psi, npsi) && finite_all(M, nm) && finite_all(st, 3 * nxy) && finite_all(f, 2 * nxy)
             && isfinite(mass);
    free(psi); free(M); free(u); free(g); free(Mo); free(m0); free(m1); free(po); free(st); free(mo);
    free(B); free(sc); free(src); free(f); free(R);
    return ok;
}

static int run_r0_case(int nx, int ny, int nth, int ns, double rc, double m_total, double motor_cfl, unsigned seed) {
    oracle_params p = {nx, ny, nth, ns, 6.283185307179586, 6.283185307179586, 1.0, 1.0, 0.5, 1.5, 0.8, 1.0,
                       0, m_total, motor_cfl, rc};
    const long ncell = oracle_r0_cells(&p, NULL);
    if (ncell < 0) return 0;
    int *cells = malloc((size_t)(ncell > 0 ? ncell : 1) * 4 * sizeof *cells);
    oracle_r0_cells(&p, cells);
    const size_t npsi = (size_t)nx * ny * nth, nxy = (size_t)nx * ny, nb = (size_t)ncell * nxy;
    double *psi = fill(npsi, &seed, 0.5, 1.5), *Mb = fill(nb > 0 ? nb : 1, &seed, 0.0, 2.0);
    double *u = fill(2 * nxy, &seed, -0.1, 0.1), *g = fill(4 * nxy, &seed, -0.1, 0.1);
    double *Mo = malloc((nb > 0 ? nb : 1) * sizeof *Mo), *co = malloc(nxy * sizeof *co);
    double *m0 = malloc(npsi * sizeof *m0), *m1 = malloc(npsi * sizeof *m1);
    double *Mf = malloc(npsi * ns * sizeof *Mf);
    oracle_r0_coarse(&p, cells, ncell, psi, Mb, co);
    oracle_r0_motor_step(&p, 2e-3, cells, ncell, Mb, Mo, NULL, NULL);
    oracle_r0_marginal(&p, cells, ncell, Mb, m0, m1);
    oracle_r0_marginal_field(&p, cells, ncell, Mb, Mf);
    oracle_r0_run(&p, 2e-3, 2, cells, ncell, psi, Mb, u, g, m0, m1, co);
    int ok = finite_all(psi, npsi) && finite_all(co, nxy);
    free(cells); free(psi); free(Mb); free(u); free(g); free(Mo); free(co); free(m0); free(m1); free(Mf);
    return ok;
}

int main(void) {
    int ok = 1;
    ok &= run_case(5, 3, 7, 9, 0, 0.0, 0.0, 1u);
    ok &= run_case(1, 1, 1, 1, 1, 0.0, 0.0, 2u);
    ok &= run_case(4, 6, 8, 16, 0, 0.05, 0.0, 3u);
    ok &= run_case(3, 5, 6, 12, 0, 0.05, 0.1, 4u);
    ok &= run_case(6, 4, 4, 3, 1, 0.0, 0.2, 5u);
    ok &= run_r0_case(12, 10, 8, 8, 0.45, 0.0, 0.0, 6u);
    ok &= run_r0_case(12, 12, 6, 10, 0.6, 0.01, 0.1, 7u);
    ok &= run_r0_case(10, 10, 4, 4, 0.05, 0.01, 0.0, 8u);
    printf(ok ? "ok\n" : "non-finite result\n");
    return ok ? 0 : 1;
}
