/*
 * oracle_sanitize_driver.c -- runs the oracle's entry points on small
 * problems so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * sees every code path: both limiters, transmissive and periodic walls, both
 * sweep orders, grids smaller than the stencil, the sampled-cell step, the
 * Cochran-Chan and reactive liquids, and the diagnostics.  Test
 * infrastructure (built and run by tests/test_oracle_sanitizers.py); it
 * includes the oracle's source so that one translation unit is instrumented.
 */
#include "oracle.c"

#include <stdio.h>

static or_problem base(int nx, int ny)
{
    or_problem P;
    memset(&P, 0, sizeof P);
    P.nx = nx; P.ny = ny; P.dx = 1.0e-5; P.dy = 1.0e-5;
    P.gamma1 = 1.4; P.pinf1 = 0.0; P.gamma2 = 4.4; P.pinf2 = 6.0e8;
    P.cfl = 0.4; P.zeps = 1.0e-6;
    P.cc_gamma0 = 1.19; P.cc_A = 0.819e9; P.cc_B = 1.51e9; P.cc_C = 4.53; P.cc_D = 1.42;
    P.cc_rho0 = 1134.0;
    P.rx_C = 2.6e9; P.rx_Ta = 11350.0; P.rx_Q = 4.46e6; P.rx_cv2 = 1714.0;
    return P;
}

/* Shocked liquid left of x = nx/4, an air bubble of radius ny/4 centred at
 * (nx/2, ny/2) with a tanh interface, reaction progress 1 (0 in the strip). */
static void bubble_prim(const or_problem *P, double *prim, double rho2, double p_hi)
{
    long N = (long)P->nx * P->ny, i, j;
    int nc = P->reactive ? 7 : 6;
    for (j = 0; j < P->ny; ++j)
        for (i = 0; i < P->nx; ++i) {
            long k = j * P->nx + i;
            double x = i + 0.5 - 0.5 * P->nx, y = j + 0.5 - 0.5 * P->ny;
            double r = sqrt(x * x + y * y), R = 0.25 * (P->ny > 2 ? P->ny : 4);
            double w = 0.5 * (1.0 - tanh(r - R));
            prim[k] = P->zeps + (1.0 - 2.0 * P->zeps) * w;
            prim[N + k] = 1.2;
            prim[2 * N + k] = rho2;
            prim[3 * N + k] = i < P->nx / 4 ? 300.0 : 0.0;
            prim[4 * N + k] = 0.0;
            prim[5 * N + k] = i < P->nx / 4 ? p_hi : 1.0e5;
            if (nc == 7) prim[6 * N + k] = i < P->nx / 4 ? 0.0 : 1.0;
        }
}

static int run_case(or_problem P, int nsteps, double rho2, double p_hi)
{
    long N = (long)P.nx * P.ny;
    int nc = P.reactive ? 7 : 6, bad = 0;
    double *prim = malloc(sizeof(double) * nc * N), *U = malloc(sizeof(double) * nc * N);
    double *out = malloc(sizeof(double) * nc * N);
    double t = 0.0, last = 0.0;
    bubble_prim(&P, prim, rho2, p_hi);
    or_prim_to_cons(&P, prim, U);
    or_cons_to_prim(&P, U, out);
    if (or_run(&P, U, 0, nsteps, &t, 0.0, &last) < 0) bad = 1;
    /* sampled-cell step on every cell, both parities */
    {
        int64_t *cells = malloc(sizeof(int64_t) * N), s;
        double *so = malloc(sizeof(double) * nc * N);
        double dt = 0.0, tn = 0.0;
        for (s = 0; s < N; ++s) cells[s] = s;
        if (or_dt(&P, U, t, 0.0, &dt, &tn) == 0) {
            or_step_cells(&P, U, nsteps, dt, cells, N, so);
            or_step_cells(&P, U, nsteps + 1, dt, cells, N, so);
        }
        free(cells); free(so);
    }
    /* diagnostics */
    {
        double *pb = malloc(sizeof(double) * P.nx), *rb = malloc(sizeof(double) * P.nx);
        double *ub = malloc(sizeof(double) * P.nx), integ[7], f[64];
        or_y_averages(&P, U, pb, rb, ub);
        or_integrals(&P, U, integ);
        or_log_histogram(&P, U, 9, 4.0, 0.1, 64, 1.0, f);
        or_log_histogram(&P, U, 6, -1.0, 0.1, 64, 1.0, f);
        if (P.reactive) or_log_histogram(&P, U, 14, 2.0, 0.2, 40, 1.0, f);
        free(pb); free(rb); free(ub);
    }
    (void)or_max_speed(&P, U);
    free(prim); free(U); free(out);
    return bad;
}

int main(void)
{
    static const int sizes[][2] = {{1, 1}, {1, 5}, {5, 1}, {2, 3}, {3, 2}, {4, 4}, {37, 23}};
    int s, lim, bc, bad = 0;
    for (s = 0; s < 7; ++s)
        for (lim = 0; lim < 2; ++lim)
            for (bc = 0; bc < 2; ++bc) {
                or_problem P = base(sizes[s][0], sizes[s][1]);
                P.limiter = lim;
                P.bc_xlo = P.bc_xhi = P.bc_ylo = P.bc_yhi = bc;
                bad |= run_case(P, 3, 1000.0, 1.0e9);
            }
    {
        or_problem P = base(40, 24);                 /* Cochran-Chan liquid */
        P.eos2 = 1;
        bad |= run_case(P, 4, 1134.0, 7.81e9);
        P.reactive = 1;                              /* reactive liquid */
        bad |= run_case(P, 4, 1134.0, 7.81e9);
        P.bc_ylo = P.bc_yhi = 1;
        bad |= run_case(P, 3, 1134.0, 7.81e9);
    }
    {
        double e[17], wl[NV], wh[NV], w0[NV] = {1.0, 999.0, 10.0, -3.0, 1.0e6, 0.3, 0.0};
        double wm[NV] = {1.1, 990.0, 12.0, -2.0, 1.1e6, 0.32, 0.0}, out[8], q[NV], w[NV], r, c2;
        double wp[NV] = {0.9, 1001.0, 9.0, -4.0, 0.9e6, 0.28, 0.0}, ref[3];
        or_problem P = base(8, 1);
        int c;
        or_log_edges(2.0, 0.5, 16, e);
        or_unit_face_states(wm, w0, wp, 1.0 / 1000.0, 2.0e9, 0.01, 0, wl, wh);
        or_unit_hllc(&P, wl, wh, out);
        for (c = 0; c < NV; ++c) q[c] = w0[c];
        q[4] = 3.0e8;
        or_unit_cons_to_prim(&P, q, w, &r, &c2);
        (void)or_unit_limiter(1.0, 2.0, 0);
        (void)or_unit_limiter(-1.0, 2.0, 1);
        P.eos2 = 1;
        or_unit_cc_reference(&P, 1300.0, ref);
        (void)or_liquid_temperature(&P, 1300.0, 2.0e9, 1714.0);
    }
    printf("oracle sanitize driver: %s\n", bad ? "a run reported a bad state" : "ok");
    return 0;
}
