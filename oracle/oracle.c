/*
 * oracle.c -- plain FP64 CPU reference of the two-fluid diffuse-interface
 * finite-volume update (Eq. (1), Sec. 2.1; scheme of Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or constant table with the HIP library.
 *
 * What it computes (per time step n, see the arithmetic contract in the design
 * notes; every formula below is written in the order the contract fixes):
 *   state U = (z1 rho1, z2 rho2, rho u, rho v, rho E, z1)       Eq. (1), Sec. 2.1
 *   mixture closure rho = sum z_k rho_k, rho e = sum z_k rho_k e_k,
 *     p1 = p2, z1 + z2 = 1                                      Sec. 2.1
 *   each phase a stiffened gas, the Mie-Grueneisen form of Eq. (2) with
 *     constant reference terms (air: p_inf = 0, ideal gas)      Sec. 2.2
 *   dt = CFL / max_cells max((|u|+c)/dx, (|v|+c)/dy)
 *   dimensionally split sweeps, X then Y on even n, Y then X on odd n
 *   each sweep: MUSCL reconstruction of primitive variables with a van Leer
 *     or minmod slope limiter, Hancock half-step predictor, HLLC fluxes,
 *     conservative update of the first five components and a non-conservative
 *     update of z1 (its advection equation in Eq. (1))         Sec. 3
 *   pointwise stage: z1 <- clamp(z1, eps, 1 - eps)             Sec. 3 (Strang)
 *   liquid as a Cochran-Chan Mie-Grueneisen material, reference curves of
 *     Eqs. (3)-(4), constants of Table 1                        Sec. 2.2
 *   reactive liquid: reactant mass z2 rho2 lambda advected as a seventh
 *     component (last line of Eq. (1)); Arrhenius source of Eq. (6) with the
 *     constants of Table 3 at the liquid temperature of Eq. (5), applied as
 *     S(dt/2) H(dt) S(dt/2) with the temperature frozen over each S
 *   diagnostics: transverse averages (Sec. 4.2), domain integrals and the
 *     remaining reactant mass (Eq. (10)), mass-weighted log-binned PDFs of
 *     pressure, density and heat-release rate (Sec. 4.5)
 *
 * Built with -O2 -ffp-contract=off and no fast-math so that every operation is
 * a separately rounded IEEE double operation in the order written.
 *
 * Rows (x sweep) and columns (y sweep) are independent, so an OpenMP loop over
 * them changes no result; the CFL maximum is order independent.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 7   /* largest number of components (with the reaction progress) */

/* Problem description passed from Python (ctypes mirrors this layout). */
typedef struct {
    int32_t nx, ny;
    double dx, dy;
    int32_t bc_xlo, bc_xhi, bc_ylo, bc_yhi; /* 0 transmissive, 1 periodic */
    double gamma1, pinf1, gamma2, pinf2;    /* phase 1 = air, phase 2 = liquid */
    double cfl, zeps;
    int32_t limiter;                        /* 0 van Leer, 1 minmod */
    int32_t eos2;                           /* liquid: 0 stiffened gas, 1 Cochran-Chan */
    double cc_gamma0, cc_A, cc_B, cc_C, cc_D, cc_rho0;   /* Eqs. (2)-(4), Table 1 */
    int32_t reactive;                       /* 1: 7th plane z2 rho2 lambda + Arrhenius */
    int32_t pad2_;
    double rx_C, rx_Ta, rx_Q, rx_cv2;       /* Eq. (6), Table 3; c_v,2 of Table 1 */
} or_problem;

/* Mixture constants.  Every phase is written in the Mie-Grueneisen form of
 * Eq. (2), so that rho_k e_k = phi_k(rho_k) + p / Gamma_k with
 * phi_k = rho_k e_ref,k - p_ref,k / Gamma_k, and the pressure-equilibrium
 * closure of Sec. 2.1 becomes  rho e = p xi + eta,  xi = sum z_k / Gamma_k,
 * eta = sum z_k phi_k(rho_k).
 * Stiffened gas: Gamma = gamma - 1, phi = gamma p_inf / (gamma - 1) =: h,
 * constant.  Cochran-Chan (Eqs. (3)-(4)): phi depends on rho_2.          */
typedef struct {
    double g1, g2, h1, h2;
    int eos2;
    double A, B, C, D, rho0, iG, kA, kB;
    int nc;                                 /* components: 6, or 7 with z2 rho2 lambda */
} mixc;

static mixc mix_constants(const or_problem *P)
{
    mixc m;
    m.g1 = 1.0 / (P->gamma1 - 1.0);
    m.h1 = (P->gamma1 * P->pinf1) * m.g1;
    m.eos2 = P->eos2;
    m.nc = P->reactive ? 7 : 6;
    if (P->eos2 == 1) {
        m.iG = 1.0 / P->cc_gamma0;
        m.g2 = m.iG;
        m.h2 = 0.0;
        m.A = P->cc_A;
        m.B = P->cc_B;
        m.C = P->cc_C;
        m.D = P->cc_D;
        m.rho0 = P->cc_rho0;
        m.kA = -P->cc_A / (P->cc_rho0 * (1.0 - P->cc_C));
        m.kB = P->cc_B / (P->cc_rho0 * (1.0 - P->cc_D));
    } else {
        m.g2 = 1.0 / (P->gamma2 - 1.0);
        m.h2 = (P->gamma2 * P->pinf2) * m.g2;
        m.iG = m.A = m.B = m.C = m.D = m.rho0 = m.kA = m.kB = 0.0;
    }
    return m;
}

/* Cochran-Chan reference curves at liquid density rho (Eqs. (3)-(4)):
 * p_ref, e_ref and rho dp_ref/drho, with v = rho0 / rho.                    */
static void cc_reference(const mixc *m, double rho, double *pref, double *eref, double *rdpref)
{
    double v = m->rho0 / rho;
    double vc = pow(v, -m->C), vd = pow(v, -m->D);
    *pref = m->A * vc - m->B * vd;
    *eref = m->kA * (v * vc - 1.0) + m->kB * (v * vd - 1.0);
    *rdpref = (m->A * m->C) * vc - (m->B * m->D) * vd;
}

/* Liquid contributions z2 phi2(rho2) to eta and z2 rho2 phi2'(rho2) to psi,
 * the term the density dependence of phi adds to the frozen sound speed:
 * rho c^2 = (p (1 + xi) + eta - psi) / xi.   rho2 = a2 / z2.              */
static void liquid_terms(const mixc *m, double a2, double z2, double *eta2, double *psi2)
{
    double rho2 = a2 / z2, pref, eref, rdpref, phi, rphi;
    cc_reference(m, rho2, &pref, &eref, &rdpref);
    phi = rho2 * eref - pref * m->iG;
    rphi = (rho2 * eref + pref) - rdpref * m->iG;
    *eta2 = z2 * phi;
    *psi2 = z2 * rphi;
}

/* ------------------------------------------------------------------------ */
/* Closure (Sec. 2.1 / Sec. 2.2).  Line-frame conserved vector:
 *   q = (a1, a2, mn, mt, E, z): partial densities, momentum normal and
 *   tangential to the sweep, total energy, air volume fraction.
 * Primitive vector w = (a1, a2, un, ut, p, z).  Also returns 1/rho and rho c^2
 * (frozen-z isentropic sound speed of the z-advection model).                */
static void cons_to_prim(const mixc *m, const double q[NV], double w[NV],
                         double *r_out, double *rc2_out)
{
    double rho = q[0] + q[1];
    double r = 1.0 / rho;
    double un = q[2] * r;
    double ut = q[3] * r;
    double ke = 0.5 * (q[2] * un + q[3] * ut);
    double rhoe = q[4] - ke;
    double z = q[5];
    double z2 = 1.0 - z;
    double xi = z * m->g1 + z2 * m->g2;
    double eta, ixi, p, rc2;
    if (m->eos2 == 1) {
        double eta2, psi2;
        liquid_terms(m, q[1], z2, &eta2, &psi2);
        eta = z * m->h1 + eta2;
        ixi = 1.0 / xi;
        p = (rhoe - eta) * ixi;
        rc2 = ((p * (1.0 + xi) + eta) - psi2) * ixi;
    } else {
        eta = z * m->h1 + z2 * m->h2;
        ixi = 1.0 / xi;
        p = (rhoe - eta) * ixi;
        rc2 = (p * (1.0 + xi) + eta) * ixi;
    }
    w[0] = q[0]; w[1] = q[1]; w[2] = un; w[3] = ut; w[4] = p; w[5] = z;
    if (m->nc == 7) w[6] = q[6] / q[1];     /* lambda: mass fraction of unreacted liquid */
    *r_out = r;
    *rc2_out = rc2;
}

/* ------------------------------------------------------------------------ */
/* Slope limiters (Sec. 3: "van Leer" limiter; minmod as the alternative
 * reading).  a = backward difference, b = forward difference.               */
static double limit_slope(double a, double b, int limiter)
{
    double ab = a * b;
    if (!(ab > 0.0)) return 0.0;
    if (limiter == 1) {                  /* minmod */
        return (a > 0.0) ? fmin(a, b) : fmax(a, b);
    }
    return (ab + ab) / (a + b);          /* van Leer: harmonic mean 2ab/(a+b) */
}

/* MUSCL reconstruction + Hancock half step (Sec. 3, "MUSCL-Hancock") in
 * primitive variables.  Inputs: primitives of cells i-1, i, i+1, and 1/rho,
 * rho c^2 of cell i; hl = dt/(2h).  Outputs the evolved boundary values at the
 * low (wl) and high (wh) faces of cell i.
 * Quasi-linear primitive system along the sweep:
 *   d a_k/dt + un d a_k/dx + a_k d un/dx = 0
 *   d un/dt  + un d un/dx + (1/rho) d p/dx = 0
 *   d ut/dt  + un d ut/dx = 0
 *   d p/dt   + un d p/dx + rho c^2 d un/dx = 0
 *   d z/dt   + un d z/dx = 0                                                */
static void face_states(const double wm[NV], const double w0[NV], const double wp[NV],
                        double r, double rc2, double hl, int limiter, int nc,
                        double wl[NV], double wh[NV])
{
    double d[NV], s[NV];
    int c;
    for (c = 0; c < nc; ++c)
        d[c] = limit_slope(w0[c] - wm[c], wp[c] - w0[c], limiter);
    {
        double un = w0[2];
        s[0] = hl * (un * d[0] + w0[0] * d[2]);
        s[1] = hl * (un * d[1] + w0[1] * d[2]);
        s[2] = hl * (un * d[2] + r * d[4]);
        s[3] = hl * (un * d[3]);
        s[4] = hl * (un * d[4] + rc2 * d[2]);
        s[5] = hl * (un * d[5]);
        if (nc == 7) s[6] = hl * (un * d[6]);   /* lambda is advected */
    }
    for (c = 0; c < nc; ++c) {
        wl[c] = (w0[c] - 0.5 * d[c]) - s[c];
        wh[c] = (w0[c] + 0.5 * d[c]) - s[c];
    }
}

/* Per-side quantities of a face state for the HLLC solver. */
typedef struct {
    double rho, un, ut, p, z, c, E;
    double U[6];   /* a1, a2, rho un, rho ut, E (, a2 lambda) */
    double F[6];   /* physical flux along the sweep           */
} side_t;

static void side_eval(const mixc *m, const double w[NV], side_t *s)
{
    double rho = w[0] + w[1];
    double un = w[2], ut = w[3], p = w[4], z = w[5];
    double z2 = 1.0 - z;
    double xi = z * m->g1 + z2 * m->g2;
    double eta, c;
    if (m->eos2 == 1) {
        double eta2, psi2;
        liquid_terms(m, w[1], z2, &eta2, &psi2);
        eta = z * m->h1 + eta2;
        c = sqrt(((p * (1.0 + xi) + eta) - psi2) / (xi * rho));
    } else {
        eta = z * m->h1 + z2 * m->h2;
        c = sqrt((p * (1.0 + xi) + eta) / (xi * rho));
    }
    double E = (p * xi + eta) + 0.5 * (rho * (un * un + ut * ut));
    double mn = rho * un;
    s->rho = rho; s->un = un; s->ut = ut; s->p = p; s->z = z; s->c = c; s->E = E;
    s->U[0] = w[0]; s->U[1] = w[1]; s->U[2] = mn; s->U[3] = rho * ut; s->U[4] = E;
    s->F[0] = w[0] * un;
    s->F[1] = w[1] * un;
    s->F[2] = mn * un + p;
    s->F[3] = mn * ut;
    s->F[4] = (E + p) * un;
    if (m->nc == 7) {
        s->U[5] = w[1] * w[6];
        s->F[5] = s->U[5] * un;
    }
}

/* HLLC star-region flux of side K (K = L with S = S_L, or R with S = S_R),
 * together with the HLLC-consistent interface velocity used by the
 * non-conservative z1 term.                                                 */
static void star_flux(const side_t *k, double S, double Ss, int nc, double out[8])
{
    double d = S - k->un;
    double chi = d / (S - Ss);
    double us[6];
    int c;
    us[0] = chi * k->U[0];
    us[1] = chi * k->U[1];
    us[2] = chi * (k->rho * Ss);
    us[3] = chi * (k->rho * k->ut);
    us[4] = chi * (k->E + (Ss - k->un) * (k->rho * Ss + k->p / d));
    for (c = 0; c < 5; ++c) out[c] = k->F[c] + S * (us[c] - k->U[c]);
    out[5] = k->un + S * (chi - 1.0);   /* interface velocity u_f */
    out[6] = k->z;                      /* upwind face value of z1 */
    if (nc == 7) {
        us[5] = chi * k->U[5];
        out[7] = k->F[5] + S * (us[5] - k->U[5]);
    }
}

/* HLLC approximate Riemann solver (Sec. 3) with Davis wave-speed bounds.
 * out = (5 flux components, u_f, z_f).                                      */
static void hllc(const mixc *m, const double wL[NV], const double wR[NV], double out[8])
{
    side_t L, R;
    double SL, SR, dL, dR, Ss;
    int c;
    side_eval(m, wL, &L);
    side_eval(m, wR, &R);
    SL = fmin(L.un - L.c, R.un - R.c);
    SR = fmax(L.un + L.c, R.un + R.c);
    dL = SL - L.un;
    dR = SR - R.un;
    Ss = ((R.p - L.p) + (L.U[2] * dL - R.U[2] * dR)) / (L.rho * dL - R.rho * dR);
    if (SL >= 0.0) {
        for (c = 0; c < 5; ++c) out[c] = L.F[c];
        out[5] = L.un; out[6] = L.z;
        if (m->nc == 7) out[7] = L.F[5];
    } else if (SR <= 0.0) {
        for (c = 0; c < 5; ++c) out[c] = R.F[c];
        out[5] = R.un; out[6] = R.z;
        if (m->nc == 7) out[7] = R.F[5];
    } else if (Ss > 0.0) {
        star_flux(&L, SL, Ss, m->nc, out);
    } else if (Ss < 0.0) {
        star_flux(&R, SR, Ss, m->nc, out);
    } else {
        double a[8], b[8];
        int no = m->nc == 7 ? 8 : 7;
        star_flux(&L, SL, Ss, m->nc, a);
        star_flux(&R, SR, Ss, m->nc, b);
        for (c = 0; c < no; ++c) out[c] = 0.5 * (a[c] + b[c]);
    }
}

/* Conservative update of the first five components and the non-conservative
 * z1 update  z -= lam * [ (z_f - z)_{+} u_{f,+} - (z_f - z)_{-} u_{f,-} ],
 * i.e. the discrete form of  dz/dt + d(uz)/dx - z du/dx = 0.               */
static void update_cell(const double q[NV], const double flo[8], const double fhi[8],
                        double lam, int nc, double qo[NV])
{
    int c;
    double z = q[5];
    for (c = 0; c < 5; ++c) qo[c] = q[c] - lam * (fhi[c] - flo[c]);
    qo[5] = z - lam * ((fhi[6] - z) * fhi[5] - (flo[6] - z) * flo[5]);
    if (nc == 7) qo[6] = q[6] - lam * (fhi[7] - flo[7]);
}

/* ------------------------------------------------------------------------ */
/* Boundary ghost-cell index map: transmissive = copy of the edge cell,
 * periodic = wrap (Sec. 2.4, Fig. 1).                                      */
static long map_index(long i, long n, int bc_lo, int bc_hi)
{
    if (i < 0) {
        if (bc_lo == 1) return ((i % n) + n) % n;
        return 0;
    }
    if (i >= n) {
        if (bc_hi == 1) return i % n;
        return n - 1;
    }
    return i;
}

/* One sweep along a line of n cells.  qin/qout: NV arrays of stride 1 in the
 * line frame.  work must hold (n + 4) * (2 NV + 2) + (n + 1) * 7 doubles.   */
static void sweep_line(const mixc *m, long n, double *const qin[NV], double *const qout[NV],
                       int bc_lo, int bc_hi, double lam, int limiter, double *work)
{
    long i, k;
    int c;
    double hl = 0.5 * lam;
    long nw = n + 4;
    double *W = work;                 /* nw * NV, cell i at (i + 2)      */
    double *rr = W + nw * NV;         /* nw                               */
    double *rc = rr + nw;             /* nw                               */
    double *WL = rc + nw;             /* nw * NV (low-face state)          */
    double *WH = WL + nw * NV;        /* nw * NV (high-face state)         */
    double *FF = WH + nw * NV;        /* (n + 1) * 8, face f between f-1, f */
    int nc = m->nc;

    for (i = -2; i < n + 2; ++i) {
        double q[NV];
        long src = map_index(i, n, bc_lo, bc_hi);
        for (c = 0; c < nc; ++c) q[c] = qin[c][src];
        cons_to_prim(m, q, &W[(i + 2) * NV], &rr[i + 2], &rc[i + 2]);
    }
    for (i = -1; i < n + 1; ++i) {
        k = i + 2;
        face_states(&W[(k - 1) * NV], &W[k * NV], &W[(k + 1) * NV], rr[k], rc[k], hl,
                    limiter, nc, &WL[k * NV], &WH[k * NV]);
    }
    for (i = 0; i <= n; ++i) {
        /* face between cell i-1 (its high face) and cell i (its low face) */
        hllc(m, &WH[(i + 1) * NV], &WL[(i + 2) * NV], &FF[i * 8]);
    }
    for (i = 0; i < n; ++i) {
        double q[NV], qo[NV];
        for (c = 0; c < nc; ++c) q[c] = qin[c][i];
        update_cell(q, &FF[i * 8], &FF[(i + 1) * 8], lam, nc, qo);
        for (c = 0; c < nc; ++c) qout[c][i] = qo[c];
    }
}

static size_t line_work_doubles(long n)
{
    return (size_t)(n + 4) * (2 * NV + 2) + (size_t)(n + 4) * NV + (size_t)(n + 1) * 8;
}

/* X sweep of the whole grid: rows are lines, normal momentum = rho u.      */
static void sweep_x(const or_problem *P, const mixc *m, const double *U, double *V, double lam)
{
    long nx = P->nx, ny = P->ny, N = nx * ny;
    long j;
#pragma omp parallel
    {
        double *work = (double *)malloc(line_work_doubles(nx) * sizeof(double));
        double *lin = (double *)malloc((size_t)nx * NV * sizeof(double));
        double *lout = (double *)malloc((size_t)nx * NV * sizeof(double));
#pragma omp for schedule(static)
        for (j = 0; j < ny; ++j) {
            double *qi[NV], *qo[NV];
            int c;
            long i;
            /* line frame: (a1, a2, rho u, rho v, E, z) -- same order as U */
            for (c = 0; c < m->nc; ++c) {
                qi[c] = lin + c * nx;
                qo[c] = lout + c * nx;
                for (i = 0; i < nx; ++i) qi[c][i] = U[c * N + j * nx + i];
            }
            sweep_line(m, nx, qi, qo, P->bc_xlo, P->bc_xhi, lam, P->limiter, work);
            for (c = 0; c < m->nc; ++c)
                for (i = 0; i < nx; ++i) V[c * N + j * nx + i] = qo[c][i];
        }
        free(work); free(lin); free(lout);
    }
}

/* Y sweep: columns are lines, normal momentum = rho v, tangential = rho u.  */
static const int ymap[NV] = {0, 1, 3, 2, 4, 5, 6};

static void sweep_y(const or_problem *P, const mixc *m, const double *U, double *V, double lam)
{
    long nx = P->nx, ny = P->ny, N = nx * ny;
    long i;
#pragma omp parallel
    {
        double *work = (double *)malloc(line_work_doubles(ny) * sizeof(double));
        double *lin = (double *)malloc((size_t)ny * NV * sizeof(double));
        double *lout = (double *)malloc((size_t)ny * NV * sizeof(double));
#pragma omp for schedule(static)
        for (i = 0; i < nx; ++i) {
            double *qi[NV], *qo[NV];
            int c;
            long j;
            for (c = 0; c < m->nc; ++c) {
                qi[c] = lin + c * ny;
                qo[c] = lout + c * ny;
                for (j = 0; j < ny; ++j) qi[c][j] = U[ymap[c] * N + j * nx + i];
            }
            sweep_line(m, ny, qi, qo, P->bc_ylo, P->bc_yhi, lam, P->limiter, work);
            for (c = 0; c < m->nc; ++c)
                for (j = 0; j < ny; ++j) V[ymap[c] * N + j * nx + i] = qo[c][j];
        }
        free(work); free(lin); free(lout);
    }
}

/* Pointwise stage of the Strang split (Sec. 3): with no reaction the source
 * step reduces to keeping z1 inside [eps, 1 - eps].                         */
static void clamp_z(const or_problem *P, double *U)
{
    long N = (long)P->nx * P->ny, k;
    double lo = P->zeps, hi = 1.0 - P->zeps;
    double *z = U + 5 * N;
    for (k = 0; k < N; ++k) z[k] = fmin(fmax(z[k], lo), hi);
}

/* ======================================================================== */
/* Exported entry points (called from Python through ctypes).               */

/* Primitive (z1, rho1, rho2, u, v, p) planes -> conserved planes.          */
void or_prim_to_cons(const or_problem *P, const double *prim, double *U)
{
    mixc m = mix_constants(P);
    long N = (long)P->nx * P->ny, k;
    for (k = 0; k < N; ++k) {
        double z = prim[k], r1 = prim[N + k], r2 = prim[2 * N + k];
        double u = prim[3 * N + k], v = prim[4 * N + k], p = prim[5 * N + k];
        double z2 = 1.0 - z;
        double a1 = z * r1, a2 = z2 * r2;
        double rho = a1 + a2;
        double xi = z * m.g1 + z2 * m.g2;
        double eta;
        if (m.eos2 == 1) {
            double eta2, psi2;
            liquid_terms(&m, a2, z2, &eta2, &psi2);
            eta = z * m.h1 + eta2;
        } else {
            eta = z * m.h1 + z2 * m.h2;
        }
        U[k] = a1;
        U[N + k] = a2;
        U[2 * N + k] = rho * u;
        U[3 * N + k] = rho * v;
        U[4 * N + k] = (p * xi + eta) + 0.5 * (rho * (u * u + v * v));
        U[5 * N + k] = z;
        if (m.nc == 7) U[6 * N + k] = a2 * prim[6 * N + k];
    }
}

/* Conserved -> (rho, u, v, p, c, z1) planes.                                */
void or_cons_to_prim(const or_problem *P, const double *U, double *out)
{
    mixc m = mix_constants(P);
    long N = (long)P->nx * P->ny, k;
    for (k = 0; k < N; ++k) {
        double q[NV], w[NV], r, rc2;
        int c;
        for (c = 0; c < m.nc; ++c) q[c] = U[c * N + k];
        cons_to_prim(&m, q, w, &r, &rc2);
        if (m.nc == 7) out[6 * N + k] = w[6];
        out[k] = w[0] + w[1];
        out[N + k] = w[2];
        out[2 * N + k] = w[3];
        out[3 * N + k] = w[4];
        out[4 * N + k] = sqrt(rc2 * r);
        out[5 * N + k] = w[5];
    }
}

/* Largest signal speed over grid spacing, max((|u|+c)/dx, (|v|+c)/dy).
 * Returns NaN if any cell is non-finite or has rho <= 0 or rho c^2 <= 0.    */
double or_max_speed(const or_problem *P, const double *U)
{
    mixc m = mix_constants(P);
    long N = (long)P->nx * P->ny, k;
    double idx = 1.0 / P->dx, idy = 1.0 / P->dy;
    double smax = 0.0;
    int bad = 0;
#pragma omp parallel for reduction(max : smax) reduction(| : bad) schedule(static)
    for (k = 0; k < N; ++k) {
        double q[NV], w[NV], r, rc2, c, s;
        int cc;
        for (cc = 0; cc < m.nc; ++cc) q[cc] = U[cc * N + k];
        cons_to_prim(&m, q, w, &r, &rc2);
        c = sqrt(rc2 * r);
        s = fmax((fabs(w[2]) + c) * idx, (fabs(w[3]) + c) * idy);
        if (!(r > 0.0) || !(rc2 > 0.0) || !(s <= 1.0e300)) bad = 1;
        else if (s > smax) smax = s;
    }
    return bad ? NAN : smax;
}

/* Pointwise source stage of the Strang split (Sec. 3) over a time h, for the
 * reactive liquid: single-step Arrhenius kinetics (Eq. (6), Table 3),
 * K = -lambda C exp(-Ta / T2), with the liquid temperature of Eq. (5)
 * (T_ref,2 = 0, constant c_v,2 and Gamma_0,2) frozen over the stage, so that
 * lambda <- lambda exp(-C exp(-Ta / T2) h) exactly; the liquid mass that
 * reacts releases Q per unit mass into rho E (the source -z2 rho2 K Q of
 * Eq. (1)).  Cells with no reactant or a non-positive temperature are left
 * alone.                                                                    */
static void react_cell(const or_problem *P, const mixc *m, double q[NV], double h)
{
    double w[NV], r, rc2, rho2, pref, eref, rdpref, T, k, lam_new;
    if (!(q[6] > 0.0)) return;
    cons_to_prim(m, q, w, &r, &rc2);
    rho2 = q[1] / (1.0 - q[5]);
    cc_reference(m, rho2, &pref, &eref, &rdpref);
    T = (w[4] - pref) / (rho2 * P->cc_gamma0 * P->rx_cv2);
    if (!(T > 0.0)) return;
    k = P->rx_C * exp(-P->rx_Ta / T);
    lam_new = w[6] * exp(-k * h);
    q[4] = q[4] + P->rx_Q * (q[6] - q[1] * lam_new);
    q[6] = q[1] * lam_new;
}

static void react_all(const or_problem *P, const mixc *m, double *U, double h)
{
    long N = (long)P->nx * P->ny, k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < N; ++k) {
        double q[NV];
        int c;
        for (c = 0; c < NV; ++c) q[c] = U[c * N + k];
        react_cell(P, m, q, h);
        U[4 * N + k] = q[4];
        U[6 * N + k] = q[6];
    }
}

/* One full time step with time-step size dt: S(dt/2), split sweeps in the
 * order set by the parity of the step index, S(dt/2), where the pointwise
 * stage S is the z1 clamp (then the reaction of a reactive liquid).
 * tmp: as many planes as U.                                                 */
void or_step(const or_problem *P, double *U, double *tmp, int64_t step, double dt)
{
    mixc m = mix_constants(P);
    double lamx = dt / P->dx, lamy = dt / P->dy;
    if (m.nc == 7) react_all(P, &m, U, 0.5 * dt);
    if ((step & 1) == 0) {
        sweep_x(P, &m, U, tmp, lamx);
        sweep_y(P, &m, tmp, U, lamy);
    } else {
        sweep_y(P, &m, U, tmp, lamy);
        sweep_x(P, &m, tmp, U, lamx);
    }
    clamp_z(P, U);
    if (m.nc == 7) react_all(P, &m, U, 0.5 * dt);
}

/* Time-step size from the CFL condition, clipped so that the run ends exactly
 * at t_end (t_end <= 0 means no end time).  Returns 0 on success, -1 when the
 * state is non-finite or has no positive signal speed.                     */
int or_dt(const or_problem *P, const double *U, double t, double t_end, double *dt_out,
          double *t_new)
{
    double smax = or_max_speed(P, U);
    double dt;
    if (!(smax > 0.0) || !(smax <= 1.0e300)) return -1;
    dt = P->cfl / smax;
    if (t_end > 0.0 && t + dt >= t_end) {
        dt = t_end - t;
        *t_new = t_end;
    } else {
        *t_new = t + dt;
    }
    *dt_out = dt;
    return 0;
}

/* Advance up to nsteps steps (dt from the CFL condition; stop at t_end when
 * t_end > 0).  Returns the number of steps taken, or -1 on a bad state.
 * On return *t holds the new time, *last_dt the last step size.            */
int64_t or_run(const or_problem *P, double *U, int64_t step0, int64_t nsteps, double *t,
               double t_end, double *last_dt)
{
    long N = (long)P->nx * P->ny;
    double *tmp = (double *)malloc((size_t)N * (P->reactive ? 7 : 6) * sizeof(double));
    int64_t n;
    for (n = 0; n < nsteps; ++n) {
        double dt, tn;
        if (t_end > 0.0 && *t >= t_end) break;
        if (or_dt(P, U, *t, t_end, &dt, &tn) != 0) { free(tmp); return -1; }
        or_step(P, U, tmp, step0 + n, dt);
        *t = tn;
        *last_dt = dt;
    }
    free(tmp);
    return n;
}

/* Updated state after one step at a list of cells only (for checking very
 * large grids cell by cell).  U: state before the step, all planes.
 * cells[k] = j * nx + i.  out: nc * ncells (component-major).               */
static void sweep_point(const mixc *m, double win[NV][5], double lam, int limiter,
                        double qo[NV])
{
    /* win[c][k]: cells -2..2 of a line-frame window centred on the target */
    double W[5][NV], r[5], rc2[5], WL[3][NV], WH[3][NV], flo[8], fhi[8], q[NV];
    int k, c;
    double hl = 0.5 * lam;
    for (k = 0; k < 5; ++k) {
        double qq[NV];
        for (c = 0; c < m->nc; ++c) qq[c] = win[c][k];
        cons_to_prim(m, qq, W[k], &r[k], &rc2[k]);
    }
    for (k = 1; k <= 3; ++k)
        face_states(W[k - 1], W[k], W[k + 1], r[k], rc2[k], hl, limiter, m->nc, WL[k - 1],
                    WH[k - 1]);
    hllc(m, WH[0], WL[1], flo);
    hllc(m, WH[1], WL[2], fhi);
    for (c = 0; c < m->nc; ++c) q[c] = win[c][2];
    update_cell(q, flo, fhi, lam, m->nc, qo);
}

static void xpoint(const or_problem *P, const mixc *m, const double *U, long i, long j,
                   double lam, double qo[NV])
{
    long nx = P->nx, N = (long)P->nx * P->ny;
    double win[NV][5];
    int k, c;
    for (k = 0; k < 5; ++k) {
        long ii = map_index(i + k - 2, nx, P->bc_xlo, P->bc_xhi);
        for (c = 0; c < m->nc; ++c) win[c][k] = U[c * N + j * nx + ii];
    }
    sweep_point(m, win, lam, P->limiter, qo);
}

static void ypoint(const or_problem *P, const mixc *m, const double *U, long i, long j,
                   double lam, double qo[NV])
{
    long nx = P->nx, ny = P->ny, N = (long)P->nx * P->ny;
    double win[NV][5], t[NV];
    int k, c;
    for (k = 0; k < 5; ++k) {
        long jj = map_index(j + k - 2, ny, P->bc_ylo, P->bc_yhi);
        for (c = 0; c < m->nc; ++c) win[c][k] = U[ymap[c] * N + jj * nx + i];
    }
    sweep_point(m, win, lam, P->limiter, t);
    for (c = 0; c < m->nc; ++c) qo[ymap[c]] = t[c];
}

void or_step_cells(const or_problem *P, const double *U, int64_t step, double dt,
                   const int64_t *cells, int64_t ncells, double *out)
{
    mixc m = mix_constants(P);
    long nx = P->nx, ny = P->ny, N = (long)P->nx * P->ny;
    double lamx = dt / P->dx, lamy = dt / P->dy;
    double *Ur = NULL;
    int64_t s;
    if (m.nc == 7) {   /* first half of the source stage on the whole state */
        Ur = (double *)malloc((size_t)N * 7 * sizeof(double));
        memcpy(Ur, U, (size_t)N * 7 * sizeof(double));
        react_all(P, &m, Ur, 0.5 * dt);
        U = Ur;
    }
    for (s = 0; s < ncells; ++s) {
        long i = (long)(cells[s] % nx), j = (long)(cells[s] / nx);
        double mid[NV][5];   /* intermediate state on the 5-cell cross line */
        double qo[NV], win_t[NV];
        int k, c;
        if ((step & 1) == 0) {
            /* X first: intermediate values along column i, rows j-2..j+2 */
            for (k = 0; k < 5; ++k) {
                long jj = map_index(j + k - 2, ny, P->bc_ylo, P->bc_yhi);
                xpoint(P, &m, U, i, jj, lamx, win_t);
                for (c = 0; c < m.nc; ++c) mid[ymap[c]][k] = win_t[c];
            }
            sweep_point(&m, mid, lamy, P->limiter, win_t);
            for (c = 0; c < m.nc; ++c) qo[ymap[c]] = win_t[c];
        } else {
            /* Y first: intermediate values along row j, columns i-2..i+2 */
            for (k = 0; k < 5; ++k) {
                long ii = map_index(i + k - 2, nx, P->bc_xlo, P->bc_xhi);
                ypoint(P, &m, U, ii, j, lamy, win_t);
                for (c = 0; c < m.nc; ++c) mid[c][k] = win_t[c];
            }
            sweep_point(&m, mid, lamx, P->limiter, qo);
        }
        {
            double lo = P->zeps, hi = 1.0 - P->zeps;
            qo[5] = fmin(fmax(qo[5], lo), hi);
        }
        if (m.nc == 7) react_cell(P, &m, qo, 0.5 * dt);
        for (c = 0; c < m.nc; ++c) out[c * ncells + s] = qo[c];
    }
    free(Ur);
}

/* Temperature of the liquid from the linearisation about its reference curve
 * (Eq. (5) with T_ref,2 = 0, constant c_v,2 and Gamma_0,2):
 *   T2 = (p - p_ref,2(rho2)) / (rho2 Gamma_0,2 c_v,2).                      */
double or_liquid_temperature(const or_problem *P, double rho2, double p, double cv2)
{
    mixc m = mix_constants(P);
    double pref, eref, rdpref;
    cc_reference(&m, rho2, &pref, &eref, &rdpref);
    return (p - pref) / (rho2 * P->cc_gamma0 * cv2);
}

void or_unit_cc_reference(const or_problem *P, double rho, double out[3])
{
    mixc m = mix_constants(P);
    cc_reference(&m, rho, &out[0], &out[1], &out[2]);
}

/* ---- building blocks exported for unit pins ----------------------------- */
void or_unit_cons_to_prim(const or_problem *P, const double q[NV], double w[NV], double *r,
                          double *rc2)
{
    mixc m = mix_constants(P);
    cons_to_prim(&m, q, w, r, rc2);
}

double or_unit_limiter(double a, double b, int32_t limiter) { return limit_slope(a, b, limiter); }

void or_unit_face_states(const double wm[NV], const double w0[NV], const double wp[NV],
                         double r, double rc2, double hl, int32_t limiter, double wl[NV],
                         double wh[NV])
{
    face_states(wm, w0, wp, r, rc2, hl, limiter, 6, wl, wh);
}

void or_unit_hllc(const or_problem *P, const double wL[NV], const double wR[NV], double out[8])
{
    mixc m = mix_constants(P);
    hllc(&m, wL, wR, out);
}

void or_unit_sweep_line(const or_problem *P, int64_t n, const double *qin, double *qout,
                        double lam)
{
    /* qin/qout: NV planes of n values, line frame; x-direction boundaries */
    mixc m = mix_constants(P);
    double *qi[NV], *qo[NV];
    double *work = (double *)malloc(line_work_doubles(n) * sizeof(double));
    int c;
    for (c = 0; c < m.nc; ++c) {
        qi[c] = (double *)qin + c * n;
        qo[c] = qout + c * n;
    }
    sweep_line(&m, n, qi, qo, P->bc_xlo, P->bc_xhi, lam, P->limiter, work);
    free(work);
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (n < 1: all processors).  The
 * results do not depend on it. */
void or_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n >= 1 ? (int)n : omp_get_num_procs());
#else
    (void)n;
#endif
}

/* ======================================================================== */
/* Diagnostics (Sec. 4.2 transverse averages; Sec. 4.5 mass-weighted PDFs).  */

/* Pressure, density and x-momentum of a cell through the closure. */
static void cell_prim(const mixc *m, const double *U, long N, long k, double *p, double *rho,
                      double *mu)
{
    double q[NV], w[NV], r, rc2;
    int c;
    for (c = 0; c < m->nc; ++c) q[c] = U[c * N + k];
    cons_to_prim(m, q, w, &r, &rc2);
    *p = w[4];
    *rho = q[0] + q[1];
    *mu = q[2];
}

/* Transverse averages over y of each column i (sums taken in increasing j):
 *   pbar(x) = (1/ny) sum_j p,  rhobar(x) = (1/ny) sum_j rho,
 *   ubar(x) = sum_j rho u / sum_j rho  (density-weighted velocity).          */
void or_y_averages(const or_problem *P, const double *U, double *pbar, double *rhobar,
                   double *ubar)
{
    mixc m = mix_constants(P);
    long nx = P->nx, ny = P->ny, N = nx * ny, i, j;
    for (i = 0; i < nx; ++i) {
        double sp = 0.0, sr = 0.0, sm = 0.0;
        for (j = 0; j < ny; ++j) {
            double p, rho, mu;
            cell_prim(&m, U, N, j * nx + i, &p, &rho, &mu);
            sp = sp + p;
            sr = sr + rho;
            sm = sm + mu;
        }
        pbar[i] = sp / (double)ny;
        rhobar[i] = sr / (double)ny;
        ubar[i] = sm / sr;
    }
}

/* Domain integrals (cell area dx*dy): z1 rho1, z2 rho2, rho u, rho v, rho E,
 * air volume z1 and, for a reactive liquid, the remaining reactant mass
 * M_2,r of Eq. (10).  Each is (sum over i of (sum over j of q)) * area, both
 * sums in increasing index order.                                           */
void or_integrals(const or_problem *P, const double *U, double out[7])
{
    long nx = P->nx, ny = P->ny, N = nx * ny, i, j;
    int c, nc = P->reactive ? 7 : 6;
    double area = P->dx * P->dy;
    for (c = 0; c < nc; ++c) {
        double tot = 0.0;
        for (i = 0; i < nx; ++i) {
            double s = 0.0;
            for (j = 0; j < ny; ++j) s = s + U[c * N + j * nx + i];
            tot = tot + s;
        }
        out[c] = tot * area;
    }
}

/* Bin edges 10^(lo + k dn), k = 0..nbins. */
void or_log_edges(double lo, double dn, int32_t nbins, double *edges)
{
    int32_t k;
    for (k = 0; k <= nbins; ++k) edges[k] = pow(10.0, lo + (double)k * dn);
}

/* Volumetric rate of energy release q = -z2 rho2 K Q of the reactive liquid
 * (Sec. 4.5), in GW/m^3, with the temperature of Eq. (5).                   */
static double heat_release(const or_problem *P, const mixc *m, const double q[NV])
{
    double w[NV], r, rc2, rho2, pref, eref, rdpref, T;
    if (!(q[6] > 0.0)) return 0.0;
    cons_to_prim(m, q, w, &r, &rc2);
    rho2 = q[1] / (1.0 - q[5]);
    cc_reference(m, rho2, &pref, &eref, &rdpref);
    T = (w[4] - pref) / (rho2 * P->cc_gamma0 * P->rx_cv2);
    if (!(T > 0.0)) return 0.0;
    return ((q[6] * P->rx_C) * exp(-P->rx_Ta / T) * P->rx_Q) * 1.0e-9;
}

/* Mass-weighted histogram of pressure (field 9), density (field 6) or the
 * heat-release rate (field 14, GW/m^3) over the log-spaced bins:
 * m_k = sum of z2 rho2 dx dy over cells with edges[k] <= v < edges[k+1];
 * f_k = m_k / (m_ref dn)  (Sec. 4.5).                                        */
void or_log_histogram(const or_problem *P, const double *U, int32_t field, double lo, double dn,
                      int32_t nbins, double m_ref, double *f)
{
    mixc m = mix_constants(P);
    long N = (long)P->nx * P->ny, k;
    double area = P->dx * P->dy;
    double *edges = (double *)malloc((size_t)(nbins + 1) * sizeof(double));
    int32_t b;
    or_log_edges(lo, dn, nbins, edges);
    for (b = 0; b < nbins; ++b) f[b] = 0.0;
    for (k = 0; k < N; ++k) {
        double p, rho, mu, v;
        int32_t a, z;
        if (field == 14) {
            double q[NV];
            int c;
            for (c = 0; c < m.nc; ++c) q[c] = U[c * N + k];
            v = heat_release(P, &m, q);
        } else {
            cell_prim(&m, U, N, k, &p, &rho, &mu);
            v = (field == 6) ? rho : p;
        }
        if (!(v >= edges[0]) || !(v < edges[nbins])) continue;
        /* largest a with edges[a] <= v */
        a = 0;
        z = nbins;
        while (z - a > 1) {
            int32_t h = (a + z) / 2;
            if (edges[h] <= v) a = h;
            else z = h;
        }
        f[a] += U[N + k] * area;
    }
    for (b = 0; b < nbins; ++b) f[b] = f[b] / (m_ref * dn);
    free(edges);
}
