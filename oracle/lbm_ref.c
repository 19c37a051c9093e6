/*
 * lbm_ref.c -- CPU oracle for the coupled D2Q9 / D2Q5 multiple-relaxation-time lattice
 * Boltzmann model for convection heat transfer in porous media at the REV scale
 * (Q. Liu, Y.-L. He, Q. Li, W.-Q. Tao, arXiv:1308.2071).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the HIP path: every formula below
 * is written out again from the paper, in FP64, as plain loops over the lattice, in the order
 * the paper states the algorithm.  It is slow on purpose.
 *
 * What it computes (paper section / equation in brackets):
 *   flow    : D2Q9 MRT collision in moment space with porosity-dependent equilibrium moments and
 *             a moment-space forcing term [Sec. 3.1, Eqs. (6)-(24)];
 *   heat    : D2Q5 MRT collision with the heat source term [Sec. 3.2, Eqs. (26)-(37a)];
 *   walls   : non-equilibrium extrapolation for both distributions [Sec. 4, ref. 43];
 *   output  : macroscopic u, p, T and the wall-averaged Nusselt numbers [Eq. (38)].
 *
 * Readings taken where the paper is silent (each is listed with its reason in the design notes):
 *   - the state kept between steps is the post-collision population field; one step is
 *     streaming -> wall reconstruction -> macroscopic recovery -> collision; observables at
 *     time n are taken after streaming and wall reconstruction;
 *   - L = nx - 1 (wall nodes sit on the walls);  T0 = (Th+Tc)/2, dT = Th-Tc from the west and
 *     east isothermal walls;  g*beta = Ma^2 cs^2 / (dT L) from Ma = U/cs, U = sqrt(g beta dT L);
 *   - tau_T = 1/2 + nu / (sigma csT^2 Pr) with nu = nu_e / J (Pr = nu / alpha_e);
 *   - m^eq is Eq. (16) with j = rho0 u (u from Eq. (21)) and m0^eq = rho0;
 *   - a wall node takes u = 0, phi*p from its inward neighbour, T from the wall (isothermal) or
 *     from the neighbour (adiabatic); all 9 + 5 of its populations are rebuilt as equilibrium at
 *     the wall plus the neighbour's non-equilibrium part; corner nodes use the diagonal neighbour;
 *   - the initial post-collision populations are the rest equilibria f_i = w_i rho0,
 *     g_i = wt_i T_init at every node;
 *   - the five-point wall derivative is the fourth-order one-sided stencil
 *     (-25, 48, -36, 16, -3)/12, averaged over the wall by the trapezoid rule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Parameters                                                                                  */
/* ------------------------------------------------------------------------------------------ */

enum { REF_ISOTHERMAL = 0, REF_ADIABATIC = 1, REF_PERIODIC = 2 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };

typedef struct {
    int32_t nx, ny;          /* lattice nodes, wall nodes included                          */
    int32_t bc[4];           /* west, east, south, north: REF_ISOTHERMAL / ADIABATIC / PERIODIC */
    double T_wall[4];        /* wall temperature where bc == REF_ISOTHERMAL                  */
    double Ra, Pr, Da, J;    /* Sec. 2 dimensionless groups                                  */
    double Ma, sigma, varpi, rho0;
    double s_e, s_eps, s_q;  /* s1, s2, s4 = s6 of Eq. (20)                                   */
    double zeta3, zeta4;     /* zeta3, zeta4 of Eq. (31)                                      */
    int32_t forchheimer;     /* 1: F_phi from Eq. (5); 0: F_phi = 0 (Brinkman-extended Darcy)  */
    double T_init;
    double ext_accel[2];     /* extra body acceleration added to G (channel flow)              */
    double tau_v, tau_T;     /* > 0: use this value; otherwise Eq. (37b)                       */
    double gbeta;            /* >= 0: use this value; negative: from Ma                        */
    int32_t uniform_rates;   /* 1: every flow rate 1/tau_v and every thermal rate 1/tau_T      */
    double Ra_I;             /* internal Rayleigh number (Sec. 2); > 0: Q''' derived from it   */
    double Qv;               /* Q''' in lattice units when Ra_I <= 0 (0: no heat source)      */
} ref_params;

/* Derived quantities, in this order, for the tests:
 * 0 L, 1 cs2, 2 csT2, 3 tau_v, 4 tau_T, 5 nu_e, 6 nu, 7 gbeta, 8 dT, 9 T0, 10 K_uniform,
 * 11 Q (the heat source Q''')                                                               */
#define REF_NDERIVED 12

typedef struct {
    double L, cs2, csT2, tau_v, tau_T, nu_e, nu, gbeta, dT, T0, K_uniform, Q;
    double s[9], zeta[5];
} ref_derived;

/* ------------------------------------------------------------------------------------------ */
/* Lattice data                                                                                */
/* ------------------------------------------------------------------------------------------ */

/* D2Q9 velocities, Eq. (8) with c = 1. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* D2Q9 weights, after Eq. (13). */
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* Transformation matrix M, Eq. (11). */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
/* Transformation matrix N, Eq. (28). */
static const double NN[5][5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {-4, 1, 1, 1, 1},
    {0, 1, -1, 1, -1}};

/* M and N have mutually orthogonal rows, so their inverses are the transposes scaled by the
 * reciprocal squared row norms.  Filled once by build_inverses(). */
static double MINV[9][9];
static double NINV[5][5];
static int inverses_built = 0;

static void build_inverses(void) {
    if (inverses_built) return;
    for (int k = 0; k < 9; ++k) {
        double nrm2 = 0;
        for (int i = 0; i < 9; ++i) nrm2 += MM[k][i] * MM[k][i];
        for (int i = 0; i < 9; ++i) MINV[i][k] = MM[k][i] / nrm2;
    }
    for (int k = 0; k < 5; ++k) {
        double nrm2 = 0;
        for (int i = 0; i < 5; ++i) nrm2 += NN[k][i] * NN[k][i];
        for (int i = 0; i < 5; ++i) NINV[i][k] = NN[k][i] / nrm2;
    }
    inverses_built = 1;
}

/* ------------------------------------------------------------------------------------------ */
/* Parameter derivation                                                                        */
/* ------------------------------------------------------------------------------------------ */

void ref_default_params(ref_params *p) {
    memset(p, 0, sizeof(*p));
    p->nx = 64;
    p->ny = 64;
    p->bc[SIDE_W] = REF_ISOTHERMAL;
    p->bc[SIDE_E] = REF_ISOTHERMAL;
    p->bc[SIDE_S] = REF_ADIABATIC;
    p->bc[SIDE_N] = REF_ADIABATIC;
    p->T_wall[SIDE_W] = 1.0; /* T_h */
    p->T_wall[SIDE_E] = 0.0; /* T_c */
    p->Ra = 1e3;
    p->Pr = 1.0;
    p->Da = 1e-2;
    p->J = 1.0;
    p->Ma = 0.1;      /* Sec. 4 */
    p->sigma = 1.0;   /* Sec. 4 */
    p->varpi = -2.0;  /* Sec. 4 */
    p->rho0 = 1.0;    /* Sec. 4 */
    p->s_e = 1.1;     /* Sec. 4 */
    p->s_eps = 1.1;
    p->s_q = 1.2;
    p->zeta3 = 1.5;
    p->zeta4 = 1.5;
    p->forchheimer = 1;
    p->T_init = 0.5;
    p->tau_v = -1;
    p->tau_T = -1;
    p->gbeta = -1;
    p->uniform_rates = 0;
    p->Ra_I = 0.0;
    p->Qv = 0.0;
}

static void derive(const ref_params *p, ref_derived *d) {
    d->L = (double)(p->nx - 1);
    d->cs2 = 1.0 / 3.0;                  /* cs = c / sqrt(3), after Eq. (13)  */
    d->csT2 = (4.0 + p->varpi) / 10.0;   /* after Eq. (37a)                   */
    /* Eq. (37b): tau_v = 1/2 + Ma J L sqrt(Pr/Ra) / (cs dt); with internal heating only
     * (Ra = 0, Sec. 4.2) Ra_I takes Ra's place */
    if (p->tau_v > 0)
        d->tau_v = p->tau_v;
    else if (p->Ra > 0)
        d->tau_v = 0.5 + p->Ma * p->J * d->L * sqrt(p->Pr / p->Ra) / sqrt(d->cs2);
    else
        d->tau_v = 0.5 + p->Ma * p->J * d->L * sqrt(p->Pr) / (sqrt(d->cs2) * sqrt(p->Ra_I));
    d->nu_e = d->cs2 * (d->tau_v - 0.5); /* Eq. (24) */
    d->nu = d->nu_e / p->J;              /* J = nu_e / nu, Sec. 2 */
    /* alpha_e = sigma csT^2 (tau_T - 1/2) (after Eq. (37a), Eq. (A9)) and Pr = nu / alpha_e */
    d->tau_T = p->tau_T > 0 ? p->tau_T : 0.5 + d->nu / (p->sigma * d->csT2 * p->Pr);
    if (p->bc[SIDE_W] == REF_ISOTHERMAL && p->bc[SIDE_E] == REF_ISOTHERMAL &&
        p->T_wall[SIDE_W] != p->T_wall[SIDE_E]) {
        d->dT = p->T_wall[SIDE_W] - p->T_wall[SIDE_E];         /* dT = Th - Tc, Sec. 4.1 */
        d->T0 = 0.5 * (p->T_wall[SIDE_W] + p->T_wall[SIDE_E]);  /* T0 = (Th + Tc)/2     */
    } else {
        d->dT = 1.0;
        d->T0 = p->T_init;
    }
    /* Ma = U / cs with U = sqrt(g beta dT L), Sec. 4 */
    d->gbeta = p->gbeta >= 0 ? p->gbeta : p->Ma * p->Ma * d->cs2 / (d->dT * d->L);
    d->K_uniform = p->Da > 0 ? p->Da * d->L * d->L : INFINITY; /* Da = K / L^2, Sec. 2 */
    /* Heat source: Ra_I = g beta Q''' L^5 / (nu alpha_e^2) (Sec. 2) with
     * alpha_e = sigma csT^2 (tau_T - 1/2) (after Eq. (37a)).  Without side heating the
     * temperature scale is dT = Q''' L^2 / alpha_e (Sec. 4.2), taken as 1. */
    if (p->Ra_I > 0) {
        const double alpha = p->sigma * d->csT2 * (d->tau_T - 0.5);
        d->Q = p->Ra_I * d->nu * alpha * alpha / (d->gbeta * pow(d->L, 5.0));
    } else {
        d->Q = p->Qv;
    }

    /* Eq. (20) with the values of Sec. 4; Eq. (31) likewise. */
    const double sv = 1.0 / d->tau_v, sT = 1.0 / d->tau_T;
    if (p->uniform_rates) {
        for (int k = 0; k < 9; ++k) d->s[k] = sv;
        for (int k = 0; k < 5; ++k) d->zeta[k] = sT;
    } else {
        const double s[9] = {1.0, p->s_e, p->s_eps, 1.0, p->s_q, 1.0, p->s_q, sv, sv};
        const double z[5] = {1.0, sT, sT, p->zeta3, p->zeta4};
        memcpy(d->s, s, sizeof s);
        memcpy(d->zeta, z, sizeof z);
    }
}

void ref_derive(const ref_params *p, double *out) {
    ref_derived d;
    derive(p, &d);
    const double v[REF_NDERIVED] = {d.L,  d.cs2,   d.csT2, d.tau_v, d.tau_T,    d.nu_e,
                                    d.nu, d.gbeta, d.dT,   d.T0,    d.K_uniform, d.Q};
    memcpy(out, v, sizeof v);
}

/* ------------------------------------------------------------------------------------------ */
/* Per-node formulas of the paper                                                              */
/* ------------------------------------------------------------------------------------------ */

/* Eq. (5): Ergun geometric function. */
static double ergun_F(double phi, int forchheimer) {
    return forchheimer ? 1.75 / sqrt(150.0 * phi * phi * phi) : 0.0;
}

/* Eq. (14): velocity part s_i(u) of the porous incompressible equilibrium. */
static double s_i(int i, double ux, double uy, double phi, double cs2) {
    const double eu = EX[i] * ux + EY[i] * uy;
    const double uu = ux * ux + uy * uy;
    return W9[i] * (eu / cs2 + eu * eu / (2.0 * phi * cs2 * cs2) - uu / (2.0 * phi * cs2));
}

/* Eq. (13): f_i^eq as a function of the product phi*p, u and phi. */
static void feq(double phip, double ux, double uy, double phi, double rho0, double cs2,
                double out[9]) {
    out[0] = rho0 - (1.0 - W9[0]) * phip / cs2 + rho0 * s_i(0, ux, uy, phi, cs2);
    for (int i = 1; i < 9; ++i) out[i] = W9[i] * phip / cs2 + rho0 * s_i(i, ux, uy, phi, cs2);
}

/* Eq. (37a): D2Q5 equilibrium with weights wt0 = (1 - varpi)/5, wt_i = (4 + varpi)/20. */
static void geq(double T, double ux, double uy, double sigma, double varpi, double out[5]) {
    const double csT2 = (4.0 + varpi) / 10.0;
    for (int i = 0; i < 5; ++i) {
        const double wt = (i == 0) ? (1.0 - varpi) / 5.0 : (4.0 + varpi) / 20.0;
        out[i] = wt * T * (1.0 + (EX[i] * ux + EY[i] * uy) / (sigma * csT2));
    }
}

/* Eq. (16): equilibrium moments, with phi*p passed as a product. */
static void meq(double phip, double ux, double uy, double phi, double rho0, double out[9]) {
    const double uu = ux * ux + uy * uy;
    out[0] = rho0;
    out[1] = -4.0 * rho0 + 6.0 * phip + 3.0 * rho0 * uu / phi;
    out[2] = 4.0 * rho0 - 9.0 * phip - 3.0 * rho0 * uu / phi;
    out[3] = rho0 * ux;
    out[4] = -rho0 * ux;
    out[5] = rho0 * uy;
    out[6] = -rho0 * uy;
    out[7] = rho0 * (ux * ux - uy * uy) / phi;
    out[8] = rho0 * ux * uy / phi;
}

/* Eq. (19): forcing term in moment space. */
static void forcing(double ux, double uy, double Fx, double Fy, double phi, double rho0,
                    double out[9]) {
    const double uF = ux * Fx + uy * Fy;
    out[0] = 0.0;
    out[1] = 6.0 * rho0 * uF / phi;
    out[2] = -6.0 * rho0 * uF / phi;
    out[3] = rho0 * Fx;
    out[4] = -rho0 * Fx;
    out[5] = rho0 * Fy;
    out[6] = -rho0 * Fy;
    out[7] = 2.0 * rho0 * (ux * Fx - uy * Fy) / phi;
    out[8] = rho0 * (ux * Fy + uy * Fx) / phi;
}

/* Eq. (29): thermal equilibrium moments (no heat source). */
static void neq(double T, double ux, double uy, double sigma, double varpi, double out[5]) {
    out[0] = T;
    out[1] = ux * T / sigma;
    out[2] = uy * T / sigma;
    out[3] = varpi * T;
    out[4] = 0.0;
}

/* Macroscopic state of one node. */
typedef struct {
    double T, ux, uy, phip, Fx, Fy, phi;
    double vv;   /* |v|^2 of Eq. (22) (a wall node carries its inward neighbour's) */
} macro_t;

/* Eqs. (36), (22), (21), (23), (4) for a fluid node from its post-streaming populations. */
static void interior_macros(const double fh[9], const double gh[5], double phi, double K,
                            const ref_params *p, const ref_derived *d, macro_t *m) {
    const double rho0 = p->rho0;
    double T = 0.0;
    for (int i = 0; i < 5; ++i) T += gh[i];
    T += 0.5 * d->Q / p->sigma;                                    /* Eq. (36), dt = 1 */
    const double Gx = p->ext_accel[0];
    const double Gy = p->ext_accel[1] + d->gbeta * (T - d->T0);    /* G = g beta (T-T0) j */
    double jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        jx += EX[i] * fh[i];
        jy += EY[i] * fh[i];
    }
    const double vx = jx / rho0 + 0.5 * phi * Gx;                  /* Eq. (22) */
    const double vy = jy / rho0 + 0.5 * phi * Gy;
    const double Fphi = ergun_F(phi, p->forchheimer);
    const double l0 = 0.5 * (1.0 + phi * 0.5 * d->nu / K);         /* after Eq. (22) */
    const double l1 = phi * 0.5 * Fphi / sqrt(K);
    const double vmag = sqrt(vx * vx + vy * vy);
    const double den = l0 + sqrt(l0 * l0 + l1 * vmag);             /* Eq. (21) */
    const double ux = vx / den, uy = vy / den;
    double sum18 = 0.0;
    for (int i = 1; i < 9; ++i) sum18 += fh[i];
    /* Eq. (23), multiplied through by phi so that the product phi*p is kept. */
    const double phip = d->cs2 / (1.0 - W9[0]) * (sum18 + rho0 * s_i(0, ux, uy, phi, d->cs2));
    const double umag = sqrt(ux * ux + uy * uy);
    m->T = T;
    m->ux = ux;
    m->uy = uy;
    m->phip = phip;
    m->Fx = -phi * d->nu / K * ux - phi * Fphi / sqrt(K) * umag * ux + phi * Gx; /* Eq. (4) */
    m->Fy = -phi * d->nu / K * uy - phi * Fphi / sqrt(K) * umag * uy + phi * Gy;
    m->phi = phi;
    m->vv = vx * vx + vy * vy;
}

/* Eq. (17) then Eq. (34) at one node: post-streaming populations -> post-collision ones. */
static void collide_node(const double fh[9], const double gh[5], const macro_t *m,
                         const ref_params *p, const ref_derived *d, double fp[9],
                         double gp[5]) {
    double mom[9], me[9], S[9], mp[9];
    for (int k = 0; k < 9; ++k) {
        mom[k] = 0.0;
        for (int i = 0; i < 9; ++i) mom[k] += MM[k][i] * fh[i];           /* Eq. (9) */
    }
    meq(m->phip, m->ux, m->uy, m->phi, p->rho0, me);
    forcing(m->ux, m->uy, m->Fx, m->Fy, m->phi, p->rho0, S);
    for (int k = 0; k < 9; ++k)                                         /* Eq. (17), dt = 1 */
        mp[k] = mom[k] - d->s[k] * (mom[k] - me[k]) + (1.0 - 0.5 * d->s[k]) * S[k];
    for (int i = 0; i < 9; ++i) {
        fp[i] = 0.0;
        for (int k = 0; k < 9; ++k) fp[i] += MINV[i][k] * mp[k];        /* f+ = M^-1 m+ */
    }
    double n[5], ne[5], np[5];
    for (int k = 0; k < 5; ++k) {
        n[k] = 0.0;
        for (int i = 0; i < 5; ++i) n[k] += NN[k][i] * gh[i];            /* Eq. (27) */
    }
    neq(m->T, m->ux, m->uy, p->sigma, p->varpi, ne);
    const double Psi[5] = {d->Q / p->sigma, 0.0, 0.0, p->varpi * d->Q / p->sigma, 0.0}; /* (30) */
    for (int k = 0; k < 5; ++k)                                         /* Eq. (34), dt = 1 */
        np[k] = n[k] - d->zeta[k] * (n[k] - ne[k]) + (1.0 - 0.5 * d->zeta[k]) * Psi[k];
    for (int i = 0; i < 5; ++i) {
        gp[i] = 0.0;
        for (int k = 0; k < 5; ++k) gp[i] += NINV[i][k] * np[k];        /* g+ = N^-1 n+ */
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Lattice context                                                                             */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    ref_params p;
    ref_derived d;
    int nx, ny;
    size_t n;
    double *f, *g;      /* post-collision populations, plane-major: f[i*n + y*nx + x]   */
    double *fh, *gh;    /* post-streaming, post-wall-reconstruction populations          */
    double *phi, *K;    /* medium per node                                               */
    macro_t *mac;       /* macroscopic state per node at the current time level          */
    int64_t step;
} ref_ctx;

static int is_wall(const ref_ctx *c, int x, int y) {
    const int32_t *bc = c->p.bc;
    return (x == 0 && bc[SIDE_W] != REF_PERIODIC) || (x == c->nx - 1 && bc[SIDE_E] != REF_PERIODIC) ||
           (y == 0 && bc[SIDE_S] != REF_PERIODIC) || (y == c->ny - 1 && bc[SIDE_N] != REF_PERIODIC);
}

void ref_destroy(ref_ctx *c) {
    if (!c) return;
    free(c->f);
    free(c->g);
    free(c->fh);
    free(c->gh);
    free(c->phi);
    free(c->K);
    free(c->mac);
    free(c);
}

/* Rest equilibrium everywhere (u = 0, phi*p = rho0 cs^2, T = T_init). */
static void set_rest(ref_ctx *c) {
    const size_t n = c->n;
    double g5[5];
    geq(c->p.T_init, 0.0, 0.0, c->p.sigma, c->p.varpi, g5);
    for (size_t k = 0; k < n; ++k) {
        for (int i = 0; i < 9; ++i) c->f[i * n + k] = W9[i] * c->p.rho0;
        for (int i = 0; i < 5; ++i) c->g[i * n + k] = g5[i];
    }
    c->step = 0;
}

/* phi, K: host arrays [ny][nx] or NULL (then phi_uniform and Da L^2 are used). */
ref_ctx *ref_create(const ref_params *p, const double *phi, double phi_uniform, const double *K) {
    build_inverses();
    ref_ctx *c = (ref_ctx *)calloc(1, sizeof(ref_ctx));
    if (!c) return NULL;
    c->p = *p;
    derive(p, &c->d);
    c->nx = p->nx;
    c->ny = p->ny;
    c->n = (size_t)p->nx * (size_t)p->ny;
    const size_t n = c->n;
    c->f = (double *)malloc(9 * n * sizeof(double));
    c->g = (double *)malloc(5 * n * sizeof(double));
    c->fh = (double *)malloc(9 * n * sizeof(double));
    c->gh = (double *)malloc(5 * n * sizeof(double));
    c->phi = (double *)malloc(n * sizeof(double));
    c->K = (double *)malloc(n * sizeof(double));
    c->mac = (macro_t *)malloc(n * sizeof(macro_t));
    if (!c->f || !c->g || !c->fh || !c->gh || !c->phi || !c->K || !c->mac) {
        ref_destroy(c);
        return NULL;
    }
    for (size_t k = 0; k < n; ++k) {
        c->phi[k] = phi ? phi[k] : phi_uniform;
        c->K[k] = K ? K[k] : c->d.K_uniform;
    }
    set_rest(c);
    return c;
}

/* Streaming, Eqs. (18) and (35): fh_i(x) = f_i(x - e_i).  Slots whose source lies outside a
 * non-periodic domain are left NaN; only wall nodes have such slots and the wall
 * reconstruction overwrites all of their populations. */
static void stream(ref_ctx *c) {
    const int nx = c->nx, ny = c->ny;
    const size_t n = c->n;
    const int perx = c->p.bc[SIDE_W] == REF_PERIODIC, pery = c->p.bc[SIDE_S] == REF_PERIODIC;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) {
                int xs = x - EX[i], ys = y - EY[i];
                if (perx) xs = (xs + nx) % nx;
                if (pery) ys = (ys + ny) % ny;
                const int inside = xs >= 0 && xs < nx && ys >= 0 && ys < ny;
                const size_t src = (size_t)ys * nx + xs;
                c->fh[i * n + k] = inside ? c->f[i * n + src] : NAN;
                if (i < 5) c->gh[i * n + k] = inside ? c->g[i * n + src] : NAN;
            }
        }
    }
}

/* Macroscopics at fluid nodes, then the non-equilibrium extrapolation at wall nodes. */
static void macros_and_walls(ref_ctx *c) {
    const int nx = c->nx, ny = c->ny;
    const size_t n = c->n;
    const ref_params *p = &c->p;
    const ref_derived *d = &c->d;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            if (is_wall(c, x, y)) continue;
            const size_t k = (size_t)y * nx + x;
            double f9[9], g5[5];
            for (int i = 0; i < 9; ++i) f9[i] = c->fh[i * n + k];
            for (int i = 0; i < 5; ++i) g5[i] = c->gh[i * n + k];
            interior_macros(f9, g5, c->phi[k], c->K[k], p, d, &c->mac[k]);
        }
    }
    /* Wall nodes read only fluid nodes (their inward neighbours), so this loop may run after
     * the fluid loop in any order. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            if (!is_wall(c, x, y)) continue;
            const int onW = x == 0 && p->bc[SIDE_W] != REF_PERIODIC;
            const int onE = x == nx - 1 && p->bc[SIDE_E] != REF_PERIODIC;
            const int onS = y == 0 && p->bc[SIDE_S] != REF_PERIODIC;
            const int onN = y == ny - 1 && p->bc[SIDE_N] != REF_PERIODIC;
            const int dx = onW ? 1 : (onE ? -1 : 0);
            const int dy = onS ? 1 : (onN ? -1 : 0);
            const size_t k = (size_t)y * nx + x;
            const size_t kf = (size_t)(y + dy) * nx + (x + dx); /* inward neighbour */
            const macro_t *mf = &c->mac[kf];
            /* wall temperature */
            const int sx = onW ? SIDE_W : (onE ? SIDE_E : -1);
            const int sy = onS ? SIDE_S : (onN ? SIDE_N : -1);
            const int isoX = sx >= 0 && p->bc[sx] == REF_ISOTHERMAL;
            const int isoY = sy >= 0 && p->bc[sy] == REF_ISOTHERMAL;
            double Tb;
            if (isoX && isoY) Tb = 0.5 * (p->T_wall[sx] + p->T_wall[sy]);
            else if (isoX) Tb = p->T_wall[sx];
            else if (isoY) Tb = p->T_wall[sy];
            else Tb = mf->T;
            const double phib = c->phi[k];
            macro_t *mb = &c->mac[k];
            mb->T = Tb;
            mb->ux = 0.0;
            mb->uy = 0.0;
            mb->phip = mf->phip;           /* phi_b p_b = phi_f p_f */
            mb->phi = phib;
            mb->vv = mf->vv;
            mb->Fx = phib * p->ext_accel[0];
            mb->Fy = phib * (p->ext_accel[1] + d->gbeta * (Tb - d->T0));
            /* f_b = f^eq(wall) + [f(x_f) - f^eq(x_f)], likewise for g */
            double fe_b[9], fe_f[9], ge_b[5], ge_f[5];
            feq(mb->phip, 0.0, 0.0, phib, p->rho0, d->cs2, fe_b);
            feq(mf->phip, mf->ux, mf->uy, mf->phi, p->rho0, d->cs2, fe_f);
            geq(Tb, 0.0, 0.0, p->sigma, p->varpi, ge_b);
            geq(mf->T, mf->ux, mf->uy, p->sigma, p->varpi, ge_f);
            for (int i = 0; i < 9; ++i)
                c->fh[i * n + k] = fe_b[i] + (c->fh[i * n + kf] - fe_f[i]);
            for (int i = 0; i < 5; ++i)
                c->gh[i * n + k] = ge_b[i] + (c->gh[i * n + kf] - ge_f[i]);
        }
    }
}

static void collide_all(ref_ctx *c) {
    const int nx = c->nx, ny = c->ny;
    const size_t n = c->n;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            double f9[9], g5[5], fp[9], gp[5];
            for (int i = 0; i < 9; ++i) f9[i] = c->fh[i * n + k];
            for (int i = 0; i < 5; ++i) g5[i] = c->gh[i * n + k];
            collide_node(f9, g5, &c->mac[k], &c->p, &c->d, fp, gp);
            for (int i = 0; i < 9; ++i) c->f[i * n + k] = fp[i];
            for (int i = 0; i < 5; ++i) c->g[i * n + k] = gp[i];
        }
    }
}

/* Advance the post-collision state by nsteps time steps. */
void ref_step(ref_ctx *c, int64_t nsteps) {
    for (int64_t s = 0; s < nsteps; ++s) {
        stream(c);
        macros_and_walls(c);
        collide_all(c);
        c->step += 1;
    }
}

/* Temperature interval outside which a run counts as diverged: [lo, hi] over T_init and the
 * isothermal walls, widened by the temperature scale dT and, with a heat source, by what the
 * source can add: |Q| Lmax^2 / (2 alpha_e) (conduction from one isothermal side across the
 * longer side, alpha_e T'' = -Q) when some side is isothermal, else |Q| t / sigma (Eq. (3)
 * with no heat leaving), Q the source Q''' of Eq. (30).  out[0] = lower, out[1] = upper. */
static void temperature_bounds(const ref_ctx *c, double out[2]) {
    const ref_params *p = &c->p;
    const ref_derived *d = &c->d;
    double lo = p->T_init, hi = p->T_init;
    int iso = 0;
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] != REF_ISOTHERMAL) continue;
        iso = 1;
        if (p->T_wall[s] < lo) lo = p->T_wall[s];
        if (p->T_wall[s] > hi) hi = p->T_wall[s];
    }
    const double Lmax = (double)((c->nx > c->ny ? c->nx : c->ny) - 1);
    const double alpha = p->sigma * d->csT2 * (d->tau_T - 0.5);
    const double rise = iso ? fabs(d->Q) * Lmax * Lmax / (2.0 * alpha)
                            : fabs(d->Q) * (double)c->step / p->sigma;
    out[0] = lo - fabs(d->dT) - (d->Q < 0 ? rise : 0.0);
    out[1] = hi + fabs(d->dT) + (d->Q > 0 ? rise : 0.0);
}

/* Observables at the current time level: u, phi*p/phi, T per node ([ny][nx], any may be NULL)
 * and out[0..7] = Nu_hot (west wall), Nu_cold (east wall), max |u|, relative total-mass error
 * of the stored post-collision populations, a divergence flag, min T, max T and
 * max |phi p - rho0 cs^2|.  The flag is 1 when
 *   - a field (u, p, T) or |v| of Eq. (22) is not finite (|v|^2 overflowing makes the
 *     denominator of Eq. (21) infinite and u = 0, so u alone cannot show it),
 *   - max |u| exceeds cs,
 *   - T leaves the interval of temperature_bounds.
 * (The level of phi p is a gauge of the step that drifts slowly in long runs; max
 * |phi p - rho0 cs^2| is reported but not judged.) */
void ref_observables(ref_ctx *c, double *ux, double *uy, double *pr, double *T, double *out) {
    stream(c);
    macros_and_walls(c);
    const int nx = c->nx, ny = c->ny;
    const size_t n = c->n;
    double umax = 0.0, tmin = INFINITY, tmax = -INFINITY, pdev = 0.0;
    int bad = 0;
    const double prest = c->p.rho0 * c->d.cs2;
    for (size_t k = 0; k < n; ++k) {
        const macro_t *m = &c->mac[k];
        if (ux) ux[k] = m->ux;
        if (uy) uy[k] = m->uy;
        if (pr) pr[k] = m->phip / m->phi;
        if (T) T[k] = m->T;
        const double um = sqrt(m->ux * m->ux + m->uy * m->uy);
        if (!(um <= umax)) umax = um;
        if (!isfinite(m->ux) || !isfinite(m->uy) || !isfinite(m->phip) || !isfinite(m->T) ||
            !isfinite(m->vv))
            bad = 1;
        if (!(m->T >= tmin)) tmin = m->T;
        if (!(m->T <= tmax)) tmax = m->T;
        const double pd = fabs(m->phip - prest);
        if (!(pd <= pdev)) pdev = pd;
    }
    /* Eq. (38) with the five-point one-sided derivative and the trapezoid rule. */
    double nu_h = 0.0, nu_c = 0.0;
    if (nx >= 5) {
        for (int y = 0; y < ny; ++y) {
            const size_t r = (size_t)y * nx;
            const double dTdx_h = (-25.0 * c->mac[r + 0].T + 48.0 * c->mac[r + 1].T -
                                   36.0 * c->mac[r + 2].T + 16.0 * c->mac[r + 3].T -
                                   3.0 * c->mac[r + 4].T) / 12.0;
            const double dTdx_c = (25.0 * c->mac[r + nx - 1].T - 48.0 * c->mac[r + nx - 2].T +
                                   36.0 * c->mac[r + nx - 3].T - 16.0 * c->mac[r + nx - 4].T +
                                   3.0 * c->mac[r + nx - 5].T) / 12.0;
            const double w = (y == 0 || y == ny - 1) ? 0.5 : 1.0;
            nu_h += w * (-c->d.L * dTdx_h / c->d.dT);
            nu_c += w * (-c->d.L * dTdx_c / c->d.dT);
        }
        nu_h /= (double)(ny - 1);
        nu_c /= (double)(ny - 1);
    }
    double mass = 0.0;
    for (size_t k = 0; k < 9 * n; ++k) mass += c->f[k];
    const double mass_ref = (double)n * c->p.rho0;
    out[0] = nu_h;
    out[1] = nu_c;
    out[2] = umax;
    out[3] = fabs(mass - mass_ref) / mass_ref;
    double tb[2];
    temperature_bounds(c, tb);
    out[4] = (bad || !(umax <= sqrt(c->d.cs2)) || !(tmin >= tb[0]) || !(tmax <= tb[1])) ? 1.0
                                                                                        : 0.0;
    out[5] = tmin;
    out[6] = tmax;
    out[7] = pdev;
}

int64_t ref_get_step(const ref_ctx *c) { return c->step; }

/* Post-collision state as plane-major arrays f[9][ny][nx], g[5][ny][nx]. */
void ref_get_state(const ref_ctx *c, double *f, double *g) {
    memcpy(f, c->f, 9 * c->n * sizeof(double));
    memcpy(g, c->g, 5 * c->n * sizeof(double));
}

void ref_set_state(ref_ctx *c, const double *f, const double *g, int64_t step) {
    memcpy(c->f, f, 9 * c->n * sizeof(double));
    memcpy(c->g, g, 5 * c->n * sizeof(double));
    c->step = step;
}

void ref_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int ref_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Single-formula entry points, exported for the pin tests                                     */
/* ------------------------------------------------------------------------------------------ */

void ref_matrices(double *M, double *Minv, double *N, double *Ninv) {
    build_inverses();
    memcpy(M, MM, sizeof MM);
    memcpy(Minv, MINV, sizeof MINV);
    memcpy(N, NN, sizeof NN);
    memcpy(Ninv, NINV, sizeof NINV);
}

void ref_feq(double phip, double ux, double uy, double phi, double rho0, double *out) {
    feq(phip, ux, uy, phi, rho0, 1.0 / 3.0, out);
}

void ref_meq(double phip, double ux, double uy, double phi, double rho0, double *out) {
    meq(phip, ux, uy, phi, rho0, out);
}

void ref_forcing(double ux, double uy, double Fx, double Fy, double phi, double rho0,
                 double *out) {
    forcing(ux, uy, Fx, Fy, phi, rho0, out);
}

void ref_geq(double T, double ux, double uy, double sigma, double varpi, double *out) {
    geq(T, ux, uy, sigma, varpi, out);
}

void ref_neq(double T, double ux, double uy, double sigma, double varpi, double *out) {
    neq(T, ux, uy, sigma, varpi, out);
}

/* Fluid-node macroscopics: out = (T, ux, uy, phi*p, Fx, Fy). */
void ref_macros(const ref_params *p, const double *fh, const double *gh, double phi, double K,
                double *out) {
    ref_derived d;
    derive(p, &d);
    macro_t m;
    interior_macros(fh, gh, phi, K, p, &d, &m);
    out[0] = m.T;
    out[1] = m.ux;
    out[2] = m.uy;
    out[3] = m.phip;
    out[4] = m.Fx;
    out[5] = m.Fy;
}

/* Fluid-node collision: post-streaming (fh, gh) -> post-collision (fp, gp). */
void ref_collide_fluid_node(const ref_params *p, const double *fh, const double *gh, double phi,
                            double K, double *fp, double *gp) {
    build_inverses();
    ref_derived d;
    derive(p, &d);
    macro_t m;
    interior_macros(fh, gh, phi, K, p, &d, &m);
    collide_node(fh, gh, &m, p, &d, fp, gp);
}
