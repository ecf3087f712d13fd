/*
 * tcp_oracle.c -- plain FP64 CPU reference of the coupled thermocapillary
 * phase-field lattice Boltzmann step (Holzer, Mitchell, Leonardi, Ruede,
 * "Development of a central-moment phase-field lattice Boltzmann model for
 * thermocapillary flows", arXiv 2401.03041).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library, and it never calls it.
 *
 * Style: slow and literal.  Every collision builds the central-moment matrix
 * T(u) of the cell numerically, transforms f, f_eq and the source, relaxes
 * each moment with its own rate and solves T f* = kappa* by Gaussian
 * elimination.  Cells are independent inside a sub-step, so the loops over
 * cells are OpenMP-parallel; nothing else is blocked, fused or reordered.
 *
 * Units: dx = dt = 1, c_s^2 = 1/3 on every stencil used here.
 * Index of a cell: c = x + nx*(y + ny*z).  The oracle stores PDFs cell-major
 * (pdf[c*Q + i]).
 *
 * Readings of passages the paper leaves silent or garbled (each is listed
 * with its justification in the design notes of the repository):
 *   R1  relaxation rates omega_phi = 1/(1/2 + M/c_s^2), omega_T = 1/(1/2 + kappa/c_s^2)
 *   R2  omega(phi) = 1/(tau(phi) + 1/2), tau_{H,L} = nu_{H,L}/c_s^2, nu = tau c_s^2
 *   R3  Allen-Cahn counter-term lambda = 4 phi (1-phi)/xi (Eq. phasefieldforce)
 *   R4  |grad phi|^2 in the Marangoni term of F_s
 *   R5  mu_phi = 4 beta phi (phi-1)(phi-1/2) - k lap(phi), beta = 12 sigma/xi, k = 3 sigma xi/2
 *   R6  p* = p/(c_s^2 rho); read back p = p* rho c_s^2
 *   R7  kappa(phi) = kappa_L + phi_c (kappa_H - kappa_L)
 *   R8  kappa is a lattice diffusivity (rho c_p == 1)
 *   R9  RK2 = midpoint rule
 *   R10 heat source nonzero for d^2 <= d_s^2 (d_s <= 0: no cut-off)
 *   R11 Dirichlet temperature by anti-bounce-back; stencil ghost 2 T_w - T
 *   R12 halfway bounce-back for h and g, moving-wall term for g, mirror ghost for phi
 *   R13 central-moment bases per stencil; kappa_eq = T(u) f_eq (discrete)
 *   R14 relaxation rate per moment
 *   R15 Guo source terms
 *   R16 strain rate from the non-equilibrium second moment of g
 *   R17 isotropic D3Q27 finite differences for gradients and Laplacians
 *   R18 time levels inside one step: the phase-field and hydrodynamic updates
 *       both see phi^n (and T^n); the thermal update sees phi^{n+1}, u^{n+1}
 *   R19 n = grad phi / sqrt(|grad phi|^2 + eps^2), eps = normal_eps (default 1e-6)
 *   R20 phi clamped to [0,1] only inside rho, tau and kappa
 *   R21 initial state: tanh droplets, PDFs at equilibrium with p* = 0
 *   R22, R23 (the App. A reference solution and channel set-up: tests only)
 *   R24 wetting: ghost phi across a wall from the contact-angle condition
 *       n_w . grad phi = -cos(theta) 4 phi (1 - phi)/xi (mirror at 90 degrees)
 *
 * Parity unpinned (no test other than oracle-vs-GPU consistency fixes them):
 *   the relaxation rates of the third- and higher-order moments (R14), the
 *   time levels of R18 away from steady states, the regularisation of R19 and
 *   the clamp of R20.  Every other function below is pinned by a CPU test
 *   against a closed form, an invariant or a textbook special case.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27
#define CS2 (1.0 / 3.0)

/* ------------------------------------------------------------------------ */
/* Stencils: velocity order of the App. B figure, weights of the App. B
 * weight equations.  Axis convention of the figure: 1/2 = +y/-y (N/S),
 * 3/4 = -x/+x (W/E), 5/6 = +z/-z (T/B).                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int q;
    int e[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} stencil;

static const int VEL27[27][3] = {
    {0, 0, 0},                                                 /* 0  C   */
    {0, 1, 0},   {0, -1, 0},  {-1, 0, 0},  {1, 0, 0},          /* 1-4 N S W E */
    {0, 0, 1},   {0, 0, -1},                                   /* 5-6 T B */
    {-1, 1, 0},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},         /* 7-10 NW NE SW SE */
    {0, 1, 1},   {0, -1, 1},  {-1, 0, 1},  {1, 0, 1},          /* 11-14 TN TS TW TE */
    {0, 1, -1},  {0, -1, -1}, {-1, 0, -1}, {1, 0, -1},         /* 15-18 BN BS BW BE */
    {1, 1, 1},   {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},        /* 19-22 TNE TNW TSE TSW */
    {1, 1, -1},  {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}        /* 23-26 BNE BNW BSE BSW */
};

static stencil ST7, ST15, ST19, ST27;
static int stencils_ready = 0;

static void fill_opp(stencil *s)
{
    for (int i = 0; i < s->q; ++i) {
        s->opp[i] = -1;
        for (int j = 0; j < s->q; ++j)
            if (s->e[j][0] == -s->e[i][0] && s->e[j][1] == -s->e[i][1] &&
                s->e[j][2] == -s->e[i][2])
                s->opp[i] = j;
    }
}

static void init_stencils(void)
{
    if (stencils_ready) return;
    /* D3Q7: w_0 = 0, w_{1..6} = 1/6 */
    ST7.q = 7;
    for (int i = 0; i < 7; ++i) {
        memcpy(ST7.e[i], VEL27[i], sizeof(int) * 3);
        ST7.w[i] = (i == 0) ? 0.0 : 1.0 / 6.0;
    }
    /* D3Q15: centre, 6 faces, then the 8 corners in the order TNE..BSW */
    ST15.q = 15;
    for (int i = 0; i < 15; ++i) {
        int src = (i < 7) ? i : i + 12;
        memcpy(ST15.e[i], VEL27[src], sizeof(int) * 3);
        ST15.w[i] = (i == 0) ? 16.0 / 72.0 : (i < 7 ? 8.0 / 72.0 : 1.0 / 72.0);
    }
    /* D3Q19: centre, 6 faces, 12 edges */
    ST19.q = 19;
    for (int i = 0; i < 19; ++i) {
        memcpy(ST19.e[i], VEL27[i], sizeof(int) * 3);
        ST19.w[i] = (i == 0) ? 12.0 / 36.0 : (i < 7 ? 2.0 / 36.0 : 1.0 / 36.0);
    }
    /* D3Q27 */
    ST27.q = 27;
    for (int i = 0; i < 27; ++i) {
        memcpy(ST27.e[i], VEL27[i], sizeof(int) * 3);
        ST27.w[i] = (i == 0) ? 64.0 / 216.0
                    : (i < 7) ? 16.0 / 216.0
                    : (i < 19) ? 4.0 / 216.0
                               : 1.0 / 216.0;
    }
    fill_opp(&ST7);
    fill_opp(&ST15);
    fill_opp(&ST19);
    fill_opp(&ST27);
    stencils_ready = 1;
}

static const stencil *get_stencil(int q)
{
    init_stencils();
    switch (q) {
    case 7: return &ST7;
    case 15: return &ST15;
    case 19: return &ST19;
    case 27: return &ST27;
    default: return NULL;
    }
}

/* ------------------------------------------------------------------------ */
/* Central-moment bases (reading R13).  A basis row is a polynomial in the
 * peculiar velocity c = e - u, given as a short sum of monomials.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;            /* number of monomials */
    double coef[3];
    int pw[3][3];     /* exponents (a,b,c) of x^a y^b z^c */
    int order;        /* polynomial degree */
    int tag;          /* 0 plain, 1 trace, 2 deviatoric diagonal, 3 off-diagonal 2nd order */
} mrow;

typedef struct {
    int q;
    mrow r[QMAX];
} mbasis;

static void mono(mrow *r, int a, int b, int c)
{
    r->n = 1;
    r->coef[0] = 1.0;
    r->pw[0][0] = a; r->pw[0][1] = b; r->pw[0][2] = c;
    r->order = a + b + c;
    r->tag = (r->order == 2 && (a == 1 || b == 1 || c == 1)) ? 3 : 0;
}

/* Monomial exponent sets of the four stencils (reading R13). */
static void basis_monomials(int q, mbasis *B)
{
    int k = 0;
    B->q = q;
    if (q == 27) {
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) mono(&B->r[k++], a, b, c);
        return;
    }
    static const int base[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                    {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    int nbase = (q == 7) ? 7 : 10;
    for (int j = 0; j < nbase; ++j) mono(&B->r[k++], base[j][0], base[j][1], base[j][2]);
    if (q == 19) {
        static const int extra[9][3] = {{2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2},
                                        {0, 1, 2}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
        for (int j = 0; j < 9; ++j) mono(&B->r[k++], extra[j][0], extra[j][1], extra[j][2]);
    } else if (q == 15) {
        static const int extra[5][3] = {{1, 2, 0}, {0, 1, 2}, {2, 0, 1}, {1, 1, 1}, {2, 2, 0}};
        for (int j = 0; j < 5; ++j) mono(&B->r[k++], extra[j][0], extra[j][1], extra[j][2]);
    }
}

/* Hydrodynamic D3Q27 basis: the three diagonal second-order monomials are
 * replaced by the trace x^2+y^2+z^2 and the deviators x^2-y^2, x^2-z^2 so
 * that bulk and shear parts relax with their own rates (reading R14).      */
static void basis_hydro(mbasis *B)
{
    basis_monomials(27, B);
    for (int j = 0; j < 27; ++j) {
        mrow *r = &B->r[j];
        int a = r->pw[0][0], b = r->pw[0][1], c = r->pw[0][2];
        if (r->order != 2 || r->tag == 3) continue;
        if (a == 2) { /* trace */
            r->n = 3;
            r->coef[0] = r->coef[1] = r->coef[2] = 1.0;
            r->pw[0][0] = 2; r->pw[0][1] = 0; r->pw[0][2] = 0;
            r->pw[1][0] = 0; r->pw[1][1] = 2; r->pw[1][2] = 0;
            r->pw[2][0] = 0; r->pw[2][1] = 0; r->pw[2][2] = 2;
            r->tag = 1;
        } else { /* x^2 - y^2 or x^2 - z^2 */
            r->n = 2;
            r->coef[0] = 1.0; r->coef[1] = -1.0;
            r->pw[1][0] = 0; r->pw[1][1] = b; r->pw[1][2] = c;
            r->pw[0][0] = 2; r->pw[0][1] = 0; r->pw[0][2] = 0;
            r->tag = 2;
        }
    }
}

static double ipow(double v, int p)
{
    double r = 1.0;
    for (int k = 0; k < p; ++k) r *= v;
    return r;
}

/* T(u)_{ji} = P_j(e_i - u) */
static void build_T(const stencil *s, const mbasis *B, const double u[3], double *T)
{
    for (int j = 0; j < s->q; ++j)
        for (int i = 0; i < s->q; ++i) {
            double cx = s->e[i][0] - u[0], cy = s->e[i][1] - u[1], cz = s->e[i][2] - u[2];
            double v = 0.0;
            for (int t = 0; t < B->r[j].n; ++t)
                v += B->r[j].coef[t] * ipow(cx, B->r[j].pw[t][0]) * ipow(cy, B->r[j].pw[t][1]) *
                     ipow(cz, B->r[j].pw[t][2]);
            T[j * s->q + i] = v;
        }
}

/* Solve A x = b (n x n, row-major, destroyed) by Gaussian elimination with
 * partial pivoting.  Returns 0 on success.                                 */
static int gauss_solve(int n, double *A, double *b, double *x)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > best) { best = fabs(A[r * n + k]); p = r; }
        if (best == 0.0) return -1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double m = A[r * n + k] / A[k * n + k];
            if (m == 0.0) continue;
            for (int c = k; c < n; ++c) A[r * n + c] -= m * A[k * n + c];
            b[r] -= m * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * x[c];
        x[k] = s / A[k * n + k];
    }
    return 0;
}

/* Central-moment collision (readings R13-R15):
 *   kappa = T f, kappa_eq = T f_eq, kappa_S = T S,
 *   kappa*_j = kappa_j + w_j (kappa_eq_j - kappa_j) + (1 - w_j/2) kappa_S_j,
 *   f* = T^{-1} kappa*.                                                     */
static int cm_collide(const stencil *s, const mbasis *B, const double *rate, const double u[3],
                      const double *f, const double *feq, const double *S, double *fout)
{
    int q = s->q;
    double T[QMAX * QMAX], ks[QMAX], x[QMAX];
    build_T(s, B, u, T);
    for (int j = 0; j < q; ++j) {
        double k = 0.0, ke = 0.0, kS = 0.0;
        for (int i = 0; i < q; ++i) {
            k += T[j * q + i] * f[i];
            ke += T[j * q + i] * feq[i];
            kS += T[j * q + i] * S[i];
        }
        ks[j] = k + rate[j] * (ke - k) + (1.0 - 0.5 * rate[j]) * kS;
    }
    int rc = gauss_solve(q, T, ks, x);
    for (int i = 0; i < q; ++i) fout[i] = x[i];
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Parameters and state                                                      */
/* ------------------------------------------------------------------------ */
#define ORA_MAX_SOURCES 16

typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_y;     /* 1: no-slip walls at y = -1/2 and y = ny - 1/2; 0: periodic */
    int32_t q_pf;        /* 15 or 27 */
    int32_t q_thermal;   /* 7, 15, 19 or 27 */
    int32_t thermal;     /* 0: lattice Boltzmann, 1: RK2, 2: RK4 */
    int32_t pad;
    double rho_h, rho_l, nu_h, nu_l, mobility, xi;
    double sigma_ref, sigma_t, t_ref, kappa_h, kappa_l;
    double g[3];
    double omega_bulk;
    double u_wall_bot[3], u_wall_top[3];
    double t_wall_bot, t_wall_top;
    double normal_eps;
    double contact_angle_bot, contact_angle_top; /* degrees, through the heavy phase (R24) */
} ora_params;

typedef struct {
    double Q, x, y, z, w, dcut;
} ora_source;

typedef struct {
    ora_params P;
    const stencil *sh, *sg, *sf;
    mbasis Bh, Bg, Bf;
    int64_t N;
    double *h[2], *g[2], *f[2];
    double *phi[2]; /* phi[cur]: current phase field (phi^n) */
    double *u;      /* 3N, cell-major */
    double *T;
    double *Twb, *Twt; /* wall temperatures, nx*nz, x fastest */
    double wet_bot, wet_top; /* (4/xi) cos(contact angle) of the two walls */
    double *rk[4];     /* RK work fields */
    int cur;
    int nsrc;
    ora_source src[ORA_MAX_SOURCES];
    double omega_phi, tau_h, tau_l;
} ora_domain;

static int64_t cidx(const ora_domain *d, int x, int y, int z)
{
    return (int64_t)x + (int64_t)d->P.nx * ((int64_t)y + (int64_t)d->P.ny * z);
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* ------------------------------------------------------------------------ */
/* Material laws                                                             */
/* ------------------------------------------------------------------------ */
static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* rho(phi), linear interpolation with phi_L = 0, phi_H = 1 (Sec. 2.2) */
static double rho_of(const ora_params *P, double phic) { return P->rho_l + phic * (P->rho_h - P->rho_l); }
/* kappa(phi) (reading R7) */
static double kappa_of(const ora_params *P, double phic) { return P->kappa_l + phic * (P->kappa_h - P->kappa_l); }
/* sigma(T) = sigma_ref + sigma_T (T - T_ref) (Sec. 2.1) */
static double sigma_of(const ora_params *P, double T) { return P->sigma_ref + P->sigma_t * (T - P->t_ref); }

/* heat source q_T (Eq. HeatSource, reading R10) */
static double heat_source(const ora_domain *d, double x, double y, double z)
{
    double q = 0.0;
    for (int k = 0; k < d->nsrc; ++k) {
        const ora_source *s = &d->src[k];
        double d2 = (x - s->x) * (x - s->x) + (y - s->y) * (y - s->y) + (z - s->z) * (z - s->z);
        if (s->dcut > 0.0 && d2 > s->dcut * s->dcut) continue;
        q += s->Q * exp(-2.0 * d2 / (s->w * s->w));
    }
    return q;
}

/* ------------------------------------------------------------------------ */
/* Scalar fields with wall ghosts and isotropic finite differences (R17)     */
/* ------------------------------------------------------------------------ */
/* phi with a wetting ghost across the y walls (reading R24): the wall normal
 * derivative of phi is -cos(theta) |grad phi| with |grad phi| = 4 phi (1 - phi)/xi
 * (the tanh interface), taken one-sided between the ghost and the adjacent
 * cell: ghost = phi_adj + cos(theta) (4/xi) phi_adj (1 - phi_adj).  A contact
 * angle of 90 degrees gives the mirror ghost (reading R12). */
static double phi_at(const ora_domain *d, const double *phi, int x, int y, int z)
{
    x = wrap(x, d->P.nx);
    z = wrap(z, d->P.nz);
    if (d->P.walls_y) {
        if (y < 0) {
            const double v = phi[cidx(d, x, 0, z)];
            return v + d->wet_bot * v * (1.0 - v);
        }
        if (y >= d->P.ny) {
            const double v = phi[cidx(d, x, d->P.ny - 1, z)];
            return v + d->wet_top * v * (1.0 - v);
        }
    } else {
        y = wrap(y, d->P.ny);
    }
    return phi[cidx(d, x, y, z)];
}

/* temperature-like field with Dirichlet ghost 2 T_w - T across y walls (R11) */
static double temp_at(const ora_domain *d, const double *T, int x, int y, int z)
{
    x = wrap(x, d->P.nx);
    z = wrap(z, d->P.nz);
    if (d->P.walls_y) {
        if (y < 0) return 2.0 * d->Twb[x + d->P.nx * z] - T[cidx(d, x, 0, z)];
        if (y >= d->P.ny) return 2.0 * d->Twt[x + d->P.nx * z] - T[cidx(d, x, d->P.ny - 1, z)];
    } else {
        y = wrap(y, d->P.ny);
    }
    return T[cidx(d, x, y, z)];
}

typedef double (*field_at_fn)(const ora_domain *, const double *, int, int, int);

/* grad psi = (1/c_s^2) sum_i w_i e_i psi(x + e_i);
 * lap psi  = (2/c_s^2) sum_i w_i (psi(x + e_i) - psi(x)), D3Q27 weights.  */
static void iso_grad_lap(const ora_domain *d, field_at_fn at, const double *psi, int x, int y, int z,
                         double grad[3], double *lap)
{
    const stencil *s = &ST27;
    double c = at(d, psi, x, y, z);
    double gx = 0, gy = 0, gz = 0, l = 0;
    for (int i = 0; i < 27; ++i) {
        double v = at(d, psi, x + s->e[i][0], y + s->e[i][1], z + s->e[i][2]);
        gx += s->w[i] * s->e[i][0] * v;
        gy += s->w[i] * s->e[i][1] * v;
        gz += s->w[i] * s->e[i][2] * v;
        l += s->w[i] * (v - c);
    }
    grad[0] = gx / CS2;
    grad[1] = gy / CS2;
    grad[2] = gz / CS2;
    if (lap) *lap = 2.0 * l / CS2;
}

/* ------------------------------------------------------------------------ */
/* Equilibria                                                                */
/* ------------------------------------------------------------------------ */
/* second-order polynomial of the equilibria of Sec. 2.2 / Eq. lb_thermal */
static double eq_poly(const int e[3], const double u[3])
{
    double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
}

/* h_eq = phi w_i [1 + ...] (phase field), also used for f_eq with T */
static void eq_scalar(const stencil *s, double psi, const double u[3], double *out)
{
    for (int i = 0; i < s->q; ++i) out[i] = psi * s->w[i] * (1.0 + eq_poly(s->e[i], u));
}

/* incompressible g_eq = w_i (p* + [...]) (Sec. 2.2) */
static void eq_hydro(const stencil *s, double pstar, const double u[3], double *out)
{
    for (int i = 0; i < s->q; ++i) out[i] = s->w[i] * (pstar + eq_poly(s->e[i], u));
}

/* Guo source in velocity form (R15): S_i = w_i [(e_i - u)/c_s^2 + (e_i.u) e_i/c_s^4] . a */
static void guo_source(const stencil *s, const double u[3], const double acc[3], double *S)
{
    for (int i = 0; i < s->q; ++i) {
        double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
        double v = 0.0;
        for (int a = 0; a < 3; ++a) v += ((s->e[i][a] - u[a]) / CS2 + eu * s->e[i][a] / (CS2 * CS2)) * acc[a];
        S[i] = s->w[i] * v;
    }
}

/* ------------------------------------------------------------------------ */
/* Pull streaming with wall rules                                            */
/* ------------------------------------------------------------------------ */
/* Returns 1 when the link x - e_i crosses a y wall; *bottom tells which.    */
static int crosses_wall(const ora_domain *d, int y, const int e[3], int *bottom)
{
    if (!d->P.walls_y) return 0;
    int ys = y - e[1];
    if (ys < 0) { *bottom = 1; return 1; }
    if (ys >= d->P.ny) { *bottom = 0; return 1; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sub-step K1: phase-field LB (Eq. lb_interface, Eq. phasefieldforce)      */
/* ------------------------------------------------------------------------ */
static int step_phase_field(ora_domain *d)
{
    const stencil *s = d->sh;
    const int q = s->q, nx = d->P.nx, ny = d->P.ny, nz = d->P.nz;
    const double *hin = d->h[d->cur], *phi_old = d->phi[d->cur];
    double *hout = d->h[1 - d->cur], *phi_new = d->phi[1 - d->cur];
    double rate[QMAX];
    for (int j = 0; j < q; ++j) rate[j] = (d->Bh.r[j].order == 1) ? d->omega_phi : 1.0;
    int err = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : err)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(d, x, y, z);
                double hp[QMAX], heq[QMAX], S[QMAX], hn[QMAX];
                /* pull, halfway bounce-back at walls */
                for (int i = 0; i < q; ++i) {
                    int bot;
                    if (crosses_wall(d, y, s->e[i], &bot))
                        hp[i] = hin[c * q + s->opp[i]];
                    else
                        hp[i] = hin[cidx(d, wrap(x - s->e[i][0], nx), wrap(y - s->e[i][1], ny),
                                         wrap(z - s->e[i][2], nz)) * q + i];
                }
                double phi = 0.0;
                for (int i = 0; i < q; ++i) phi += hp[i];
                /* interface normal from the previous phase field (R18, R19) */
                double gr[3];
                iso_grad_lap(d, phi_at, phi_old, x, y, z, gr, NULL);
                double ne = d->P.normal_eps;
                double nrm = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + ne * ne);
                double lam = 4.0 * phi * (1.0 - phi) / d->P.xi;
                double F[3] = {lam * gr[0] / nrm, lam * gr[1] / nrm, lam * gr[2] / nrm};
                const double *u = &d->u[c * 3];
                eq_scalar(s, phi, u, heq);
                for (int i = 0; i < q; ++i)
                    S[i] = s->w[i] * (s->e[i][0] * F[0] + s->e[i][1] * F[1] + s->e[i][2] * F[2]);
                err |= cm_collide(s, &d->Bh, rate, u, hp, heq, S, hn);
                for (int i = 0; i < q; ++i) hout[c * q + i] = hn[i];
                phi_new[c] = phi;
            }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Sub-step K2: hydrodynamic LB with forces (Sec. 2.1, Sec. 2.2)            */
/* ------------------------------------------------------------------------ */
static int step_hydro(ora_domain *d)
{
    const stencil *s = d->sg;
    const int q = s->q, nx = d->P.nx, ny = d->P.ny, nz = d->P.nz;
    const ora_params *P = &d->P;
    const double *gin = d->g[d->cur];
    double *gout = d->g[1 - d->cur];
    const double *phi_old = d->phi[d->cur];
    const double drho = P->rho_h - P->rho_l;
    int err = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : err)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(d, x, y, z);
                double gp[QMAX], geq[QMAX], S[QMAX], gn[QMAX], rate[QMAX];
                for (int i = 0; i < q; ++i) {
                    int bot;
                    if (crosses_wall(d, y, s->e[i], &bot)) {
                        const double *uw = bot ? P->u_wall_bot : P->u_wall_top;
                        double eu = s->e[i][0] * uw[0] + s->e[i][1] * uw[1] + s->e[i][2] * uw[2];
                        gp[i] = gin[c * q + s->opp[i]] + 2.0 * s->w[i] * eu / CS2;
                    } else {
                        gp[i] = gin[cidx(d, wrap(x - s->e[i][0], nx), wrap(y - s->e[i][1], ny),
                                         wrap(z - s->e[i][2], nz)) * q + i];
                    }
                }
                /* zeroth and first moments: p* and the force-free velocity u0 */
                double pstar = 0.0, u0[3] = {0, 0, 0};
                for (int i = 0; i < q; ++i) {
                    pstar += gp[i];
                    for (int a = 0; a < 3; ++a) u0[a] += gp[i] * s->e[i][a];
                }
                /* phase field and temperature at the start of the step, phi^n and T^n (R18) */
                double phi = phi_old[c], gphi[3], lphi, T = d->T[c], gT[3];
                iso_grad_lap(d, phi_at, phi_old, x, y, z, gphi, &lphi);
                iso_grad_lap(d, temp_at, d->T, x, y, z, gT, NULL);
                double phic = clamp01(phi);
                double rho = rho_of(P, phic);
                double tau = d->tau_l + phic * (d->tau_h - d->tau_l);
                double omega = 1.0 / (tau + 0.5);
                double nu = tau * CS2;
                /* chemical potential and surface tension (R4, R5) */
                double sig = sigma_of(P, T);
                double beta = 12.0 * sig / P->xi, kap = 1.5 * sig * P->xi;
                double mu = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kap * lphi;
                double gp2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
                double gTgp = gT[0] * gphi[0] + gT[1] * gphi[1] + gT[2] * gphi[2];
                /* strain rate from the non-equilibrium second moment (R16) */
                double geq0[QMAX];
                eq_hydro(s, pstar, u0, geq0);
                double Sr[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double m = 0.0;
                        for (int i = 0; i < q; ++i) m += s->e[i][a] * s->e[i][b] * (gp[i] - geq0[i]);
                        Sr[a][b] = -omega / CS2 * m;
                    }
                double F[3];
                for (int a = 0; a < 3; ++a) {
                    double Fs = mu * gphi[a] + 1.5 * P->xi * P->sigma_t * (gp2 * gT[a] - gTgp * gphi[a]);
                    double Fb = rho * P->g[a];
                    double Fp = -pstar * CS2 * drho * gphi[a];
                    double Fm = nu * drho * (Sr[a][0] * gphi[0] + Sr[a][1] * gphi[1] + Sr[a][2] * gphi[2]);
                    F[a] = Fs + Fb + Fp + Fm;
                }
                double acc[3] = {F[0] / rho, F[1] / rho, F[2] / rho};
                double u[3] = {u0[0] + 0.5 * acc[0], u0[1] + 0.5 * acc[1], u0[2] + 0.5 * acc[2]};
                eq_hydro(s, pstar, u, geq);
                guo_source(s, u, acc, S);
                /* rates per moment (R14) */
                for (int j = 0; j < q; ++j) {
                    int tg = d->Bg.r[j].tag;
                    rate[j] = (tg == 2 || tg == 3) ? omega : (tg == 1 ? P->omega_bulk : 1.0);
                }
                err |= cm_collide(s, &d->Bg, rate, u, gp, geq, S, gn);
                for (int i = 0; i < q; ++i) gout[c * q + i] = gn[i];
                for (int a = 0; a < 3; ++a) d->u[c * 3 + a] = u[a];
            }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Sub-step K3: thermal LB (Eq. lb_thermal, Eq. thlbm-tau)                   */
/* ------------------------------------------------------------------------ */
static int step_thermal_lb(ora_domain *d)
{
    const stencil *s = d->sf;
    const int q = s->q, nx = d->P.nx, ny = d->P.ny, nz = d->P.nz;
    const double *fin = d->f[d->cur];
    double *fout = d->f[1 - d->cur];
    const double *phi_new = d->phi[1 - d->cur];
    int err = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : err)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(d, x, y, z);
                double fp[QMAX], feq[QMAX], S[QMAX], fn[QMAX], rate[QMAX];
                for (int i = 0; i < q; ++i) {
                    int bot;
                    if (crosses_wall(d, y, s->e[i], &bot)) {
                        double tw = bot ? d->Twb[x + nx * z] : d->Twt[x + nx * z];
                        fp[i] = -fin[c * q + s->opp[i]] + 2.0 * s->w[i] * tw;
                    } else {
                        fp[i] = fin[cidx(d, wrap(x - s->e[i][0], nx), wrap(y - s->e[i][1], ny),
                                         wrap(z - s->e[i][2], nz)) * q + i];
                    }
                }
                double T = 0.0;
                for (int i = 0; i < q; ++i) T += fp[i];
                const double *u = &d->u[c * 3];
                double kap = kappa_of(&d->P, clamp01(phi_new[c]));
                double omT = 1.0 / (0.5 + kap / CS2);
                eq_scalar(s, T, u, feq);
                for (int i = 0; i < q; ++i) S[i] = 0.0;
                for (int j = 0; j < q; ++j) rate[j] = (d->Bf.r[j].order == 1) ? omT : 1.0;
                err |= cm_collide(s, &d->Bf, rate, u, fp, feq, S, fn);
                double qT = heat_source(d, x, y, z);
                for (int i = 0; i < q; ++i) fout[c * q + i] = fn[i] + s->w[i] * qT;
                d->T[c] = T;
            }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Energy equation right-hand side (Eq. temperature with R7, R8, R17)       */
/*   R(Theta) = -u.grad Theta + grad kappa . grad Theta + kappa lap Theta + q_T */
/* ------------------------------------------------------------------------ */
static void energy_rhs(const ora_domain *d, const double *theta, double *out)
{
    const int nx = d->P.nx, ny = d->P.ny, nz = d->P.nz;
    const double *phi_new = d->phi[1 - d->cur];
    const double dk = d->P.kappa_h - d->P.kappa_l;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(d, x, y, z);
                double gth[3], lth, gphi[3];
                iso_grad_lap(d, temp_at, theta, x, y, z, gth, &lth);
                iso_grad_lap(d, phi_at, phi_new, x, y, z, gphi, NULL);
                const double *u = &d->u[c * 3];
                double kap = kappa_of(&d->P, clamp01(phi_new[c]));
                double adv = u[0] * gth[0] + u[1] * gth[1] + u[2] * gth[2];
                double cond = dk * (gphi[0] * gth[0] + gphi[1] * gth[1] + gphi[2] * gth[2]);
                out[c] = -adv + cond + kap * lth + heat_source(d, x, y, z);
            }
}

/* Eq. rk4 (classical) and Eq. rk2 read as the midpoint rule (R9) */
static void step_thermal_rk(ora_domain *d)
{
    int64_t N = d->N;
    double *k = d->rk[0], *th = d->rk[1], *acc = d->rk[2];
    if (d->P.thermal == 1) {
        energy_rhs(d, d->T, k);
        for (int64_t c = 0; c < N; ++c) th[c] = d->T[c] + 0.5 * k[c];
        energy_rhs(d, th, k);
        for (int64_t c = 0; c < N; ++c) d->T[c] += k[c];
        return;
    }
    /* RK4: K1..K4 with the stage values T^n + K/2, T^n + K/2, T^n + K */
    static const double stage_shift[3] = {0.5, 0.5, 1.0};
    static const double weight[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    for (int64_t c = 0; c < N; ++c) acc[c] = 0.0;
    const double *arg = d->T;
    for (int s = 0; s < 4; ++s) {
        energy_rhs(d, arg, k);
        for (int64_t c = 0; c < N; ++c) {
            acc[c] += weight[s] * k[c];
            if (s < 3) th[c] = d->T[c] + stage_shift[s] * k[c];
        }
        arg = th;
    }
    for (int64_t c = 0; c < N; ++c) d->T[c] += acc[c];
}

/* ------------------------------------------------------------------------ */
/* Public C interface used by the Python test harness                       */
/* ------------------------------------------------------------------------ */
void ora_destroy(ora_domain *d);

/* cosine of an angle in degrees, exactly zero at 90 */
static double cos_deg(double a)
{
    return a == 90.0 ? 0.0 : cos(a * (3.14159265358979323846 / 180.0));
}

ora_domain *ora_create(const ora_params *P)
{
    init_stencils();
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return NULL;
    if (P->q_pf != 15 && P->q_pf != 27) return NULL;
    if (!get_stencil(P->q_thermal)) return NULL;
    if (P->thermal < 0 || P->thermal > 2) return NULL;
    ora_domain *d = (ora_domain *)calloc(1, sizeof(ora_domain));
    if (!d) return NULL;
    d->P = *P;
    d->sh = get_stencil(P->q_pf);
    d->sg = get_stencil(27);
    d->wet_bot = 4.0 / P->xi * cos_deg(P->contact_angle_bot);
    d->wet_top = 4.0 / P->xi * cos_deg(P->contact_angle_top);
    d->sf = get_stencil(P->q_thermal);
    basis_monomials(P->q_pf, &d->Bh);
    basis_hydro(&d->Bg);
    basis_monomials(P->q_thermal, &d->Bf);
    d->N = (int64_t)P->nx * P->ny * P->nz;
    int64_t N = d->N;
    int ok = 1;
    for (int b = 0; b < 2; ++b) {
        ok &= (d->h[b] = (double *)calloc((size_t)N * d->sh->q, sizeof(double))) != NULL;
        ok &= (d->g[b] = (double *)calloc((size_t)N * 27, sizeof(double))) != NULL;
        ok &= (d->f[b] = (double *)calloc((size_t)N * d->sf->q, sizeof(double))) != NULL;
        ok &= (d->phi[b] = (double *)calloc((size_t)N, sizeof(double))) != NULL;
    }
    ok &= (d->u = (double *)calloc((size_t)N * 3, sizeof(double))) != NULL;
    ok &= (d->T = (double *)calloc((size_t)N, sizeof(double))) != NULL;
    ok &= (d->Twb = (double *)calloc((size_t)P->nx * P->nz, sizeof(double))) != NULL;
    ok &= (d->Twt = (double *)calloc((size_t)P->nx * P->nz, sizeof(double))) != NULL;
    for (int k = 0; k < 3; ++k) ok &= (d->rk[k] = (double *)calloc((size_t)N, sizeof(double))) != NULL;
    if (!ok) { ora_destroy(d); return NULL; }
    for (int64_t k = 0; k < (int64_t)P->nx * P->nz; ++k) {
        d->Twb[k] = P->t_wall_bot;
        d->Twt[k] = P->t_wall_top;
    }
    /* R1, R2 */
    d->omega_phi = 1.0 / (0.5 + P->mobility / CS2);
    d->tau_h = P->nu_h / CS2;
    d->tau_l = P->nu_l / CS2;
    return d;
}

void ora_destroy(ora_domain *d)
{
    if (!d) return;
    for (int b = 0; b < 2; ++b) { free(d->h[b]); free(d->g[b]); free(d->f[b]); free(d->phi[b]); }
    free(d->u); free(d->T); free(d->Twb); free(d->Twt);
    for (int k = 0; k < 3; ++k) free(d->rk[k]);
    free(d);
}

/* which: 0 phi, 1 ux, 2 uy, 3 uz, 4 T; host arrays in x-fastest order */
int ora_set_field(ora_domain *d, int which, const double *src)
{
    int64_t N = d->N;
    switch (which) {
    case 0: for (int64_t c = 0; c < N; ++c) d->phi[d->cur][c] = src[c]; return 0;
    case 1: case 2: case 3:
        for (int64_t c = 0; c < N; ++c) d->u[c * 3 + which - 1] = src[c];
        return 0;
    case 4: for (int64_t c = 0; c < N; ++c) d->T[c] = src[c]; return 0;
    default: return -1;
    }
}

/* Initial phase field from spherical droplets (Sec. 3.1 interface profile,
 * reading R21): phi = max_k [1/2 + 1/2 tanh(2 (R_k - r_k)/xi)].  The box is
 * the part of a global domain of size gdim starting at origin; distances use
 * the minimum image along the global periodic axes.  drops: n x 4 (x,y,z,R). */
int ora_set_droplets(ora_domain *d, const double *drops, int n, const int64_t gdim[3],
                     const int64_t origin[3], const int32_t periodic[3])
{
    const int nx = d->P.nx, ny = d->P.ny, nz = d->P.nz;
    double *phi = d->phi[d->cur];
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double pos[3] = {(double)(origin[0] + x), (double)(origin[1] + y), (double)(origin[2] + z)};
                double best = 0.0;
                for (int k = 0; k < n; ++k) {
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double dd = pos[a] - drops[4 * k + a];
                        if (periodic[a]) {
                            double L = (double)gdim[a];
                            dd = fmod(dd, L);
                            if (dd > 0.5 * L) dd -= L;
                            if (dd < -0.5 * L) dd += L;
                        }
                        r2 += dd * dd;
                    }
                    double v = 0.5 + 0.5 * tanh(2.0 * (drops[4 * k + 3] - sqrt(r2)) / d->P.xi);
                    if (k == 0 || v > best) best = v;
                }
                phi[cidx(d, x, y, z)] = (n > 0) ? best : 0.0;
            }
    return 0;
}

int ora_set_heat_sources(ora_domain *d, const double *s, int n)
{
    if (n < 0 || n > ORA_MAX_SOURCES) return -1;
    d->nsrc = n;
    for (int k = 0; k < n; ++k) {
        d->src[k].Q = s[6 * k + 0];
        d->src[k].x = s[6 * k + 1];
        d->src[k].y = s[6 * k + 2];
        d->src[k].z = s[6 * k + 3];
        d->src[k].w = s[6 * k + 4];
        d->src[k].dcut = s[6 * k + 5];
    }
    return 0;
}

/* wall 0: bottom (y = -1/2), 1: top (y = ny - 1/2); Tw has nx*nz values */
int ora_set_wall_temperature(ora_domain *d, int wall, const double *Tw)
{
    double *dst = wall == 0 ? d->Twb : (wall == 1 ? d->Twt : NULL);
    if (!dst) return -1;
    for (int64_t k = 0; k < (int64_t)d->P.nx * d->P.nz; ++k) dst[k] = Tw[k];
    return 0;
}

/* PDFs := equilibrium of the current fields with p* = 0 (R21) */
int ora_initialize(ora_domain *d)
{
    int64_t N = d->N;
    const int qh = d->sh->q, qf = d->sf->q;
    double *phi_cur = d->phi[d->cur];
    for (int64_t c = 0; c < N; ++c) {
        const double *u = &d->u[c * 3];
        eq_scalar(d->sh, phi_cur[c], u, &d->h[d->cur][c * qh]);
        eq_hydro(d->sg, 0.0, u, &d->g[d->cur][c * 27]);
        eq_scalar(d->sf, d->T[c], u, &d->f[d->cur][c * qf]);
        d->phi[1 - d->cur][c] = phi_cur[c];
    }
    return 0;
}

/* One step = K1 phase field, K2 hydrodynamics, K3 thermal LB or RK (Alg. 1/2) */
int ora_step(ora_domain *d, int64_t nsteps)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        int err = 0;
        err |= step_phase_field(d);
        err |= step_hydro(d);
        if (d->P.thermal == 0)
            err |= step_thermal_lb(d);
        else
            step_thermal_rk(d);
        if (err) return -2;
        d->cur = 1 - d->cur;
    }
    return 0;
}

/* Temperature initialisation (Sec. 4.1): phi and u are imposed, T is found by
 * running the thermal solver by itself until it settles.  Each update is the
 * thermal part of a step with phi^{n+1} = phi^n and u held; the change is the
 * largest |T_new - T_old| of one update, taken after every check_every updates
 * and after the last; the loop ends once it is at most tol or after max_steps. */
int ora_warm_temperature(ora_domain *d, int64_t max_steps, double tol, int64_t check_every, int64_t *steps_done,
                         double *change)
{
    if (max_steps < 0 || check_every < 1 || !(tol >= 0.0)) return -1;
    const int64_t N = d->N;
    const int start = d->cur;
    memcpy(d->phi[1 - start], d->phi[start], (size_t)N * sizeof(double));
    double *prev = malloc((size_t)N * sizeof(double));
    if (!prev) return -3;
    int64_t n = 0;
    double last = 0.0;
    int err = 0;
    while (n < max_steps) {
        memcpy(prev, d->T, (size_t)N * sizeof(double));
        if (d->P.thermal == 0) {
            err |= step_thermal_lb(d);
            d->cur = 1 - d->cur;
        } else {
            step_thermal_rk(d);
        }
        ++n;
        if (n % check_every == 0 || n == max_steps) {
            last = 0.0;
            for (int64_t c = 0; c < N; ++c) {
                const double dv = fabs(d->T[c] - prev[c]);
                if (dv > last || dv != dv) last = dv;
            }
            if (last <= tol) break;
        }
    }
    free(prev);
    /* the thermal PDFs go back to the parity of the other PDFs */
    if (d->cur != start) {
        const int qf = d->sf->q;
        memcpy(d->f[start], d->f[d->cur], (size_t)N * qf * sizeof(double));
        d->cur = start;
    }
    if (steps_done) *steps_done = n;
    if (change) *change = last;
    return err ? -2 : 0;
}

/* which: 0 phi, 1 ux, 2 uy, 3 uz, 4 p, 5 p*, 6 T, 7 rho */
int ora_get_field(const ora_domain *d, int which, double *out)
{
    int64_t N = d->N;
    const double *phi = d->phi[d->cur];
    const double *g = d->g[d->cur];
    for (int64_t c = 0; c < N; ++c) {
        double pstar = 0.0;
        if (which == 4 || which == 5)
            for (int i = 0; i < 27; ++i) pstar += g[c * 27 + i];
        double rho = rho_of(&d->P, clamp01(phi[c]));
        switch (which) {
        case 0: out[c] = phi[c]; break;
        case 1: case 2: case 3: out[c] = d->u[c * 3 + which - 1]; break;
        case 4: out[c] = pstar * rho * CS2; break;
        case 5: out[c] = pstar; break;
        case 6: out[c] = d->T[c]; break;
        case 7: out[c] = rho; break;
        default: return -1;
        }
    }
    return 0;
}

/* Post-collision PDFs of field 0 (h), 1 (g), 2 (f) in x-fastest SoA order:
 * out[i*N + c].                                                              */
int ora_get_pdfs(const ora_domain *d, int which, double *out)
{
    const double *src = which == 0 ? d->h[d->cur] : which == 1 ? d->g[d->cur] : which == 2 ? d->f[d->cur] : NULL;
    int q = which == 0 ? d->sh->q : which == 1 ? 27 : d->sf->q;
    if (!src) return -1;
    for (int64_t c = 0; c < d->N; ++c)
        for (int i = 0; i < q; ++i) out[(int64_t)i * d->N + c] = src[c * q + i];
    return 0;
}

int ora_set_pdfs(ora_domain *d, int which, const double *in)
{
    double *dst = which == 0 ? d->h[d->cur] : which == 1 ? d->g[d->cur] : which == 2 ? d->f[d->cur] : NULL;
    int q = which == 0 ? d->sh->q : which == 1 ? 27 : d->sf->q;
    if (!dst) return -1;
    for (int64_t c = 0; c < d->N; ++c)
        for (int i = 0; i < q; ++i) dst[c * q + i] = in[(int64_t)i * d->N + c];
    return 0;
}

/* FP64 mass and centroid with integer cell coordinates */
int ora_reduce(const ora_domain *d, double *mass, double centroid[3])
{
    const double *phi = d->phi[d->cur];
    double m = 0, cx = 0, cy = 0, cz = 0;
    for (int z = 0; z < d->P.nz; ++z)
        for (int y = 0; y < d->P.ny; ++y)
            for (int x = 0; x < d->P.nx; ++x) {
                double p = phi[cidx(d, x, y, z)];
                m += p; cx += p * x; cy += p * y; cz += p * z;
            }
    *mass = m;
    centroid[0] = cx / m; centroid[1] = cy / m; centroid[2] = cz / m;
    return 0;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Building blocks exposed for the pin tests                                 */
/* ------------------------------------------------------------------------ */
int ora_stencil(int q, int *e_out, double *w_out, int *opp_out)
{
    const stencil *s = get_stencil(q);
    if (!s) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) e_out[3 * i + a] = s->e[i][a];
        w_out[i] = s->w[i];
        opp_out[i] = s->opp[i];
    }
    return 0;
}

/* kind: 0 monomial basis of stencil q, 1 hydrodynamic basis (q = 27).
 * Writes T(u) (q x q, row-major), the order and tag of every row.           */
int ora_moment_matrix(int q, int kind, const double u[3], double *T, int *order, int *tag)
{
    const stencil *s = get_stencil(q);
    if (!s || (kind == 1 && q != 27)) return -1;
    mbasis B;
    if (kind == 1) basis_hydro(&B); else basis_monomials(q, &B);
    build_T(s, &B, u, T);
    for (int j = 0; j < q; ++j) { order[j] = B.r[j].order; tag[j] = B.r[j].tag; }
    return 0;
}

int ora_cm_collide(int q, int kind, const double *rate, const double u[3], const double *f,
                   const double *feq, const double *S, double *fout)
{
    const stencil *s = get_stencil(q);
    if (!s || (kind == 1 && q != 27)) return -1;
    mbasis B;
    if (kind == 1) basis_hydro(&B); else basis_monomials(q, &B);
    return cm_collide(s, &B, rate, u, f, feq, S, fout);
}

/* equilibria: kind 0 scalar (phi or T), 1 incompressible hydrodynamic */
int ora_equilibrium(int q, int kind, double zeroth, const double u[3], double *out)
{
    const stencil *s = get_stencil(q);
    if (!s) return -1;
    if (kind == 0) eq_scalar(s, zeroth, u, out); else eq_hydro(s, zeroth, u, out);
    return 0;
}

/* isotropic gradient and Laplacian (pin tests of R12, R11, R17); ghost 0: the
 * phase-field mirror ghost, 1: the Dirichlet temperature ghost */
int ora_iso_grad_lap(const ora_domain *d, const double *psi, int x, int y, int z, int ghost, double *grad,
                     double *lap)
{
    iso_grad_lap(d, ghost ? temp_at : phi_at, psi, x, y, z, grad, lap);
    return 0;
}

/* hydrodynamic Guo source (pin tests of R15) */
int ora_guo_source(const double u[3], const double acc[3], double *S)
{
    guo_source(get_stencil(27), u, acc, S);
    return 0;
}

/* heat-source density at a point (pin tests of R10) */
double ora_heat_source(const ora_domain *d, double x, double y, double z) { return heat_source(d, x, y, z); }
