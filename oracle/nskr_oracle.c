/*
 * nskr_oracle.c -- plain FP64 CPU reference of the DGSEM discretisation of the
 * relaxation models 1 and 2 of the non-isothermal Navier-Stokes-Korteweg
 * equations (Keim, Munz, Rohde, arXiv 2208.05310).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  It shares no code, header, table or helper with the HIP
 * path.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product never calls it.
 *
 * Everything is written to be read against the paper, not to be fast: loops
 * follow the order of the method, every quantity is FP64, and nothing is
 * blocked, fused or reordered beyond what the definitions state.  OpenMP is
 * used only to spread independent elements over threads; every global sum is
 * taken sequentially in element order.
 *
 * Paper passages followed (section numbers of the arXiv text):
 *   Sec. 2.1        van der Waals Helmholtz energy, pressure law, reduced
 *                   constants R=8/3, a=3, b=1/3, c_v (eq. helmholtzfreeenergyvol,
 *                   eq. pressure).
 *   Sec. 2.3.1      speed of sound (eq. speedofsound), Stokes hypothesis for
 *                   the viscous stress.
 *   Sec. 2.3.2      relaxation energy (eq. totalenergyalpha), chemical potential
 *                   and order-parameter source, simplified energy flux j_e,
 *                   relaxation model 1 fluxes F^C, F^V and source S
 *                   (eq. navierstokeskorteweg_p); relaxation model 2: the
 *                   modified pressure p_alpha (eq. modified_pressure) and its
 *                   fluxes and source (eq. navierstokeskorteweg_palpha).
 *   Sec. 2.4        wall boundary conditions of the relaxation model
 *                   (eq. bc_nsk_alpha), cubic wall energy and its derivative
 *                   (eq. helmfreesurftot_derivative), surface tension
 *                   (eq. surftenscoef, read with the factor sqrt(2*gamma)).
 *   Sec. 3.1        DGSEM on Legendre-Gauss nodes with collocation, Rusanov
 *                   flux (HLLC for model 2), BR1 lifting, point-wise non-conservative sources,
 *                   explicit low-storage RK4, CFL = 0.9 (Sec. 4 preamble).
 *   Sec. 3.2        boundary conditions enforced weakly through the face flux;
 *                   the tabulated sigma_vl for varying wall temperatures.
 *   Sec. 4.1.1      tanh droplet profile (eq. staticbubble1D).
 *   Sec. 4.3        colliding droplets with given velocities and bulk
 *                   densities (Tables 4, 5); Sec. 4.4.1 the liquid pillar
 *                   (a cylinder between two walls).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - rho*e is the conserved total energy of eq. totalenergyalpha, so the
 *     temperature needs the lifted grad c (a first BR1 pass), and grad theta
 *     needs a second pass.
 *   - Delta c in the order-parameter flux and in j_e is a BR1 divergence
 *     lifting of the lifted grad c, with a central face value.
 *   - Lifted variables are the primitives rho, u, v, w, c, then theta.
 *   - Face primitives come from the prolonged conserved state.
 *   - Rusanov wave speed uses sqrt(|c_s^2|) where c_s^2 < 0.
 *   - Walls: no-slip isothermal wall with static contact angle (possibly
 *     moving tangentially), slip adiabatic neutral wall (gamma_1 = gamma_4 = 0,
 *     so zeta_c = 0 on the wall), or the generalized Navier-slip wall of
 *     eq. bc_nsk_alpha with gamma_1, gamma_2, gamma_4 and either a fixed
 *     temperature or the heat-transfer condition with gamma_3.
 *   - A wall temperature that varies along the wall (linearly in x) or in
 *     time (linearly in t, evaluated at each RK stage's time t + c_s dt)
 *     takes sigma and the Maxwell states from the table of Sec. 3.2
 *     (15-point Gauss rule, 10000 points on [0.3, 1], linear interpolation),
 *     the Maxwell states tabulated alongside sigma.
 *   - Model 2 walls use the mirrored-ghost Rusanov flux with p_alpha and
 *     the wave speed sqrt(c_s^2 + alpha rho); interior faces the HLLC flux
 *     with Davis wave-speed estimates, c carried as a passive scalar.
 *   - Time integration: Carpenter-Kennedy 5-stage 2N-storage RK4(3)5.
 *   - Time step: advective limit with 1D Rusanov stability constants, and a
 *     parabolic/source limit with 1D BR1 spectral radii.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXP 10 /* polynomial degree up to 9 */

/* ------------------------------------------------------------------------ */
/* Parameter and mesh descriptions (plain structs, passed from Python).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double R, a, b, cv;       /* van der Waals constants (Sec. 2.1)          */
    double mu, kappa, gam;    /* viscosity, heat conductivity, capillarity   */
    double alpha, beta;       /* Korteweg and relaxation parameters          */
    double cfl;               /* CFL number (0.9 in the paper)               */
    int model;                /* relaxation model 1 (0 reads as 1) or 2      */
} orc_params;

typedef struct {
    int N;                    /* polynomial degree                            */
    int n[3];                 /* elements per direction                       */
    double lo[3], len[3];     /* box origin and extent                        */
    int periodic[3];          /* 1 = periodic along that axis                 */
    int side_kind[6];         /* x-,x+,y-,y+,z-,z+ : 1 no-slip isothermal with
                                 contact angle, 2 slip adiabatic neutral,
                                 3 generalized Navier slip (eq. bc_nsk_alpha) */
    double side_twall[6];     /* wall temperature (kinds 1, 3)                */
    double side_theta[6];     /* static contact angle in degrees (kinds 1, 3) */
    double curve_amp;         /* amplitude of the smooth sine perturbation    */
    double side_uwall[6][3];  /* wall velocity (kinds 1, 3; tangential)       */
    double side_g1[6], side_g2[6], side_g4[6]; /* gamma_1, gamma_2, gamma_4 (kind 3) */
    double side_g3[6];        /* gamma_3 (kind 3); infinite = isothermal wall */
    double side_tgrad[6][3];  /* wall temperature gradient (kinds 1, 3): the
                                 wall temperature at x is twall + tgrad . x,
                                 evaluated through the sigma/Maxwell table  */
    double side_trate[6];     /* wall temperature rate: + trate * t          */
    int ngeo;                 /* geometry degree: each element is the degree-ngeo
                                 interpolant of the map through its Gauss-Lobatto
                                 points (0 or >= N: degree N)                 */
} orc_box;

typedef struct {
    int N, P, n2, n3, E;
    orc_params pr;
    orc_box box;
    /* 1D Gauss ingredients */
    double xg[MAXP], wg[MAXP];
    double D[MAXP][MAXP];     /* D_ij = l_j'(x_i)                              */
    double Dh[MAXP][MAXP];    /* Dhat_ij = -(w_j/w_i) D_ji                     */
    double lm[MAXP], lp[MAXP];   /* l_j(-1), l_j(+1)                          */
    double lhm[MAXP], lhp[MAXP]; /* l_j(-1)/w_j, l_j(+1)/w_j                  */
    /* mesh */
    int *nbr;                 /* [E][6] neighbour element, -1 on a wall       */
    int *kind;                /* [E][6] 0 interior/periodic, 1/2 wall kinds   */
    int *side;                /* [E][6] box side index of a wall face, else -1 */
    double *Ja;               /* [E][n3][3][3]  Ja[d][m] = J d xi^d / d x_m    */
    double *J;                /* [E][n3]                                      */
    double *nv;               /* [E][6][n2][3] outward n dS                    */
    double *xyz;              /* [E][n3][3]                                   */
    /* wall constants per box side: Maxwell states, sigma, cos(theta) */
    double wrv[6], wrl[6], wsig[6], wcos[6];
    int wvar[6];              /* side with a varying wall temperature        */
    double time;              /* time at which orc_rhs evaluates (walls whose
                                 temperature changes in time); orc_rk_step
                                 sets it to each stage's time               */
    double *stab;             /* [ORC_NTAB][3] sigma/sqrt(2 gamma), rv, rl   */
} orc_ctx;

/* Wall-temperature table of Sec. 3.2: ORC_NTAB equidistant temperatures on
 * [0.3, 1]; sigma by the 15-point Gauss rule, linear interpolation. */
#define ORC_NTAB 10000
#define ORC_TAB_T0 0.3
#define ORC_TAB_T1 1.0

/* ------------------------------------------------------------------------ */
/* 1D polynomial machinery (Sec. 3.1: Lagrange basis on Legendre-Gauss       */
/* nodes, collocated Gauss quadrature).                                      */
/* ------------------------------------------------------------------------ */
static void legendre(int n, double x, double *Pn, double *dPn)
{
    /* Bonnet recursion for P_n and its derivative. */
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *Pn = 1.0; *dPn = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        double d2 = d0 + (2.0 * k - 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *Pn = p1; *dPn = d1;
}

/* Legendre-Gauss nodes and weights with N+1 points, ascending. */
static void gauss_nodes(int N, double *x, double *w)
{
    int n = N + 1;
    for (int i = 0; i < n; ++i) {
        double xi = -cos((2.0 * i + 1.0) * M_PI / (2.0 * n));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, xi, &P, &dP);
            double dx = P / dP;
            xi -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double P, dP;
        legendre(n, xi, &P, &dP);
        x[i] = xi;
        w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
    }
}

/* Legendre-Gauss-Lobatto nodes with N+1 points (geometry interpolation). */
static void lobatto_nodes(int N, double *x)
{
    x[0] = -1.0; x[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double xi = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            /* roots of P_N'(x): Newton on q = P_N', q' from Legendre's ODE */
            double P, dP;
            legendre(N, xi, &P, &dP);
            double d2P = (2.0 * xi * dP - N * (N + 1.0) * P) / (1.0 - xi * xi);
            double dx = dP / d2P;
            xi -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        x[i] = xi;
    }
}

/* l_j(x) for the nodes xn[0..n-1], by the product formula. */
static double lagrange(int n, const double *xn, int j, double x)
{
    double v = 1.0;
    for (int k = 0; k < n; ++k)
        if (k != j) v *= (x - xn[k]) / (xn[j] - xn[k]);
    return v;
}

/* Differentiation matrix D_ij = l_j'(x_i) from barycentric weights; the
 * diagonal is minus the off-diagonal row sum (exact for constants). */
static void diff_matrix(int n, const double *xn, double D[MAXP][MAXP])
{
    double lam[MAXP];
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (xn[j] - xn[k]);
        lam[j] = 1.0 / p;
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i][j] = (lam[j] / lam[i]) / (xn[i] - xn[j]);
            s += D[i][j];
        }
        D[i][i] = -s;
    }
}

/* ------------------------------------------------------------------------ */
/* Index helpers.  Node (i,j,k) with i along xi^1; element-local index        */
/* i + P*(j + P*k).  Face f = 2d + s (d = direction, s = 0 at xi^d = -1,      */
/* s = 1 at +1).  Face point (p,q) = the two remaining indices in increasing  */
/* order, stored as p + P*q.                                                  */
/* ------------------------------------------------------------------------ */
static inline int nidx(int P, int i, int j, int k) { return i + P * (j + P * k); }

static inline int line_node(int P, int d, int l, int p, int q)
{
    if (d == 0) return nidx(P, l, p, q);
    if (d == 1) return nidx(P, p, l, q);
    return nidx(P, p, q, l);
}

/* For node (i,j,k) and direction d: its index along d and its face point. */
static inline void node_split(int P, int node, int d, int *l, int *fp)
{
    int i = node % P, j = (node / P) % P, k = node / (P * P);
    if (d == 0) { *l = i; *fp = j + P * k; }
    else if (d == 1) { *l = j; *fp = i + P * k; }
    else { *l = k; *fp = i + P * j; }
}

/* ------------------------------------------------------------------------ */
/* Thermodynamics of the reduced van der Waals fluid (Sec. 2.1, 2.3.1).       */
/* ------------------------------------------------------------------------ */
static double vdw_p(const orc_params *pr, double rho, double T)
{
    return rho * pr->R * T / (1.0 - pr->b * rho) - pr->a * rho * rho;
}

/* Isothermal pressure derivative (dp/drho)_T = rho * psi''. */
static double vdw_dpdrho_T(const orc_params *pr, double rho, double T)
{
    double q = 1.0 - pr->b * rho;
    return pr->R * T / (q * q) - 2.0 * pr->a * rho;
}

/* Square of the isentropic speed of sound, eq. speedofsound evaluated for the
 * Helmholtz energy of Sec. 2.1: (1 + 1/c_v) R T / (1 - b rho)^2 - 2 a rho. */
static double vdw_cs2(const orc_params *pr, double rho, double T)
{
    double q = 1.0 - pr->b * rho;
    return (1.0 + 1.0 / pr->cv) * pr->R * T / (q * q) - 2.0 * pr->a * rho;
}

/* rho-dependent part of the chemical potential d psi / d rho at fixed T. */
static double vdw_mu(const orc_params *pr, double rho, double T)
{
    double q = 1.0 - pr->b * rho;
    return pr->R * T * log(pr->b * rho / q) + pr->R * T / q - 2.0 * pr->a * rho;
}

/* Part of psi(rho,T) that is not linear in rho (linear parts cancel against
 * the bitangent in eq. surftenscoef). */
static double vdw_psi_nl(const orc_params *pr, double rho, double T)
{
    return rho * pr->R * T * log(pr->b * rho / (1.0 - pr->b * rho)) - pr->a * rho * rho;
}

/* Spinodal densities: zeros of (dp/drho)_T (Sec. 2.1), found by bisection on
 * both sides of the maximum of R T / ((1-b rho)^2 2 a rho).  Returns 0 when
 * T is supercritical. */
int orc_spinodal(double R, double a, double b, double T, double *rsv, double *rsl)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    /* g(rho) = (dp/drho)_T is positive near 0 and near 1/b and has a single
     * minimum inside; locate the minimum by golden search, then bisect. */
    double lo = 1e-12, hi = 1.0 / b - 1e-12;
    double gr = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    for (int it = 0; it < 300; ++it) {
        if (vdw_dpdrho_T(&pr, x1, T) < vdw_dpdrho_T(&pr, x2, T)) { hi = x2; }
        else { lo = x1; }
        x1 = hi - gr * (hi - lo); x2 = lo + gr * (hi - lo);
    }
    double rmin = 0.5 * (lo + hi);
    if (vdw_dpdrho_T(&pr, rmin, T) >= 0.0) return 0;
    double A = 1e-12, B = rmin;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (A + B);
        if (vdw_dpdrho_T(&pr, m, T) > 0.0) A = m; else B = m;
    }
    *rsv = 0.5 * (A + B);
    A = rmin; B = 1.0 / b - 1e-12;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (A + B);
        if (vdw_dpdrho_T(&pr, m, T) < 0.0) A = m; else B = m;
    }
    *rsl = 0.5 * (A + B);
    return 1;
}

/* Root of p(rho) = p0 on the branch [A,B] where p is increasing. */
static double root_increasing(const orc_params *pr, double T, double p0, double A, double B)
{
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (A + B);
        if (vdw_p(pr, m, T) < p0) A = m; else B = m;
    }
    return 0.5 * (A + B);
}

/* Inverse of the pressure law rho(T, p) on the vapour (branch 0) or liquid
 * (branch 1) side of the spinodal, as used for the Young-Laplace adjusted
 * densities of Sec. 4.3. */
double orc_rho_of_p(double R, double a, double b, double T, double p, int branch)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    double rsv, rsl;
    if (!orc_spinodal(R, a, b, T, &rsv, &rsl)) return NAN;
    if (branch == 0) return root_increasing(&pr, T, p, 1e-14, rsv);
    return root_increasing(&pr, T, p, rsl, 1.0 / b - 1e-14);
}

/* Maxwell construction (Sec. 2.1): equal pressure and equal chemical
 * potential of vapour and liquid.  Plain nested bisection: for a trial
 * pressure p the two branch roots rho_v(p), rho_l(p) are found by bisection,
 * and mu(rho_l) - mu(rho_v), which decreases monotonically in p, is bisected
 * to zero. */
int orc_maxwell(double R, double a, double b, double T, double *rv, double *rl, double *psat)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    double rsv, rsl;
    if (!orc_spinodal(R, a, b, T, &rsv, &rsl)) return 0;
    double plo = vdw_p(&pr, rsl, T), phi = vdw_p(&pr, rsv, T);
    if (plo < 0.0) plo = 0.0;
    for (int it = 0; it < 200; ++it) {
        double pm = 0.5 * (plo + phi);
        double v = root_increasing(&pr, T, pm, 1e-14, rsv);
        double l = root_increasing(&pr, T, pm, rsl, 1.0 / b - 1e-14);
        double f = vdw_mu(&pr, l, T) - vdw_mu(&pr, v, T);
        if (f > 0.0) plo = pm; else phi = pm;
        if (phi - plo <= 0.0) break;
    }
    double pm = 0.5 * (plo + phi);
    *rv = root_increasing(&pr, T, pm, 1e-14, rsv);
    *rl = root_increasing(&pr, T, pm, rsl, 1.0 / b - 1e-14);
    if (psat) *psat = pm;
    return 1;
}

/* Integrand sqrt(psi - psi_M) of eq. surftenscoef. */
static double sigma_integrand(const orc_params *pr, double T, double rv, double rho)
{
    double psiM = vdw_psi_nl(pr, rv, T) + (rho - rv) * vdw_mu(pr, rv, T);
    double d = vdw_psi_nl(pr, rho, T) - psiM;
    return d > 0.0 ? sqrt(d) : 0.0;
}

/* Equilibrium surface tension sigma_vl(T) of eq. surftenscoef, with the
 * prefactor read as sqrt(2 gamma) (the printed sqrt(2/gamma) contradicts the
 * tabulated sigma values).  The integrand is analytic on [rho_v, rho_l]
 * (it vanishes linearly at both ends), so a composite Gauss-Legendre rule
 * converges spectrally; npanel panels of 20 points each. */
double orc_sigma_panels(double R, double a, double b, double T, double gam, int npanel)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    double rv, rl, x[32], w[32];
    if (!orc_maxwell(R, a, b, T, &rv, &rl, NULL)) return 0.0;
    gauss_nodes(19, x, w);
    double h = (rl - rv) / npanel, I = 0.0;
    for (int k = 0; k < npanel; ++k) {
        double A = rv + k * h, s = 0.0;
        for (int i = 0; i < 20; ++i)
            s += w[i] * sigma_integrand(&pr, T, rv, A + 0.5 * h * (x[i] + 1.0));
        I += 0.5 * h * s;
    }
    return sqrt(2.0 * gam) * I;
}

double orc_sigma(double R, double a, double b, double T, double gam)
{
    return orc_sigma_panels(R, a, b, T, gam, 64);
}

/* The same integral with a single 15-point Gauss rule, the quadrature the
 * paper states for its tabulation (Sec. 3.2); reported beside the reference. */
double orc_sigma_gauss15(double R, double a, double b, double T, double gam)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    double rv, rl, x[32], w[32];
    if (!orc_maxwell(R, a, b, T, &rv, &rl, NULL)) return 0.0;
    gauss_nodes(14, x, w);
    double I = 0.0;
    for (int i = 0; i < 15; ++i) {
        double rho = 0.5 * (rv + rl) + 0.5 * (rl - rv) * x[i];
        I += 0.5 * (rl - rv) * w[i] * sigma_integrand(&pr, T, rv, rho);
    }
    return sqrt(2.0 * gam) * I;
}

/* Entry k of the wall-temperature table at T_k = 0.3 + k (0.7/(ORC_NTAB-1)):
 * sigma/sqrt(2 gamma) by the 15-point Gauss rule over [rv, rl] and the
 * Maxwell states; the last entry is the critical point (sigma = 0, rv = rl =
 * 1/(3b)). */
static void table_entry(double R, double a, double b, int k, double out[3])
{
    double T = ORC_TAB_T0 + k * ((ORC_TAB_T1 - ORC_TAB_T0) / (ORC_NTAB - 1));
    double rv, rl;
    if (k == ORC_NTAB - 1 || !orc_maxwell(R, a, b, T, &rv, &rl, NULL)) {
        out[0] = 0.0; out[1] = out[2] = 1.0 / (3.0 * b);
        return;
    }
    out[0] = orc_sigma_gauss15(R, a, b, T, 0.5);  /* sqrt(2 gamma) = 1 */
    out[1] = rv; out[2] = rl;
}

void orc_table_build(double R, double a, double b, double *tab)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int k = 0; k < ORC_NTAB; ++k) table_entry(R, a, b, k, tab + 3 * k);
}

/* Linear interpolation in the table at temperature T (clamped to the grid). */
void orc_table_lookup(const double *tab, double T, double out[3])
{
    double sx = (T - ORC_TAB_T0) / ((ORC_TAB_T1 - ORC_TAB_T0) / (ORC_NTAB - 1));
    int k = (int)floor(sx);
    if (k < 0) k = 0;
    if (k > ORC_NTAB - 2) k = ORC_NTAB - 2;
    double w = sx - k;
    for (int v = 0; v < 3; ++v) out[v] = (1.0 - w) * tab[3 * k + v] + w * tab[3 * (k + 1) + v];
}

/* Derivative of the cubic wall energy, eq. helmfreesurftot_derivative. */
double orc_dpsiwall_dc(double c, double rv, double rl, double sigma, double costheta)
{
    double d = rl - rv;
    return 6.0 * (c - rl) * (c - rv) / (d * d * d) * sigma * costheta;
}

/* The cubic wall energy itself (used by the tests of its defining
 * properties); sigma_sv and sigma_sl are the two wall energies. */
double orc_psiwall(double c, double rv, double rl, double ssv, double ssl)
{
    double d = rl - rv;
    return ((c - rl) * (c - rl) * (2.0 * c + rl - 3.0 * rv) * ssv -
            (c - rv) * (c - rv) * (2.0 * c + rv - 3.0 * rl) * ssl) / (d * d * d);
}

/* ------------------------------------------------------------------------ */
/* Point-wise physics of relaxation model 1 (Sec. 2.3.2).                     */
/* ------------------------------------------------------------------------ */

/* Temperature from eq. totalenergyalpha: rho*e minus kinetic, relaxation and
 * gradient energy gives rho*eps, and eps = R c_v T - a rho (the internal
 * energy of the Helmholtz energy of Sec. 2.1). */
static double temperature(const orc_params *pr, const double U[6], const double qc[3])
{
    double rho = U[0];
    double kin = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
    double rel = 0.5 * pr->alpha * (rho - U[5]) * (rho - U[5]);
    double grd = 0.5 * pr->gam * (qc[0] * qc[0] + qc[1] * qc[1] + qc[2] * qc[2]);
    double reps = U[4] - kin - rel - grd;
    return (reps / rho + pr->a * rho) / (pr->R * pr->cv);
}

/* Pressure in the convective flux: p for relaxation model 1; for model 2 the
 * modified pressure p_alpha = p + alpha/2 rho^2 of eq. modified_pressure. */
static double p_conv(const orc_params *pr, double rho, double T)
{
    double p = vdw_p(pr, rho, T);
    return pr->model == 2 ? p + 0.5 * pr->alpha * rho * rho : p;
}

/* Speed of sound of the convective flux, sqrt(|(dp/drho)_s|) (reading Q3 for
 * model 1); model 2 uses p_alpha, whose derivative adds alpha rho (the
 * eigenvalues u.n +- sqrt((dp_alpha/drho)_s) of Sec. 2.3.2). */
static double wave_speed(const orc_params *pr, double rho, double T)
{
    double a2 = vdw_cs2(pr, rho, T);
    if (pr->model == 2) a2 += pr->alpha * rho;
    return sqrt(fabs(a2));
}

/* Full local state needed for the fluxes at one point. */
typedef struct {
    double U[6];
    double T;
    double gu[3][3];   /* gu[j][i] = d u_j / d x_i (lifted) */
    double gT[3];      /* lifted grad theta                  */
    double gc[3];      /* lifted grad c                       */
    double lapc;       /* lifted div(grad c)                  */
} point_state;

/* Convective flux F^{C,i}, i = 0..2, of eq. navierstokeskorteweg_p (model 1)
 * or eq. navierstokeskorteweg_palpha (model 2, p replaced by p_alpha). */
static void flux_conv(const orc_params *pr, const point_state *s, double Fc[3][6])
{
    double rho = s->U[0];
    double u[3] = {s->U[1] / rho, s->U[2] / rho, s->U[3] / rho};
    double p = p_conv(pr, rho, s->T);
    for (int i = 0; i < 3; ++i) {
        Fc[i][0] = s->U[1 + i];
        for (int j = 0; j < 3; ++j)
            Fc[i][1 + j] = s->U[1 + i] * u[j] + (i == j ? p : 0.0);
        Fc[i][4] = (s->U[4] + p) * u[i];
        Fc[i][5] = s->U[5] * u[i];
    }
}

/* Viscous stress with the Stokes hypothesis (Sec. 2.3.1). */
static void viscous_stress(const orc_params *pr, const double gu[3][3], double Tv[3][3])
{
    double div = gu[0][0] + gu[1][1] + gu[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Tv[i][j] = pr->mu * (gu[i][j] + gu[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
}

/* Viscous flux F^{V,i} of eq. navierstokeskorteweg_p with the simplified
 * energy flux j_e = k grad T - gamma c grad c div u + gamma grad c zeta_c,
 * zeta_c = -beta chi_c = beta (gamma lap c + alpha (rho - c)). */
static void flux_visc(const orc_params *pr, const point_state *s, double Fv[3][6])
{
    double rho = s->U[0], c = s->U[5];
    double u[3] = {s->U[1] / rho, s->U[2] / rho, s->U[3] / rho};
    double Tv[3][3];
    viscous_stress(pr, s->gu, Tv);
    double div = s->gu[0][0] + s->gu[1][1] + s->gu[2][2];
    double zeta = pr->beta * (pr->gam * s->lapc + pr->alpha * (rho - c));
    for (int i = 0; i < 3; ++i) {
        double je = pr->kappa * s->gT[i] - pr->gam * c * s->gc[i] * div + pr->gam * s->gc[i] * zeta;
        Fv[i][0] = 0.0;
        for (int j = 0; j < 3; ++j) Fv[i][1 + j] = Tv[j][i];
        Fv[i][4] = Tv[i][0] * u[0] + Tv[i][1] * u[1] + Tv[i][2] * u[2] + je;
        Fv[i][5] = pr->gam * pr->beta * s->gc[i];
    }
}

/* Non-conservative source S of eq. navierstokeskorteweg_p (model 1), or of
 * eq. navierstokeskorteweg_palpha (model 2: the alpha rho grad rho and
 * alpha/2 rho^2 div u parts moved into p_alpha), evaluated point-wise with
 * the lifted gradients (Sec. 3.1). */
static void source(const orc_params *pr, const double U[6], const double grho[3],
                   const double gu[3][3], const double gc[3], double S[6])
{
    double rho = U[0], c = U[5];
    double u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
    double div = gu[0][0] + gu[1][1] + gu[2][2];
    if (pr->model == 2) {
        double gc2 = gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2];
        double cc = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) cc += gc[i] * gc[j] * gu[j][i];
        S[0] = 0.0;
        for (int m = 0; m < 3; ++m) S[1 + m] = pr->alpha * rho * gc[m];
        S[4] = pr->alpha * rho * (gc[0] * u[0] + gc[1] * u[1] + gc[2] * u[2]) + 0.5 * pr->alpha * c * c * div +
               pr->gam * (0.5 * gc2 * div - cc);
        S[5] = pr->alpha * pr->beta * (rho - c);
        return;
    }
    double d[3] = {gc[0] - grho[0], gc[1] - grho[1], gc[2] - grho[2]};
    double gc2 = gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2];
    double cc = 0.0; /* grad c (x) grad c : grad (x) u = sum_ij c_i c_j du_j/dx_i */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) cc += gc[i] * gc[j] * gu[j][i];
    S[0] = 0.0;
    for (int m = 0; m < 3; ++m) S[1 + m] = pr->alpha * rho * d[m];
    S[4] = pr->alpha * rho * (d[0] * u[0] + d[1] * u[1] + d[2] * u[2]) +
           0.5 * pr->alpha * (c * c - rho * rho) * div + pr->gam * (0.5 * gc2 * div - cc);
    S[5] = pr->alpha * pr->beta * (rho - c);
}

/* ------------------------------------------------------------------------ */
/* Mesh and metric terms.                                                    */
/* ------------------------------------------------------------------------ */

/* Geometry map of the box: element-wise affine reference box, optionally
 * perturbed by amp * sin(2 pi X1/L1) sin(2 pi X2/L2) sin(2 pi X3/L3) added to
 * every component (a smooth curved mesh with the same periodicity).
 * Evaluated in extended precision (the metric terms below are too). */
typedef long double ldbl;

static void geom_map(const orc_box *bx, const ldbl X[3], ldbl x[3])
{
    ldbl s = 1.0L;
    for (int d = 0; d < 3; ++d) s *= sinl(2.0L * 3.14159265358979323846264338327950288L * (X[d] - bx->lo[d]) / bx->len[d]);
    for (int d = 0; d < 3; ++d) x[d] = X[d] + (ldbl)bx->curve_amp * s;
}

static void lobatto_nodes_ld(int N, ldbl *x)
{
    x[0] = -1.0L; x[N] = 1.0L;
    for (int i = 1; i < N; ++i) {
        ldbl xi = -cosl(3.14159265358979323846264338327950288L * i / N);
        for (int it = 0; it < 100; ++it) {
            ldbl p0 = 1.0L, p1 = xi, d0 = 0.0L, d1 = 1.0L;
            for (int k = 2; k <= N; ++k) {
                ldbl p2 = ((2.0L * k - 1.0L) * xi * p1 - (k - 1.0L) * p0) / k;
                ldbl d2 = d0 + (2.0L * k - 1.0L) * p1;
                p0 = p1; p1 = p2; d0 = d1; d1 = d2;
            }
            ldbl d2P = (2.0L * xi * d1 - N * (N + 1.0L) * p1) / (1.0L - xi * xi);
            ldbl dx = d1 / d2P;
            xi -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        x[i] = xi;
    }
}

static ldbl lagrange_ld(int n, const ldbl *xn, int j, ldbl x)
{
    ldbl v = 1.0L;
    for (int k = 0; k < n; ++k)
        if (k != j) v *= (x - xn[k]) / (xn[j] - xn[k]);
    return v;
}

static void diff_matrix_ld(int n, const ldbl *xn, ldbl D[MAXP][MAXP])
{
    ldbl lam[MAXP];
    for (int j = 0; j < n; ++j) {
        ldbl p = 1.0L;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (xn[j] - xn[k]);
        lam[j] = 1.0L / p;
    }
    for (int i = 0; i < n; ++i) {
        ldbl s = 0.0L;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i][j] = (lam[j] / lam[i]) / (xn[i] - xn[j]);
            s += D[i][j];
        }
        D[i][i] = -s;
    }
}

/* Metric terms by the conservative curl form of Kopriva (2006):
 *   Ja^i_n = -( curl_xi ( I^N( X_l grad_xi X_m ) ) )_i,  (n,m,l) cyclic,
 * evaluated on Gauss-Lobatto points of degree N, then interpolated to the
 * Gauss volume nodes and evaluated at xi^d = +-1 on the faces.  The element's
 * geometry X is the Gauss-Lobatto interpolant of the map of degree ngeo <= N
 * (Sec. 3.1, curved elements of geometry degree N_geo), and the node
 * coordinates are its values at the Gauss nodes.  All of it in extended
 * precision, rounded once to FP64 at the end. */
static void build_metrics(orc_ctx *c)
{
    int N = c->N, P = c->P, n3 = c->n3, n2 = c->n2;
    int ng = (c->box.ngeo >= 1 && c->box.ngeo < N) ? c->box.ngeo : N;
    ldbl xgl[MAXP], Dgl[MAXP][MAXP], V[MAXP][MAXP], xgs[MAXP], xgg[MAXP], Vg[MAXP][MAXP];
    lobatto_nodes_ld(N, xgl);
    lobatto_nodes_ld(ng, xgg);
    diff_matrix_ld(P, xgl, Dgl);
    for (int a = 0; a < P; ++a) xgs[a] = c->xg[a];
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) V[a][b] = lagrange_ld(P, xgl, b, xgs[a]); /* GL -> Gauss */
    for (int a = 0; a < P; ++a)
        for (int b = 0; b <= ng; ++b) Vg[a][b] = lagrange_ld(ng + 1, xgg, b, xgl[a]); /* GL(ngeo) -> GL(N) */

    size_t sz = (size_t)n3;
    ldbl *X = malloc(sizeof(ldbl) * 3 * sz);
    ldbl *dX = malloc(sizeof(ldbl) * 9 * sz);       /* dX[m][d] */
    ldbl *Rv = malloc(sizeof(ldbl) * 3 * sz);
    ldbl *JaGL = malloc(sizeof(ldbl) * 9 * sz);     /* [i][n] */
    ldbl *tmp = malloc(sizeof(ldbl) * sz), *tmp2 = malloc(sizeof(ldbl) * sz);

    for (int ez = 0; ez < c->box.n[2]; ++ez)
    for (int ey = 0; ey < c->box.n[1]; ++ey)
    for (int ex = 0; ex < c->box.n[0]; ++ex) {
        int e = ex + c->box.n[0] * (ey + c->box.n[1] * ez);
        int ee[3] = {ex, ey, ez};
        /* geometry at GL points: the map at the degree-ngeo GL points,
         * interpolated to the degree-N GL points */
        for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
        for (int i = 0; i < P; ++i) {
            int ii[3] = {i, j, k};
            ldbl acc[3] = {0.0L, 0.0L, 0.0L};
            for (int c3 = 0; c3 <= ng; ++c3)
            for (int c2 = 0; c2 <= ng; ++c2)
            for (int c1 = 0; c1 <= ng; ++c1) {
                int cc[3] = {c1, c2, c3};
                ldbl wgt = 1.0L, Xr[3], x[3];
                for (int d = 0; d < 3; ++d) {
                    ldbl h = (ldbl)c->box.len[d] / c->box.n[d];
                    Xr[d] = c->box.lo[d] + h * (ee[d] + 0.5L * (xgg[cc[d]] + 1.0L));
                    wgt *= ng == N ? (cc[d] == ii[d] ? 1.0L : 0.0L) : Vg[ii[d]][cc[d]];
                }
                if (wgt == 0.0L) continue;
                geom_map(&c->box, Xr, x);
                for (int m = 0; m < 3; ++m) acc[m] += wgt * x[m];
            }
            for (int m = 0; m < 3; ++m) X[m * sz + nidx(P, i, j, k)] = acc[m];
        }
        /* dX_m / d xi^d on GL points */
        for (int m = 0; m < 3; ++m)
            for (int d = 0; d < 3; ++d)
                for (int nd = 0; nd < n3; ++nd) {
                    int l, fp; node_split(P, nd, d, &l, &fp);
                    int p = fp % P, q = fp / P;
                    ldbl s = 0.0L;
                    for (int r = 0; r < P; ++r) s += Dgl[l][r] * X[m * sz + line_node(P, d, r, p, q)];
                    dX[(m * 3 + d) * sz + nd] = s;
                }
        /* curl form; the product uses coordinates relative to the element's
         * first geometry node (the curl of grad X_m vanishes, so a constant
         * shift of X_l changes nothing but the size of the round-off) */
        for (int n = 0; n < 3; ++n) {
            int m = (n + 1) % 3, l = (n + 2) % 3;
            for (int jj = 0; jj < 3; ++jj)
                for (int nd = 0; nd < n3; ++nd)
                    Rv[jj * sz + nd] = (X[l * sz + nd] - X[l * sz]) * dX[(m * 3 + jj) * sz + nd];
            for (int i = 0; i < 3; ++i) {
                /* (curl R)_i = d_{i+1} R_{i+2} - d_{i+2} R_{i+1} */
                int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
                for (int nd = 0; nd < n3; ++nd) {
                    int l1, fp1, l2, fp2;
                    node_split(P, nd, i1, &l1, &fp1);
                    node_split(P, nd, i2, &l2, &fp2);
                    ldbl s1 = 0.0L, s2 = 0.0L;
                    for (int r = 0; r < P; ++r) {
                        s1 += Dgl[l1][r] * Rv[i2 * sz + line_node(P, i1, r, fp1 % P, fp1 / P)];
                        s2 += Dgl[l2][r] * Rv[i1 * sz + line_node(P, i2, r, fp2 % P, fp2 / P)];
                    }
                    JaGL[(i * 3 + n) * sz + nd] = -(s1 - s2);
                }
            }
        }
        /* interpolate Ja (9 fields) and dX (9 fields) from GL to Gauss nodes,
         * one direction at a time; dX is overwritten with its Gauss values */
        for (int fld = 0; fld < 18; ++fld) {
            ldbl *src = fld < 9 ? JaGL + fld * sz : dX + (fld - 9) * sz;
            memcpy(tmp, src, sizeof(ldbl) * sz);
            for (int d = 0; d < 3; ++d) {
                for (int nd = 0; nd < n3; ++nd) {
                    int l, fp; node_split(P, nd, d, &l, &fp);
                    ldbl s = 0.0L;
                    for (int r = 0; r < P; ++r) s += V[l][r] * tmp[line_node(P, d, r, fp % P, fp / P)];
                    tmp2[nd] = s;
                }
                memcpy(tmp, tmp2, sizeof(ldbl) * sz);
            }
            if (fld < 9)
                for (int nd = 0; nd < n3; ++nd) c->Ja[((size_t)e * n3 + nd) * 9 + fld] = (double)tmp[nd];
            else
                memcpy(src, tmp, sizeof(ldbl) * sz);
        }
        /* J = det(dx/dxi) at Gauss nodes; node coordinates at Gauss nodes */
        for (int nd = 0; nd < n3; ++nd) {
            ldbl A[3][3];
            for (int m = 0; m < 3; ++m)
                for (int d = 0; d < 3; ++d) A[m][d] = dX[(m * 3 + d) * sz + nd];
            c->J[(size_t)e * n3 + nd] = (double)(
                A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]));
            int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
            for (int m = 0; m < 3; ++m) {
                ldbl x = 0.0L;
                for (int c3 = 0; c3 < P; ++c3)
                    for (int c2 = 0; c2 < P; ++c2)
                        for (int c1 = 0; c1 < P; ++c1)
                            x += V[i][c1] * V[j][c2] * V[k][c3] * X[m * sz + nidx(P, c1, c2, c3)];
                c->xyz[((size_t)e * n3 + nd) * 3 + m] = (double)x;
            }
        }
        /* Face metrics: Ja^d at xi^d = +-1 (GL endpoint), interpolated along
         * the two tangential directions to the Gauss face points; outward
         * n dS = (2s-1) Ja^d. */
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                int f = 2 * d + s;
                int lgl = s ? N : 0;
                for (int m = 0; m < 3; ++m) {
                    ldbl G[MAXP][MAXP], H[MAXP][MAXP];
                    for (int q = 0; q < P; ++q)
                        for (int p = 0; p < P; ++p)
                            G[q][p] = JaGL[(d * 3 + m) * sz + line_node(P, d, lgl, p, q)];
                    for (int q = 0; q < P; ++q)
                        for (int p = 0; p < P; ++p) {
                            ldbl v = 0.0L;
                            for (int r = 0; r < P; ++r) v += V[p][r] * G[q][r];
                            H[q][p] = v;
                        }
                    for (int q = 0; q < P; ++q)
                        for (int p = 0; p < P; ++p) {
                            ldbl v = 0.0L;
                            for (int r = 0; r < P; ++r) v += V[q][r] * H[r][p];
                            c->nv[(((size_t)e * 6 + f) * n2 + p + P * q) * 3 + m] = (double)((s ? 1.0L : -1.0L) * v);
                        }
                }
            }
    }
    free(X); free(dX); free(Rv); free(JaGL); free(tmp); free(tmp2);

    /* Interior faces: the element on the + side of a face ("master") keeps
     * its n dS and the neighbour uses the exact negative. */
    for (int e = 0; e < c->E; ++e)
        for (int d = 0; d < 3; ++d) {
            int f = 2 * d; /* minus face of e: slave side */
            int ne = c->nbr[e * 6 + f];
            if (ne < 0) continue;
            for (int fp = 0; fp < n2; ++fp)
                for (int m = 0; m < 3; ++m)
                    c->nv[(((size_t)e * 6 + f) * n2 + fp) * 3 + m] =
                        -c->nv[(((size_t)ne * 6 + f + 1) * n2 + fp) * 3 + m];
        }
}

/* ------------------------------------------------------------------------ */
/* Context creation.                                                         */
/* ------------------------------------------------------------------------ */
void *orc_create(const orc_params *pr, const orc_box *bx, char *err, int errlen)
{
    if (bx->N < 1 || bx->N >= MAXP) { snprintf(err, errlen, "N out of range"); return NULL; }
    if (pr->model < 0 || pr->model > 2) { snprintf(err, errlen, "model must be 1 or 2"); return NULL; }
    for (int d = 0; d < 3; ++d)
        if (bx->n[d] < 1 || bx->len[d] <= 0) { snprintf(err, errlen, "bad box"); return NULL; }
    orc_ctx *c = calloc(1, sizeof(orc_ctx));
    c->pr = *pr; c->box = *bx;
    c->N = bx->N; c->P = bx->N + 1; c->n2 = c->P * c->P; c->n3 = c->n2 * c->P;
    c->E = bx->n[0] * bx->n[1] * bx->n[2];
    int P = c->P;
    gauss_nodes(c->N, c->xg, c->wg);
    diff_matrix(P, c->xg, c->D);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) c->Dh[i][j] = -(c->wg[j] / c->wg[i]) * c->D[j][i];
    for (int j = 0; j < P; ++j) {
        c->lm[j] = lagrange(P, c->xg, j, -1.0);
        c->lp[j] = lagrange(P, c->xg, j, 1.0);
        c->lhm[j] = c->lm[j] / c->wg[j];
        c->lhp[j] = c->lp[j] / c->wg[j];
    }
    size_t E = c->E;
    c->nbr = malloc(sizeof(int) * E * 6);
    c->kind = malloc(sizeof(int) * E * 6);
    c->side = malloc(sizeof(int) * E * 6);
    c->Ja = malloc(sizeof(double) * E * c->n3 * 9);
    c->J = malloc(sizeof(double) * E * c->n3);
    c->nv = malloc(sizeof(double) * E * 6 * c->n2 * 3);
    c->xyz = malloc(sizeof(double) * E * c->n3 * 3);
    /* structured connectivity */
    for (int ez = 0; ez < bx->n[2]; ++ez)
    for (int ey = 0; ey < bx->n[1]; ++ey)
    for (int ex = 0; ex < bx->n[0]; ++ex) {
        int e = ex + bx->n[0] * (ey + bx->n[1] * ez);
        int ee[3] = {ex, ey, ez};
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                int f = 2 * d + s;
                int nn[3] = {ex, ey, ez};
                nn[d] += s ? 1 : -1;
                int inside = nn[d] >= 0 && nn[d] < bx->n[d];
                if (!inside && bx->periodic[d]) { nn[d] = (nn[d] + bx->n[d]) % bx->n[d]; inside = 1; }
                if (inside) {
                    c->nbr[e * 6 + f] = nn[0] + bx->n[0] * (nn[1] + bx->n[1] * nn[2]);
                    c->kind[e * 6 + f] = 0;
                    c->side[e * 6 + f] = -1;
                } else {
                    int k = bx->side_kind[f];
                    int bad = (k != 1 && k != 2 && k != 3);
                    if (k == 3)
                        bad = !(bx->side_g1[f] >= 0 && bx->side_g2[f] >= 0 && bx->side_g3[f] >= 0 &&
                                bx->side_g4[f] >= 0);
                    if (bad) {
                        snprintf(err, errlen, "non-periodic side %d needs a wall kind (1, 2, 3 with "
                                 "non-negative coefficients)", f);
                        free(c->nbr); free(c->kind); free(c->side); free(c->Ja); free(c->J);
                        free(c->nv); free(c->xyz); free(c);
                        return NULL;
                    }
                    c->nbr[e * 6 + f] = -1;
                    c->kind[e * 6 + f] = k;
                    c->side[e * 6 + f] = f;
                }
                (void)ee;
            }
    }
    /* wall constants: Maxwell states and sigma at the wall temperature */
    for (int f = 0; f < 6; ++f) {
        c->wrv[f] = c->wrl[f] = c->wsig[f] = 0.0; c->wcos[f] = 0.0;
        if (bx->periodic[f / 2] || (bx->side_kind[f] != 1 && bx->side_kind[f] != 3)) continue;
        double rv, rl;
        if (!orc_maxwell(pr->R, pr->a, pr->b, bx->side_twall[f], &rv, &rl, NULL)) {
            snprintf(err, errlen, "wall temperature %d is not subcritical", f);
            free(c->nbr); free(c->kind); free(c->side); free(c->Ja); free(c->J);
            free(c->nv); free(c->xyz); free(c->stab); free(c);
            return NULL;
        }
        c->wrv[f] = rv; c->wrl[f] = rl;
        c->wsig[f] = orc_sigma(pr->R, pr->a, pr->b, bx->side_twall[f], pr->gam);
        c->wcos[f] = cos(bx->side_theta[f] * M_PI / 180.0);
        const double *tg = bx->side_tgrad[f];
        c->wvar[f] = tg[0] != 0.0 || tg[1] != 0.0 || tg[2] != 0.0 || bx->side_trate[f] != 0.0;
        if (c->wvar[f]) {
            /* the wall temperature must stay inside the table's subcritical
             * part on the whole side (its extremes are at the side's corners) */
            int d = f / 2;
            for (int q = 0; q < 4; ++q) {
                double x[3], T = bx->side_twall[f];
                int bit = 0;
                for (int m = 0; m < 3; ++m) {
                    x[m] = bx->lo[m] + (m == d ? (f & 1) * bx->len[m] : ((q >> bit++) & 1) * bx->len[m]);
                    T += tg[m] * x[m];
                }
                if (!(T >= 0.3 && T <= 0.99)) {
                    snprintf(err, errlen, "wall temperature of side %d leaves [0.3, 0.99]", f);
                    free(c->nbr); free(c->kind); free(c->side); free(c->Ja); free(c->J);
                    free(c->nv); free(c->xyz); free(c->stab); free(c);
                    return NULL;
                }
            }
            if (!c->stab) {
                c->stab = malloc(sizeof(double) * 3 * ORC_NTAB);
                orc_table_build(pr->R, pr->a, pr->b, c->stab);
            }
        }
    }
    build_metrics(c);
    return c;
}

void orc_destroy(void *vc)
{
    orc_ctx *c = vc;
    if (!c) return;
    free(c->nbr); free(c->kind); free(c->side); free(c->Ja); free(c->J);
    free(c->nv); free(c->xyz); free(c->stab); free(c);
}

long orc_nnodes(void *vc) { orc_ctx *c = vc; return (long)c->E * c->n3; }
int orc_nelems(void *vc) { orc_ctx *c = vc; return c->E; }

void orc_node_coords(void *vc, double *xyz)
{
    orc_ctx *c = vc;
    size_t nn = (size_t)c->E * c->n3;
    for (size_t a = 0; a < nn; ++a)
        for (int m = 0; m < 3; ++m) xyz[m * nn + a] = c->xyz[a * 3 + m];
}

/* Exports the metric terms for the tests: Ja as [9][E*n3] (index d*3+m),
 * J as [E*n3], n dS as [3][E][6][n2]. */
void orc_metrics(void *vc, double *Ja, double *J, double *nv)
{
    orc_ctx *c = vc;
    size_t nn = (size_t)c->E * c->n3, nf = (size_t)c->E * 6 * c->n2;
    for (size_t a = 0; a < nn; ++a) {
        for (int k = 0; k < 9; ++k) Ja[k * nn + a] = c->Ja[a * 9 + k];
        J[a] = c->J[a];
    }
    for (size_t a = 0; a < nf; ++a)
        for (int m = 0; m < 3; ++m) nv[m * nf + a] = c->nv[a * 3 + m];
}

/* 1D operators for the tests. */
void orc_basis(int N, double *x, double *w, double *D, double *Dh, double *lm, double *lp)
{
    int P = N + 1;
    double DD[MAXP][MAXP];
    gauss_nodes(N, x, w);
    diff_matrix(P, x, DD);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            D[i * P + j] = DD[i][j];
            Dh[i * P + j] = -(w[j] / w[i]) * DD[j][i];
        }
    for (int j = 0; j < P; ++j) {
        lm[j] = lagrange(P, x, j, -1.0);
        lp[j] = lagrange(P, x, j, 1.0);
    }
}

void orc_lobatto(int N, double *x) { lobatto_nodes(N, x); }

/* ------------------------------------------------------------------------ */
/* Discrete operators.                                                       */
/* ------------------------------------------------------------------------ */

/* Prolongation of one nodal field (element e, stride over nodes) to face f:
 * value at face point (p,q) = sum_l l_l(+-1) u(l along the face normal). */
static void prolong(const orc_ctx *c, const double *u, int f, double *out)
{
    int P = c->P, d = f / 2, s = f % 2;
    const double *L = s ? c->lp : c->lm;
    for (int q = 0; q < P; ++q)
        for (int p = 0; p < P; ++p) {
            double v = 0.0;
            for (int l = 0; l < P; ++l) v += L[l] * u[line_node(P, d, l, p, q)];
            out[p + P * q] = v;
        }
}

/* BR1 lifting of one scalar w on element e (Sec. 3.1):
 *   J q_m = sum_d sum_l Dhat_{i_d l} (Ja^d_m w)_l
 *           + sum_faces lhat^{+-}_{i_d} w*(face point) (n dS)_m,
 * returned as q_m = (J q_m)/J for m = 0..2 (out[m*n3 + node]). */
static void lift_scalar(const orc_ctx *c, int e, const double *w, const double *wstar, double *out)
{
    int P = c->P, n3 = c->n3, n2 = c->n2;
    const double *Ja = c->Ja + (size_t)e * n3 * 9;
    const double *nv = c->nv + (size_t)e * 6 * n2 * 3;
    for (int nd = 0; nd < n3; ++nd)
        for (int m = 0; m < 3; ++m) {
            double acc = 0.0;
            for (int d = 0; d < 3; ++d) {
                int l, fp; node_split(P, nd, d, &l, &fp);
                int p = fp % P, q = fp / P;
                for (int r = 0; r < P; ++r) {
                    int nr = line_node(P, d, r, p, q);
                    acc += c->Dh[l][r] * Ja[nr * 9 + d * 3 + m] * w[nr];
                }
                acc += c->lhm[l] * wstar[(2 * d) * n2 + fp] * nv[((2 * d) * n2 + fp) * 3 + m];
                acc += c->lhp[l] * wstar[(2 * d + 1) * n2 + fp] * nv[((2 * d + 1) * n2 + fp) * 3 + m];
            }
            out[m * n3 + nd] = acc / c->J[(size_t)e * n3 + nd];
        }
}

/* BR1 divergence lifting of the vector field v (3 x n3) on element e:
 *   J div = sum_d sum_l Dhat_{i_d l} (sum_m Ja^d_m v_m)_l
 *           + sum_faces lhat^{+-}_{i_d} flux*(face point),
 * where flux* is the face value of v . (n dS). */
static void lift_div(const orc_ctx *c, int e, const double *v, const double *fstar, double *out)
{
    int P = c->P, n3 = c->n3, n2 = c->n2;
    const double *Ja = c->Ja + (size_t)e * n3 * 9;
    for (int nd = 0; nd < n3; ++nd) {
        double acc = 0.0;
        for (int d = 0; d < 3; ++d) {
            int l, fp; node_split(P, nd, d, &l, &fp);
            int p = fp % P, q = fp / P;
            for (int r = 0; r < P; ++r) {
                int nr = line_node(P, d, r, p, q);
                double ft = 0.0;
                for (int m = 0; m < 3; ++m) ft += Ja[nr * 9 + d * 3 + m] * v[m * n3 + nr];
                acc += c->Dh[l][r] * ft;
            }
            acc += c->lhm[l] * fstar[(2 * d) * n2 + fp];
            acc += c->lhp[l] * fstar[(2 * d + 1) * n2 + fp];
        }
        out[nd] = acc / c->J[(size_t)e * n3 + nd];
    }
}

/* Workspace of one RHS evaluation. */
typedef struct {
    double *Uf;    /* [E][6 faces][6 vars][n2]   prolonged conserved state     */
    double *q;     /* [E][15][n3] lifted grad of rho, u1, u2, u3, c            */
    double *qcf;   /* [E][6][3][n2] prolonged grad c                           */
    double *T;     /* [E][n3]                                                  */
    double *Tf;    /* [E][6][n2]                                               */
    double *qT;    /* [E][3][n3]                                               */
    double *lapc;  /* [E][n3]                                                  */
    double *gf;    /* [E][6][13][n2] prolonged grad u (9), grad T (3), lap c   */
    double *Fs;    /* [E][6][6][n2] (F* . n) dS on each face of each element   */
} work_t;

static void work_alloc(const orc_ctx *c, work_t *w)
{
    size_t E = c->E, n3 = c->n3, n2 = c->n2;
    w->Uf = malloc(sizeof(double) * E * 36 * n2);
    w->q = malloc(sizeof(double) * E * 15 * n3);
    w->qcf = malloc(sizeof(double) * E * 18 * n2);
    w->T = malloc(sizeof(double) * E * n3);
    w->Tf = malloc(sizeof(double) * E * 6 * n2);
    w->qT = malloc(sizeof(double) * E * 3 * n3);
    w->lapc = malloc(sizeof(double) * E * n3);
    w->gf = malloc(sizeof(double) * E * 6 * 13 * n2);
    w->Fs = malloc(sizeof(double) * E * 36 * n2);
}

static void work_free(work_t *w)
{
    free(w->Uf); free(w->q); free(w->qcf); free(w->T); free(w->Tf); free(w->qT);
    free(w->lapc); free(w->gf); free(w->Fs);
}

/* Gather the conserved state of element e into a local [6][n3] array. */
static void gather_U(const orc_ctx *c, const double *U, int e, double *Ue)
{
    size_t nn = (size_t)c->E * c->n3;
    for (int v = 0; v < 6; ++v)
        memcpy(Ue + v * c->n3, U + v * nn + (size_t)e * c->n3, sizeof(double) * c->n3);
}

/* Primitive value (rho, u1, u2, u3, c)[k] of a conserved state. */
static double prim(const double *U6, int k)
{
    if (k == 0) return U6[0];
    if (k == 4) return U6[5];
    return U6[k] / U6[0];
}

/* Step 1: prolong U to all faces. */
static void step_prolong(const orc_ctx *c, const double *U, work_t *w)
{
    int n2 = c->n2, n3 = c->n3;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        double Ue[6 * MAXP * MAXP * MAXP];
        gather_U(c, U, e, Ue);
        for (int f = 0; f < 6; ++f)
            for (int v = 0; v < 6; ++v)
                prolong(c, Ue + v * n3, f, w->Uf + (((size_t)e * 6 + f) * 6 + v) * n2);
    }
}

/* Face state of element e, face f, point fp as a 6-vector. */
static void face_U(const orc_ctx *c, const work_t *w, int e, int f, int fp, double U6[6])
{
    for (int v = 0; v < 6; ++v) U6[v] = w->Uf[(((size_t)e * 6 + f) * 6 + v) * c->n2 + fp];
}

static void unit_normal(const orc_ctx *c, int e, int f, int fp, double n[3], double *dS)
{
    const double *nv = c->nv + (((size_t)e * 6 + f) * c->n2 + fp) * 3;
    double s = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    n[0] = nv[0] / s; n[1] = nv[1] / s; n[2] = nv[2] / s;
    *dS = s;
}

/* Step 2: BR1 pass 1 for w in (rho, u1, u2, u3, c).  Interior faces use the
 * central value w* = (w- + w+)/2.  Walls: rho* = rho-, c* = c-, and u* = the
 * wall velocity on the no-slip wall or the tangential part of u- on the slip
 * and Navier-slip walls. */
static void step_lift1(const orc_ctx *c, const double *U, work_t *w)
{
    int n2 = c->n2, n3 = c->n3;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        double Ue[6 * MAXP * MAXP * MAXP], wv[MAXP * MAXP * MAXP];
        double ws[6 * MAXP * MAXP];
        gather_U(c, U, e, Ue);
        for (int k = 0; k < 5; ++k) {
            for (int nd = 0; nd < n3; ++nd) {
                double U6[6];
                for (int v = 0; v < 6; ++v) U6[v] = Ue[v * n3 + nd];
                wv[nd] = prim(U6, k);
            }
            for (int f = 0; f < 6; ++f)
                for (int fp = 0; fp < n2; ++fp) {
                    double Um[6];
                    face_U(c, w, e, f, fp, Um);
                    int ne = c->nbr[e * 6 + f];
                    double val;
                    if (ne >= 0) {
                        double Up[6];
                        face_U(c, w, ne, f ^ 1, fp, Up);
                        val = 0.5 * (prim(Um, k) + prim(Up, k));
                    } else if (k == 0 || k == 4) {
                        val = prim(Um, k);
                    } else if (c->kind[e * 6 + f] == 1) {
                        val = c->box.side_uwall[c->side[e * 6 + f]][k - 1]; /* no-slip */
                    } else {
                        double n[3], dS, un;
                        unit_normal(c, e, f, fp, n, &dS);
                        un = (Um[1] * n[0] + Um[2] * n[1] + Um[3] * n[2]) / Um[0];
                        val = prim(Um, k) - un * n[k - 1];
                    }
                    ws[f * n2 + fp] = val;
                }
            lift_scalar(c, e, wv, ws, w->q + ((size_t)e * 15 + 3 * k) * n3);
        }
    }
}

/* Physical position of face point fp of face f of element e (face points
 * ordered p + P q over the two tangential directions in axis order). */
static void face_point_x(const orc_ctx *c, int e, int f, int fp, double x[3])
{
    int P = c->P, d = f / 2, t[2] = {fp % P, fp / P}, it = 0;
    int ee[3] = {e % c->box.n[0], (e / c->box.n[0]) % c->box.n[1], e / (c->box.n[0] * c->box.n[1])};
    ldbl Xr[3], xx[3];
    for (int m = 0; m < 3; ++m) {
        ldbl xi = (m == d) ? ((f & 1) ? 1.0L : -1.0L) : (ldbl)c->xg[t[it++]];
        ldbl h = (ldbl)c->box.len[m] / c->box.n[m];
        Xr[m] = c->box.lo[m] + h * (ee[m] + 0.5L * (xi + 1.0L));
    }
    geom_map(&c->box, Xr, xx);
    for (int m = 0; m < 3; ++m) x[m] = (double)xx[m];
}

/* Wall temperature and the contact-angle constants at one wall face point:
 * the side's constants for a fixed wall temperature; for a varying one,
 * T_w = twall + tgrad . x + trate t and sigma, rv, rl interpolated in the
 * table. */
typedef struct { double Tw, rv, rl, sig, cs; } wall_pt;
static void wall_point(const orc_ctx *c, int e, int f, int fp, wall_pt *w)
{
    int sd = c->side[e * 6 + f];
    w->cs = c->wcos[sd];
    w->Tw = c->box.side_twall[sd];
    if (!c->wvar[sd]) {
        w->rv = c->wrv[sd]; w->rl = c->wrl[sd]; w->sig = c->wsig[sd];
        return;
    }
    double x[3], v[3];
    const double *tg = c->box.side_tgrad[sd];
    face_point_x(c, e, f, fp, x);
    w->Tw += tg[0] * x[0] + tg[1] * x[1] + tg[2] * x[2];
    w->Tw += c->box.side_trate[sd] * c->time;
    orc_table_lookup(c->stab, w->Tw, v);
    w->sig = sqrt(2.0 * c->pr.gam) * v[0];
    w->rv = v[1]; w->rl = v[2];
}

/* Contact-angle flux g = grad c . n on a wall of kind 1 or 3, from the
 * constitutive relation eq. bc_contactangle_alpha: g = (gamma_1 div u -
 * dpsi/dc) / gamma, with gamma_1 = 0 on the no-slip wall; div u is the trace
 * of the lifted velocity gradient at the wall. */
static double wall_g(const orc_ctx *c, int kind, int f_side, const wall_pt *wp, double cm, double div)
{
    double g = -orc_dpsiwall_dc(cm, wp->rv, wp->rl, wp->sig, wp->cs) / c->pr.gam;
    if (kind == 3) g += c->box.side_g1[f_side] * div / c->pr.gam;
    return g;
}

/* Isothermal wall: theta* = T_wall in the lifting and the conductive flux
 * from the lifted gradient (kind 1, and kind 3 with gamma_3 infinite). */
static int wall_isothermal(const orc_ctx *c, int kind, int f_side)
{
    return kind == 1 || (kind == 3 && isinf(c->box.side_g3[f_side]));
}

/* Step 3: temperature at nodes and faces, then BR1 pass 2 for theta and the
 * divergence lifting of grad c.  Walls: theta* = T_wall (isothermal) or
 * theta- (adiabatic and heat-transfer walls); (grad c . n)* = g (contact
 * angle, kinds 1 and 3) or 0 (slip). */
static void step_lift2(const orc_ctx *c, const double *U, work_t *w)
{
    int n2 = c->n2, n3 = c->n3;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        double Ue[6 * MAXP * MAXP * MAXP];
        gather_U(c, U, e, Ue);
        const double *qe = w->q + (size_t)e * 15 * n3;
        for (int nd = 0; nd < n3; ++nd) {
            double U6[6], qc[3];
            for (int v = 0; v < 6; ++v) U6[v] = Ue[v * n3 + nd];
            for (int m = 0; m < 3; ++m) qc[m] = qe[(12 + m) * n3 + nd];
            w->T[(size_t)e * n3 + nd] = temperature(&c->pr, U6, qc);
        }
        for (int f = 0; f < 6; ++f) {
            for (int m = 0; m < 3; ++m)
                prolong(c, qe + (12 + m) * n3, f, w->qcf + (((size_t)e * 6 + f) * 3 + m) * n2);
            for (int fp = 0; fp < n2; ++fp) {
                double U6[6], qc[3];
                face_U(c, w, e, f, fp, U6);
                for (int m = 0; m < 3; ++m) qc[m] = w->qcf[(((size_t)e * 6 + f) * 3 + m) * n2 + fp];
                w->Tf[((size_t)e * 6 + f) * n2 + fp] = temperature(&c->pr, U6, qc);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        double Ts[6 * MAXP * MAXP], fs[6 * MAXP * MAXP];
        for (int f = 0; f < 6; ++f)
            for (int fp = 0; fp < n2; ++fp) {
                int ne = c->nbr[e * 6 + f];
                double Tm = w->Tf[((size_t)e * 6 + f) * n2 + fp];
                const double *nv = c->nv + (((size_t)e * 6 + f) * n2 + fp) * 3;
                if (ne >= 0) {
                    double Tp = w->Tf[((size_t)ne * 6 + (f ^ 1)) * n2 + fp];
                    Ts[f * n2 + fp] = 0.5 * (Tm + Tp);
                    double s = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        double qm = w->qcf[(((size_t)e * 6 + f) * 3 + m) * n2 + fp];
                        double qp = w->qcf[(((size_t)ne * 6 + (f ^ 1)) * 3 + m) * n2 + fp];
                        s += 0.5 * (qm + qp) * nv[m];
                    }
                    fs[f * n2 + fp] = s;
                } else {
                    int sd = c->side[e * 6 + f];
                    double dS = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
                    int kd = c->kind[e * 6 + f];
                    wall_pt wp;
                    wall_point(c, e, f, fp, &wp);
                    Ts[f * n2 + fp] = wall_isothermal(c, kd, sd) ? wp.Tw : Tm;
                    if (kd == 2) {
                        fs[f * n2 + fp] = 0.0;
                    } else {
                        double cm = w->Uf[(((size_t)e * 6 + f) * 6 + 5) * n2 + fp];
                        double div = 0.0;
                        if (kd == 3) {
                            /* trace of the lifted div u: d u/dx + d v/dy + d w/dz */
                            const double *qe = w->q + (size_t)e * 15 * n3;
                            double tr[MAXP * MAXP];
                            for (int m = 0; m < 3; ++m) {
                                prolong(c, qe + (3 + 4 * m) * n3, f, tr);
                                div += tr[fp];
                            }
                        }
                        fs[f * n2 + fp] = wall_g(c, kd, sd, &wp, cm, div) * dS;
                    }
                }
            }
        lift_scalar(c, e, w->T + (size_t)e * n3, Ts, w->qT + (size_t)e * 3 * n3);
        lift_div(c, e, w->q + ((size_t)e * 15 + 12) * n3, fs, w->lapc + (size_t)e * n3);
    }
}

/* Collect the point state at face point fp of face f of element e. */
static void face_state(const orc_ctx *c, const work_t *w, int e, int f, int fp, point_state *s)
{
    int n2 = c->n2;
    face_U(c, w, e, f, fp, s->U);
    s->T = w->Tf[((size_t)e * 6 + f) * n2 + fp];
    const double *g = w->gf + ((size_t)e * 6 + f) * 13 * n2;
    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) s->gu[j][i] = g[(3 * j + i) * n2 + fp];
    for (int i = 0; i < 3; ++i) s->gT[i] = g[(9 + i) * n2 + fp];
    s->lapc = g[12 * n2 + fp];
    for (int m = 0; m < 3; ++m) s->gc[m] = w->qcf[(((size_t)e * 6 + f) * 3 + m) * n2 + fp];
}

/* Rusanov (local Lax-Friedrichs) flux of the convective part, Sec. 3.1:
 * 1/2 (F^C(U-) + F^C(U+)) . n - 1/2 lambda (U+ - U-), with
 * lambda = max(|u- . n| + c~-, |u+ . n| + c~+), c~ = sqrt(|c_s^2|). */
static void rusanov(const orc_params *pr, const point_state *sm, const point_state *sp,
                    const double n[3], double out[6])
{
    double Fm[3][6], Fp[3][6];
    flux_conv(pr, sm, Fm);
    flux_conv(pr, sp, Fp);
    double unm = (sm->U[1] * n[0] + sm->U[2] * n[1] + sm->U[3] * n[2]) / sm->U[0];
    double unp = (sp->U[1] * n[0] + sp->U[2] * n[1] + sp->U[3] * n[2]) / sp->U[0];
    double lm = fabs(unm) + wave_speed(pr, sm->U[0], sm->T);
    double lp = fabs(unp) + wave_speed(pr, sp->U[0], sp->T);
    double lam = lm > lp ? lm : lp;
    for (int v = 0; v < 6; ++v) {
        double a = 0.0;
        for (int i = 0; i < 3; ++i) a += 0.5 * (Fm[i][v] + Fp[i][v]) * n[i];
        out[v] = a - 0.5 * lam * (sp->U[v] - sm->U[v]);
    }
}

/* HLLC flux (Toro 2009, Sec. 10.4) of the convective part for relaxation
 * model 2, in the frame of the unit normal n from side m (left) to side p
 * (right): wave speeds S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L,
 * u_R + a_R) (Davis) with a = sqrt((dp_alpha/drho)_s) and u the normal
 * velocity; contact speed S*; star states with the tangential velocity and
 * c/rho of their side; the order parameter rides along as a passive scalar. */
static void hllc(const orc_params *pr, const point_state *sm, const point_state *sp, const double n[3],
                 double out[6])
{
    const point_state *st[2] = {sm, sp};
    double rho[2], un[2], p[2], a[2], F[2][6];
    for (int k = 0; k < 2; ++k) {
        const double *U = st[k]->U;
        rho[k] = U[0];
        un[k] = (U[1] * n[0] + U[2] * n[1] + U[3] * n[2]) / U[0];
        p[k] = p_conv(pr, U[0], st[k]->T);
        a[k] = wave_speed(pr, U[0], st[k]->T);
        double Fc[3][6];
        flux_conv(pr, st[k], Fc);
        for (int v = 0; v < 6; ++v) F[k][v] = Fc[0][v] * n[0] + Fc[1][v] * n[1] + Fc[2][v] * n[2];
    }
    double SL = fmin(un[0] - a[0], un[1] - a[1]);
    double SR = fmax(un[0] + a[0], un[1] + a[1]);
    if (SL >= 0.0) { for (int v = 0; v < 6; ++v) out[v] = F[0][v]; return; }
    if (SR <= 0.0) { for (int v = 0; v < 6; ++v) out[v] = F[1][v]; return; }
    double Ss = (p[1] - p[0] + rho[0] * un[0] * (SL - un[0]) - rho[1] * un[1] * (SR - un[1])) /
                (rho[0] * (SL - un[0]) - rho[1] * (SR - un[1]));
    int k = Ss >= 0.0 ? 0 : 1;       /* the star region adjacent to x/t = 0 */
    double S = k == 0 ? SL : SR;
    const double *U = st[k]->U;
    double f = rho[k] * (S - un[k]) / (S - Ss);
    double Us[6];
    Us[0] = f;
    for (int m = 0; m < 3; ++m) Us[1 + m] = f * (U[1 + m] / U[0] + (Ss - un[k]) * n[m]);
    Us[4] = f * (U[4] / U[0] + (Ss - un[k]) * (Ss + p[k] / (rho[k] * (S - un[k]))));
    Us[5] = f * U[5] / U[0];
    for (int v = 0; v < 6; ++v) out[v] = F[k][v] + S * (Us[v] - U[v]);
}

/* The interior numerical flux of the convective part for two face states
 * (conserved U and temperature T on each side) and a unit normal: Rusanov for
 * model 1, HLLC for model 2.  For the tests of the flux alone. */
void orc_numflux(const orc_params *pr, const double *UL, double TL, const double *UR, double TR, const double *n,
                 double *out)
{
    point_state sm, sp;
    memset(&sm, 0, sizeof(sm));
    memset(&sp, 0, sizeof(sp));
    for (int v = 0; v < 6; ++v) { sm.U[v] = UL[v]; sp.U[v] = UR[v]; }
    sm.T = TL;
    sp.T = TR;
    if (pr->model == 2)
        hllc(pr, &sm, &sp, n, out);
    else
        rusanov(pr, &sm, &sp, n, out);
}

/* Wall flux (F* . n) of Sec. 3.2 for the readings of eq. bc_nsk_alpha.
 * Convective part: Rusanov against a ghost state with the same density,
 * order parameter and temperature, and the velocity reflected about the
 * wall velocity (2 u_w - u, no-slip wall) or stripped of twice its normal
 * part (slip and Navier-slip walls).  Viscous part F^V . n:
 *   no-slip (kind 1): traction T^V n; energy (T^V n) . u_w + k grad T . n
 *     - gamma c g div u; order parameter gamma beta g.
 *   slip (kind 2): the normal traction only; no energy or c flux.
 *   Navier slip (kind 3): normal traction plus the tangential traction of
 *     eq. bc_navierstokes_alpha, t = gamma_1 div u grad_G c - gamma_2 (u_t -
 *     u_w); energy t . u_t + q - gamma c g div u + gamma g zeta_c with the
 *     wall value zeta_c = -gamma_1 gamma_4 div u of eq. bc_relaxation_alpha
 *     and q = k grad T . n (gamma_3 infinite: isothermal) or -gamma_3 (1/T_w
 *     - 1/T-) (eq. bc_energy_alpha); order parameter gamma beta g.
 * g is the contact-angle flux of wall_g; grad_G c and u_t are the tangential
 * parts of the lifted grad c and of u- at the face. */
static void wall_flux(const orc_ctx *c, int e, int f, int fp, const point_state *sm, const double n[3],
                      double out[6])
{
    const orc_params *pr = &c->pr;
    const orc_box *bx = &c->box;
    int kd = c->kind[e * 6 + f], sd = c->side[e * 6 + f];
    wall_pt wp;
    wall_point(c, e, f, fp, &wp);
    const double *uw = bx->side_uwall[sd];
    double rho = sm->U[0], u[3], un = 0.0;
    for (int m = 0; m < 3; ++m) {
        u[m] = sm->U[1 + m] / rho;
        un += u[m] * n[m];
    }
    point_state sg = *sm;
    if (kd == 1) {
        double ke = 0.0, keg = 0.0;
        for (int m = 0; m < 3; ++m) {
            double ug = 2.0 * uw[m] - u[m];
            sg.U[1 + m] = 2.0 * rho * uw[m] - sm->U[1 + m];
            ke += u[m] * u[m];
            keg += ug * ug;
        }
        if (uw[0] != 0.0 || uw[1] != 0.0 || uw[2] != 0.0) sg.U[4] = sm->U[4] + 0.5 * rho * (keg - ke);
    } else {
        double mn = sm->U[1] * n[0] + sm->U[2] * n[1] + sm->U[3] * n[2];
        for (int m = 0; m < 3; ++m) sg.U[1 + m] = sm->U[1 + m] - 2.0 * mn * n[m];
    }
    double fc[6];
    rusanov(pr, sm, &sg, n, fc);

    double Tv[3][3];
    viscous_stress(pr, sm->gu, Tv);
    double fv[6] = {0, 0, 0, 0, 0, 0};
    double tn[3];
    for (int i = 0; i < 3; ++i) tn[i] = Tv[i][0] * n[0] + Tv[i][1] * n[1] + Tv[i][2] * n[2];
    double div = sm->gu[0][0] + sm->gu[1][1] + sm->gu[2][2];
    double gTn = sm->gT[0] * n[0] + sm->gT[1] * n[1] + sm->gT[2] * n[2];
    if (kd == 1) {
        double g = wall_g(c, kd, sd, &wp, sm->U[5], div);
        for (int m = 0; m < 3; ++m) fv[1 + m] = tn[m];
        fv[4] = (tn[0] * uw[0] + tn[1] * uw[1] + tn[2] * uw[2]) + pr->kappa * gTn - pr->gam * sm->U[5] * g * div;
        fv[5] = pr->gam * pr->beta * g;
    } else if (kd == 2) {
        double nn = tn[0] * n[0] + tn[1] * n[1] + tn[2] * n[2];
        for (int m = 0; m < 3; ++m) fv[1 + m] = nn * n[m];
    } else {
        double g1 = bx->side_g1[sd], g2 = bx->side_g2[sd], g3 = bx->side_g3[sd], g4 = bx->side_g4[sd];
        double g = wall_g(c, kd, sd, &wp, sm->U[5], div);
        double nn = tn[0] * n[0] + tn[1] * n[1] + tn[2] * n[2];
        double gcn = sm->gc[0] * n[0] + sm->gc[1] * n[1] + sm->gc[2] * n[2];
        double uwn = uw[0] * n[0] + uw[1] * n[1] + uw[2] * n[2];
        double work = 0.0;
        for (int m = 0; m < 3; ++m) {
            double ut = u[m] - un * n[m];
            double t = g1 * div * (sm->gc[m] - gcn * n[m]) - g2 * (ut - (uw[m] - uwn * n[m]));
            fv[1 + m] = nn * n[m] + t;
            work += t * ut;
        }
        double q = wall_isothermal(c, kd, sd) ? pr->kappa * gTn : -g3 * (1.0 / wp.Tw - 1.0 / sm->T);
        double zeta = -g1 * g4 * div;
        fv[4] = work + q - pr->gam * sm->U[5] * g * div + pr->gam * g * zeta;
        fv[5] = pr->gam * pr->beta * g;
    }
    for (int v = 0; v < 6; ++v) out[v] = fc[v] - fv[v];
}

/* Step 4: prolong the remaining gradients and compute the face fluxes.  The
 * master side of each interior face evaluates (F* . n) dS and the slave side
 * takes its negative; walls are evaluated by their only element. */
static void step_faces(const orc_ctx *c, work_t *w)
{
    int n2 = c->n2, n3 = c->n3;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        const double *qe = w->q + (size_t)e * 15 * n3;
        for (int f = 0; f < 6; ++f) {
            double *g = w->gf + ((size_t)e * 6 + f) * 13 * n2;
            for (int k = 0; k < 9; ++k) prolong(c, qe + (3 + k) * n3, f, g + k * n2);
            for (int k = 0; k < 3; ++k) prolong(c, w->qT + ((size_t)e * 3 + k) * n3, f, g + (9 + k) * n2);
            prolong(c, w->lapc + (size_t)e * n3, f, g + 12 * n2);
        }
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e)
        for (int f = 0; f < 6; ++f) {
            int ne = c->nbr[e * 6 + f];
            if (ne >= 0 && (f % 2) == 0) continue; /* slave side */
            for (int fp = 0; fp < n2; ++fp) {
                point_state sm;
                double n[3], dS, out[6];
                face_state(c, w, e, f, fp, &sm);
                unit_normal(c, e, f, fp, n, &dS);
                if (ne >= 0) {
                    point_state sp;
                    double Fvm[3][6], Fvp[3][6];
                    face_state(c, w, ne, f ^ 1, fp, &sp);
                    if (c->pr.model == 2)
                        hllc(&c->pr, &sm, &sp, n, out);
                    else
                        rusanov(&c->pr, &sm, &sp, n, out);
                    flux_visc(&c->pr, &sm, Fvm);
                    flux_visc(&c->pr, &sp, Fvp);
                    for (int v = 0; v < 6; ++v)
                        for (int i = 0; i < 3; ++i) out[v] -= 0.5 * (Fvm[i][v] + Fvp[i][v]) * n[i];
                } else {
                    wall_flux(c, e, f, fp, &sm, n, out);
                }
                for (int v = 0; v < 6; ++v) w->Fs[(((size_t)e * 6 + f) * 6 + v) * n2 + fp] = out[v] * dS;
            }
        }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e)
        for (int f = 0; f < 6; f += 2) {
            int ne = c->nbr[e * 6 + f];
            if (ne < 0) continue;
            for (int v = 0; v < 6; ++v)
                for (int fp = 0; fp < n2; ++fp)
                    w->Fs[(((size_t)e * 6 + f) * 6 + v) * n2 + fp] =
                        -w->Fs[(((size_t)ne * 6 + f + 1) * 6 + v) * n2 + fp];
        }
}

/* Step 5: volume integral with the contravariant fluxes
 * Ftilde^d = sum_m Ja^d_m (F^C_m - F^V_m), surface integral with lhat, the
 * point-wise source, and J U_t = -V - surface + J S. */
static void step_assemble(const orc_ctx *c, const double *U, work_t *w, double *Ut)
{
    int P = c->P, n2 = c->n2, n3 = c->n3;
    size_t nn = (size_t)c->E * n3;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < c->E; ++e) {
        static __thread double Ft[3][6][MAXP * MAXP * MAXP];
        double Ue[6 * MAXP * MAXP * MAXP];
        gather_U(c, U, e, Ue);
        const double *qe = w->q + (size_t)e * 15 * n3;
        const double *Ja = c->Ja + (size_t)e * n3 * 9;
        for (int nd = 0; nd < n3; ++nd) {
            point_state s;
            for (int v = 0; v < 6; ++v) s.U[v] = Ue[v * n3 + nd];
            s.T = w->T[(size_t)e * n3 + nd];
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) s.gu[j][i] = qe[(3 + 3 * j + i) * n3 + nd];
            for (int i = 0; i < 3; ++i) s.gT[i] = w->qT[((size_t)e * 3 + i) * n3 + nd];
            for (int i = 0; i < 3; ++i) s.gc[i] = qe[(12 + i) * n3 + nd];
            s.lapc = w->lapc[(size_t)e * n3 + nd];
            double Fc[3][6], Fv[3][6];
            flux_conv(&c->pr, &s, Fc);
            flux_visc(&c->pr, &s, Fv);
            for (int d = 0; d < 3; ++d)
                for (int v = 0; v < 6; ++v) {
                    double a = 0.0;
                    for (int m = 0; m < 3; ++m) a += Ja[nd * 9 + d * 3 + m] * (Fc[m][v] - Fv[m][v]);
                    Ft[d][v][nd] = a;
                }
        }
        for (int nd = 0; nd < n3; ++nd) {
            double acc[6] = {0, 0, 0, 0, 0, 0};
            for (int d = 0; d < 3; ++d) {
                int l, fp; node_split(P, nd, d, &l, &fp);
                int p = fp % P, q = fp / P;
                for (int v = 0; v < 6; ++v) {
                    double a = 0.0;
                    for (int r = 0; r < P; ++r) a += c->Dh[l][r] * Ft[d][v][line_node(P, d, r, p, q)];
                    a += c->lhm[l] * w->Fs[(((size_t)e * 6 + 2 * d) * 6 + v) * n2 + fp];
                    a += c->lhp[l] * w->Fs[(((size_t)e * 6 + 2 * d + 1) * 6 + v) * n2 + fp];
                    acc[v] += a;
                }
            }
            double U6[6], grho[3], gu[3][3], gc[3], S[6];
            for (int v = 0; v < 6; ++v) U6[v] = Ue[v * n3 + nd];
            for (int i = 0; i < 3; ++i) grho[i] = qe[i * n3 + nd];
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) gu[j][i] = qe[(3 + 3 * j + i) * n3 + nd];
            for (int i = 0; i < 3; ++i) gc[i] = qe[(12 + i) * n3 + nd];
            source(&c->pr, U6, grho, gu, gc, S);
            double J = c->J[(size_t)e * n3 + nd];
            for (int v = 0; v < 6; ++v) Ut[v * nn + (size_t)e * n3 + nd] = -acc[v] / J + S[v];
        }
    }
}

/* U_t = L(U), the semi-discrete DGSEM operator. */
void orc_rhs(void *vc, const double *U, double *Ut)
{
    orc_ctx *c = vc;
    work_t w;
    work_alloc(c, &w);
    step_prolong(c, U, &w);
    step_lift1(c, U, &w);
    step_lift2(c, U, &w);
    step_faces(c, &w);
    step_assemble(c, U, &w, Ut);
    work_free(&w);
}

/* Lifted gradients of pass 1: out [15][E*n3], field 3k+m = d w_k / d x_m for
 * w = (rho, u1, u2, u3, c). */
void orc_lift1(void *vc, const double *U, double *out)
{
    orc_ctx *c = vc;
    work_t w;
    work_alloc(c, &w);
    step_prolong(c, U, &w);
    step_lift1(c, U, &w);
    size_t nn = (size_t)c->E * c->n3;
    for (int e = 0; e < c->E; ++e)
        for (int k = 0; k < 15; ++k)
            memcpy(out + k * nn + (size_t)e * c->n3, w.q + ((size_t)e * 15 + k) * c->n3, sizeof(double) * c->n3);
    work_free(&w);
}

/* Pass 2 results: out [5][E*n3] = theta, grad theta (3), lifted lap c. */
void orc_lift2(void *vc, const double *U, double *out)
{
    orc_ctx *c = vc;
    work_t w;
    work_alloc(c, &w);
    step_prolong(c, U, &w);
    step_lift1(c, U, &w);
    step_lift2(c, U, &w);
    size_t nn = (size_t)c->E * c->n3, n3 = c->n3;
    for (int e = 0; e < c->E; ++e) {
        memcpy(out + (size_t)e * n3, w.T + (size_t)e * n3, sizeof(double) * n3);
        for (int k = 0; k < 3; ++k)
            memcpy(out + (1 + k) * nn + (size_t)e * n3, w.qT + ((size_t)e * 3 + k) * n3, sizeof(double) * n3);
        memcpy(out + 4 * nn + (size_t)e * n3, w.lapc + (size_t)e * n3, sizeof(double) * n3);
    }
    work_free(&w);
}

/* ------------------------------------------------------------------------ */
/* Time integration.                                                         */
/* ------------------------------------------------------------------------ */

/* Carpenter & Kennedy 5-stage 2N-storage RK4(3)5 (the low-storage fourth-
 * order scheme family of Kennedy, Carpenter, Lewis 2000 cited in Sec. 3.1). */
static const double RK_A[5] = {0.0,
    -567301805773.0 / 1357537059087.0,
    -2404267990393.0 / 2016746695238.0,
    -3550918686646.0 / 2091501179385.0,
    -1275806237668.0 / 842570457699.0};
static const double RK_B[5] = {
    1432997174477.0 / 9575080441755.0,
    5161836677717.0 / 13612068292357.0,
    1720146321549.0 / 2090206949498.0,
    3134564353537.0 / 4481467310338.0,
    2277821191437.0 / 14882151754819.0};
static const double RK_C[5] = {0.0,
    1432997174477.0 / 9575080441755.0,
    2526269341429.0 / 6820363962896.0,
    2006345519317.0 / 3224310063776.0,
    2802321613138.0 / 2924317926251.0};

void orc_set_time(void *vc, double t) { ((orc_ctx *)vc)->time = t; }

void orc_rk_coeffs(double *A, double *B, double *C)
{
    for (int s = 0; s < 5; ++s) { A[s] = RK_A[s]; B[s] = RK_B[s]; C[s] = RK_C[s]; }
}

/* One step: for each stage R <- A_s R + dt L(U) (assigned in stage 1),
 * U <- U + B_s R. */
void orc_rk_step(void *vc, double *U, double *R, double t, double dt)
{
    orc_ctx *c = vc;
    size_t n = (size_t)6 * c->E * c->n3;
    double *Ut = malloc(sizeof(double) * n);
    for (int s = 0; s < 5; ++s) {
        c->time = t + RK_C[s] * dt;  /* stage time of the 2N scheme */
        orc_rhs(c, U, Ut);
        for (size_t a = 0; a < n; ++a) {
            R[a] = (s == 0) ? dt * Ut[a] : RK_A[s] * R[a] + dt * Ut[a];
            U[a] += RK_B[s] * R[a];
        }
    }
    free(Ut);
}

void orc_run(void *vc, double *U, double *R, double t, double dt, int nsteps)
{
    for (int k = 0; k < nsteps; ++k) orc_rk_step(vc, U, R, t + k * dt, dt);
}

/* Stability constants of the time-step rule for N = 1..7 (1D periodic
 * Gauss DGSEM spectra under the RK4(3)5 stability polynomial): T_N is the
 * largest stable dt*a/h for Rusanov advection, RHO_N the spectral radius of
 * the BR1 diffusion operator at h = 1, RK_REAL the stability interval of the
 * scheme on the negative real axis.  Only N = 2..5 are tabulated. */
static double tN(int N)
{
    static const double T[6] = {0, 0, 0.3521, 0.2200, 0.1523, 0.1126};
    return (N >= 2 && N <= 5) ? T[N] : 0.0;
}
static double rhoN(int N)
{
    static const double R[6] = {0, 0, 64.8, 176.2, 387.0, 745.2};
    return (N >= 2 && N <= 5) ? R[N] : 0.0;
}
#define RK_REAL 4.6567
/* Wall limit (generalized Navier-slip walls with gamma_1 > 0): SIGMA_N is the
 * spectral radius of the BR1 lifted first derivative on the reference element
 * over the Bloch spectrum of the periodic Gauss DGSEM, RK_IMAG the stability
 * interval of the scheme on the imaginary axis. */
static double sigmaN(int N)
{
    static const double S[6] = {0, 0, 4.0406, 6.6385, 9.8386, 13.6629};
    return (N >= 2 && N <= 5) ? S[N] : 0.0;
}
#define RK_IMAG 3.3407

/* Stiffness of the gamma_1 terms of eq. bc_navierstokes_alpha and
 * eq. bc_contactangle_alpha at one node of an element with Navier-slip wall
 * faces.  Both enter through the surface lifting of the wall face (weight
 * Lambda_N = sum_j l_j(-1)^2 / w_j = (N+1)^2/2 on Gauss nodes, times
 * |Ja^n|/J of the face direction n) and act on the tangential derivatives
 * of u (SIGMA_N |Ja^d|/J per tangential direction d):
 *   traction gamma_1 div u grad_G c: a wall viscosity gamma_1 |grad_G c|/rho,
 *     lambda_t = SIGMA_N Lambda_N (|Ja^n|/J) gamma_1 sum_d |grad c . Ja^d|/(J rho);
 *   c-flux beta gamma_1 div u, closed through alpha grad c in the momentum
 *     source: lambda_c = SIGMA_N sqrt(alpha beta gamma_1 Lambda_N (|Ja^n|/J)
 *     sum_d (|Ja^d|/J)^2).
 * Both eigenvalues lie near the imaginary axis.  Returns the sum over the
 * element's Navier-slip faces of lambda_t + lambda_c. */
static double wall_rate(const orc_ctx *c, int e, const double *Ja, double J, double rho, const double gc[3])
{
    const orc_params *pr = &c->pr;
    double lam = 0.5 * (c->N + 1) * (c->N + 1), r = 0.0;
    for (int f = 0; f < 6; ++f) {
        if (c->kind[e * 6 + f] != 3) continue;
        double g1 = c->box.side_g1[c->side[e * 6 + f]];
        if (!(g1 > 0.0)) continue;
        int dn = f / 2;
        const double *An = Ja + dn * 3;
        double an = sqrt(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]) / J, st = 0.0, gt = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (d == dn) continue;
            const double *A = Ja + d * 3;
            double nd = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]) / J;
            st += nd * nd;
            gt += fabs(gc[0] * A[0] + gc[1] * A[1] + gc[2] * A[2]) / J;
        }
        r += sigmaN(c->N) * (lam * an * g1 * gt / rho + sqrt(pr->alpha * pr->beta * g1 * lam * an * st));
    }
    return r;
}

/* Time step: min of an advective limit CFL T_N 2 / max sum_d lambda^d with
 * lambda^d = (|u . Ja^d| + c~ |Ja^d|)/J, a parabolic/source limit
 * CFL RK_REAL / (alpha beta + RHO_N nu_max max sum_d (|Ja^d|/(2J))^2), with
 * nu_max = max(4 mu/(3 rho), k/(rho R c_v), gamma beta), and a wall limit
 * CFL RK_IMAG / max wall_rate on elements with Navier-slip walls of
 * gamma_1 > 0.  Needs the temperature and the lifted grad c, hence one
 * lifting pass. */
double orc_dt(void *vc, const double *U)
{
    orc_ctx *c = vc;
    const orc_params *pr = &c->pr;
    work_t w;
    work_alloc(c, &w);
    step_prolong(c, U, &w);
    step_lift1(c, U, &w);
    size_t nn = (size_t)c->E * c->n3;
    double lmax = 0.0, gmax = 0.0, nmax = 0.0, wmax = 0.0;
    for (int e = 0; e < c->E; ++e)
        for (int nd = 0; nd < c->n3; ++nd) {
            size_t a = (size_t)e * c->n3 + nd;
            double U6[6], qc[3];
            for (int v = 0; v < 6; ++v) U6[v] = U[v * nn + a];
            for (int m = 0; m < 3; ++m) qc[m] = w.q[((size_t)e * 15 + 12 + m) * c->n3 + nd];
            double T = temperature(pr, U6, qc);
            double cs = wave_speed(pr, U6[0], T);
            double J = c->J[a], sl = 0.0, sg = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double *Ja = c->Ja + a * 9 + d * 3;
                double un = (U6[1] * Ja[0] + U6[2] * Ja[1] + U6[3] * Ja[2]) / U6[0];
                double nJ = sqrt(Ja[0] * Ja[0] + Ja[1] * Ja[1] + Ja[2] * Ja[2]);
                sl += (fabs(un) + cs * nJ) / J;
                sg += (nJ / (2.0 * J)) * (nJ / (2.0 * J));
            }
            double nu = 4.0 * pr->mu / (3.0 * U6[0]);
            double nu2 = pr->kappa / (U6[0] * pr->R * pr->cv);
            if (nu2 > nu) nu = nu2;
            if (pr->gam * pr->beta > nu) nu = pr->gam * pr->beta;
            if (sl > lmax) lmax = sl;
            if (sg > gmax) gmax = sg;
            if (nu > nmax) nmax = nu;
            double wr = wall_rate(c, e, c->Ja + a * 9, J, U6[0], qc);
            if (wr > wmax) wmax = wr;
        }
    work_free(&w);
    double dt_adv = pr->cfl * tN(c->N) * 2.0 / lmax;
    double den = pr->alpha * pr->beta + rhoN(c->N) * nmax * gmax;
    double dt_par = den > 0.0 ? pr->cfl * RK_REAL / den : INFINITY;
    double dt_wall = wmax > 0.0 ? pr->cfl * RK_IMAG / wmax : INFINITY;
    double dt = dt_adv < dt_par ? dt_adv : dt_par;
    return dt < dt_wall ? dt : dt_wall;
}

/* ------------------------------------------------------------------------ */
/* Initial state and integrals.                                              */
/* ------------------------------------------------------------------------ */

/* Droplets: rho = rho_v + sum_j (rho_l - rho_v)/2 (1 + tanh((r_j - d_j)/w)),
 * the tanh profile of Sec. 4.1.1, 4.2 and 4.3 with the width written
 * directly, distances as minimum images along periodic axes; rho_v, rho_l the
 * Maxwell densities at T0 unless both rv_in and rl_in are positive (the
 * Young-Laplace densities of the collision cases, Table 5); plus the given
 * per-node noise; c = rho.  Velocity: each droplet j carries its velocity
 * v_j (vel[3j..3j+2], or 0 when vel is NULL) weighted by its indicator
 * (1 + tanh((r_j - d_j)/w))/2, so a droplet moves with v_j and the vapour far
 * from it is at rest (the collision velocity field of Sec. 4.3 read as
 * u_rel/2 per droplet); m = rho u.  rho e from eq. totalenergyalpha with the
 * lifted grad c and the kinetic energy, so the recovered temperature is T0.
 * noise and vel may be NULL.  cyl_axis in 0..2 makes every droplet a
 * cylinder along that axis (the liquid pillar of Sec. 4.4.1): d_j is then
 * measured in the plane normal to it; -1 keeps spheres. */
int orc_init_droplets(void *vc, double T0, int nd, const double *cen, const double *rad,
                      double width, const double *noise, double *U, const double *vel, double rv_in,
                      double rl_in, int cyl_axis)
{
    orc_ctx *c = vc;
    const orc_params *pr = &c->pr;
    double rv, rl;
    if (rv_in > 0.0 && rl_in > 0.0) {
        rv = rv_in;
        rl = rl_in;
    } else if (!orc_maxwell(pr->R, pr->a, pr->b, T0, &rv, &rl, NULL)) {
        return -1;
    }
    size_t nn = (size_t)c->E * c->n3;
    for (size_t a = 0; a < nn; ++a) {
        double rho = rv, u[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < nd; ++j) {
            double d2 = 0.0;
            for (int m = 0; m < 3; ++m) {
                if (m == cyl_axis) continue;
                double dx = c->xyz[a * 3 + m] - cen[3 * j + m];
                if (c->box.periodic[m]) dx -= c->box.len[m] * round(dx / c->box.len[m]);
                d2 += dx * dx;
            }
            double th = tanh((rad[j] - sqrt(d2)) / width);
            rho += 0.5 * (rl - rv) * (1.0 + th);
            if (vel)
                for (int m = 0; m < 3; ++m) u[m] += vel[3 * j + m] * 0.5 * (1.0 + th);
        }
        if (noise) rho += noise[a];
        U[a] = rho;
        U[nn + a] = rho * u[0];
        U[2 * nn + a] = rho * u[1];
        U[3 * nn + a] = rho * u[2];
        U[4 * nn + a] = 0.0;
        U[5 * nn + a] = rho;
    }
    double *q = malloc(sizeof(double) * 15 * nn);
    orc_lift1(c, U, q);
    for (size_t a = 0; a < nn; ++a) {
        double rho = U[a];
        double g2 = q[12 * nn + a] * q[12 * nn + a] + q[13 * nn + a] * q[13 * nn + a] + q[14 * nn + a] * q[14 * nn + a];
        double m2 = U[nn + a] * U[nn + a] + U[2 * nn + a] * U[2 * nn + a] + U[3 * nn + a] * U[3 * nn + a];
        U[4 * nn + a] = rho * (pr->R * pr->cv * T0 - pr->a * rho) + 0.5 * pr->gam * g2 + 0.5 * m2 / rho;
    }
    free(q);
    return 0;
}

/* Integrals (Gauss quadrature with J) and counters, in element order:
 *  0 mass, 1-3 momentum, 4 total energy, 5 int c, 6 kinetic energy,
 *  7 gradient energy gamma/2 |grad c|^2, 8 relaxation energy alpha/2 (rho-c)^2,
 *  9 int (rho-c)^2, 10 min rho, 11 max rho, 12 min T, 13 max T,
 *  14 non-finite values, 15 rho outside (0,1/b), 16 T <= 0, 17 c_s^2 < 0,
 *  18 mathematical entropy -int rho eta, 19 volume. */
void orc_reduce(void *vc, const double *U, double *out)
{
    orc_ctx *c = vc;
    const orc_params *pr = &c->pr;
    size_t nn = (size_t)c->E * c->n3;
    double *q = malloc(sizeof(double) * 15 * nn);
    orc_lift1(c, U, q);
    for (int k = 0; k < 20; ++k) out[k] = 0.0;
    out[10] = out[12] = INFINITY;
    out[11] = out[13] = -INFINITY;
    int P = c->P;
    for (int e = 0; e < c->E; ++e)
        for (int nd = 0; nd < c->n3; ++nd) {
            size_t a = (size_t)e * c->n3 + nd;
            int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
            double wJ = c->wg[i] * c->wg[j] * c->wg[k] * c->J[a];
            double U6[6], qc[3];
            int bad = 0;
            for (int v = 0; v < 6; ++v) { U6[v] = U[v * nn + a]; if (!isfinite(U6[v])) bad = 1; }
            for (int m = 0; m < 3; ++m) qc[m] = q[(12 + m) * nn + a];
            if (bad) { out[14] += 1.0; continue; }
            double rho = U6[0];
            double T = temperature(pr, U6, qc);
            if (!(rho > 0.0 && rho * pr->b < 1.0)) out[15] += 1.0;
            if (!(T > 0.0)) out[16] += 1.0;
            if (vdw_cs2(pr, rho, T) < 0.0) out[17] += 1.0;
            double g2 = qc[0] * qc[0] + qc[1] * qc[1] + qc[2] * qc[2];
            out[0] += wJ * rho;
            for (int m = 0; m < 3; ++m) out[1 + m] += wJ * U6[1 + m];
            out[4] += wJ * U6[4];
            out[5] += wJ * U6[5];
            out[6] += wJ * 0.5 * (U6[1] * U6[1] + U6[2] * U6[2] + U6[3] * U6[3]) / rho;
            out[7] += wJ * 0.5 * pr->gam * g2;
            out[8] += wJ * 0.5 * pr->alpha * (rho - U6[5]) * (rho - U6[5]);
            out[9] += wJ * (rho - U6[5]) * (rho - U6[5]);
            if (rho < out[10]) out[10] = rho;
            if (rho > out[11]) out[11] = rho;
            if (T < out[12]) out[12] = T;
            if (T > out[13]) out[13] = T;
            if (pr->b > 0.0 && T > 0.0 && rho > 0.0 && rho * pr->b < 1.0) {
                double eta = pr->R * pr->cv * log(T) - pr->R * log(pr->b * rho / (1.0 - pr->b * rho));
                out[18] += -wJ * rho * eta;
            }
            out[19] += wJ;
        }
    free(q);
}

/* Point-wise helpers exported for the tests. */
double orc_pressure(double R, double a, double b, double rho, double T)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    return vdw_p(&pr, rho, T);
}
double orc_cs2(double R, double a, double b, double cv, double rho, double T)
{
    orc_params pr = {R, a, b, cv, 0, 0, 0, 0, 0, 0, 1};
    return vdw_cs2(&pr, rho, T);
}
double orc_chempot(double R, double a, double b, double rho, double T)
{
    orc_params pr = {R, a, b, 1.0, 0, 0, 0, 0, 0, 0, 1};
    return vdw_mu(&pr, rho, T);
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
