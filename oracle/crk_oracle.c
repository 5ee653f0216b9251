/*
 * crk_oracle.c -- plain, slow, FP64 CPU reference of compact Runge-Kutta
 * flux reconstruction (cRKFR) with entropy-conservative (EC) and
 * kinetic-energy-preserving (KEP) two-point volume fluxes
 * (Babbar, Chen, Ranocha, arXiv 2604.02125).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the HIP library: everything below (Gauss-Lobatto nodes,
 * differentiation matrix, physics, fluxes, the step) is written out here
 * again from the mathematics, in the paper's order and notation, with no
 * blocking or fusion.
 *
 * Notation (paper, Section 2): reference element [0,1], solution points
 * xi_0 < ... < xi_N = Gauss-Lobatto-Legendre (GLL) nodes, weights w_p,
 * D_pq = l_q'(xi_p) (eq:diff.matrix).  State layout of every array that
 * crosses this file's interface: u[v][e][node], v = conserved variable,
 * e = ey*nx + ex, node = j*(N+1) + i (x index fastest).
 *
 * Parity status: every function here is pinned by a CPU test against a
 * closed form, an invariant or a textbook special case, except where the
 * function header says "parity unpinned".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 8           /* highest supported polynomial degree        */
#define ORC_MAXNP 81         /* (ORC_MAXN+1)^2                               */
#define ORC_MAXM 9           /* conserved variables: GLM-MHD has 9           */
#define ORC_MAXS 8           /* Runge-Kutta stages                           */

enum { ORC_EULER = 0, ORC_MHD = 1 };
enum { ORC_VOL_CENTRAL = 0, ORC_VOL_KG = 1, ORC_VOL_RANOCHA = 2, ORC_VOL_DERIGS = 3 };
enum { ORC_LIM_NONE = 0, ORC_LIM_BLEND_MODAL = 1, ORC_LIM_BLEND_GIVEN = 2 };
enum { ORC_SURF_RUSANOV = 0, ORC_SURF_EC = 1 };

/* Problem description.  Field order is mirrored by oracle/__init__.py. */
typedef struct {
    int dim, nx, ny, N, eq;
    double x0, x1, y0, y1, gamma;
    int stages;
    double A[ORC_MAXS * ORC_MAXS];  /* Butcher A, row-major, strictly lower */
    double b[ORC_MAXS];
    int vol_flux;
    int limiter;
    double alpha_max, alpha_min;
    double cfl;
    double ch;                        /* GLM cleaning speed (MHD), fixed per step */
    int nthreads;
    int bc[2];                        /* per direction: ORC_BC_PERIODIC or ORC_BC_WALL */
    int nc_stagewise;                 /* MHD interface flux: 0 reduced form, 1 stage-wise */
} orc_problem;

enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1 };

/* ------------------------------------------------------------------ */
/* Small helpers                                                        */
/* ------------------------------------------------------------------ */
int orc_nvar(const orc_problem *P) { return P->eq == ORC_MHD ? 9 : P->dim + 2; }
static int np_of(const orc_problem *P) { return P->dim == 2 ? (P->N + 1) * (P->N + 1) : P->N + 1; }
static long nelem_of(const orc_problem *P) { return P->dim == 2 ? (long)P->nx * P->ny : (long)P->nx; }
static double dx_of(const orc_problem *P, int d)
{
    return d == 0 ? (P->x1 - P->x0) / P->nx : (P->y1 - P->y0) / P->ny;
}
static int nthreads_of(const orc_problem *P) { return P->nthreads > 0 ? P->nthreads : 1; }

/* ------------------------------------------------------------------ */
/* Layer 0: reference element (Section 2: GLL solution points on [0,1],  */
/* eq:diff.matrix).                                                     */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n and its derivative at x by the three-term
 * recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1} and
 * P'_{n+1} = P'_{n-1} + (2n+1) P_n. */
static void legendre(int n, double x, double *P, double *dP)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

/* GLL nodes xi and weights w on [0,1] for degree N >= 1: the endpoints and
 * the N-1 roots of P_N', found by Newton's method on P_N' with
 * P_N'' = (2x P_N' - N(N+1) P_N)/(1-x^2) (Legendre's equation); weights
 * 2/(N(N+1) P_N(x)^2) on [-1,1], halved for [0,1]. */
int orc_gll(int N, double *xi, double *w)
{
    if (N < 1 || N > ORC_MAXN) return -1;
    double x[ORC_MAXN + 1];
    x[0] = -1.0; x[N] = 1.0;
    for (int k = 1; k < N; ++k) {
        double t = -cos(M_PI * k / N);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, t, &P, &dP);
            double d2P = (2.0 * t * dP - N * (N + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[k] = t;
    }
    for (int k = 0; k <= N; ++k) {
        double P, dP;
        legendre(N, x[k], &P, &dP);
        xi[k] = 0.5 * (x[k] + 1.0);
        w[k] = 0.5 * 2.0 / (N * (N + 1.0) * P * P);
    }
    return 0;
}

/* D_pq = l_q'(xi_p), eq:diff.matrix, from the product form of the
 * Lagrange polynomial l_q(x) = prod_{m != q} (x - xi_m)/(xi_q - xi_m):
 * l_q'(x) = sum_{k != q} 1/(xi_q - xi_k) prod_{m != q,k} (x - xi_m)/(xi_q - xi_m). */
void orc_diffmat(int N, const double *xi, double *D)
{
    for (int p = 0; p <= N; ++p)
        for (int q = 0; q <= N; ++q) {
            double s = 0.0;
            for (int k = 0; k <= N; ++k) {
                if (k == q) continue;
                double prod = 1.0 / (xi[q] - xi[k]);
                for (int m = 0; m <= N; ++m) {
                    if (m == q || m == k) continue;
                    prod *= (xi[p] - xi[m]) / (xi[q] - xi[m]);
                }
                s += prod;
            }
            D[p * (N + 1) + q] = s;
        }
}

/* Derivatives of the g2 correction functions at the nodes (Section 2.3:
 * GLL points with g2).  Huynh's g2 is the left Radau combination
 * g_L = (N R_{N+1} + (N+1) R_N)/(2N+1) with R_k = (-1)^k (P_k - P_{k-1})/2
 * on [-1,1] (value 1 at -1, 0 at +1); on [0,1] d/dxi = 2 d/dx, and
 * g_R(xi) = g_L(1 - xi).  Used only by the semi-discrete FR operator. */
void orc_g2_derivatives(int N, const double *xi, double *dgL, double *dgR)
{
    for (int p = 0; p <= N; ++p) {
        double x = 2.0 * xi[p] - 1.0;
        double P1, dP1, P0, dP0, Pm, dPm;
        legendre(N + 1, x, &P1, &dP1);
        legendre(N, x, &P0, &dP0);
        legendre(N - 1, x, &Pm, &dPm);
        double sN1 = ((N + 1) % 2 == 0) ? 1.0 : -1.0;
        double sN = (N % 2 == 0) ? 1.0 : -1.0;
        double dR_N1 = sN1 * 0.5 * (dP1 - dP0);
        double dR_N = sN * 0.5 * (dP0 - dPm);
        dgL[p] = 2.0 * (N * dR_N1 + (N + 1) * dR_N) / (2.0 * N + 1.0);
        /* g_R(xi) = g_L(1 - xi)  =>  g_R'(xi_p) = -g_L'(1 - xi_p); by node
         * symmetry 1 - xi_p = xi_{N-p}, filled below. */
    }
    for (int p = 0; p <= N; ++p) dgR[p] = -dgL[N - p];
}

/* ------------------------------------------------------------------ */
/* Layer 1: physics (eq:flux.and.non.cons).                             */
/* Euler: u = (rho, rho v_1[, rho v_2], E), p = (gamma-1)(E - rho|v|^2/2).*/
/* GLM-MHD: u = (rho, rho v, E, B, psi) with v, B in R^3,                */
/*   E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2 + psi^2/2.                   */
/* ------------------------------------------------------------------ */
typedef struct {
    double rho, v[3], p, B[3], psi;
} prim_t;

static prim_t to_prim(const orc_problem *P, const double *u)
{
    prim_t s;
    memset(&s, 0, sizeof s);
    s.rho = u[0];
    if (P->eq == ORC_EULER) {
        int D = P->dim;
        for (int d = 0; d < D; ++d) s.v[d] = u[1 + d] / s.rho;
        double ke = 0.0;
        for (int d = 0; d < D; ++d) ke += 0.5 * s.rho * s.v[d] * s.v[d];
        s.p = (P->gamma - 1.0) * (u[D + 1] - ke);
    } else {
        for (int d = 0; d < 3; ++d) s.v[d] = u[1 + d] / s.rho;
        for (int d = 0; d < 3; ++d) s.B[d] = u[5 + d];
        s.psi = u[8];
        double v2 = s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2];
        double B2 = s.B[0] * s.B[0] + s.B[1] * s.B[1] + s.B[2] * s.B[2];
        s.p = (P->gamma - 1.0) * (u[4] - 0.5 * s.rho * v2 - 0.5 * B2 - 0.5 * s.psi * s.psi);
    }
    return s;
}

double orc_pressure(const orc_problem *P, const double *u) { return to_prim(P, u).p; }

/* physical flux f_d(u) in direction d */
void orc_phys_flux(const orc_problem *P, int d, const double *u, double *f)
{
    prim_t s = to_prim(P, u);
    double g = P->gamma;
    if (P->eq == ORC_EULER) {
        int D = P->dim;
        double vd = s.v[d];
        f[0] = s.rho * vd;
        for (int k = 0; k < D; ++k) f[1 + k] = s.rho * vd * s.v[k] + (k == d ? s.p : 0.0);
        f[D + 1] = (u[D + 1] + s.p) * vd;
    } else {
        double vd = s.v[d], Bd = s.B[d];
        double v2 = s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2];
        double B2 = s.B[0] * s.B[0] + s.B[1] * s.B[1] + s.B[2] * s.B[2];
        double vB = s.v[0] * s.B[0] + s.v[1] * s.B[1] + s.v[2] * s.B[2];
        f[0] = s.rho * vd;
        for (int k = 0; k < 3; ++k)
            f[1 + k] = s.rho * vd * s.v[k] - Bd * s.B[k] + (k == d ? s.p + 0.5 * B2 : 0.0);
        f[4] = vd * (0.5 * s.rho * v2 + g * s.p / (g - 1.0) + B2) - Bd * vB + P->ch * s.psi * Bd;
        for (int k = 0; k < 3; ++k)
            f[5 + k] = (k == d) ? P->ch * s.psi : vd * s.B[k] - Bd * s.v[k];
        f[8] = P->ch * Bd;
    }
}

/* Largest |eigenvalue| of f'(u) + B(u) g'(u) in direction d
 * (eq:rusanov.wave.speed, eq:combined.wave.speed).  Euler: |v_d| + c.
 * GLM-MHD: max(|v_d| + c_f, c_h), c_f the fast magnetosonic speed and
 * +-c_h the speeds of the divergence-cleaning subsystem. */
double orc_wave_speed(const orc_problem *P, int d, const double *u)
{
    prim_t s = to_prim(P, u);
    double a2 = P->gamma * s.p / s.rho;
    if (P->eq == ORC_EULER) return fabs(s.v[d]) + sqrt(a2);
    double B2 = s.B[0] * s.B[0] + s.B[1] * s.B[1] + s.B[2] * s.B[2];
    double t = a2 + B2 / s.rho;
    double cf = sqrt(0.5 * (t + sqrt(t * t - 4.0 * a2 * s.B[d] * s.B[d] / s.rho)));
    double lam = fabs(s.v[d]) + cf;
    return lam > P->ch ? lam : P->ch;
}

/* MHD fast-wave speed without the cleaning speed; c_h is its global max. */
static double mhd_fast_speed(const orc_problem *P, int d, const double *u)
{
    prim_t s = to_prim(P, u);
    double a2 = P->gamma * s.p / s.rho;
    double B2 = s.B[0] * s.B[0] + s.B[1] * s.B[1] + s.B[2] * s.B[2];
    double t = a2 + B2 / s.rho;
    double cf = sqrt(0.5 * (t + sqrt(t * t - 4.0 * a2 * s.B[d] * s.B[d] / s.rho)));
    return fabs(s.v[d]) + cf;
}

/* Non-conservative product B(u) g(u)_x (eq:flux.and.non.cons) for GLM-MHD:
 * Powell term phi_P(u) d_d B_d with phi_P = (0, B, v.B, v, 0) and GLM term
 * phi_G(u) d_d psi with phi_G = (0, 0, v_d psi, 0, v_d).  g_d(u) = (B_d, psi).
 * Returns B_d(u_a) applied to the g-vector (gB, gpsi). */
static void mhd_B_times(const orc_problem *P, int d, const double *ua, double gB, double gpsi, double *out)
{
    prim_t s = to_prim(P, ua);
    double vB = s.v[0] * s.B[0] + s.v[1] * s.B[1] + s.v[2] * s.B[2];
    out[0] = 0.0;
    for (int k = 0; k < 3; ++k) out[1 + k] = s.B[k] * gB;
    out[4] = vB * gB + s.v[d] * s.psi * gpsi;
    for (int k = 0; k < 3; ++k) out[5 + k] = s.v[k] * gB;
    out[8] = s.v[d] * gpsi;
}

/* (Bg)_NS(u_p, u_q) = B(u_p) g(u_q), eq:entropy.cons.noncons.dev; zero for Euler. */
void orc_nc_two_point(const orc_problem *P, int d, const double *up, const double *uq, double *out)
{
    int M = orc_nvar(P);
    if (P->eq != ORC_MHD) { for (int v = 0; v < M; ++v) out[v] = 0.0; return; }
    mhd_B_times(P, d, up, uq[5 + d], uq[8], out);
}

/* ------------------------------------------------------------------ */
/* Layer 2: two-point volume fluxes (eq:entropy.cons.flux.dev).         */
/* ------------------------------------------------------------------ */

/* Logarithmic mean (x - y)/(ln x - ln y).  Near x = y it uses
 * ln(x/y) = 2 artanh(f), f = (x-y)/(x+y), so with u = f^2 the mean is
 * (x + y)/(2 (1 + u/3 + u^2/5 + u^3/7)); switch at u < 1e-4. */
double orc_lnmean(double x, double y)
{
    double f = (x - y) / (x + y);
    double u = f * f;
    if (u < 1e-4) return (x + y) / (2.0 * (1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0));
    return (y - x) / log(y / x);
}

#define AVG(a, b) (0.5 * ((a) + (b)))

/* Symmetric two-point flux f_S,d(uL, uR) in direction d. */
void orc_two_point(const orc_problem *P, int d, const double *uL, const double *uR, double *f)
{
    int M = orc_nvar(P);
    double g = P->gamma;
    if (P->vol_flux == ORC_VOL_CENTRAL) {
        /* (f(uL) + f(uR))/2: recovers eq:flux.dev */
        double fL[ORC_MAXM], fR[ORC_MAXM];
        orc_phys_flux(P, d, uL, fL);
        orc_phys_flux(P, d, uR, fR);
        for (int v = 0; v < M; ++v) f[v] = AVG(fL[v], fR[v]);
        return;
    }
    prim_t L = to_prim(P, uL), R = to_prim(P, uR);
    if (P->eq == ORC_EULER) {
        int D = P->dim;
        if (P->vol_flux == ORC_VOL_KG) {
            /* Kennedy & Gruber: arithmetic means of rho, v, p and e = E/rho */
            double rho = AVG(L.rho, R.rho), vd = AVG(L.v[d], R.v[d]), p = AVG(L.p, R.p);
            double e = AVG(uL[D + 1] / L.rho, uR[D + 1] / R.rho);
            f[0] = rho * vd;
            for (int k = 0; k < D; ++k) f[1 + k] = rho * vd * AVG(L.v[k], R.v[k]) + (k == d ? p : 0.0);
            f[D + 1] = (rho * e + p) * vd;
        } else {
            /* Ranocha: EC and KEP, log means of rho and of rho/p */
            double rho_ln = orc_lnmean(L.rho, R.rho);
            double bet_ln = orc_lnmean(L.rho / L.p, R.rho / R.p);
            double vd = AVG(L.v[d], R.v[d]);
            double vv = 0.0;
            for (int k = 0; k < D; ++k) vv += 0.5 * L.v[k] * R.v[k];
            f[0] = rho_ln * vd;
            for (int k = 0; k < D; ++k) f[1 + k] = f[0] * AVG(L.v[k], R.v[k]) + (k == d ? AVG(L.p, R.p) : 0.0);
            f[D + 1] = f[0] * (1.0 / ((g - 1.0) * bet_ln) + vv) + 0.5 * (L.p * R.v[d] + R.p * L.v[d]);
        }
        return;
    }
    /* GLM-MHD, EC flux in the form of Derigs et al. (2018) with beta = rho/(2p) */
    double bL = 0.5 * L.rho / L.p, bR = 0.5 * R.rho / R.p;
    double rho_ln = orc_lnmean(L.rho, R.rho), b_ln = orc_lnmean(bL, bR);
    double rho_a = AVG(L.rho, R.rho), b_a = AVG(bL, bR), psi_a = AVG(L.psi, R.psi);
    double va[3], Ba[3];
    for (int k = 0; k < 3; ++k) { va[k] = AVG(L.v[k], R.v[k]); Ba[k] = AVG(L.B[k], R.B[k]); }
    double v2L = 0, v2R = 0, B2L = 0, B2R = 0, vBL = 0, vBR = 0;
    for (int k = 0; k < 3; ++k) {
        v2L += L.v[k] * L.v[k]; v2R += R.v[k] * R.v[k];
        B2L += L.B[k] * L.B[k]; B2R += R.B[k] * R.B[k];
        vBL += L.v[k] * L.B[k]; vBR += R.v[k] * R.B[k];
    }
    double ch = P->ch;
    f[0] = rho_ln * va[d];
    for (int k = 0; k < 3; ++k)
        f[1 + k] = f[0] * va[k] - Ba[d] * Ba[k] + (k == d ? rho_a / (2.0 * b_a) + 0.5 * AVG(B2L, B2R) : 0.0);
    for (int k = 0; k < 3; ++k)
        f[5 + k] = (k == d) ? ch * psi_a : va[d] * Ba[k] - va[k] * Ba[d];
    f[8] = ch * Ba[d];
    f[4] = f[0] * (1.0 / (2.0 * (g - 1.0) * b_ln) - 0.5 * AVG(v2L, v2R))
         + f[1] * va[0] + f[2] * va[1] + f[3] * va[2]
         + f[5] * Ba[0] + f[6] * Ba[1] + f[7] * Ba[2] + f[8] * psi_a
         - 0.5 * AVG(L.v[d] * B2L, R.v[d] * B2R) + Ba[d] * AVG(vBL, vBR)
         - ch * AVG(L.B[d] * L.psi, R.B[d] * R.psi);
    (void)M;
}

/* Entropy quantities used by the pins: S = -rho s/(gamma-1) with
 * s = ln p - gamma ln rho; entropy variables w = dS/du; entropy flux
 * q_d = S v_d; flux potential psi_d = w.f_d - q_d. */
double orc_entropy(const orc_problem *P, const double *u)
{
    prim_t s = to_prim(P, u);
    return -s.rho * (log(s.p) - P->gamma * log(s.rho)) / (P->gamma - 1.0);
}

void orc_entropy_vars(const orc_problem *P, const double *u, double *w)
{
    prim_t s = to_prim(P, u);
    double g = P->gamma, ent = log(s.p) - g * log(s.rho);
    double beta = 0.5 * s.rho / s.p;
    if (P->eq == ORC_EULER) {
        int D = P->dim;
        double v2 = 0.0;
        for (int k = 0; k < D; ++k) v2 += s.v[k] * s.v[k];
        w[0] = (g - ent) / (g - 1.0) - beta * v2;
        for (int k = 0; k < D; ++k) w[1 + k] = 2.0 * beta * s.v[k];
        w[D + 1] = -2.0 * beta;
    } else {
        double v2 = s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2];
        w[0] = (g - ent) / (g - 1.0) - beta * v2;
        for (int k = 0; k < 3; ++k) w[1 + k] = 2.0 * beta * s.v[k];
        w[4] = -2.0 * beta;
        for (int k = 0; k < 3; ++k) w[5 + k] = 2.0 * beta * s.B[k];
        w[8] = 2.0 * beta * s.psi;
    }
}

double orc_entropy_flux(const orc_problem *P, int d, const double *u)
{
    prim_t s = to_prim(P, u);
    return orc_entropy(P, u) * s.v[d];
}

double orc_flux_potential(const orc_problem *P, int d, const double *u)
{
    int M = orc_nvar(P);
    double w[ORC_MAXM], f[ORC_MAXM], wf = 0.0;
    orc_entropy_vars(P, u, w);
    orc_phys_flux(P, d, u, f);
    for (int v = 0; v < M; ++v) wf += w[v] * f[v];
    return wf - orc_entropy_flux(P, d, u);
}

/* ------------------------------------------------------------------ */
/* Layer 3: flux-differencing volume term of one element               */
/* (eq:entropy.cons.flux.dev, eq:entropy.cons.noncons.dev):             */
/*   R_p = sum_d 1/dx_d sum_q [2 D_pq f_S,d(u_p,u_q) + D_pq (Bg)_NS,d(u_p,u_q)] */
/* q runs over the nodes on the d-line through p, q = p included.       */
/* ue and R are [node][v] for one element.                              */
/* ------------------------------------------------------------------ */
typedef struct {
    int N, np, M;
    double xi[ORC_MAXN + 1], w[ORC_MAXN + 1], D[(ORC_MAXN + 1) * (ORC_MAXN + 1)];
} refel_t;

static void make_refel(const orc_problem *P, refel_t *r)
{
    r->N = P->N; r->np = np_of(P); r->M = orc_nvar(P);
    orc_gll(P->N, r->xi, r->w);
    orc_diffmat(P->N, r->xi, r->D);
}

static int node_index(const orc_problem *P, int i, int j) { return P->dim == 2 ? j * (P->N + 1) + i : i; }

static void volume_residual(const orc_problem *P, const refel_t *r, const double *ue, double *R)
{
    int N = P->N, M = r->M;
    for (int p = 0; p < r->np; ++p) for (int v = 0; v < M; ++v) R[p * M + v] = 0.0;
    for (int p = 0; p < r->np; ++p) {
        int ip = p % (N + 1), jp = p / (N + 1);
        for (int d = 0; d < P->dim; ++d) {
            double idx = 1.0 / dx_of(P, d);
            int pd = (d == 0) ? ip : jp;
            for (int qd = 0; qd <= N; ++qd) {
                int q = (d == 0) ? node_index(P, qd, jp) : node_index(P, ip, qd);
                double fs[ORC_MAXM], nc[ORC_MAXM];
                orc_two_point(P, d, ue + p * M, ue + q * M, fs);
                orc_nc_two_point(P, d, ue + p * M, ue + q * M, nc);
                double Dpq = r->D[pd * (N + 1) + qd];
                for (int v = 0; v < M; ++v) R[p * M + v] += idx * (2.0 * Dpq * fs[v] + Dpq * nc[v]);
            }
        }
    }
}

/* Exposed for the pins: volume term of one element, ue/R in [node][v]. */
void orc_volume_residual(const orc_problem *P, const double *ue, double *R)
{
    refel_t r;
    make_refel(P, &r);
    volume_residual(P, &r, ue, R);
}

/* ------------------------------------------------------------------ */
/* Mesh connectivity (uniform Cartesian, periodic).                      */
/* face f = 2*d + side; side 0: xi_d = 0, side 1: xi_d = 1.              */
/* ------------------------------------------------------------------ */
static long neighbour(const orc_problem *P, long e, int d, int side)
{
    if (P->dim == 1) return side ? (e + 1) % P->nx : (e - 1 + P->nx) % P->nx;
    long ex = e % P->nx, ey = e / P->nx;
    if (d == 0) ex = side ? (ex + 1) % P->nx : (ex - 1 + P->nx) % P->nx;
    else ey = side ? (ey + 1) % P->ny : (ey - 1 + P->ny) % P->ny;
    return ey * P->nx + ex;
}

/* Reflective (slip) walls: a face of direction d on the boundary of the
 * domain (the paper does not state the boundary conditions of its
 * Richtmyer-Meshkov test; walls are this oracle's reading).  Outside the
 * wall lies the mirror image of the element: the state with the normal
 * momentum negated, evolving as the mirror image of the element. */
static int at_wall(const orc_problem *P, long e, int d, int side)
{
    if (P->bc[d] != ORC_BC_WALL) return 0;
    long ex = P->dim == 1 ? e : e % P->nx, ey = P->dim == 1 ? 0 : e / P->nx;
    long i = d == 0 ? ex : ey, n = d == 0 ? P->nx : P->ny;
    return side ? i == n - 1 : i == 0;
}

/* the face neighbour, or e itself across a wall (its mirror image) */
static long neighbour_or_self(const orc_problem *P, long e, int d, int side)
{
    return at_wall(P, e, d, side) ? e : neighbour(P, e, d, side);
}

/* mirror image across a wall normal to direction d (Euler): rho v_d -> -rho v_d */
static void mirror_state(const orc_problem *P, int d, const double *u, double *out)
{
    int M = orc_nvar(P);
    for (int v = 0; v < M; ++v) out[v] = u[v];
    out[1 + d] = -u[1 + d];
}

static int nface_nodes(const orc_problem *P) { return P->dim == 2 ? P->N + 1 : 1; }

/* node of face (d, side) with face-node index k */
static int face_node(const orc_problem *P, int d, int side, int k)
{
    int end = side ? P->N : 0;
    if (P->dim == 1) return end;
    return d == 0 ? node_index(P, end, k) : node_index(P, k, end);
}

static void gather_elem(const orc_problem *P, const double *u, long e, double *ue)
{
    int M = orc_nvar(P), np = np_of(P);
    long E = nelem_of(P);
    for (int p = 0; p < np; ++p)
        for (int v = 0; v < M; ++v) ue[p * M + v] = u[((long)v * E + e) * np + p];
}

static void scatter_elem(const orc_problem *P, double *u, long e, const double *ue)
{
    int M = orc_nvar(P), np = np_of(P);
    long E = nelem_of(P);
    for (int p = 0; p < np; ++p)
        for (int v = 0; v < M; ++v) u[((long)v * E + e) * np + p] = ue[p * M + v];
}

/* ------------------------------------------------------------------ */
/* Layer 7: time step.  dt = CFL / ((N+1) max_{e,p} sum_d lambda_d/dx_d). */
/* For MHD, c_h = max_{e,p,d} (|v_d| + c_f) of u^n is returned first and  */
/* enters lambda_d.  (The paper does not give its CFL rule.)             */
/* ------------------------------------------------------------------ */
double orc_compute_ch(const orc_problem *P, const double *u)
{
    if (P->eq != ORC_MHD) return 0.0;
    int M = orc_nvar(P), np = np_of(P);
    long E = nelem_of(P);
    double ch = 0.0;
    for (long e = 0; e < E; ++e)
        for (int p = 0; p < np; ++p) {
            double up[ORC_MAXM];
            for (int v = 0; v < M; ++v) up[v] = u[((long)v * E + e) * np + p];
            for (int d = 0; d < P->dim; ++d) {
                double l = mhd_fast_speed(P, d, up);
                if (l > ch) ch = l;
            }
        }
    return ch;
}

double orc_compute_dt(const orc_problem *P, const double *u)
{
    int M = orc_nvar(P), np = np_of(P);
    long E = nelem_of(P);
    double mx = 0.0;
    for (long e = 0; e < E; ++e)
        for (int p = 0; p < np; ++p) {
            double up[ORC_MAXM], s = 0.0;
            for (int v = 0; v < M; ++v) up[v] = u[((long)v * E + e) * np + p];
            for (int d = 0; d < P->dim; ++d) s += orc_wave_speed(P, d, up) / dx_of(P, d);
            if (s > mx) mx = s;
        }
    return P->cfl / ((P->N + 1) * mx);
}

/* ------------------------------------------------------------------ */
/* Blending limiter indicator: modal energy of eps = rho*p in the        */
/* orthonormal Legendre basis phi_k(xi) = sqrt(2k+1) P_k(2xi-1), the     */
/* Hennemann-Gassner form (the paper uses the blending limiter of its     */
/* cited works with alpha_max; the indicator itself is not printed).     */
/* alpha_raw per element; features = m_kl^2 / sum m^2 (np values).      */
/* ------------------------------------------------------------------ */

/* solve V m = eps by Gaussian elimination with partial pivoting (n <= 9) */
static void solve_dense(int n, const double *Vin, const double *rhs, double *x)
{
    double A[(ORC_MAXN + 1) * (ORC_MAXN + 1)], bb[ORC_MAXN + 1];
    memcpy(A, Vin, sizeof(double) * n * n);
    memcpy(bb, rhs, sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r) if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            double t = bb[c]; bb[c] = bb[piv]; bb[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double fct = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= fct * A[c * n + k];
            bb[r] -= fct * bb[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = bb[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
}

static void modal_coefficients(const orc_problem *P, const refel_t *r, const double *eps, double *m)
{
    int n = P->N + 1;
    double V[(ORC_MAXN + 1) * (ORC_MAXN + 1)];
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < n; ++k) {
            double Pk, dPk;
            legendre(k, 2.0 * r->xi[p] - 1.0, &Pk, &dPk);
            V[p * n + k] = sqrt(2.0 * k + 1.0) * Pk;
        }
    if (P->dim == 1) { solve_dense(n, V, eps, m); return; }
    /* eps(xi_i, eta_j) = sum_kl m_kl phi_k(xi_i) phi_l(eta_j): solve in x for
     * every row j, then in y for every mode k. */
    double t[ORC_MAXNP], col[ORC_MAXN + 1], sol[ORC_MAXN + 1];
    for (int j = 0; j < n; ++j) solve_dense(n, V, eps + j * n, t + j * n);   /* t[j][k] */
    for (int k = 0; k < n; ++k) {
        for (int j = 0; j < n; ++j) col[j] = t[j * n + k];
        solve_dense(n, V, col, sol);
        for (int l = 0; l < n; ++l) m[l * n + k] = sol[l];                  /* m[l][k] */
    }
}

static double indicator_element(const orc_problem *P, const refel_t *r, const double *ue, double *feat)
{
    int N = P->N, n = N + 1, M = r->M;
    double eps[ORC_MAXNP], m[ORC_MAXNP];
    for (int p = 0; p < r->np; ++p) {
        prim_t s = to_prim(P, ue + p * M);
        eps[p] = s.rho * s.p;
    }
    modal_coefficients(P, r, eps, m);
    double tot = 0.0, c1 = 0.0, c2 = 0.0;
    for (int p = 0; p < r->np; ++p) {
        int k = p % n, l = (P->dim == 2) ? p / n : 0;
        double e2 = m[p] * m[p];
        tot += e2;
        if (k <= N - 1 && l <= N - 1) c1 += e2;
        if (k <= N - 2 && l <= N - 2) c2 += e2;
    }
    if (feat) for (int p = 0; p < r->np; ++p) feat[p] = m[p] * m[p] / tot;
    double E1 = (tot - c1) / tot, E2 = (c1 - c2) / c1;
    double Ener = E1 > E2 ? E1 : E2;
    double T = 0.5 * pow(10.0, -1.8 * pow(N + 1.0, 0.25));
    double s = log((1.0 - 1e-4) / 1e-4);
    double a = 1.0 / (1.0 + exp(-(s / T) * (Ener - T)));
    if (a < P->alpha_min) a = 0.0;
    if (a > 1.0 - P->alpha_min) a = 1.0;
    if (a > P->alpha_max) a = P->alpha_max;
    return a;
}

/* Smoothing of the blending coefficients over face neighbours:
 * alpha_e <- max(alpha_e, max over face neighbours of alpha_nb / 2)
 * (beyond a wall the neighbour is the element's mirror image, whose
 * coefficient is its own). */
void orc_smooth_alpha(const orc_problem *P, const double *alpha_raw, double *alpha)
{
    long E = nelem_of(P);
    for (long e = 0; e < E; ++e) {
        double a = alpha_raw[e];
        for (int d = 0; d < P->dim; ++d)
            for (int side = 0; side < 2; ++side) {
                double an = 0.5 * alpha_raw[neighbour_or_self(P, e, d, side)];
                if (an > a) a = an;
            }
        alpha[e] = a;
    }
}

/* alpha_raw[e] (clipped, capped) and alpha[e] after smoothing. */
int orc_indicator(const orc_problem *P, const double *u, double *alpha_raw, double *alpha, double *features)
{
    refel_t r;
    make_refel(P, &r);
    long E = nelem_of(P);
    int np = r.np;
#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, u, e, ue);
        alpha_raw[e] = indicator_element(P, &r, ue, features ? features + e * np : NULL);
    }
    orc_smooth_alpha(P, alpha_raw, alpha);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Layers 3-6: one cRKFR step (eq:crkfr.inner, eq:crkfr.non.cons.final,  */
/* eq:disc.avg.flux, eq:local.time.avg.non.cons, eq:numflux.cons and the  */
/* reduced-communication non-conservative interface flux of Section 2.3,  */
/* with the EC/KEP volume terms of Section 3).                            */
/*                                                                       */
/* Readings where the paper is silent:                                   */
/*  - the Rusanov speed lambda uses the u^n traces of both sides;        */
/*  - the non-conservative interface flux is 1/2 B(u^{n,+-}) (g(U^-) +     */
/*    g(U^+)), the factor 1/2 of eq:non.cons.num.flux.basic kept;         */
/*  - with GLL points and g2, dg_R/dxi = delta_{pN}/w_N and                */
/*    dg_L/dxi = -delta_{p0}/w_0 at the nodes;                            */
/*  - blending: u^{n+1} = (1-alpha_e) u^H + alpha_e u^L, u^L first-order   */
/*    Rusanov FV on the GLL subcells (widths w_k dx) from u^n; at element  */
/*    faces both schemes use F = (1-a) F^H + a f^L(u^n-, u^n+) with        */
/*    a = (alpha_e + alpha_nb)/2.                                          */
/* traces: Ut/Ft/Fnct[e][face][k][v].                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    double *Ut, *Ft, *Fnct;
    /* at wall faces, the traces of the mirror image beyond the wall:
     * sum_j b_j R u^(j) and sum_j b_j f_d(R u^(j)) (NULL without walls) */
    double *UGt, *FGt;
    /* stage-wise non-conservative interface flux: the stage states u^(j) at
     * the face nodes, [e][face][k][j][v] (NULL otherwise) */
    double *Ust;
} traces_t;

static long tr_index(const orc_problem *P, long e, int face, int k, int v)
{
    int nf = nface_nodes(P), M = orc_nvar(P);
    return (((e * (2 * P->dim) + face) * nf + k) * M + v);
}

static long st_index(const orc_problem *P, long e, int face, int k, int j, int v)
{
    int nf = nface_nodes(P), M = orc_nvar(P);
    return ((((e * (2 * P->dim) + face) * nf + k) * P->stages + j) * M + v);
}

static int has_walls(const orc_problem *P) { return P->bc[0] == ORC_BC_WALL || (P->dim == 2 && P->bc[1] == ORC_BC_WALL); }

static void traces_alloc(const orc_problem *P, traces_t *T)
{
    long ntr = nelem_of(P) * 2 * P->dim * nface_nodes(P) * orc_nvar(P);
    T->Ut = malloc(sizeof(double) * ntr);
    T->Ft = malloc(sizeof(double) * ntr);
    T->Fnct = malloc(sizeof(double) * ntr);
    T->UGt = has_walls(P) ? calloc(ntr, sizeof(double)) : NULL;
    T->FGt = has_walls(P) ? calloc(ntr, sizeof(double)) : NULL;
    T->Ust = P->nc_stagewise ? malloc(sizeof(double) * ntr * P->stages) : NULL;
}

static void traces_free(traces_t *T)
{
    free(T->Ut); free(T->Ft); free(T->Fnct); free(T->UGt); free(T->FGt); free(T->Ust);
}

/* inner stages, time averages and traces of element e; V[node][v] */
static void local_stages(const orc_problem *P, const refel_t *r, const double *un_e, double dt,
                         double *V, traces_t *T, long e)
{
    int M = r->M, np = r->np, S = P->stages;
    double *us = malloc(sizeof(double) * S * np * M);
    double *R = malloc(sizeof(double) * S * np * M);
    for (int i = 0; i < S; ++i) {
        /* u^(i) = u^n - dt sum_{j<i} a_ij R^(j)   (eq:crkfr.inner) */
        for (int p = 0; p < np; ++p)
            for (int v = 0; v < M; ++v) {
                double acc = 0.0;
                for (int j = 0; j < i; ++j) acc += P->A[i * ORC_MAXS + j] * R[(j * np + p) * M + v];
                us[(i * np + p) * M + v] = un_e[p * M + v] - dt * acc;
            }
        volume_residual(P, r, us + i * np * M, R + i * np * M);
    }
    /* time-averaged volume term V = sum_j b_j R^(j) */
    for (int p = 0; p < np; ++p)
        for (int v = 0; v < M; ++v) {
            double acc = 0.0;
            for (int j = 0; j < S; ++j) acc += P->b[j] * R[(j * np + p) * M + v];
            V[p * M + v] = acc;
        }
    /* traces: U = sum b_j u^(j), F = sum b_j f_d(u^(j)), Fnc = sum b_j B_d(u^(j)) g_d(u^(j)) */
    for (int d = 0; d < P->dim; ++d)
        for (int side = 0; side < 2; ++side)
            for (int k = 0; k < nface_nodes(P); ++k) {
                int p = face_node(P, d, side, k), face = 2 * d + side;
                for (int v = 0; v < M; ++v) {
                    T->Ut[tr_index(P, e, face, k, v)] = 0.0;
                    T->Ft[tr_index(P, e, face, k, v)] = 0.0;
                    T->Fnct[tr_index(P, e, face, k, v)] = 0.0;
                    if (T->UGt) T->UGt[tr_index(P, e, face, k, v)] = T->FGt[tr_index(P, e, face, k, v)] = 0.0;
                }
                int wall = at_wall(P, e, d, side);
                for (int j = 0; j < S; ++j) {
                    const double *uj = us + (j * np + p) * M;
                    double f[ORC_MAXM], nc[ORC_MAXM];
                    orc_phys_flux(P, d, uj, f);
                    orc_nc_two_point(P, d, uj, uj, nc);
                    for (int v = 0; v < M; ++v) {
                        T->Ut[tr_index(P, e, face, k, v)] += P->b[j] * uj[v];
                        T->Ft[tr_index(P, e, face, k, v)] += P->b[j] * f[v];
                        T->Fnct[tr_index(P, e, face, k, v)] += P->b[j] * nc[v];
                    }
                    if (wall) {
                        /* the mirror image evolves as the mirror of the element */
                        double um[ORC_MAXM], fm[ORC_MAXM];
                        mirror_state(P, d, uj, um);
                        orc_phys_flux(P, d, um, fm);
                        for (int v = 0; v < M; ++v) {
                            T->UGt[tr_index(P, e, face, k, v)] += P->b[j] * um[v];
                            T->FGt[tr_index(P, e, face, k, v)] += P->b[j] * fm[v];
                        }
                    }
                    if (T->Ust)
                        for (int v = 0; v < M; ++v) T->Ust[st_index(P, e, face, k, j, v)] = uj[v];
                }
            }
    free(us);
    free(R);
}

static void rusanov(const orc_problem *P, int d, double lam, const double *fL, const double *fR,
                    const double *uL, const double *uR, double *out)
{
    int M = orc_nvar(P);
    for (int v = 0; v < M; ++v) out[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]);
}

/* Conservative interface flux at face node k of face (d, side) of element
 * e (eq:numflux.cons): Rusanov flux of the time averages with lambda from
 * the u^n traces of both sides, blended with the first-order flux of u^n by
 * a = (alpha_e + alpha_nb)/2 when alpha != NULL.  uno, unn: u^n at this
 * face node and at the neighbour's facing node. */
static void interface_flux(const orc_problem *P, const traces_t *T, const double *alpha, long e, long en, int d,
                           int side, int k, const double *uno, const double *unn, double *Fnum)
{
    int M = orc_nvar(P), face = 2 * d + side, nface = 2 * d + (1 - side);
    const double *Uo = T->Ut + tr_index(P, e, face, k, 0);
    const double *Fo = T->Ft + tr_index(P, e, face, k, 0);
    const double *Un = T->Ut + tr_index(P, en, nface, k, 0);
    const double *Fn = T->Ft + tr_index(P, en, nface, k, 0);
    if (at_wall(P, e, d, side)) {
        /* beyond a wall: the mirror image's traces (en = e, unn = R uno) */
        Un = T->UGt + tr_index(P, e, face, k, 0);
        Fn = T->FGt + tr_index(P, e, face, k, 0);
    }
    /* left (-) and right (+) states of this interface */
    const double *UL = side ? Uo : Un, *UR = side ? Un : Uo;
    const double *FL = side ? Fo : Fn, *FR = side ? Fn : Fo;
    const double *uL = side ? uno : unn, *uR = side ? unn : uno;
    double lL = orc_wave_speed(P, d, uL), lR = orc_wave_speed(P, d, uR);
    double lam = lL > lR ? lL : lR;
    rusanov(P, d, lam, FL, FR, UL, UR, Fnum);
    if (alpha) {
        double fL[ORC_MAXM], fR[ORC_MAXM], flo[ORC_MAXM];
        orc_phys_flux(P, d, uL, fL);
        orc_phys_flux(P, d, uR, fR);
        rusanov(P, d, lam, fL, fR, uL, uR, flo);
        double a = 0.5 * (alpha[e] + alpha[en]);
        for (int v = 0; v < M; ++v) Fnum[v] = (1.0 - a) * Fnum[v] + a * flo[v];
    }
}

int orc_crk_step(const orc_problem *P, const double *un, double dt, const double *alpha_in,
                 double *unew, double *alpha_out)
{
    if (P->N < 1 || P->N > ORC_MAXN || P->stages < 1 || P->stages > ORC_MAXS) return -1;
    if (P->limiter != ORC_LIM_NONE && P->eq != ORC_EULER) return -2;
    if (has_walls(P) && P->eq != ORC_EULER) return -3;
    refel_t r;
    make_refel(P, &r);
    int M = r.M, np = r.np, N = P->N, nf = nface_nodes(P);
    long E = nelem_of(P);
    double *V = malloc(sizeof(double) * E * np * M);
    traces_t T;
    traces_alloc(P, &T);
    double *alpha = calloc(E, sizeof(double));

#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, un, e, ue);
        local_stages(P, &r, ue, dt, V + e * np * M, &T, e);
    }

    if (P->limiter == ORC_LIM_BLEND_MODAL) {
        double *araw = malloc(sizeof(double) * E);
        orc_indicator(P, un, araw, alpha, NULL);
        free(araw);
    } else if (P->limiter == ORC_LIM_BLEND_GIVEN) {
        for (long e = 0; e < E; ++e) alpha[e] = alpha_in[e];
    }
    if (alpha_out) for (long e = 0; e < E; ++e) alpha_out[e] = alpha[e];

#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM], uH[ORC_MAXNP * ORC_MAXM], uLo[ORC_MAXNP * ORC_MAXM];
        double Fstar[4][ORC_MAXN + 1][ORC_MAXM];
        gather_elem(P, un, e, ue);
        for (int p = 0; p < np; ++p)
            for (int v = 0; v < M; ++v) uH[p * M + v] = ue[p * M + v] - dt * V[(e * np + p) * M + v];
        for (int d = 0; d < P->dim; ++d) {
            double idx = 1.0 / dx_of(P, d);
            for (int side = 0; side < 2; ++side) {
                long en = neighbour_or_self(P, e, d, side);
                int wall = at_wall(P, e, d, side);
                int face = 2 * d + side, nface = 2 * d + (1 - side);
                double une[ORC_MAXNP * ORC_MAXM];
                gather_elem(P, un, en, une);
                for (int k = 0; k < nf; ++k) {
                    int p = face_node(P, d, side, k), pn = face_node(P, d, 1 - side, k);
                    const double *Uo = T.Ut + tr_index(P, e, face, k, 0);
                    const double *Fo = T.Ft + tr_index(P, e, face, k, 0);
                    const double *Fnco = T.Fnct + tr_index(P, e, face, k, 0);
                    const double *Un = T.Ut + tr_index(P, en, nface, k, 0);
                    const double *uno = ue + p * M, *unn = une + pn * M;
                    double umir[ORC_MAXM];
                    if (wall) {
                        mirror_state(P, d, uno, umir);
                        unn = umir;
                    }
                    const double *UL = side ? Uo : Un, *UR = side ? Un : Uo;
                    double Fnum[ORC_MAXM];
                    interface_flux(P, &T, P->limiter != ORC_LIM_NONE ? alpha : NULL, e, en, d, side, k, uno, unn,
                                   Fnum);
                    for (int v = 0; v < M; ++v) Fstar[face][k][v] = Fnum[v];
                    double ncn[ORC_MAXM];
                    for (int v = 0; v < M; ++v) ncn[v] = 0.0;
                    if (P->eq == ORC_MHD && !P->nc_stagewise) {
                        /* non-conservative interface flux of the own side, reduced
                         * form: 1/2 B(u^n_own) (g(U^-) + g(U^+)) */
                        double gB = UL[5 + d] + UR[5 + d], gpsi = UL[8] + UR[8];
                        mhd_B_times(P, d, uno, 0.5 * gB, 0.5 * gpsi, ncn);
                    } else if (P->eq == ORC_MHD) {
                        /* stage-wise form (eq:bad.numflux.non.cons):
                         * sum_j b_j 1/2 B(u^(j)_own) (g(u^(j),-) + g(u^(j),+)) */
                        for (int j = 0; j < P->stages; ++j) {
                            const double *uo_j = T.Ust + st_index(P, e, face, k, j, 0);
                            const double *un_j = T.Ust + st_index(P, en, nface, k, j, 0);
                            double o[ORC_MAXM];
                            mhd_B_times(P, d, uo_j, 0.5 * (uo_j[5 + d] + un_j[5 + d]), 0.5 * (uo_j[8] + un_j[8]), o);
                            for (int v = 0; v < M; ++v) ncn[v] += P->b[j] * o[v];
                        }
                    }
                    /* eq:crkfr.non.cons.final with dg_R = delta_pN/w_N, dg_L = -delta_p0/w_0 */
                    for (int v = 0; v < M; ++v) {
                        double jump = Fnum[v] + ncn[v] - Fo[v] - Fnco[v];
                        if (side) uH[p * M + v] -= dt * idx * jump / r.w[N];
                        else uH[p * M + v] += dt * idx * jump / r.w[0];
                    }
                }
            }
        }
        if (P->limiter == ORC_LIM_NONE) {
            scatter_elem(P, unew, e, uH);
            continue;
        }
        /* low-order scheme: first-order Rusanov FV on the GLL subcells */
        for (int p = 0; p < np; ++p) for (int v = 0; v < M; ++v) uLo[p * M + v] = ue[p * M + v];
        for (int d = 0; d < P->dim; ++d) {
            double idx = 1.0 / dx_of(P, d);
            for (int k = 0; k < nf; ++k) {
                /* the line of nodes along direction d with transverse index k */
                int line[ORC_MAXN + 1];
                for (int c = 0; c <= N; ++c)
                    line[c] = (P->dim == 1) ? c : (d == 0 ? node_index(P, c, k) : node_index(P, k, c));
                /* subcell interface fluxes fl[c] at the right end of subcell c, c=-1..N */
                double fl[ORC_MAXN + 2][ORC_MAXM];
                for (int v = 0; v < M; ++v) {
                    fl[0][v] = Fstar[2 * d + 0][k][v];
                    fl[N + 1][v] = Fstar[2 * d + 1][k][v];
                }
                for (int c = 0; c < N; ++c) {
                    const double *a = ue + line[c] * M, *b = ue + line[c + 1] * M;
                    double fa[ORC_MAXM], fb[ORC_MAXM];
                    orc_phys_flux(P, d, a, fa);
                    orc_phys_flux(P, d, b, fb);
                    double la = orc_wave_speed(P, d, a), lb = orc_wave_speed(P, d, b);
                    rusanov(P, d, la > lb ? la : lb, fa, fb, a, b, fl[c + 1]);
                }
                for (int c = 0; c <= N; ++c)
                    for (int v = 0; v < M; ++v)
                        uLo[line[c] * M + v] -= dt * idx / r.w[c] * (fl[c + 1][v] - fl[c][v]);
            }
        }
        double ub[ORC_MAXNP * ORC_MAXM];
        for (int p = 0; p < np; ++p)
            for (int v = 0; v < M; ++v) ub[p * M + v] = (1.0 - alpha[e]) * uH[p * M + v] + alpha[e] * uLo[p * M + v];
        scatter_elem(P, unew, e, ub);
    }
    free(V); traces_free(&T); free(alpha);
    return 0;
}

/* Stage volume term, time averages and traces of the whole mesh, for the
 * pins and for parity of the local-stage phase.  V in the state layout
 * [v][e][node]; traces Ut/Ft/Fnct as [e][face][k][v]. */
int orc_local_phase(const orc_problem *P, const double *un, double dt, double *V, double *Ut, double *Ft, double *Fnct)
{
    refel_t r;
    make_refel(P, &r);
    int M = r.M, np = r.np;
    long E = nelem_of(P), ntr = E * 2 * P->dim * nface_nodes(P) * M;
    traces_t T;
    traces_alloc(P, &T);
    double *Ve = malloc(sizeof(double) * E * np * M);
#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, un, e, ue);
        local_stages(P, &r, ue, dt, Ve + e * np * M, &T, e);
    }
    for (long e = 0; e < E; ++e) scatter_elem(P, V, e, Ve + e * np * M);
    memcpy(Ut, T.Ut, sizeof(double) * ntr);
    memcpy(Ft, T.Ft, sizeof(double) * ntr);
    memcpy(Fnct, T.Fnct, sizeof(double) * ntr);
    free(Ve);
    traces_free(&T);
    return 0;
}

/* Interface fluxes of one cRKFR step: Fstar[e][face][k][v] (the layout of
 * the traces) from the local phase's time averages and u^n; alpha = NULL
 * for no blending. */
int orc_face_fluxes(const orc_problem *P, const double *un, double dt, const double *alpha, double *Fstar)
{
    if (has_walls(P) && P->eq != ORC_EULER) return -3;
    refel_t r;
    make_refel(P, &r);
    int M = r.M, nf = nface_nodes(P);
    long E = nelem_of(P);
    traces_t T;
    traces_alloc(P, &T);
#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM], V[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, un, e, ue);
        local_stages(P, &r, ue, dt, V, &T, e);
    }
#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM], une[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, un, e, ue);
        for (int d = 0; d < P->dim; ++d)
            for (int side = 0; side < 2; ++side) {
                long en = neighbour_or_self(P, e, d, side);
                gather_elem(P, un, en, une);
                for (int k = 0; k < nf; ++k) {
                    int p = face_node(P, d, side, k), pn = face_node(P, d, 1 - side, k);
                    double umir[ORC_MAXM];
                    const double *unn = une + pn * M;
                    if (at_wall(P, e, d, side)) {
                        mirror_state(P, d, ue + p * M, umir);
                        unn = umir;
                    }
                    interface_flux(P, &T, alpha, e, en, d, side, k, ue + p * M, unn,
                                   Fstar + tr_index(P, e, 2 * d + side, k, 0));
                }
            }
    }
    traces_free(&T);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Semi-discrete FR operator (eq:general.non.conservative.fr.one with    */
/* the flux-differencing volume term), written with the g2 correction     */
/* derivatives from the Radau construction rather than the lifting 1/w.   */
/* Used by the pins (s=1 equivalence, EC surface flux => zero entropy     */
/* rate) and by the standard multi-stage RKFR step (eq:rkfr.non.cons).    */
/* rhs = du/dt in the state layout.                                       */
/* ------------------------------------------------------------------ */
int orc_fr_rhs(const orc_problem *P, const double *u, int surface, double *rhs)
{
    if (has_walls(P) && P->eq != ORC_EULER) return -3;
    refel_t r;
    make_refel(P, &r);
    int M = r.M, np = r.np, N = P->N, nf = nface_nodes(P);
    long E = nelem_of(P);
    double dgL[ORC_MAXN + 1], dgR[ORC_MAXN + 1];
    orc_g2_derivatives(N, r.xi, dgL, dgR);
#pragma omp parallel for num_threads(nthreads_of(P)) schedule(static)
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM], R[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, u, e, ue);
        volume_residual(P, &r, ue, R);
        for (int p = 0; p < np; ++p) for (int v = 0; v < M; ++v) R[p * M + v] = -R[p * M + v];
        for (int d = 0; d < P->dim; ++d) {
            double idx = 1.0 / dx_of(P, d);
            for (int side = 0; side < 2; ++side) {
                long en = neighbour_or_self(P, e, d, side);
                double une[ORC_MAXNP * ORC_MAXM];
                gather_elem(P, u, en, une);
                for (int k = 0; k < nf; ++k) {
                    int p = face_node(P, d, side, k), pn = face_node(P, d, 1 - side, k);
                    const double *uo = ue + p * M, *unb = une + pn * M;
                    double umir[ORC_MAXM];
                    if (at_wall(P, e, d, side)) {
                        /* beyond a wall: the mirror image of this node */
                        mirror_state(P, d, uo, umir);
                        unb = umir;
                    }
                    const double *uL = side ? uo : unb, *uR = side ? unb : uo;
                    double fnum[ORC_MAXM], fo[ORC_MAXM], nco[ORC_MAXM], ncn[ORC_MAXM];
                    if (surface == ORC_SURF_EC) {
                        orc_two_point(P, d, uL, uR, fnum);
                    } else {
                        double fL[ORC_MAXM], fR[ORC_MAXM];
                        orc_phys_flux(P, d, uL, fL);
                        orc_phys_flux(P, d, uR, fR);
                        double lL = orc_wave_speed(P, d, uL), lR = orc_wave_speed(P, d, uR);
                        rusanov(P, d, lL > lR ? lL : lR, fL, fR, uL, uR, fnum);
                    }
                    orc_phys_flux(P, d, uo, fo);
                    orc_nc_two_point(P, d, uo, uo, nco);
                    if (P->eq == ORC_MHD) {
                        mhd_B_times(P, d, uo, 0.5 * (uL[5 + d] + uR[5 + d]), 0.5 * (uL[8] + uR[8]), ncn);
                    } else {
                        for (int v = 0; v < M; ++v) ncn[v] = 0.0;
                    }
                    /* the correction acts on every node of the line */
                    for (int c = 0; c <= N; ++c) {
                        int q = (P->dim == 1) ? c : (d == 0 ? node_index(P, c, k) : node_index(P, k, c));
                        double dg = side ? dgR[c] : dgL[c];
                        for (int v = 0; v < M; ++v)
                            R[q * M + v] -= idx * (fnum[v] + ncn[v] - fo[v] - nco[v]) * dg;
                    }
                }
            }
        }
        scatter_elem(P, rhs, e, R);
    }
    return 0;
}

/* Standard s-stage RKFR step (eq:rkfr.non.cons): s interface exchanges. */
int orc_rkfr_step(const orc_problem *P, const double *un, double dt, double *unew)
{
    int M = orc_nvar(P), np = np_of(P), S = P->stages;
    long n = nelem_of(P) * np * M;
    double *K = malloc(sizeof(double) * S * n), *ui = malloc(sizeof(double) * n);
    for (int i = 0; i < S; ++i) {
        for (long t = 0; t < n; ++t) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += P->A[i * ORC_MAXS + j] * K[j * n + t];
            ui[t] = un[t] + dt * acc;
        }
        orc_fr_rhs(P, ui, ORC_SURF_RUSANOV, K + i * n);
    }
    for (long t = 0; t < n; ++t) {
        double acc = 0.0;
        for (int j = 0; j < S; ++j) acc += P->b[j] * K[j * n + t];
        unew[t] = un[t] + dt * acc;
    }
    free(K); free(ui);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Diagnostics (FP64): out[0..M-1] = totals sum_e sum_p w_p u_p |Omega_e|, */
/* out[M] = total entropy, out[M+1] = min rho, out[M+2] = min p,           */
/* out[M+3] = number of non-finite values, out[M+4] = first element that   */
/* is non-finite or has rho <= 0 or p <= 0 (-1 if none).                   */
/* ------------------------------------------------------------------ */
int orc_diagnostics(const orc_problem *P, const double *u, double *out)
{
    refel_t r;
    make_refel(P, &r);
    int M = r.M, np = r.np, N = P->N;
    long E = nelem_of(P);
    double vol = dx_of(P, 0) * (P->dim == 2 ? dx_of(P, 1) : 1.0);
    double tot[ORC_MAXM] = {0}, ent = 0.0, minr = INFINITY, minp = INFINITY, nbad = 0.0;
    long first = -1;
    for (long e = 0; e < E; ++e) {
        double ue[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, u, e, ue);
        int bad = 0;
        for (int p = 0; p < np; ++p) {
            int i = p % (N + 1), j = (P->dim == 2) ? p / (N + 1) : 0;
            double wq = r.w[i] * (P->dim == 2 ? r.w[j] : 1.0) * vol;
            for (int v = 0; v < M; ++v) {
                if (!isfinite(ue[p * M + v])) { nbad += 1.0; bad = 1; }
                tot[v] += wq * ue[p * M + v];
            }
            double rho = ue[p * M], pr = orc_pressure(P, ue + p * M);
            if (!(rho > 0.0) || !(pr > 0.0)) bad = 1;
            if (rho < minr) minr = rho;
            if (pr < minp) minp = pr;
            if (rho > 0.0 && pr > 0.0) ent += wq * orc_entropy(P, ue + p * M);
        }
        if (bad && first < 0) first = e;
    }
    for (int v = 0; v < M; ++v) out[v] = tot[v];
    out[M] = ent; out[M + 1] = minr; out[M + 2] = minp; out[M + 3] = nbad; out[M + 4] = (double)first;
    return 0;
}

/* Input of the learned indicator: the modal energy fractions f on a log
 * scale, 1 + log10(max(f, 1e-16))/16. */
void orc_feature_transform(long n, const double *f, double *out)
{
    for (long k = 0; k < n; ++k) out[k] = 1.0 + log10(f[k] > 1e-16 ? f[k] : 1e-16) / 16.0;
}

/* ------------------------------------------------------------------ */
/* Training labels of the learned indicator (a-posteriori troubled flag): */
/* element e is troubled (label 1) if the unlimited high-order update uH  */
/* has, at some node, rho or p outside [m (1 - tol), M (1 + tol)] where m, */
/* M are the min and max of that quantity over the nodes of e and of its   */
/* face neighbours in un, tol = 1e-3; or if uH is non-finite or has       */
/* rho <= 0 or p <= 0 there.  (The paper does not give a learned          */
/* indicator; this is the target its blending coefficient is trained on.) */
/* ------------------------------------------------------------------ */
int orc_labels(const orc_problem *P, const double *un, const double *uH, double tol, double *labels)
{
    int M = orc_nvar(P), np = np_of(P);
    long E = nelem_of(P);
    for (long e = 0; e < E; ++e) {
        double rmin = INFINITY, rmax = -INFINITY, pmin = INFINITY, pmax = -INFINITY;
        long list[5];
        int nl = 0;
        list[nl++] = e;
        for (int d = 0; d < P->dim; ++d)
            for (int side = 0; side < 2; ++side) list[nl++] = neighbour_or_self(P, e, d, side);
        for (int k = 0; k < nl; ++k) {
            double ue[ORC_MAXNP * ORC_MAXM];
            gather_elem(P, un, list[k], ue);
            for (int p = 0; p < np; ++p) {
                double r = ue[p * M], pr = orc_pressure(P, ue + p * M);
                if (r < rmin) rmin = r;
                if (r > rmax) rmax = r;
                if (pr < pmin) pmin = pr;
                if (pr > pmax) pmax = pr;
            }
        }
        double uh[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, uH, e, uh);
        int bad = 0;
        for (int p = 0; p < np; ++p) {
            for (int v = 0; v < M; ++v) if (!isfinite(uh[p * M + v])) bad = 1;
            double r = uh[p * M], pr = orc_pressure(P, uh + p * M);
            if (!(r > 0.0) || !(pr > 0.0)) bad = 1;
            if (r < rmin * (1.0 - tol) || r > rmax * (1.0 + tol)) bad = 1;
            if (pr < pmin * (1.0 - tol) || pr > pmax * (1.0 + tol)) bad = 1;
        }
        labels[e] = bad ? 1.0 : 0.0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Learned troubled-cell indicator: MLP nin -> H -> H -> 1 with ReLU and   */
/* output alpha_max * sigmoid(z).  Parameters packed as                    */
/* W1[H][nin], b1[H], W2[H][H], b2[H], W3[H], b3.  FP64 reference of the    */
/* forward pass, of the gradient of the mean binary cross-entropy loss of */
/* sigmoid(z) against labels y in [0,1] and of one Adam step.             */
/* ------------------------------------------------------------------ */
long orc_mlp_nparams(int nin, int H) { return (long)H * nin + H + (long)H * H + H + H + 1; }

int orc_mlp_forward(int nin, int H, const double *theta, long n, const double *x, double alpha_max, double *z_out, double *alpha_out)
{
    const double *W1 = theta, *b1 = W1 + H * nin, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
    double *h1 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    for (long s = 0; s < n; ++s) {
        const double *xs = x + s * nin;
        for (int a = 0; a < H; ++a) {
            double acc = b1[a];
            for (int c = 0; c < nin; ++c) acc += W1[a * nin + c] * xs[c];
            h1[a] = acc > 0.0 ? acc : 0.0;
        }
        for (int a = 0; a < H; ++a) {
            double acc = b2[a];
            for (int c = 0; c < H; ++c) acc += W2[a * H + c] * h1[c];
            h2[a] = acc > 0.0 ? acc : 0.0;
        }
        double z = b3[0];
        for (int c = 0; c < H; ++c) z += W3[c] * h2[c];
        if (z_out) z_out[s] = z;
        if (alpha_out) alpha_out[s] = alpha_max / (1.0 + exp(-z));
    }
    free(h1); free(h2);
    return 0;
}

/* loss = mean_s [ -y log sig(z) - (1-y) log(1 - sig(z)) ]; grad = dloss/dtheta */
double orc_mlp_loss_grad(int nin, int H, const double *theta, long n, const double *x, const double *y, double *grad)
{
    const double *W1 = theta, *b1 = W1 + H * nin, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
    long np = orc_mlp_nparams(nin, H);
    double *gW1 = grad, *gb1 = gW1 + H * nin, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + H;
    for (long k = 0; k < np; ++k) grad[k] = 0.0;
    double *a1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
    double *a2 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *d2 = malloc(sizeof(double) * H), *d1 = malloc(sizeof(double) * H);
    double loss = 0.0;
    for (long s = 0; s < n; ++s) {
        const double *xs = x + s * nin;
        for (int a = 0; a < H; ++a) {
            double acc = b1[a];
            for (int c = 0; c < nin; ++c) acc += W1[a * nin + c] * xs[c];
            a1[a] = acc; h1[a] = acc > 0.0 ? acc : 0.0;
        }
        for (int a = 0; a < H; ++a) {
            double acc = b2[a];
            for (int c = 0; c < H; ++c) acc += W2[a * H + c] * h1[c];
            a2[a] = acc; h2[a] = acc > 0.0 ? acc : 0.0;
        }
        double z = b3[0];
        for (int c = 0; c < H; ++c) z += W3[c] * h2[c];
        double sg = 1.0 / (1.0 + exp(-z));
        /* BCE with logits: log(1+e^z) - y z, written stably */
        loss += (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y[s] * z;
        double dz = (sg - y[s]) / (double)n;
        gb3[0] += dz;
        for (int c = 0; c < H; ++c) { gW3[c] += dz * h2[c]; d2[c] = a2[c] > 0.0 ? dz * W3[c] : 0.0; }
        for (int a = 0; a < H; ++a) {
            gb2[a] += d2[a];
            for (int c = 0; c < H; ++c) gW2[a * H + c] += d2[a] * h1[c];
        }
        for (int c = 0; c < H; ++c) {
            double acc = 0.0;
            for (int a = 0; a < H; ++a) acc += W2[a * H + c] * d2[a];
            d1[c] = a1[c] > 0.0 ? acc : 0.0;
        }
        for (int a = 0; a < H; ++a) {
            gb1[a] += d1[a];
            for (int c = 0; c < nin; ++c) gW1[a * nin + c] += d1[a] * xs[c];
        }
    }
    free(a1); free(h1); free(a2); free(h2); free(d2); free(d1);
    return loss / (double)n;
}

/* Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * theta <- theta - lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps). */
void orc_adam_step(long np, double *theta, double *m, double *v, const double *g,
                   double lr, double b1, double b2, double eps, int t)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (long k = 0; k < np; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        theta[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}
