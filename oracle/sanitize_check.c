/* Memory and undefined-behaviour check of the oracle (test infrastructure).
 *
 * Built by tests/test_oracle_sanitize.py together with crk_oracle.c (this
 * file includes it, so that one translation unit sees the problem struct)
 * under gcc's AddressSanitizer and UndefinedBehaviorSanitizer, and run as a
 * plain executable: every exported routine of the oracle is driven on small
 * meshes over the configurations the tests use (Euler 1D/2D, degrees 1..4
 * and 8, central / Kennedy-Gruber / Ranocha volume fluxes, blending with the
 * modal and a given coefficient, periodic and wall boundaries; GLM-MHD with
 * the Derigs-form flux, both non-conservative interface forms; the
 * semi-discrete operator with both surface fluxes; the multi-stage RKFR step;
 * diagnostics, labels and the MLP routines).  Any out-of-bounds access, use
 * of freed memory, leak or undefined operation aborts with a report; the run
 * prints "sanitize: ok" and a count of the cases otherwise.  Results are only
 * checked for finiteness: the numerical pins live in the Python tests.
 */
#include "crk_oracle.c"

#include <stdio.h>

static const double TWO_PI = 6.283185307179586;

/* 64-bit LCG (Knuth's MMIX constants) for the multiplicative node noise. */
static uint64_t lcg_state = 88172645463325252ull;
static double noise01(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static void set_tableau(orc_problem *P)
{
    memset(P->A, 0, sizeof P->A);
    memset(P->b, 0, sizeof P->b);
    if (P->N >= 4) {
        static const double A5[6][6] = {{0, 0, 0, 0, 0, 0},
                                        {0.25, 0, 0, 0, 0, 0},
                                        {0.125, 0.125, 0, 0, 0, 0},
                                        {0, -0.5, 1, 0, 0, 0},
                                        {3.0 / 16, 0, 0, 9.0 / 16, 0, 0},
                                        {-3.0 / 7, 2.0 / 7, 12.0 / 7, -12.0 / 7, 8.0 / 7, 0}};
        static const double b5[6] = {7.0 / 90, 0, 32.0 / 90, 12.0 / 90, 32.0 / 90, 7.0 / 90};
        P->stages = 6;
        for (int i = 0; i < 6; ++i) {
            P->b[i] = b5[i];
            for (int j = 0; j < 6; ++j) P->A[i * ORC_MAXS + j] = A5[i][j];
        }
    } else {
        P->stages = 4;
        P->A[1 * ORC_MAXS + 0] = 0.5;
        P->A[2 * ORC_MAXS + 1] = 0.5;
        P->A[3 * ORC_MAXS + 2] = 1.0;
        P->b[0] = P->b[3] = 1.0 / 6;
        P->b[1] = P->b[2] = 1.0 / 3;
    }
}

/* Smooth positive state at the nodes (x fastest), times 1 + amp U(-1,1). */
static void fill_state(const orc_problem *P, double *u, double amp)
{
    double xi[ORC_MAXN + 1], w[ORC_MAXN + 1];
    orc_gll(P->N, xi, w);
    int n1 = P->N + 1, np = np_of(P), M = orc_nvar(P);
    long E = nelem_of(P);
    double hx = (P->x1 - P->x0) / P->nx, hy = (P->y1 - P->y0) / (P->dim == 2 ? P->ny : 1);
    for (long e = 0; e < E; ++e)
        for (int p = 0; p < np; ++p) {
            int ex = (int)(e % P->nx), ey = (int)(e / P->nx);
            int i = p % n1, j = p / n1;
            double x = P->x0 + hx * (ex + 0.5 * (xi[i] + 1.0));
            double y = P->dim == 2 ? P->y0 + hy * (ey + 0.5 * (xi[j] + 1.0)) : 0.0;
            double s = sin(TWO_PI * x), c = cos(TWO_PI * y);
            double rho = 1.0 + 0.2 * s * c, pr = 1.0 + 0.1 * cos(TWO_PI * (x + y));
            double v[3] = {0.3 * c, P->dim == 2 ? -0.2 * s : 0.0, 0.1 * s};
            double q[ORC_MAXM];
            if (P->eq == ORC_EULER) {
                double ke = 0.0;
                q[0] = rho;
                for (int d = 0; d < P->dim; ++d) {
                    q[1 + d] = rho * v[d];
                    ke += 0.5 * rho * v[d] * v[d];
                }
                q[P->dim + 1] = pr / (P->gamma - 1.0) + ke;
            } else {
                double B[3] = {0.4 * c, 0.3 * s, 0.1}, psi = 0.01 * s;
                double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double me = 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                q[0] = rho;
                for (int d = 0; d < 3; ++d) { q[1 + d] = rho * v[d]; q[5 + d] = B[d]; }
                q[4] = pr / (P->gamma - 1.0) + ke + me + 0.5 * psi * psi;
                q[8] = psi;
            }
            for (int v2 = 0; v2 < M; ++v2)
                u[((long)v2 * E + e) * np + p] = q[v2] * (1.0 + amp * (2.0 * noise01() - 1.0));
        }
}

static int all_finite(const double *a, long n)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(a[k])) return 0;
    return 1;
}

static int failures = 0, cases = 0;

static void expect(int ok, const char *what, const orc_problem *P)
{
    if (!ok) {
        ++failures;
        fprintf(stderr, "sanitize: %s failed (dim %d, N %d, eq %d, flux %d, limiter %d, bc %d/%d)\n", what, P->dim,
                P->N, P->eq, P->vol_flux, P->limiter, P->bc[0], P->bc[1]);
    }
}

static void run_case(orc_problem *P, double amp)
{
    ++cases;
    set_tableau(P);
    int M = orc_nvar(P), np = np_of(P), nf = P->dim == 2 ? P->N + 1 : 1;
    long E = nelem_of(P), n = E * np * M, ntr = E * 2 * P->dim * nf * M;
    double *u = malloc(sizeof(double) * n), *u1 = malloc(sizeof(double) * n), *u2 = malloc(sizeof(double) * n);
    double *V = malloc(sizeof(double) * n), *rhs = malloc(sizeof(double) * n);
    double *Ut = malloc(sizeof(double) * ntr), *Ft = malloc(sizeof(double) * ntr);
    double *Fnct = malloc(sizeof(double) * ntr), *Fs = malloc(sizeof(double) * ntr);
    double *araw = malloc(sizeof(double) * E), *alpha = malloc(sizeof(double) * E);
    double *feat = malloc(sizeof(double) * E * np), *ftr = malloc(sizeof(double) * E * np);
    double *lab = malloc(sizeof(double) * E), *aout = malloc(sizeof(double) * E);
    double diag[ORC_MAXM + 5];

    fill_state(P, u, amp);
    P->ch = orc_compute_ch(P, u);
    double dt = orc_compute_dt(P, u);
    expect(isfinite(dt) && dt > 0.0, "compute_dt", P);
    if (P->eq == ORC_EULER) {
        expect(orc_indicator(P, u, araw, alpha, feat) == 0, "indicator", P);
        orc_feature_transform(E * np, feat, ftr);
        expect(all_finite(ftr, E * np), "feature_transform", P);
    } else {
        for (long e = 0; e < E; ++e) alpha[e] = 0.0;
    }
    expect(orc_crk_step(P, u, dt, alpha, u1, aout) == 0 && all_finite(u1, n), "crk_step", P);
    expect(orc_local_phase(P, u, dt, V, Ut, Ft, Fnct) == 0 && all_finite(V, n), "local_phase", P);
    expect(orc_face_fluxes(P, u, dt, P->limiter ? alpha : NULL, Fs) == 0 && all_finite(Fs, ntr), "face_fluxes", P);
    for (int surf = 0; surf < 2; ++surf)
        expect(orc_fr_rhs(P, u, surf, rhs) == 0 && all_finite(rhs, n), "fr_rhs", P);
    expect(orc_rkfr_step(P, u, dt, u2) == 0 && all_finite(u2, n), "rkfr_step", P);
    expect(orc_diagnostics(P, u1, diag) == 0 && all_finite(diag, M + 5), "diagnostics", P);
    if (P->eq == ORC_EULER) {
        expect(orc_labels(P, u, u1, 1e-3, lab) == 0, "labels", P);
        /* a single-element volume term */
        double ue[ORC_MAXNP * ORC_MAXM], R[ORC_MAXNP * ORC_MAXM];
        gather_elem(P, u, E - 1, ue);
        orc_volume_residual(P, ue, R);
        expect(all_finite(R, (long)np * M), "volume_residual", P);
    }
    free(u); free(u1); free(u2); free(V); free(rhs); free(Ut); free(Ft); free(Fnct); free(Fs);
    free(araw); free(alpha); free(feat); free(ftr); free(lab); free(aout);
}

static void run_mlp(void)
{
    ++cases;
    const int nin = 16, H = 8;
    const long ns = 37, npar = orc_mlp_nparams(nin, H);
    double *th = malloc(sizeof(double) * npar), *g = malloc(sizeof(double) * npar);
    double *m = calloc(npar, sizeof(double)), *v = calloc(npar, sizeof(double));
    double *x = malloc(sizeof(double) * ns * nin), *y = malloc(sizeof(double) * ns);
    double *z = malloc(sizeof(double) * ns), *a = malloc(sizeof(double) * ns);
    for (long k = 0; k < npar; ++k) th[k] = 0.3 * (2.0 * noise01() - 1.0);
    for (long k = 0; k < ns * nin; ++k) x[k] = noise01();
    for (long k = 0; k < ns; ++k) y[k] = noise01() < 0.3 ? 1.0 : 0.0;
    orc_problem dummy;
    memset(&dummy, 0, sizeof dummy);
    for (int t = 1; t <= 3; ++t) {
        expect(orc_mlp_forward(nin, H, th, ns, x, 0.5, z, a) == 0 && all_finite(a, ns), "mlp_forward", &dummy);
        double loss = orc_mlp_loss_grad(nin, H, th, ns, x, y, g);
        expect(isfinite(loss) && all_finite(g, npar), "mlp_loss_grad", &dummy);
        orc_adam_step(npar, th, m, v, g, 1e-3, 0.9, 0.999, 1e-8, t);
    }
    free(th); free(g); free(m); free(v); free(x); free(y); free(z); free(a);
}

static orc_problem base(int dim, int N, int nx, int ny)
{
    orc_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    P.N = N;
    P.nx = nx;
    P.ny = dim == 2 ? ny : 1;
    P.eq = ORC_EULER;
    P.x0 = 0.0; P.x1 = 1.0; P.y0 = 0.0; P.y1 = 0.8;
    P.gamma = 1.4;
    P.cfl = 0.4;
    P.alpha_max = 0.5;
    P.alpha_min = 1e-3;
    P.nthreads = 1;
    return P;
}

int main(void)
{
    /* Euler: every degree the tests use (and the largest supported), every
     * volume flux, both limiters, periodic and wall boundaries */
    const int degrees[] = {1, 2, 3, 4, ORC_MAXN};
    for (int dim = 1; dim <= 2; ++dim)
        for (int di = 0; di < 5; ++di)
            for (int flux = ORC_VOL_CENTRAL; flux <= ORC_VOL_RANOCHA; ++flux)
                for (int lim = ORC_LIM_NONE; lim <= ORC_LIM_BLEND_MODAL; ++lim)
                    for (int bcx = 0; bcx <= 1; ++bcx) {
                        int N = degrees[di];
                        orc_problem P = base(dim, N, N == ORC_MAXN ? 3 : 5, N == ORC_MAXN ? 2 : 4);
                        P.vol_flux = flux;
                        P.limiter = lim;
                        P.bc[0] = bcx ? ORC_BC_WALL : ORC_BC_PERIODIC;
                        P.bc[1] = (dim == 2 && bcx) ? ORC_BC_WALL : ORC_BC_PERIODIC;
                        run_case(&P, lim ? 0.05 : 1e-3);
                    }
    /* a given blending coefficient */
    {
        orc_problem P = base(2, 3, 4, 3);
        P.vol_flux = ORC_VOL_KG;
        P.limiter = ORC_LIM_BLEND_GIVEN;
        run_case(&P, 0.0);
    }
    /* GLM-MHD, Derigs-form flux, reduced and stage-wise interface forms */
    for (int N = 2; N <= 4; ++N)
        for (int sw = 0; sw <= 1; ++sw) {
            orc_problem P = base(2, N, 4, 3);
            P.eq = ORC_MHD;
            P.gamma = 5.0 / 3.0;
            P.vol_flux = ORC_VOL_DERIGS;
            P.nc_stagewise = sw;
            run_case(&P, 1e-3);
        }
    run_mlp();
    if (failures) {
        fprintf(stderr, "sanitize: %d of the checks failed\n", failures);
        return 1;
    }
    printf("sanitize: ok, %d cases\n", cases);
    return 0;
}
