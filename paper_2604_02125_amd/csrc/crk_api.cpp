// crk_api.cpp -- the C ABI of include/crk.h: argument checking, reference
// element tables, workspace layout and kernel dispatch.  No device memory is
// allocated here; every buffer comes from the caller.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/crk.h"
#include "crk_dispatch.hpp"

using namespace crk;

namespace crk {
hipError_t launch_mlp_alpha(const uint16_t *theta, const float *features, const float *lo, const float *hi, long nelem,
                            double alpha_max, double alpha_min, double *alpha_raw, const Tables *t, int *tiles,
                            hipStream_t s);
hipError_t launch_labels(const Tables &t, int prec, const void *un, const void *uh, double tol, float *labels,
                         hipStream_t s);
}

namespace {

thread_local std::string g_err;

crk_status fail(crk_status st, const char *msg)
{
    g_err = msg;
    return st;
}

crk_status hip_fail(hipError_t e, const char *where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    g_err = buf;
    return CRK_ERR_HIP;
}

// Legendre P_n(x) by the three-term recurrence.
double legendre(int n, double x)
{
    if (n == 0) return 1.0;
    double a = 1.0, b = x;
    for (int k = 2; k <= n; ++k) {
        const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    return b;
}

// GLL nodes of degree N on [-1,1] are the roots of P_{N+1} - P_{N-1}
// (proportional to (1 - x^2) P_N'); its derivative is (2N+1) P_N, so
// Newton reads x <- x - (P_{N+1} - P_{N-1}) / ((2N+1) P_N).
// Weights 2/(N(N+1) P_N^2); both mapped to [0,1].
void gll_nodes(int N, double *xi, double *w)
{
    for (int k = 0; k <= N; ++k) {
        double x = -std::cos(M_PI * k / N);
        if (k > 0 && k < N) {
            for (int it = 0; it < 60; ++it) {
                const double q = legendre(N + 1, x) - legendre(N - 1, x);
                const double dx = q / ((2 * N + 1) * legendre(N, x));
                x -= dx;
                if (std::fabs(dx) < 1e-17) break;
            }
        }
        const double PN = legendre(N, x);
        xi[k] = 0.5 * (x + 1.0);
        w[k] = 1.0 / (N * (N + 1.0) * PN * PN);
    }
}

// Differentiation matrix by barycentric weights lam_j = 1/prod_{k!=j}(xi_j - xi_k):
// D_ij = (lam_j/lam_i)/(xi_i - xi_j) (i != j), D_ii = -sum_{j!=i} D_ij.
void diff_matrix(int N, const double *xi, double *D)
{
    double lam[MAXN + 1];
    for (int j = 0; j <= N; ++j) {
        double p = 1.0;
        for (int k = 0; k <= N; ++k)
            if (k != j) p *= xi[j] - xi[k];
        lam[j] = 1.0 / p;
    }
    for (int i = 0; i <= N; ++i) {
        double s = 0.0;
        for (int j = 0; j <= N; ++j) {
            if (j == i) continue;
            const double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[i * (N + 1) + j] = v;
            s += v;
        }
        D[i * (N + 1) + i] = -s;
    }
}

// Nodal -> modal map for the orthonormal Legendre basis phi_k = sqrt(2k+1) P_k(2xi-1).
// GLL quadrature is exact for degree <= 2N-1, so the basis is discretely
// orthogonal; only the top mode has a discrete norm gamma_N != 1.  Hence
// V^{-1} = diag(1/gamma_k) V^T diag(w).
void modal_inverse(int N, const double *xi, const double *w, double Vinv[MAXN + 1][MAXN + 1])
{
    for (int k = 0; k <= N; ++k) {
        double g = 0.0, phi[MAXN + 1];
        for (int i = 0; i <= N; ++i) {
            phi[i] = std::sqrt(2.0 * k + 1.0) * legendre(k, 2.0 * xi[i] - 1.0);
            g += w[i] * phi[i] * phi[i];
        }
        for (int i = 0; i <= N; ++i) Vinv[k][i] = w[i] * phi[i] / g;
    }
}

bool is_aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

} // namespace

struct crk_solver {
    crk_mesh_desc mesh;
    int flux, limiter, prec;
    Tables t;
    size_t elem_bytes;
    size_t state_bytes, trace_bytes;
    size_t off_partials, off_slots, off_araw, off_alpha, off_features, off_tiles, off_diag, off_traces, ws_bytes;
    size_t off_stage;  // stage-wise non-conservative interface flux: stage states at the face nodes
    bool stagewise;
    long ntiles;     // local-phase tiles (two flag sets of ntiles ints in the workspace)
    int tparity;     // flag set of the next local phase
    bool tiles_valid; // the flag set covers the raw coefficients in the workspace
    const uint16_t *mlp;          // learned indicator parameters (BF16, device) or nullptr
    const float *mlp_lo, *mlp_hi; // feature range the network was trained on
    char *ws;
    bool prepared;   // crk_prepare has initialised the pipelined-step state of this workspace
};

namespace {

// Tile flags (pipelined step with the limiter, 2D, Kennedy-Gruber or
// Ranocha flux; the learned indicator flags from its own coefficients as
// well): flagged-clear tiles take the local-phase instance without the
// blending code, whose register count allows a fourth wavefront per SIMD in
// FP64 with Kennedy-Gruber (120 instead of 156 VGPRs) and a seventh in FP32;
// with the Ranocha flux it stays at three wavefronts in FP64 but issues 6 %
// fewer instructions (77 instead of 83 us on the 256^2 KHI state), a little
// more than the nearly empty second launch costs.  A 1D mesh small enough
// for crk_run's single launch keeps the blending instance so that both give
// the same bits.
bool use_tile_flags(const crk_solver *s)
{
    return s->limiter == CRK_LIM_BLEND && s->mesh.dim == 2 && (s->flux == CRK_VOL_KG || s->flux == CRK_VOL_RANOCHA);
}

template <class F>
hipError_t dispatch(const crk_solver *s, F &&f)
{
    const bool f64 = s->prec == CRK_FP64;
    if (s->mesh.equation == CRK_GLM_MHD) return f64 ? f(Family<double, EQ_MHD, 2>()) : f(Family<float, EQ_MHD, 2>());
    if (s->mesh.dim == 1) return f64 ? f(Family<double, EQ_EULER, 1>()) : f(Family<float, EQ_EULER, 1>());
    return f64 ? f(Family<double, EQ_EULER, 2>()) : f(Family<float, EQ_EULER, 2>());
}

crk_status need_ws(const crk_solver *s)
{
    if (!s) return fail(CRK_ERR_ARG, "null solver");
    if (!s->ws) return fail(CRK_ERR_STATE, "no workspace bound (crk_set_workspace)");
    return CRK_OK;
}

} // namespace

extern "C" {

const char *crk_last_error(void) { return g_err.c_str(); }

crk_status crk_reference_element(int N, double *xi, double *w, double *D)
{
    if (N < 1 || N > MAXN) return fail(CRK_ERR_UNSUPPORTED, "degree must be 1..4");
    double x[MAXN + 1], ww[MAXN + 1], DD[(MAXN + 1) * (MAXN + 1)];
    gll_nodes(N, x, ww);
    diff_matrix(N, x, DD);
    if (xi) std::memcpy(xi, x, sizeof(double) * (N + 1));
    if (w) std::memcpy(w, ww, sizeof(double) * (N + 1));
    if (D) std::memcpy(D, DD, sizeof(double) * (N + 1) * (N + 1));
    return CRK_OK;
}

} // extern "C"

namespace crk {

const char *set_error(crk_status st, const char *msg)
{
    (void)st;
    g_err = msg;
    return g_err.c_str();
}

// Validate a mesh + scheme description and build the kernel tables.
crk_status fill_tables(const crk_mesh_desc *m, const crk_scheme_desc *sc, Tables *tp)
{
    if (!m || !sc || !tp) return fail(CRK_ERR_ARG, "null argument");
    if (m->dim != 1 && m->dim != 2) return fail(CRK_ERR_ARG, "dim must be 1 or 2");
    if (m->nx < 1 || (m->dim == 2 && m->ny < 1)) return fail(CRK_ERR_ARG, "element counts must be positive");
    if (m->degree < 1 || m->degree > MAXN) return fail(CRK_ERR_UNSUPPORTED, "degree must be 1..4");
    if (m->equation != CRK_EULER && m->equation != CRK_GLM_MHD) return fail(CRK_ERR_ARG, "unknown equation");
    if (m->equation == CRK_GLM_MHD && m->dim != 2) return fail(CRK_ERR_UNSUPPORTED, "GLM-MHD is 2D only");
    if (m->precision != CRK_FP64 && m->precision != CRK_FP32) return fail(CRK_ERR_ARG, "unknown precision");
    if (!(m->gamma > 1.0)) return fail(CRK_ERR_ARG, "gamma must exceed 1");
    if (!(m->x1 > m->x0) || (m->dim == 2 && !(m->y1 > m->y0))) return fail(CRK_ERR_ARG, "empty domain");
    if (!flux_supported(m->equation == CRK_GLM_MHD ? EQ_MHD : EQ_EULER, sc->volume_flux))
        return fail(CRK_ERR_UNSUPPORTED, "volume flux not available for this equation");
    if (sc->limiter != CRK_LIM_NONE && sc->limiter != CRK_LIM_BLEND) return fail(CRK_ERR_ARG, "unknown limiter");
    if (sc->limiter == CRK_LIM_BLEND && m->equation != CRK_EULER)
        return fail(CRK_ERR_UNSUPPORTED, "the blending limiter is implemented for Euler only");
    if (!(sc->cfl > 0.0)) return fail(CRK_ERR_ARG, "cfl must be positive");
    for (int d = 0; d < 2; ++d)
        if (m->boundary[d] != CRK_BC_PERIODIC && m->boundary[d] != CRK_BC_WALL)
            return fail(CRK_ERR_ARG, "unknown boundary kind");
    const bool walls = m->boundary[0] == CRK_BC_WALL || (m->dim == 2 && m->boundary[1] == CRK_BC_WALL);
    if (walls && m->equation != CRK_EULER) return fail(CRK_ERR_UNSUPPORTED, "reflective walls are implemented for Euler only");
    if (sc->nc_interface != CRK_NC_REDUCED && sc->nc_interface != CRK_NC_STAGEWISE)
        return fail(CRK_ERR_ARG, "unknown non-conservative interface flux");
    if (sc->nc_interface == CRK_NC_STAGEWISE && m->equation != CRK_GLM_MHD)
        return fail(CRK_ERR_UNSUPPORTED, "the stage-wise non-conservative interface flux is an MHD option");
    const long nnode = m->dim == 2 ? (long)(m->degree + 1) * (m->degree + 1) : m->degree + 1;
    const long nelem = m->dim == 2 ? (long)m->nx * m->ny : m->nx;
    if (nelem * nnode >= (1L << 31)) return fail(CRK_ERR_ARG, "mesh too large");

    Tables &t = *tp;
    std::memset(&t, 0, sizeof t);
    t.dim = m->dim;
    t.nx = m->nx;
    t.ny = m->dim == 2 ? m->ny : 1;
    t.N = m->degree;
    t.M = m->equation == CRK_GLM_MHD ? 9 : m->dim + 2;
    t.nelem = (int)nelem;
    t.nnode = (int)nnode;
    t.nface = m->dim == 2 ? m->degree + 1 : 1;
    t.wall[0] = m->boundary[0] == CRK_BC_WALL ? 1 : 0;
    t.wall[1] = (m->dim == 2 && m->boundary[1] == CRK_BC_WALL) ? 1 : 0;
    t.invdx[0] = m->nx / (m->x1 - m->x0);
    {
        int l = 0;
        while ((1L << l) < m->nx) ++l;
        t.nx_s = 31 + l;
        t.nx_m = (unsigned)((1ULL << t.nx_s) / (unsigned long long)m->nx + 1);
    }
    t.invdx[1] = m->dim == 2 ? m->ny / (m->y1 - m->y0) : 0.0;
    t.gamma = m->gamma;
    t.cfl = sc->cfl;
    if (sc->A && sc->b) {
        if (sc->stages < 1 || sc->stages > MAXS) return fail(CRK_ERR_UNSUPPORTED, "stages must be 1..6");
        t.stages = sc->stages;
        for (int i = 0; i < t.stages; ++i) {
            t.b[i] = sc->b[i];
            for (int j = 0; j < t.stages; ++j) {
                const double a = sc->A[i * t.stages + j];
                if (j >= i && a != 0.0) return fail(CRK_ERR_ARG, "A must be strictly lower triangular");
                t.A[i][j] = a;
            }
        }
    } else if (m->degree <= 3) {
        // classical RK4
        t.stages = 4;
        t.A[1][0] = 0.5; t.A[2][1] = 0.5; t.A[3][2] = 1.0;
        t.b[0] = 1.0 / 6; t.b[1] = 1.0 / 3; t.b[2] = 1.0 / 3; t.b[3] = 1.0 / 6;
    } else {
        // Butcher's six-stage fifth-order method
        t.stages = 6;
        t.A[1][0] = 0.25;
        t.A[2][0] = 0.125; t.A[2][1] = 0.125;
        t.A[3][1] = -0.5; t.A[3][2] = 1.0;
        t.A[4][0] = 3.0 / 16; t.A[4][3] = 9.0 / 16;
        t.A[5][0] = -3.0 / 7; t.A[5][1] = 2.0 / 7; t.A[5][2] = 12.0 / 7; t.A[5][3] = -12.0 / 7; t.A[5][4] = 8.0 / 7;
        t.b[0] = 7.0 / 90; t.b[2] = 32.0 / 90; t.b[3] = 12.0 / 90; t.b[4] = 32.0 / 90; t.b[5] = 7.0 / 90;
    }
    {
        // classical RK4 gets a kernel that keeps one pending stage increment;
        // a six-stage matrix with Butcher's zero pattern one that forms only
        // the partial stage sums that pattern couples
        const double A4[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1, 0}};
        bool rk4 = t.stages == 4;
        for (int i = 0; rk4 && i < 4; ++i)
            for (int j = 0; j < 4; ++j) rk4 = rk4 && t.A[i][j] == A4[i][j];
        bool b6 = t.stages == 6;
        for (int k = 0; b6 && k < 6; ++k)
            for (int i = 0; i < 6; ++i) b6 = b6 && (stage_coupled<2>(k, i) || t.A[k][i] == 0.0);
        t.tableau = rk4 ? 1 : (b6 ? 2 : 0);
    }
    double xi[MAXN + 1], w[MAXN + 1], D[(MAXN + 1) * (MAXN + 1)];
    gll_nodes(t.N, xi, w);
    diff_matrix(t.N, xi, D);
    for (int p = 0; p <= t.N; ++p) {
        t.w[p] = w[p];
        t.invw_dx[0][p] = t.invdx[0] / w[p];
        t.invw_dx[1][p] = t.invdx[1] / w[p];
        for (int q = 0; q <= t.N; ++q) t.D[p][q] = D[p * (t.N + 1) + q];
    }
    if (sc->nc_interface == CRK_NC_STAGEWISE && !((t.stages == 4 && t.tableau == 1) || (t.stages == 6 && t.tableau == 2)))
        return fail(CRK_ERR_UNSUPPORTED,
                    "the stage-wise interface flux is compiled for classical RK4 and Butcher's six-stage method");
    modal_inverse(t.N, xi, w, t.Vinv);
    for (int d = 0; d < 2; ++d)
        for (int r = 0; r <= t.N; ++r) {
            for (int k = 0; k <= t.N; ++k) {
                const int q = r + k <= t.N ? r + k : r + k - (t.N + 1);
                t.dk[d][r][k] = 2.0 * t.D[r][q] * t.invdx[d];
                t.dkf[d][r][k] = (float)t.dk[d][r][k];
            }
            t.invw_dxf[d][r] = (float)t.invw_dx[d][r];
        }
    for (int i = 0; i < MAXS; ++i) {
        t.bf[i] = (float)t.b[i];
        for (int j = 0; j < MAXS; ++j) t.Af[i][j] = (float)t.A[i][j];
    }
    t.gm1 = t.gamma - 1.0;
    t.inv_gm1 = 1.0 / (t.gamma - 1.0);
    t.gammaf = (float)t.gamma;
    t.gm1f = (float)t.gm1;
    t.inv_gm1f = (float)t.inv_gm1;
    t.ind_threshold = 0.5 * std::pow(10.0, -1.8 * std::pow(t.N + 1.0, 0.25));
    t.ind_sharpness = std::log((1.0 - 1e-4) / 1e-4);
    t.ind_slope = t.ind_sharpness / t.ind_threshold;
    // the logistic value 1/(1 + exp(-slope (E - threshold))) equals alpha_min
    // at E* = threshold - ln(1/alpha_min - 1)/slope; 0.1 % of the threshold
    // below E* it is smaller by a factor (1 - 0.009) or so, far beyond the
    // few-ulp error of evaluating it, so the comparison with alpha_min cannot
    // go the other way
    t.ind_en_zero = (sc->alpha_min > 0.0 && sc->alpha_min < 0.5)
                        ? t.ind_threshold - std::log(1.0 / sc->alpha_min - 1.0) / t.ind_slope - 1e-3 * t.ind_threshold
                        : -INFINITY;
    t.alpha_min = sc->alpha_min;
    t.alpha_max = sc->alpha_max;
    return CRK_OK;
}

} // namespace crk

extern "C" {

crk_status crk_create(const crk_mesh_desc *m, const crk_scheme_desc *sc, crk_solver **out)
{
    if (!m || !sc || !out) return fail(CRK_ERR_ARG, "null argument");
    *out = nullptr;
    Tables t;
    crk_status st = fill_tables(m, sc, &t);
    if (st) return st;
    crk_solver *s = new (std::nothrow) crk_solver();
    if (!s) return fail(CRK_ERR_ARG, "out of host memory");
    s->mesh = *m;
    s->flux = sc->volume_flux;
    s->limiter = sc->limiter;
    s->prec = m->precision;
    s->t = t;
    const long nnode = t.nnode, nelem = t.nelem;
    s->elem_bytes = s->prec == CRK_FP64 ? 8 : 4;
    s->state_bytes = (size_t)t.M * nelem * nnode * s->elem_bytes;
    // per face node: the element's share of the interface flux (M values),
    // for MHD also the time-averaged normal field and psi, and the wave speed
    const int nc = t.M + (m->equation == CRK_GLM_MHD ? 2 : 0) + 1;
    s->trace_bytes = (size_t)2 * t.dim * nc * nelem * t.nface * s->elem_bytes;
    size_t off = 0;
    const long epb = tile_block_rt((int)nnode) / nnode;   // elements per interface-phase workgroup
    const long elem_blocks = (nelem + epb - 1) / epb;
    const long nparts = elem_blocks > RED_BLOCKS * 16 ? elem_blocks : RED_BLOCKS * 16;
    s->off_partials = off; off = align256(off + sizeof(double) * nparts);
    s->off_slots = off; off = align256(off + sizeof(double) * DT_SLOTS);
    s->off_araw = off; off = align256(off + sizeof(double) * nelem);
    s->off_alpha = off; off = align256(off + sizeof(double) * nelem);
    s->off_features = off; off = align256(off + sizeof(float) * nelem * nnode);
    s->ntiles = elem_blocks;
    s->off_tiles = off; off = align256(off + sizeof(int) * 2 * elem_blocks);
    s->off_diag = off; off = align256(off + sizeof(double) * (t.M + 5));
    s->off_traces = off; off = align256(off + s->trace_bytes);
    s->stagewise = sc->nc_interface == CRK_NC_STAGEWISE;
    s->off_stage = off;
    if (s->stagewise) off = align256(off + (size_t)2 * t.dim * t.stages * t.M * nelem * t.nface * s->elem_bytes);
    s->ws_bytes = off;
    s->ws = nullptr;
    s->prepared = false;
    s->tparity = 0;
    s->tiles_valid = false;
    s->mlp = nullptr;
    s->mlp_lo = s->mlp_hi = nullptr;
    *out = s;
    return CRK_OK;
}

crk_status crk_destroy(crk_solver *s)
{
    delete s;
    return CRK_OK;
}

crk_status crk_state_layout(const crk_solver *s, int64_t *nvar, int64_t *nelem, int64_t *nnode, size_t *bytes)
{
    if (!s) return fail(CRK_ERR_ARG, "null solver");
    if (nvar) *nvar = s->t.M;
    if (nelem) *nelem = s->t.nelem;
    if (nnode) *nnode = s->t.nnode;
    if (bytes) *bytes = s->state_bytes;
    return CRK_OK;
}

crk_status crk_trace_bytes(const crk_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CRK_ERR_ARG, "null argument");
    *bytes = s->trace_bytes;
    return CRK_OK;
}

crk_status crk_workspace_bytes(const crk_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CRK_ERR_ARG, "null argument");
    *bytes = s->ws_bytes;
    return CRK_OK;
}

crk_status crk_set_workspace(crk_solver *s, void *dev, size_t bytes)
{
    if (!s || !dev) return fail(CRK_ERR_ARG, "null argument");
    if (!is_aligned(dev)) return fail(CRK_ERR_ARG, "workspace must be 256-byte aligned");
    if (bytes < s->ws_bytes) return fail(CRK_ERR_ARG, "workspace too small");
    s->ws = (char *)dev;
    s->prepared = false;
    return CRK_OK;
}

} // extern "C"

namespace crk {
// CFL time step of u with caller-chosen storage for the reduction partials
// (for entry points outside this file); at most max_parts partials are used,
// else CRK_ERR_ARG before anything is launched.
crk_status solver_dt(crk_solver *s, const void *u, double *parts, int max_parts, double *dt_dev, hipStream_t stream)
{
    if (!s) return fail(CRK_ERR_ARG, "null solver");
    if (!u || !dt_dev || !parts) return fail(CRK_ERR_ARG, "null pointer");
    if (reduction_blocks(s->t) > max_parts) return fail(CRK_ERR_ARG, "more reduction partials than the scratch holds");
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::dt(s->t, u, parts, dt_dev, stream); });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "compute dt");
}
crk_status fail_with(crk_status st, const char *msg) { return fail(st, msg); }
} // namespace crk

extern "C" {

crk_status crk_compute_dt(crk_solver *s, const void *u, double *dt_dev, crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u || !dt_dev) return fail(CRK_ERR_ARG, "null pointer");
    double *parts = (double *)(s->ws + s->off_partials);
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::dt(s->t, u, parts, dt_dev, (hipStream_t)stream); });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_compute_dt");
}

crk_status crk_fr_rhs(crk_solver *s, const void *u, const double *dt_dev, int surface, void *rhs, crk_stream stream)
{
    if (!s || !u || !rhs) return fail(CRK_ERR_ARG, "null argument");
    if (!is_aligned(u) || !is_aligned(rhs)) return fail(CRK_ERR_ARG, "device arrays must be 256-byte aligned");
    if (u == rhs) return fail(CRK_ERR_ARG, "u and rhs must not alias");
    if (surface != CRK_SURF_RUSANOV && surface != CRK_SURF_EC) return fail(CRK_ERR_ARG, "unknown surface flux");
    if (s->mesh.equation == CRK_GLM_MHD && !dt_dev) return fail(CRK_ERR_ARG, "MHD needs c_h in dt_dev[1]");
    hipError_t e = dispatch(s, [&](auto fam) {
        return decltype(fam)::fr_rhs(s->t, s->flux, u, s->mesh.equation == CRK_GLM_MHD ? dt_dev : nullptr, surface,
                                     rhs, (hipStream_t)stream);
    });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_fr_rhs");
}

crk_status crk_rkfr_workspace_bytes(const crk_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CRK_ERR_ARG, "null argument");
    *bytes = (size_t)(s->t.stages + 2) * align256(s->state_bytes);
    return CRK_OK;
}

crk_status crk_rkfr_step(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, int flags, void *rk_ws,
                         size_t rk_ws_bytes, crk_stream stream)
{
    if (!s || !u_in || !u_out || !dt_dev || !rk_ws) return fail(CRK_ERR_ARG, "null argument");
    if (u_in == u_out) return fail(CRK_ERR_ARG, "u_in and u_out must not alias");
    if (!is_aligned(u_in) || !is_aligned(u_out) || !is_aligned(rk_ws))
        return fail(CRK_ERR_ARG, "buffers must be 256-byte aligned");
    if (flags & ~CRK_STEP_COMPUTE_DT) return fail(CRK_ERR_ARG, "unknown flag bits");
    if (s->limiter != CRK_LIM_NONE) return fail(CRK_ERR_UNSUPPORTED, "the standard RKFR step has no limiter");
    size_t need = 0;
    crk_rkfr_workspace_bytes(s, &need);
    if (rk_ws_bytes < need) return fail(CRK_ERR_ARG, "RKFR workspace too small (crk_rkfr_workspace_bytes)");
    char *w = (char *)rk_ws;
    const char *ui = (const char *)u_in, *uo = (const char *)u_out;
    if ((uo + s->state_bytes > w && uo < w + need) || (ui + s->state_bytes > w && ui < w + need))
        return fail(CRK_ERR_ARG, "u_in or u_out overlaps the RKFR workspace");
    if (flags & CRK_STEP_COMPUTE_DT) {
        crk_status st = crk_compute_dt(s, u_in, dt_dev, stream);
        if (st) return st;
    }
    const size_t sb = align256(s->state_bytes);
    RkPtrs p{};
    p.u_n = u_in;
    p.k = w + 2 * sb;
    p.dt = dt_dev;
    // the K arrays are packed at the state's own size (the kernel indexes them by m * nvar * nodes)
    hipError_t e = dispatch(s, [&](auto fam) {
        return decltype(fam)::rkfr(s->t, s->flux, p, w, w + sb, u_out, (hipStream_t)stream);
    });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_rkfr_step");
}

crk_status crk_indicator(crk_solver *s, const void *u, double *alpha_raw, double *alpha, crk_stream stream)
{
    if (!s || !u) return fail(CRK_ERR_ARG, "null argument");
    if (s->mesh.equation != CRK_EULER) return fail(CRK_ERR_UNSUPPORTED, "indicator is implemented for Euler only");
    double *araw = alpha_raw;
    if (!araw || s->mlp) {
        crk_status st = need_ws(s);
        if (st) return st;
    }
    if (!araw) {
        araw = (double *)(s->ws + s->off_araw);
        s->tiles_valid = false;   // the tile flags no longer describe these coefficients
    }
    float *feat = s->mlp ? (float *)(s->ws + s->off_features) : nullptr;
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::indicator(s->t, u, araw, nullptr, feat, hs); });
    if (e == hipSuccess && s->mlp)
        e = launch_mlp_alpha(s->mlp, feat, s->mlp_lo, s->mlp_hi, s->t.nelem, s->t.alpha_max, s->t.alpha_min, araw,
                             nullptr, nullptr, hs);
    if (e == hipSuccess && alpha) {
        hipLaunchKernelGGL(k_smooth, dim3((s->t.nelem + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, hs, s->t,
                           (const double *)araw, alpha);
        e = hipGetLastError();
    }
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_indicator");
}

crk_status crk_features(crk_solver *s, const void *u, float *features, crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u || !features) return fail(CRK_ERR_ARG, "null argument");
    if (s->mesh.equation != CRK_EULER) return fail(CRK_ERR_UNSUPPORTED, "features are defined for Euler only");
    double *araw = (double *)(s->ws + s->off_araw);
    // the workspace's raw coefficients now describe u, not the state of a
    // pipelined sequence: crk_advance needs crk_prepare again, and the next
    // local phase may not trust the tile flags
    s->prepared = false;
    s->tiles_valid = false;
    hipError_t e = dispatch(s, [&](auto fam) {
        return decltype(fam)::indicator(s->t, u, araw, nullptr, features, (hipStream_t)stream);
    });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_features");
}

crk_status crk_labels(crk_solver *s, const void *u_n, const void *u_high, double tol, float *labels, crk_stream stream)
{
    if (!s || !u_n || !u_high || !labels) return fail(CRK_ERR_ARG, "null argument");
    if (s->mesh.equation != CRK_EULER || s->mesh.dim != 2) return fail(CRK_ERR_UNSUPPORTED, "labels are for 2D Euler");
    hipError_t e = launch_labels(s->t, s->prec, u_n, u_high, tol, labels, (hipStream_t)stream);
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_labels");
}

crk_status crk_set_mlp(crk_solver *s, const uint16_t *theta_bf16, const float *feat_lo, const float *feat_hi)
{
    if (!s) return fail(CRK_ERR_ARG, "null solver");
    if (!theta_bf16) {
        s->mlp = nullptr;
        s->mlp_lo = s->mlp_hi = nullptr;
        return CRK_OK;
    }
    if (!feat_lo || !feat_hi) return fail(CRK_ERR_ARG, "the training feature range is required");
    if (s->limiter != CRK_LIM_BLEND || s->mesh.equation != CRK_EULER || s->mesh.dim != 2 || s->t.N != 3)
        return fail(CRK_ERR_UNSUPPORTED, "the learned indicator needs 2D Euler, degree 3, blending limiter");
    s->mlp = theta_bf16;
    s->mlp_lo = feat_lo;
    s->mlp_hi = feat_hi;
    return CRK_OK;
}

crk_status crk_local_stages(crk_solver *s, const void *u_in, const double *dt_dev, const double *alpha, void *u_out,
                            void *traces, crk_stream stream)
{
    if (!s || !u_in || !dt_dev || !u_out || !traces) return fail(CRK_ERR_ARG, "null argument");
    if (u_in == u_out) return fail(CRK_ERR_ARG, "u_in and u_out must not alias");
    if (!is_aligned(u_in) || !is_aligned(u_out) || !is_aligned(traces)) return fail(CRK_ERR_ARG, "buffers must be 256-byte aligned");
    if (s->stagewise && !s->ws) return fail(CRK_ERR_STATE, "the stage-wise interface flux keeps its stage traces in the workspace");
    StepPtrs p{};
    p.u_in = u_in; p.u_out = u_out; p.dt = dt_dev; p.traces = traces;
    p.stage_tr = s->stagewise ? s->ws + s->off_stage : nullptr;
    p.alpha = s->limiter == CRK_LIM_BLEND ? alpha : nullptr;
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::face_speed(s->t, s->flux, p, (hipStream_t)stream); });
    if (e == hipSuccess)
        e = dispatch(s, [&](auto fam) { return decltype(fam)::local(s->t, s->flux, p, (hipStream_t)stream); });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_local_stages");
}

crk_status crk_interface_update(crk_solver *s, const void *u_in, const void *traces, const double *dt_dev,
                                void *u_inout, crk_stream stream)
{
    if (!s || !u_in || !traces || !dt_dev || !u_inout) return fail(CRK_ERR_ARG, "null argument");
    if (u_in == u_inout) return fail(CRK_ERR_ARG, "u_in and u_inout must not alias");
    if (!is_aligned(u_in) || !is_aligned(u_inout) || !is_aligned(traces))
        return fail(CRK_ERR_ARG, "buffers must be 256-byte aligned");
    if (s->stagewise && !s->ws) return fail(CRK_ERR_STATE, "the stage-wise interface flux keeps its stage traces in the workspace");
    StepPtrs p{};
    p.u_in = u_in; p.u_out = u_inout; p.dt = dt_dev; p.traces = const_cast<void *>(traces);
    p.stage_tr = s->stagewise ? s->ws + s->off_stage : nullptr;
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::interface(s->t, s->flux, p, (hipStream_t)stream); });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_interface_update");
}

crk_status crk_step(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, const double *alpha_in, int flags,
                    crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u_in || !u_out || !dt_dev) return fail(CRK_ERR_ARG, "null pointer");
    if (u_in == u_out) return fail(CRK_ERR_ARG, "u_in and u_out must not alias");
    if (flags & CRK_STEP_COMPUTE_DT) {
        st = crk_compute_dt(s, u_in, dt_dev, stream);
        if (st) return st;
    }
    const double *alpha = nullptr;
    if (s->limiter == CRK_LIM_BLEND) {
        if (alpha_in) {
            alpha = alpha_in;
        } else {
            double *a = (double *)(s->ws + s->off_alpha);
            st = crk_indicator(s, u_in, (double *)(s->ws + s->off_araw), a, stream);
            if (st) return st;
            alpha = a;
        }
    }
    // the workspace's face data and indicator now describe u_in: a pipelined
    // sequence must start again from crk_prepare
    s->prepared = false;
    void *tr = s->ws + s->off_traces;
    st = crk_local_stages(s, u_in, dt_dev, alpha, u_out, tr, stream);
    if (st) return st;
    return crk_interface_update(s, u_in, tr, dt_dev, u_out, stream);
}

crk_status crk_prepare(crk_solver *s, const void *u, double *dt_dev, crk_stream stream)
{
    crk_status st = crk_compute_dt(s, u, dt_dev, stream);
    if (st) return st;
    if (s->limiter == CRK_LIM_BLEND) st = crk_indicator(s, u, (double *)(s->ws + s->off_araw), nullptr, stream);
    if (st) return st;
    StepPtrs p{};
    p.u_in = u; p.traces = s->ws + s->off_traces;
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::face_speed(s->t, s->flux, p, (hipStream_t)stream); });
    // the wave-speed slots the interface phases merge into start at zero
    // (a fill kernel, not a memset: safe inside a captured graph)
    if (e == hipSuccess) e = launch_zero((double *)(s->ws + s->off_slots), DT_SLOTS, (hipStream_t)stream);
    // tile flags of u (pipelined limiter with the modal indicator): both sets
    // cleared, set 0 marked from the raw coefficients
    s->tparity = 0;
    s->tiles_valid = false;
    if (e == hipSuccess && use_tile_flags(s)) {
        int *tiles = (int *)(s->ws + s->off_tiles);
        e = launch_zero_int(tiles, (int)(2 * s->ntiles), (hipStream_t)stream);
        if (e == hipSuccess) {
            const long epb = tile_block_rt((int)s->t.nnode) / s->t.nnode;
            const dim3 g((unsigned)((s->t.nelem + BLOCK - 1) / BLOCK));
            const double *araw = (const double *)(s->ws + s->off_araw);
            hipLaunchKernelGGL(k_mark_tiles<2>, g, dim3(BLOCK), 0, (hipStream_t)stream, s->t, araw, (int)epb, tiles);
            e = hipGetLastError();
        }
        s->tiles_valid = e == hipSuccess;
    }
    if (e != hipSuccess) return hip_fail(e, "crk_prepare");
    s->prepared = true;
    return CRK_OK;
}

crk_status crk_advance(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, int phases, crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u_in || !u_out || !dt_dev) return fail(CRK_ERR_ARG, "null pointer");
    if (u_in == u_out) return fail(CRK_ERR_ARG, "u_in and u_out must not alias");
    if (!is_aligned(u_in) || !is_aligned(u_out)) return fail(CRK_ERR_ARG, "buffers must be 256-byte aligned");
    if (phases & ~(CRK_PHASE_LOCAL | CRK_PHASE_INTERFACE | CRK_PHASE_LOCAL_PLAIN | CRK_PHASE_LOCAL_BLEND))
        return fail(CRK_ERR_ARG, "unknown phase bits");
    if (!s->prepared) return fail(CRK_ERR_STATE, "crk_prepare must run before crk_advance");
    const bool lim = s->limiter == CRK_LIM_BLEND;
    double *araw = (double *)(s->ws + s->off_araw);
    double *alpha = (double *)(s->ws + s->off_alpha);
    void *tr = s->ws + s->off_traces;
    // tile flags: set tparity is this step's, the other one the next step's
    const bool flags = use_tile_flags(s);
    int *tiles = (int *)(s->ws + s->off_tiles);
    int *t_cur = tiles + (size_t)s->tparity * s->ntiles, *t_next = tiles + (size_t)(1 - s->tparity) * s->ntiles;
    hipError_t e = hipSuccess;
    const int instances = ((phases & CRK_PHASE_LOCAL) ? 3 : 0) | ((phases & CRK_PHASE_LOCAL_PLAIN) ? 1 : 0) |
                          ((phases & CRK_PHASE_LOCAL_BLEND) ? 2 : 0);
    if (instances) {
        StepPtrs p{};
        p.instances = instances;
        p.u_in = u_in; p.u_out = u_out; p.dt = dt_dev; p.traces = tr;
        p.stage_tr = s->stagewise ? s->ws + s->off_stage : nullptr;
        p.alpha_raw = lim ? araw : nullptr;
        p.alpha_s = alpha;
        if (flags && s->tiles_valid) {
            p.tiles_in = t_cur;
            p.tiles_out = t_next;
        }
        e = dispatch(s, [&](auto fam) { return decltype(fam)::local(s->t, s->flux, p, (hipStream_t)stream); });
        if (e != hipSuccess) return hip_fail(e, "crk_advance (local phase)");
    }
    if (phases & CRK_PHASE_INTERFACE) {
        StepPtrs p{};
        p.u_in = u_in; p.u_out = u_out; p.dt = dt_dev; p.traces = tr;
        p.stage_tr = s->stagewise ? s->ws + s->off_stage : nullptr;
        p.alpha_raw_out = lim ? araw : nullptr;
        p.partials = (double *)(s->ws + s->off_slots);
        p.dt_out = dt_dev;
        p.features = (lim && s->mlp) ? (float *)(s->ws + s->off_features) : nullptr;
        // marks only add to the next step's set: a set that the local phase
        // did not clear is a superset, which is safe (flagged tiles blend
        // with whatever coefficients they find)
        if (flags) p.tiles_out = t_next;
        e = dispatch(s, [&](auto fam) { return decltype(fam)::interface(s->t, s->flux, p, (hipStream_t)stream); });
        if (e == hipSuccess && p.features)
            e = launch_mlp_alpha(s->mlp, p.features, s->mlp_lo, s->mlp_hi, s->t.nelem, s->t.alpha_max,
                                 s->t.alpha_min, araw, &s->t, p.tiles_out, (hipStream_t)stream);
        if (e != hipSuccess) {
            s->prepared = false;   // the slots may not be back at zero
            return hip_fail(e, "crk_advance (interface phase)");
        }
        if (flags) {
            s->tparity ^= 1;
            s->tiles_valid = true;
        }
    }
    return CRK_OK;
}

crk_status crk_run(crk_solver *s, void *u0, void *u1, double *dt_dev, int nsteps, crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u0 || !u1 || !dt_dev) return fail(CRK_ERR_ARG, "null pointer");
    if (u0 == u1) return fail(CRK_ERR_ARG, "u0 and u1 must not alias");
    if (nsteps < 0) return fail(CRK_ERR_ARG, "negative step count");
    if (!is_aligned(u0) || !is_aligned(u1)) return fail(CRK_ERR_ARG, "buffers must be 256-byte aligned");
    if (!s->prepared) return fail(CRK_ERR_STATE, "crk_prepare must run before crk_run");
    if (nsteps == 0) return CRK_OK;
    const bool lim = s->limiter == CRK_LIM_BLEND;
    if (s->mesh.dim == 1 && (long)s->t.nelem * s->t.nnode <= RUN_BLOCK && !s->mlp) {
        StepPtrs p{};
        p.u_in = u0; p.u_out = u1; p.dt = dt_dev; p.traces = s->ws + s->off_traces;
        p.alpha_raw = lim ? (double *)(s->ws + s->off_araw) : nullptr;
        p.alpha_s = (double *)(s->ws + s->off_alpha);
        p.alpha_raw_out = lim ? (double *)(s->ws + s->off_araw) : nullptr;
        p.partials = (double *)(s->ws + s->off_partials);
        hipError_t e = dispatch(s, [&](auto fam) {
            return decltype(fam)::run(s->t, s->flux, p, dt_dev, nsteps, (hipStream_t)stream); });
        if (e == hipSuccess) {
            s->tiles_valid = false;   // the fused steps keep no tile flags
            return CRK_OK;
        }
        if (e != hipErrorNotSupported) return hip_fail(e, "crk_run");
    }
    for (int k = 0; k < nsteps; ++k) {
        st = crk_advance(s, k % 2 ? u1 : u0, k % 2 ? u0 : u1, dt_dev, CRK_PHASE_LOCAL | CRK_PHASE_INTERFACE, stream);
        if (st) return st;
    }
    return CRK_OK;
}

crk_status crk_diagnostics(crk_solver *s, const void *u, double *out_dev, crk_stream stream)
{
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u || !out_dev) return fail(CRK_ERR_ARG, "null pointer");
    double *parts = (double *)(s->ws + s->off_partials);
    hipError_t e = dispatch(s, [&](auto fam) { return decltype(fam)::diag(s->t, u, parts, out_dev, (hipStream_t)stream); });
    return e == hipSuccess ? CRK_OK : hip_fail(e, "crk_diagnostics");
}

crk_status crk_check(crk_solver *s, const void *u, int64_t *first_bad, double *diag_host, crk_stream stream)
{
    if (first_bad) *first_bad = -1;
    crk_status st = need_ws(s);
    if (st) return st;
    if (!u) return fail(CRK_ERR_ARG, "null state");
    if (!is_aligned(u)) return fail(CRK_ERR_ARG, "state must be 256-byte aligned");
    const int M = s->t.M;
    double *dev = (double *)(s->ws + s->off_diag);
    st = crk_diagnostics(s, u, dev, stream);
    if (st) return st;
    double h[9 + 5];
    hipError_t e = hipMemcpyAsync(h, dev, sizeof(double) * (M + 5), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "crk_check");
    if (diag_host) std::memcpy(diag_host, h, sizeof(double) * (M + 5));
    const double nonfinite = h[M + 3], first = h[M + 4];
    if (first_bad) *first_bad = (int64_t)first;
    if (nonfinite > 0.0) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "%.0f non-finite values; first bad element %.0f", nonfinite, first);
        return fail(CRK_ERR_NOT_FINITE, buf);
    }
    if (first >= 0.0) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "rho <= 0 or p <= 0 (min rho %.3e, min p %.3e); first bad element %.0f",
                      h[M + 1], h[M + 2], first);
        return fail(CRK_ERR_NONPHYSICAL, buf);
    }
    return CRK_OK;
}

} // extern "C"
