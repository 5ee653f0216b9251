/*
 * crk.h -- C ABI of the MI355X (gfx950) compact Runge-Kutta flux
 * reconstruction (cRKFR) library with entropy-conservative (EC) and
 * kinetic-energy-preserving (KEP) two-point volume fluxes.
 *
 * Method: Babbar, Chen, Ranocha, "Compact Runge-Kutta flux reconstruction
 * methods with entropy- and/or kinetic energy-preserving fluxes",
 * arXiv 2604.02125.  Section 2 defines the cRKFR step for
 *   u_t + f(u)_x + B(u) g(u)_x = 0                      (eq:flux.and.non.cons)
 * on GLL solution points with g2 correction functions: element-local inner
 * stages (eq:crkfr.inner), time-averaged fluxes (eq:disc.avg.flux,
 * eq:local.time.avg.non.cons), one interface numerical flux per step
 * (eq:numflux.cons and the reduced-communication non-conservative flux
 * B(u^n) g^avg(U)) and the final update (eq:crkfr.non.cons.final).
 * Section 3 replaces the volume derivatives by flux differencing with a
 * symmetric two-point flux (eq:entropy.cons.flux.dev) and a non-symmetric
 * non-conservative term (eq:entropy.cons.noncons.dev).
 *
 * Conventions for every entry point:
 *  - Return CRK_OK (0) or a negative crk_status; nothing throws.  After an
 *    error crk_last_error() returns a message (thread-local).
 *  - Device pointers are allocated and owned by the caller; the library
 *    never allocates device memory and never frees caller memory.  Device
 *    buffers must be 256-byte aligned.
 *  - State layout (SoA, nodal): u[v][e][node], v < nvar, e = ey*nx + ex,
 *    node = j*(N+1) + i (x index fastest); element type = double (CRK_FP64)
 *    or float (CRK_FP32).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default
 *    stream) and runs asynchronously; argument checks are synchronous.
 *    Apart from crk_check, nothing reads back to the host, so the calls can
 *    be captured in a HIP graph.  Calls that share a workspace must not run
 *    concurrently.
 *  - dt_dev points to 2 device doubles: dt_dev[0] = time step,
 *    dt_dev[1] = GLM cleaning speed c_h (MHD; 0 for Euler).
 */
#ifndef CRK_H
#define CRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRK_OK = 0,
    CRK_ERR_ARG = -1,          /* invalid argument (null, size, alias)          */
    CRK_ERR_UNSUPPORTED = -2,  /* configuration not compiled in                 */
    CRK_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed    */
    CRK_ERR_NONPHYSICAL = -4,  /* crk_check: rho <= 0 or p <= 0 somewhere       */
    CRK_ERR_NOT_FINITE = -5,   /* crk_check: a value is NaN or infinite         */
    CRK_ERR_STATE = -6         /* missing workspace or wrong call order         */
} crk_status;

typedef enum { CRK_EULER = 0, CRK_GLM_MHD = 1 } crk_equation;        /* nvar = dim+2, 9 */
typedef enum {
    CRK_VOL_CENTRAL = 0,   /* (f(u_p)+f(u_q))/2: recovers eq:flux.dev                    */
    CRK_VOL_KG = 1,        /* Kennedy-Gruber KEP flux (Euler)                             */
    CRK_VOL_RANOCHA = 2,   /* Ranocha EC+KEP flux (Euler)                                 */
    CRK_VOL_DERIGS = 3     /* EC flux of Derigs et al. form + local Powell/GLM (MHD)      */
} crk_volume_flux;
typedef enum { CRK_FP64 = 0, CRK_FP32 = 1 } crk_precision;
typedef enum { CRK_LIM_NONE = 0, CRK_LIM_BLEND = 1 } crk_limiter;
/* numerical flux at element faces of the semi-discrete operator crk_fr_rhs */
typedef enum {
    CRK_SURF_RUSANOV = 0,  /* eq:numflux.cons with lambda from both traces     */
    CRK_SURF_EC = 1        /* the volume flux f_S on the two traces            */
} crk_surface_flux;

/* Boundary of a direction of the mesh.  A reflective (slip) wall has the
 * mirror image of the element beyond it (the state with the normal momentum
 * negated): the Rusanov flux of the element's traces and their mirror image
 * leaves no mass, tangential momentum or energy through the wall.  The paper
 * states no boundary conditions for its Richtmyer-Meshkov test (Section
 * 4.3); walls are this library's reading.  Euler only. */
typedef enum { CRK_BC_PERIODIC = 0, CRK_BC_WALL = 1 } crk_boundary;

/* Uniform Cartesian mesh of nx (x ny) elements on [x0,x1] (x [y0,y1]). */
typedef struct {
    int dim;            /* 1 or 2                                   */
    int nx, ny;         /* elements per direction (ny ignored in 1D) */
    double x0, x1, y0, y1;
    int degree;         /* N, 1 <= N <= 4                           */
    int equation;       /* crk_equation (MHD: dim = 2)              */
    double gamma;
    int precision;      /* crk_precision                            */
    int boundary[2];    /* crk_boundary of x and y (0: periodic)    */
} crk_mesh_desc;

/* Non-conservative interface flux of the MHD step (end of Section 2).
 * REDUCED: 1/2 B(u^{n,+-}) (g(U^-) + g(U^+)) from the time averages U that
 * the conservative flux exchanges anyway (the paper's choice, one exchange
 * of the usual size).  STAGEWISE: eq:bad.numflux.non.cons,
 * sum_j b_j 1/2 B(u^{(j),+-}) (g(u^{(j),-}) + g(u^{(j),+})), which needs
 * every stage's traces of both sides (an s-fold larger exchange). */
typedef enum { CRK_NC_REDUCED = 0, CRK_NC_STAGEWISE = 1 } crk_nc_interface;

/* Scheme: explicit RK tableau (eq:butcher), volume flux, CFL number,
 * blending limiter.  A (stages x stages, row-major, strictly lower) and b
 * may be NULL: then classical RK4 (N <= 3) or Butcher's six-stage
 * fifth-order method (N = 4) is used. */
typedef struct {
    int stages;                /* 1..6 (ignored when A == NULL)              */
    const double *A;           /* host pointer, copied at create             */
    const double *b;           /* host pointer, copied at create             */
    int volume_flux;           /* crk_volume_flux                            */
    double cfl;                /* dt = cfl / ((N+1) max sum_d lambda_d/dx_d) */
    int limiter;               /* crk_limiter                                */
    double alpha_max, alpha_min;
    int nc_interface;          /* crk_nc_interface (MHD; 0: reduced form)    */
} crk_scheme_desc;

typedef struct crk_solver crk_solver;
typedef void *crk_stream;      /* hipStream_t */

/* Create a solver for one mesh + scheme.  Host-only; copies the descriptors. */
crk_status crk_create(const crk_mesh_desc *mesh, const crk_scheme_desc *scheme, crk_solver **out);
crk_status crk_destroy(crk_solver *s);

/* Sizes: nvar, nelem, nodes per element, bytes of one state array. */
crk_status crk_state_layout(const crk_solver *s, int64_t *nvar, int64_t *nelem, int64_t *nnode, size_t *bytes);

/* Face data handed from the local-stage phase to the interface phase.
 * The blended Rusanov interface flux (eq:numflux.cons) is a sum of one term
 * per side, F* = P^- + P^+, with
 *   P^- = (1-a)(F^-/2 + lambda U^-/2) + a(f_d(u^-)/2 + lambda u^-/2),
 *   P^+ = (1-a)(F^+/2 - lambda U^+/2) + a(f_d(u^+)/2 - lambda u^+/2),
 * U = sum_j b_j u^(j), F = sum_j b_j f_d(u^(j)) the time averages at the
 * face node (eq:disc.avg.flux), u = u^n, lambda = max of the wave speeds of
 * u^n on both sides, a = (alpha_e + alpha_nb)/2 (0 without blending).
 * Layout trace[face][c][e][k], face = 2*d + side (side 0: xi_d = 0, side 1:
 * xi_d = 1), k = face node (j for x faces, i for y faces; 0 in 1D):
 * c < nvar: the element's own share P; for MHD also c = nvar: U of the
 * normal field B_d, c = nvar + 1: U of psi; last component (c = nvar, MHD
 * nvar + 2): the wave speed of direction d of the step's initial state at
 * the face node, |v_d| + c (Euler) or |v_d| + c_f (MHD; lambda also takes
 * c_h), from which the local phase forms lambda.  Element type = the
 * precision. */
crk_status crk_trace_bytes(const crk_solver *s, size_t *bytes);

/* Scratch for crk_step and the reductions (traces, blending coefficients,
 * reduction partials).  The caller allocates it once (any contents) and
 * passes it to crk_set_workspace; it stays bound until destroy or rebind. */
crk_status crk_workspace_bytes(const crk_solver *s, size_t *bytes);
crk_status crk_set_workspace(crk_solver *s, void *dev, size_t bytes);

/* GLL nodes xi, weights w on [0,1] and D_pq = l_q'(xi_p) (eq:diff.matrix),
 * row-major, of degree N (host arrays of N+1, N+1, (N+1)^2 doubles; any may
 * be NULL).  Host-only. */
crk_status crk_reference_element(int degree, double *xi, double *w, double *D);

/* dt_dev[0] = cfl / ((N+1) max_{e,p} sum_d lambda_d(u)/dx_d) with
 * lambda_d = |v_d| + c (Euler) or max(|v_d| + c_f, c_h) (MHD), and
 * dt_dev[1] = c_h = max_{e,p,d} (|v_d| + c_f) (MHD).  Needs the workspace. */
crk_status crk_compute_dt(crk_solver *s, const void *u, double *dt_dev, crk_stream stream);

/* As crk_compute_dt, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): needs no workspace and allocates nothing.  The reduction
 * partials go to a static scratch array of the library (8 KiB per GPU,
 * enough for every mesh the library accepts: the reduction uses at most 1024
 * partials; CRK_ERR_ARG beyond that).  Every call on a GPU shares that GPU's
 * scratch, so calls that overlap on one GPU (concurrent streams, threads)
 * race; stream-ordered calls do not.  The scratch keeps the previous call's
 * partials, which a call never reads (it writes every partial it uses). */
crk_status crk_compute_dt_noalloc(crk_solver *s, const void *u, double *dt_dev, crk_stream stream);

/* Blending coefficients of the subcell-FV limiter (Hennemann-Gassner modal
 * energy of rho*p, clipped at alpha_min, capped at alpha_max):
 * alpha_raw[e], and alpha[e] = max(alpha_raw[e], max over face neighbours
 * of alpha_raw/2).  Device arrays of nelem doubles; either may be NULL. */
crk_status crk_indicator(crk_solver *s, const void *u, double *alpha_raw, double *alpha, crk_stream stream);

/* Test operator: the semi-discrete FR right-hand side rhs = du/dt of
 * eq:general.non.conservative.fr.one, with the flux-differencing volume term
 * of Section 3 (the solver's volume flux, plus B_d(u_p) g_d(u_q) for MHD) and
 * the g2 surface correction (Huynh's g2 on GLL points: only the end nodes of
 * a line, with weight 1/(w dx)) of the numerical flux of
 * eq:combined.num.flux.fr: surface = CRK_SURF_RUSANOV, or CRK_SURF_EC, the
 * volume flux on the two traces (with an entropy-conservative volume flux,
 * zero semi-discrete entropy rate on the periodic mesh); MHD adds
 * 1/2 B_d(u)(g_d(u^-) + g_d(u^+)) - B_d(u) g_d(u).  u and rhs: device state
 * arrays (layout of crk_state_layout), distinct, 256-byte aligned.  dt_dev:
 * device [dt, c_h]; only c_h is read, and only for MHD (may be NULL for
 * Euler).  No workspace; stream-ordered; CRK_ERR_ARG on a null, misaligned
 * or aliased pointer or an unknown surface flux. */
crk_status crk_fr_rhs(crk_solver *s, const void *u, const double *dt_dev, int surface, void *rhs,
                      crk_stream stream);

#define CRK_STEP_COMPUTE_DT 1   /* flag of crk_step and crk_rkfr_step: compute dt first */

/* Standard s-stage RKFR step of eq:rkfr.non.cons, the scheme cRKFR is
 * compared with: every stage applies the semi-discrete operator of
 * crk_fr_rhs (the solver's volume flux, Rusanov faces with lambda from both
 * stage traces, MHD: 1/2 B(u)(g^- + g^+) at the faces) to the stage state,
 * so a step needs s interface exchanges instead of one:
 *   K_i = L(u^(i)), u^(i) = u_in + dt sum_{m<i} a_im K_m,
 *   u_out = u_in + dt sum_i b_i K_i.
 * flags & CRK_STEP_COMPUTE_DT: dt_dev from u_in first (needs the solver's
 * workspace), else dt_dev is an input ([dt, c_h]; c_h is held fixed over
 * the step).  rk_ws: caller-owned device scratch of crk_rkfr_workspace_bytes
 * (two stage states and the s stage derivatives).  No limiter
 * (CRK_ERR_UNSUPPORTED when the solver has one).  u_in, u_out distinct, not
 * in rk_ws, 256-byte aligned; stream-ordered. */
crk_status crk_rkfr_workspace_bytes(const crk_solver *s, size_t *bytes);
crk_status crk_rkfr_step(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, int flags, void *rk_ws,
                         size_t rk_ws_bytes, crk_stream stream);

/* Local phase (eq:crkfr.inner, eq:disc.avg.flux, Section 3 volume terms):
 * for every element the s inner stages with flux differencing, then
 *   u_out = u_in - dt [(1-alpha_e) V + alpha_e L]   (V = sum_j b_j R^(j);
 * L = interior part of the first-order subcell FV update; alpha == NULL or
 * limiter off means alpha_e = 0), and at the face nodes the element's own
 * part of the lifting of eq:crkfr.non.cons.final: its share P of the
 * interface flux minus (1-alpha_e) F (for MHD also its half of
 * 1/2 B(u^n)(g(U^-) + g(U^+)) minus the own non-conservative trace), with
 * dg_R/dxi = delta_pN/w_N, dg_L/dxi = -delta_p0/w_0; the face data (layout
 * above) for the neighbours.  alpha (device, nelem doubles) is read for the
 * element and its face neighbours.  The face wave speeds of u_in are written
 * into traces first (a separate pass; the pipelined crk_advance gets them
 * from the previous interface phase instead).  u_in and u_out must not
 * alias. */
crk_status crk_local_stages(crk_solver *s, const void *u_in, const double *dt_dev, const double *alpha,
                            void *u_out, void *traces, crk_stream stream);

/* Interface phase (eq:numflux.cons, eq:crkfr.non.cons.final): adds to
 * every face node of u_inout (the local phase's output, in place) the
 * lifted share P of the neighbour across each face it lies on (for MHD
 * also 1/2 B(u^n_own) g(U_nb), which reads u_in, the state the step started
 * from; Euler does not read u_in).  traces = the local phase's face data. */
crk_status crk_interface_update(crk_solver *s, const void *u_in, const void *traces, const double *dt_dev,
                                void *u_inout, crk_stream stream);

/* One full cRKFR step u_out = step(u_in).  flags & CRK_STEP_COMPUTE_DT:
 * compute dt_dev from u_in first (else dt_dev is an input).  With the
 * limiter on, alpha_in (device, nelem doubles, final blending coefficients)
 * is used if non-NULL, else the indicator runs on u_in.  Needs the
 * workspace; u_in and u_out must not alias.  Uses the workspace state of
 * the pipelined calls below: after crk_step, crk_advance needs crk_prepare
 * again (CRK_ERR_STATE otherwise). */
crk_status crk_step(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, const double *alpha_in,
                    int flags, crk_stream stream);

/* Pipelined time stepping.  crk_prepare computes, for a state u, dt_dev
 * (as crk_compute_dt), the face wave speeds of u and, with the limiter on,
 * the raw blending indicator of u, the last two kept in the workspace.
 * crk_advance then performs one step u_out = step(u_in) using dt_dev and the
 * kept data, all of which must belong to u_in (from crk_prepare or from the
 * previous crk_advance), and computes them for u_out while the new state is
 * still in registers: on
 * return dt_dev holds the time step of u_out.  The step is the same
 * arithmetic as crk_step; only the CFL reduction and the indicator move
 * into the interface phase.  `phases` selects CRK_PHASE_LOCAL and/or
 * CRK_PHASE_INTERFACE (both = one full step; the phases of one step must
 * be issued in this order on one stream).  Needs the workspace.  The
 * interface phase merges per-workgroup wave-speed maxima into a small slot
 * array of the workspace that crk_prepare sets to zero and each interface
 * phase leaves at zero; two pipelined sequences must therefore not run on
 * one solver at once, and a failed interface phase requires crk_prepare
 * again (CRK_ERR_STATE). */
#define CRK_PHASE_LOCAL 1
#define CRK_PHASE_INTERFACE 2
/* The local phase in its two launches, for timing each on its own: the
 * element tiles where no blending coefficient can be positive run a kernel
 * instance without the blending code (PLAIN), the others the instance with
 * it (BLEND).  CRK_PHASE_LOCAL = both; issued separately, PLAIN comes first
 * and both come before the interface phase. */
#define CRK_PHASE_LOCAL_PLAIN 4
#define CRK_PHASE_LOCAL_BLEND 8
crk_status crk_prepare(crk_solver *s, const void *u, double *dt_dev, crk_stream stream);
crk_status crk_advance(crk_solver *s, const void *u_in, void *u_out, double *dt_dev, int phases, crk_stream stream);

/* nsteps pipelined steps (as nsteps calls of crk_advance with both phases,
 * alternating u0 -> u1 -> u0 ...): after an even count the state is in u0,
 * after an odd count in u1; dt_dev as for crk_advance.  A one-dimensional
 * Euler mesh of at most 256 nodes (without a bound network) runs all steps
 * in one launch of one workgroup; other meshes issue the steps one by one.
 * Needs crk_prepare on u0 first and the workspace. */
crk_status crk_run(crk_solver *s, void *u0, void *u1, double *dt_dev, int nsteps, crk_stream stream);

/* FP64 diagnostics of u into out_dev (device, nvar + 5 doubles):
 * totals sum_e sum_p w_p u_p |Omega_e| (nvar), total entropy
 * sum w_p S(u_p) |Omega_e| with S = -rho (ln p - gamma ln rho)/(gamma-1),
 * min rho, min p, count of non-finite values, first element index that is
 * non-finite or has rho <= 0 or p <= 0 (-1 if none).  Needs the workspace. */
crk_status crk_diagnostics(crk_solver *s, const void *u, double *out_dev, crk_stream stream);

/* Crash detection on the host: the diagnostics of u (as crk_diagnostics,
 * into the workspace), waited for on `stream` and read back.  Returns
 * CRK_ERR_NOT_FINITE if a value of u is NaN or infinite, else
 * CRK_ERR_NONPHYSICAL if rho <= 0 or p <= 0 at some node, else CRK_OK; in
 * every case *first_bad (if non-NULL) = the first element index that is
 * non-finite or non-physical (-1 if none) and diag_host (if non-NULL, nvar
 * + 5 host doubles) receives the diagnostics.  Synchronises `stream`, so it
 * cannot be captured in a HIP graph.  Needs the workspace. */
crk_status crk_check(crk_solver *s, const void *u, int64_t *first_bad, double *diag_host, crk_stream stream);

/* ---------------------------------------------------------------- learned indicator
 * A multilayer perceptron 16 -> 64 -> 64 -> 1 (ReLU; output alpha_max *
 * sigmoid(z)) gives the blending coefficient from the 16 modal energy
 * fractions of rho*p of a degree-3 quadrilateral (the quantities of the
 * modal indicator), on a log scale (crk_features).  Parameters: one vector theta of crk_mlp_param_count values,
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3, stored as BF16 for the
 * network (FP32 arithmetic) and as FP32 master copy for training.  The
 * paper gives no learned indicator; this replaces its modal one where the
 * network is trusted. */
crk_status crk_mlp_param_count(int nin, int hidden, int64_t *count);
/* z[n] (may be NULL) and alpha[n] = alpha_max sigmoid(z) (may be NULL) of x[n][16]. */
crk_status crk_mlp_forward(int nin, int hidden, const uint16_t *theta_bf16, const float *x, int64_t n,
                           double alpha_max, float *z, double *alpha, crk_stream stream);
/* grad[count] of the mean binary cross-entropy of sigmoid(z) against labels
 * y[n] in [0,1], and the loss (device float, may be NULL).  Deterministic
 * (fixed reduction order).  workspace: crk_mlp_grad_workspace_bytes. */
crk_status crk_mlp_grad_workspace_bytes(int nin, int hidden, int64_t n, size_t *bytes);
crk_status crk_mlp_loss_grad(int nin, int hidden, const uint16_t *theta_bf16, const float *x, const float *y, int64_t n,
                             float *grad, float *loss, void *workspace, size_t ws_bytes, crk_stream stream);
/* One Adam step (bias-corrected, step number t >= 1) on the FP32 master
 * parameters, refreshing the BF16 copy when theta_bf16 != NULL. */
crk_status crk_mlp_adam(int64_t count, float *theta, float *m, float *v, const float *grad, double lr, double b1,
                        double b2, double eps, int t, uint16_t *theta_bf16, crk_stream stream);
crk_status crk_mlp_to_bf16(int64_t count, const float *theta, uint16_t *theta_bf16, crk_stream stream);
/* Features of the state u (FP32): features[e][node] = 1 + log10(max(f,
 * 1e-16))/16 with f = m_kl^2 / sum m^2 the modal energy fractions of rho*p
 * (in [0, 1]).  Needs the workspace; overwrites the indicator that the
 * pipelined calls keep there, so crk_advance and crk_run return
 * CRK_ERR_STATE until crk_prepare runs again. */
crk_status crk_features(crk_solver *s, const void *u, float *features, crk_stream stream);
/* Training labels (1/0 per element, FP32) of the unlimited update u_high
 * of u_n: 1 if at a node of the element rho or p leaves
 * [min (1 - tol), max (1 + tol)] of that quantity over the element and its
 * face neighbours in u_n, or the update is non-finite or has rho <= 0 or
 * p <= 0.  2D Euler. */
crk_status crk_labels(crk_solver *s, const void *u_n, const void *u_high, double tol, float *labels, crk_stream stream);
/* Use the network (device BF16 parameters, device feature range lo[16],
 * hi[16]) for the blending coefficient of crk_indicator, crk_step,
 * crk_prepare and crk_advance; where a feature is outside [lo, hi] or the
 * output is not finite the modal coefficient is kept.  theta_bf16 = NULL
 * restores the modal indicator.  2D Euler, degree 3, blending limiter. */
crk_status crk_set_mlp(crk_solver *s, const uint16_t *theta_bf16, const float *feat_lo, const float *feat_hi);

/* ---------------------------------------------------------------- batches
 * Many independent periodic 2D Euler meshes (degree 3 with classical RK4,
 * degree 4 with Butcher's RK5, one precision, Kennedy-Gruber or Ranocha
 * volume flux, no limiter) advanced together by pipelined steps.  The
 * element tiles of all problems form one work list (degree-3 tiles first);
 * each phase is one launch per degree over the tiles of that degree, or one
 * launch over all of them (tuning.merged), with one workgroup per tile or a
 * fixed grid of persistent workgroups (tuning);
 * each problem has its own CFL time step.  Each problem i occupies the values
 * [offsets[i], offsets[i+1]) of a state buffer, laid out as u[v][e][node]
 * of that problem. */
typedef struct crk_batch crk_batch;
typedef struct {
    int block;          /* lanes per workgroup: 64, 128 or 256 (0: 256)           */
    int grid_per_cu;    /* persistent workgroups per compute unit; 0: one per tile */
    int merged;         /* 1: one launch per phase over the tiles of both degrees,
                           each tile taking its degree's path; 0: one per degree  */
} crk_batch_tuning;
/* meshes[nprob]; scheme->A and ->b must be NULL.  tuning may be NULL. */
crk_status crk_batch_create(const crk_mesh_desc *meshes, int nprob, const crk_scheme_desc *scheme,
                            const crk_batch_tuning *tuning, crk_batch **out);
crk_status crk_batch_destroy(crk_batch *b);
/* offsets[nprob+1] (values), degrees[nprob], bytes of one state buffer, of
 * the workspace, and the number of work items; any pointer may be NULL. */
crk_status crk_batch_layout(const crk_batch *b, int64_t *offsets, int *degrees, size_t *state_bytes,
                            size_t *workspace_bytes, int64_t *ntiles);
/* Bind the two state buffers u0, u1, the time steps dt_dev[2*nprob]
 * (dt_dev[2i] = dt of problem i) and the workspace; uploads the work list
 * (synchronises `stream`). */
crk_status crk_batch_bind(crk_batch *b, void *u0, void *u1, double *dt_dev, void *workspace, size_t ws_bytes,
                          crk_stream stream);
/* dt of every problem from state src (0: u0, 1: u1). */
crk_status crk_batch_prepare(crk_batch *b, int src, crk_stream stream);
/* One pipelined step from state src into the other buffer (phases:
 * CRK_PHASE_LOCAL and/or CRK_PHASE_INTERFACE, as for crk_advance); leaves the
 * dt of the new states in dt_dev. */
crk_status crk_batch_advance(crk_batch *b, int src, int phases, crk_stream stream);
/* Capture two steps u0 -> u1 -> u0 into a HIP graph (stream must not be the
 * default stream), and replay it. */
crk_status crk_batch_graph_capture(crk_batch *b, crk_stream stream);
crk_status crk_batch_graph_launch(crk_batch *b, crk_stream stream);

/* Message of the last error on this thread ("" if none). */
const char *crk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CRK_H */
