// crk_kernels.hpp -- HIP kernels of one cRKFR step on gfx950.
//
// Mapping: one lane per solution node, the (N+1)^d nodes of an element in
// consecutive lanes; single-wavefront workgroups where whole elements fit a
// wavefront, else 128-lane workgroups of floor(128/(N+1)^d) elements (the
// reductions and the indicator use 256-lane workgroups).
// A stage stages its per-node fields (primitives, logarithms) in LDS so that
// every lane can form the two-point fluxes with the nodes on its x- and
// y-lines; the stage states, stage residuals and time averages stay in
// registers.  State and trace arrays are SoA with the node (or face-node)
// index fastest, so a wavefront touches contiguous memory.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include "crk_physics.hpp"

namespace crk {

constexpr int MAXN = 4;      // highest compiled degree
constexpr int MAXS = 6;      // highest stage count
constexpr int BLOCK = 256;   // lanes per workgroup of the element kernels
constexpr int RED_BLOCKS = 1024;  // max workgroups of the reduction kernels
#ifndef CRK_WIDE_TILE
#define CRK_WIDE_TILE 128
#endif
#ifndef CRK_WAVE_TILE
#define CRK_WAVE_TILE 64
#endif
// Workgroup of the local-stage and interface kernels for elements of NP
// nodes: when whole elements fit a wavefront those kernels need no
// workgroup barrier, and smaller workgroups finish the grid more evenly.
// Otherwise (N = 2, 4 in 2D) two wavefronts: a workgroup barrier then waits
// for one other wavefront only, and the degree-4 MHD kernel, held at one
// wavefront per SIMD by its registers, fits two workgroups per CU in LDS
// (Orszag-Tang 192^2: 409 -> 369 us per local phase against 256 lanes;
// 192 lanes leave one SIMD idle, 64 lanes hold two elements in 50 lanes).
template <int NP>
constexpr int tile_block() { return 64 % NP == 0 ? CRK_WAVE_TILE : CRK_WIDE_TILE; }
inline int tile_block_rt(int np) { return 64 % np == 0 ? CRK_WAVE_TILE : CRK_WIDE_TILE; }

// XCD-aware tile order.  Workgroups are dispatched round-robin over the
// eight XCDs (b -> XCD b mod 8), each with its own L2.  Giving XCD x the
// contiguous tile range [x G/8, (x+1) G/8) (plus one of the G mod 8 spare
// tiles) keeps horizontally adjacent element tiles, which share the cache
// lines of their face data, on one XCD and close in time.  A bijection of
// [0, G) for every G.
// Tiles per workgroup of the two local-phase instances (single-wavefront
// tiles): the instance with the blending code, which skips every tile that
// cannot blend, runs several per workgroup.
#ifndef CRK_LOCAL_WPB_PLAIN
#define CRK_LOCAL_WPB_PLAIN 1
#endif
#ifndef CRK_LOCAL_WPB_BLEND
#define CRK_LOCAL_WPB_BLEND 4
#endif

constexpr int NXCD = 8;
__device__ __forceinline__ long xcd_tile(long b, long G)
{
    const long x = b % NXCD, q = G / NXCD, r = G % NXCD;
    return x * q + (x < r ? x : r) + b / NXCD;
}

// Chunked variant for the local phase: each XCD takes chunks of XCD_CHUNK
// consecutive tiles in turn (chunk c on XCD c mod NXCD), so that a region
// of flagged tiles, which is contiguous in space, is spread over every XCD
// instead of loading the few that own its part of the mesh; blocks past the
// last whole round of chunks keep their own index.  A bijection on [0, G).
constexpr long XCD_CHUNK = 16;
__device__ __forceinline__ long xcd_chunk_tile(long b, long G)
{
    const long round = NXCD * XCD_CHUNK, gm = (G / round) * round;
    if (b >= gm) return b;
    const long x = b % NXCD, j = b / NXCD;
    return ((j / XCD_CHUNK) * NXCD + x) * XCD_CHUNK + j % XCD_CHUNK;
}

// Everything a kernel needs besides its pointers; passed by value.
struct Tables {
    int dim, nx, ny, N, M, nelem, nnode, nface;  // nface = nodes per face
    int wall[2];                      // per direction: reflective walls instead of periodic wrap
    double invdx[2];
    double gamma;
    int stages;
    int tableau;                      // sparsity class of A: see stage_coupled()
    double A[MAXS][MAXS];
    double b[MAXS];
    double D[MAXN + 1][MAXN + 1];     // D_pq = l_q'(xi_p) on [0,1]
    double w[MAXN + 1];               // GLL weights on [0,1]
    double invw_dx[2][MAXN + 1];      // 1/(w_p dx_d)
    double Vinv[MAXN + 1][MAXN + 1];  // nodal -> orthonormal Legendre modal
    double cfl;
    double ind_threshold, ind_sharpness, alpha_min, alpha_max;
    // formed once on the host for the local stages (the float copies for the
    // FP32 kernels, each the rounded double): dk[d][r][k] = 2 D_{r,(r+k) mod
    // (N+1)} / dx_d (k = 0: the diagonal), gamma - 1 and 1/(gamma - 1)
    double dk[2][MAXN + 1][MAXN + 1];
    float dkf[2][MAXN + 1][MAXN + 1];
    float invw_dxf[2][MAXN + 1];
    float Af[MAXS][MAXS], bf[MAXS];
    double gm1, inv_gm1;
    float gammaf, gm1f, inv_gm1f;
    // modal indicator: sharpness / threshold, and an energy below which the
    // logistic value is under alpha_min by a wide margin (so the coefficient
    // is zero without evaluating it)
    double ind_slope, ind_en_zero;
    // row of an element without a division: ey = floor(e / nx) = (e nx_m) >> nx_s
    // for every 0 <= e < 2^31 (nx_s = 31 + ceil(log2 nx), nx_m = floor(2^nx_s / nx) + 1;
    // Granlund and Montgomery's multiply-and-shift division)
    unsigned nx_m;   // < 2^32 for dividends below 2^31
    int nx_s;
};

// The host-formed coefficients in the kernel's precision.
template <typename real> struct Tab;
template <> struct Tab<double> {
    static __device__ __forceinline__ double dk(const Tables &t, int d, int r, int k) { return t.dk[d][r][k]; }
    // D_{r,q} / dx_d: half of dk at rotation (q - r) mod (N+1), exactly (a power of two)
    static __device__ __forceinline__ double dn(const Tables &t, int d, int r, int q)
    {
        return 0.5 * t.dk[d][r][q - r < 0 ? q - r + t.N + 1 : q - r];
    }
    static __device__ __forceinline__ double invw(const Tables &t, int d, int r) { return t.invw_dx[d][r]; }
    static __device__ __forceinline__ double A(const Tables &t, int i, int j) { return t.A[i][j]; }
    static __device__ __forceinline__ double b(const Tables &t, int i) { return t.b[i]; }
};
template <> struct Tab<float> {
    static __device__ __forceinline__ float dk(const Tables &t, int d, int r, int k) { return t.dkf[d][r][k]; }
    static __device__ __forceinline__ float dn(const Tables &t, int d, int r, int q)
    {
        return 0.5f * t.dkf[d][r][q - r < 0 ? q - r + t.N + 1 : q - r];
    }
    static __device__ __forceinline__ float invw(const Tables &t, int d, int r) { return t.invw_dxf[d][r]; }
    static __device__ __forceinline__ float A(const Tables &t, int i, int j) { return t.Af[i][j]; }
    static __device__ __forceinline__ float b(const Tables &t, int i) { return t.bf[i]; }
};

// Which entries a_ki (k > i) of the stage matrix a kernel may treat as
// non-zero: TAB 0 any, TAB 1 only a_{i+1,i} (classical RK4), TAB 2 the
// pattern of Butcher's six-stage fifth-order method (a_10; a_20, a_21;
// a_31, a_32; a_40, a_43; a_5j).  The values always come from Tables::A; the
// pattern only decides which partial stage sums Z_k = sum_j a_kj R^(j) are
// formed, so that those still pending stay few (registers).
template <int TAB>
__host__ __device__ constexpr bool stage_coupled(int k, int i)
{
    if (k <= i) return false;
    if (TAB == 1) return k == i + 1;
    if (TAB == 2) {
        switch (k) {
        case 1: return i == 0;
        case 2: return i <= 1;
        case 3: return i == 1 || i == 2;
        case 4: return i == 0 || i == 3;
        default: return true;
        }
    }
    return true;
}

struct StepPtrs {
    const void *u_in;
    void *u_out;
    const double *dt;      // [dt, c_h]
    const double *alpha;   // final blending coefficients or nullptr
    void *traces;
    // pipelined step (crk_advance): the local phase smooths the raw indicator
    // of u_in itself; the interface phase computes dt and the raw indicator
    // of u_out while the new state is in registers.
    const double *alpha_raw;  // local phase: raw indicator of u_in, or nullptr
    double *alpha_s;          // local phase: smoothed coefficients written for the interface phase
    double *alpha_raw_out;    // interface phase: raw indicator of u_out, or nullptr
    double *partials;         // interface phase: wave-speed maxima (k_interface: DT_SLOTS slots, zero on entry)
    double *dt_out;           // interface phase: dt and c_h of u_out (finished by k_dt_slots), or nullptr
    float *features;          // interface phase: learned-indicator features of u_out, or nullptr
    // Pipelined step with the limiter: one flag per local-phase tile, set when
    // a raw coefficient within two faces of one of its elements is positive
    // (only such tiles can blend).  Local phase: tiles_in are the step's
    // flags, tiles_out (the next step's) are cleared; interface phase: the
    // flags of u_out are marked into tiles_out.  nullptr: no flags.
    const int *tiles_in;
    int *tiles_out;
    // local phase: which instances to launch, bit 0 the one without the
    // blending code, bit 1 the one with it (0: both); either launches only
    // where the configuration uses it
    int instances;
    // MHD with the stage-wise non-conservative interface flux: the stage
    // states u^(j) at the face nodes, [face][j][v][e][k] (local phase
    // writes, interface phase reads); nullptr: the reduced form
    void *stage_tr;
};

// Pointers of one stage of the standard multi-stage RKFR step (crk_rhs.hpp).
struct RkPtrs {
    const void *u_n;    // u^n
    const void *x_in;   // u^(i) (u^n for i = 0)
    void *x_out;        // u^(i+1), or u^{n+1} after the last stage
    void *k;            // K_0 .. K_{s-1}, each a state array
    const double *dt;   // [dt, c_h]
};

// ---------------------------------------------------------------- helpers
// element coordinates and the four (two in 1D) face neighbours; e < 2^31.
// The row index comes from the host-formed multiply-and-shift (exact, see
// Tables::nx_m): far cheaper per lane than an integer division.  A face on
// a reflective wall has the element itself as neighbour (beyond the wall
// lies its mirror image, whose blending coefficient and wave speeds are the
// element's own) and its bit 2d + side set in `wall`: the kernels that read
// the neighbour's state or face data take the mirror image there instead.
struct Nbrs {
    long n[2][2];   // [d][side]
    int wall;       // bit 2d + side: that face lies on a wall
};
// (WALLS = false: the caller has checked that the mesh has no walls)
template <int DIM, bool WALLS = true>
__device__ __forceinline__ Nbrs neighbours(const Tables &t, long e)
{
    Nbrs r;
    const int nx = t.nx, ei = (int)e;
    if constexpr (DIM == 1) {
        const bool w0 = WALLS && t.wall[0] && ei == 0, w1 = WALLS && t.wall[0] && ei + 1 == nx;
        r.n[0][0] = w0 ? ei : (ei == 0 ? nx - 1 : ei - 1);
        r.n[0][1] = w1 ? ei : (ei + 1 == nx ? 0 : ei + 1);
        r.n[1][0] = r.n[1][1] = e;
        r.wall = (w0 ? 1 : 0) | (w1 ? 2 : 0);
        return r;
    }
    const int ey = (int)(((unsigned long long)(unsigned)ei * (unsigned long long)t.nx_m) >> t.nx_s);
    const int row = ey * nx;
    const int ex = ei - row;
    const bool wx0 = WALLS && t.wall[0] && ex == 0, wx1 = WALLS && t.wall[0] && ex + 1 == nx;
    const bool wy0 = WALLS && t.wall[1] && ey == 0, wy1 = WALLS && t.wall[1] && ey + 1 == t.ny;
    r.n[0][0] = wx0 ? ei : row + (ex == 0 ? nx - 1 : ex - 1);
    r.n[0][1] = wx1 ? ei : row + (ex + 1 == nx ? 0 : ex + 1);
    r.n[1][0] = wy0 ? ei : (ey == 0 ? (t.ny - 1) * nx : row - nx) + ex;
    r.n[1][1] = wy1 ? ei : (ey + 1 == t.ny ? 0 : row + nx) + ex;
    r.wall = (wx0 ? 1 : 0) | (wx1 ? 2 : 0) | (wy0 ? 4 : 0) | (wy1 ? 8 : 0);
    return r;
}
__device__ __forceinline__ Nbrs neighbours_any(const Tables &t, long e)
{
    return t.dim == 1 ? neighbours<1>(t, e) : neighbours<2>(t, e);
}

template <typename real, int EQ, int DIM, int FLUX> struct PhysOf;
template <typename real, int DIM, int FLUX> struct PhysOf<real, EQ_EULER, DIM, FLUX> { using type = EulerP<real, DIM, FLUX>; };
template <typename real, int DIM, int FLUX> struct PhysOf<real, EQ_MHD, DIM, FLUX> { using type = MhdP<real, FLUX>; };

template <typename real>
__device__ __forceinline__ Ctx<real> make_ctx(const Tables &t, const double *dt)
{
    Ctx<real> c;
    if constexpr (sizeof(real) == 8) {
        c.gamma = real(t.gamma);
        c.gm1 = real(t.gm1);
        c.inv_gm1 = real(t.inv_gm1);
    } else {
        c.gamma = real(t.gammaf);
        c.gm1 = real(t.gm1f);
        c.inv_gm1 = real(t.inv_gm1f);
    }
    c.ch = dt ? real(dt[1]) : real(0);
    return c;
}

// Face data between the two phases, [face][c][e][k] (face = 2d + side, k =
// face node): c < M the element's share of the interface flux; MHD: c = M,
// M + 1 the time-averaged normal field and psi; last component the wave
// speed of direction d of the state at the face node, |v_d| + c (Euler) or
// |v_d| + c_f (MHD), from which the local phase forms the Rusanov lambda.
template <int EQ, int M>
struct FaceData {
    static constexpr int NC = EQ == EQ_MHD ? M + 2 : M;   // flux-share (+ MHD) components
    static constexpr int SPEED = NC;                       // component of the wave speed
    static constexpr int NCT = NC + 1;                     // components per face node
};

template <typename real, int EQ, int DIM, int FLUX>
__device__ __forceinline__ real face_speed(int d, const real *nd, const Ctx<real> &ctx)
{
    if constexpr (EQ == EQ_MHD) return MhdP<real, FLUX>::fast(d, nd, ctx);
    else return EulerP<real, DIM, FLUX>::speed(d, nd, ctx);
}

// One tile of BLK lanes (a lane per node): the wave speeds of the face nodes of u.
template <typename real, int EQ, int DIM, int N, int FLUX, int BLK>
__device__ __forceinline__ void face_speed_tile(const Tables &t, const void *u_, void *traces, long e0)
{
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int M = Phys::M;
    constexpr int nf = DIM == 2 ? n1 : 1;
    using FD = FaceData<EQ, M>;
    const int tid = threadIdx.x;
    const int le = tid / NP;
    const int node = tid - le * NP;
    const long e = e0 + le;
    if (le >= BLK / NP || e >= t.nelem) return;
    const int pd[2] = {node % n1, DIM == 2 ? node / n1 : 0};
    bool face_lane = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) face_lane |= (pd[d] == 0 || pd[d] == N);
    if (!face_lane) return;
    const long E = t.nelem;
    const real *u = (const real *)u_;
    real us[M], nd[Phys::NF];
#pragma unroll
    for (int v = 0; v < M; ++v) us[v] = u[((long)v * E + e) * NP + node];
    const Ctx<real> ctx = make_ctx<real>(t, nullptr);
    Phys::node_basic(us, nd, ctx);
    real *tr = (real *)traces;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (!(pd[d] == 0 || pd[d] == N)) continue;
        const int face = 2 * d + (pd[d] == N ? 1 : 0);
        const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
        tr[((long)(face * FD::NCT + FD::SPEED) * E + e) * nf + kk] = face_speed<real, EQ, DIM, FLUX>(d, nd, ctx);
    }
}

template <typename real, int EQ, int DIM, int N, int FLUX>
__global__ void __launch_bounds__(BLOCK) k_face_speed(const Tables t, const void *u, void *traces)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    face_speed_tile<real, EQ, DIM, N, FLUX, BLOCK>(t, u, traces, (long)blockIdx.x * (BLOCK / NP));
}

// ---------------------------------------------------------------- K2: local stages
// For every element: S inner stages u^(i) = u^n - dt sum_{j<i} a_ij R^(j)
// with R^(i)_p = sum_d 1/dx_d sum_q [2 D_pq f_S,d(u_p,u_q) + D_pq B_d(u_p) g_d(u_q)]
// (eq:crkfr.inner with the volume terms of Section 3), the element's share
// of the interface flux and the provisional update (see crk_local_stages).
//
// Pairs along a line are visited by rotation: lane p pairs with
// q = (p + k) mod (N+1), k = 1..N.  Rotation k and N+1-k visit the same
// unordered pairs, so each lane evaluates only the rotations k < (N+1)/2
// (and k = (N+1)/2 when N+1 is even) and takes the mirrored symmetric
// fluxes f_S(u_p, u_q) = f_S(u_q, u_p) from its line neighbour through LDS.
template <int N, int DIM>
__device__ __forceinline__ int line_node(const int *pd, int d, int qd)
{
    constexpr int n1 = N + 1;
    return (DIM == 1) ? qd : (d == 0 ? pd[1] * n1 + qd : qd * n1 + pd[0]);
}

// Synchronisation of the lanes of one element.  When a wavefront holds
// whole elements (64 divisible by (N+1)^d: N = 1, 3; or single-wavefront
// workgroups), every LDS exchange of the local stages stays inside one
// wavefront, so ordering the wavefront's own LDS accesses suffices and the
// waves of a workgroup never wait for each other; otherwise the workgroup
// barrier.
template <int NP, int BLK = BLOCK>
__device__ __forceinline__ void element_sync()
{
    if constexpr (64 % NP == 0 || BLK <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// LDS slots (of BLK values each) used by the local-stage tile (BL: the
// instance with the blending code)
template <typename real, int EQ, int DIM, int N, int FLUX, bool BL = true>
struct LocalShape {
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    static constexpr int n1 = N + 1;
    // the conservative two-point fluxes are symmetric for both systems (the
    // MHD non-conservative term is formed separately)
    static constexpr bool SYM = N >= 2;
    static constexpr int NPRIM = SYM ? (n1 - 1) / 2 : 0;           // rotations whose mirror comes from LDS
    static constexpr int KSELF = (SYM && n1 % 2 == 0) ? n1 / 2 : 0;  // self-mirrored rotation, evaluated directly
    static constexpr int NX = SYM ? DIM * NPRIM * Phys::M : 0;
    // ASL slots carry the blending coefficients of each element and of its
    // face neighbours ((2 DIM + 1) values per element of NP lanes; only in
    // the instance with the blending code)
    static constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    static constexpr int ASL = BL ? (2 * DIM + 1 + NP - 1) / NP : 0;
    // Euler, whole elements per wavefront, instance with the blending code:
    // one slot for the sound speed of u^n, shared by the subcell fluxes
    static constexpr int CS = (BL && EQ == EQ_EULER && 64 % NP == 0) ? 1 : 0;
    // 2D, N+1 even: the pairs of the self-mirrored rotation (p, p + (N+1)/2)
    // along x and along y are as many as the nodes.  With the Ranocha flux
    // each lane evaluates one of them (the x pair when exactly one of its
    // indices is below (N+1)/2, else the y pair) and takes the other from
    // the lane that evaluated it (M slots), so that every unordered pair of
    // the element is evaluated once.  (For the cheap KG flux the selects and
    // the exchange cost as much as the pair.)
    static constexpr bool BAL = DIM == 2 && SYM && KSELF > 0 && EQ == EQ_EULER && FLUX == VOL_RANOCHA;
    static constexpr int XB = BAL ? Phys::M : 0;
    // FP64 Euler in 2D, degree 4, and degree 3 with the Ranocha flux: the
    // coefficients 2 D_{p,q}/dx_d of the lane's rotations and diagonal come
    // from a table in LDS (one slot) instead of 2 (N+1) registers each, so
    // that one more wavefront per SIMD fits in registers and LDS (three at
    // degree 4, four for Ranocha at degree 3).  Otherwise at degree 4 (MHD,
    // bound at one wavefront by its registers; FP32, not register-bound) the
    // node fields alternate between two sets of slots from stage to stage,
    // so that a stage may overwrite them without waiting for the previous
    // stage's readers (one barrier fewer per stage).
    static constexpr bool DTAB = DIM == 2 && EQ == EQ_EULER && sizeof(real) == 8 &&
                                 (N == 4 || (N == 3 && FLUX == VOL_RANOCHA));
    static constexpr bool DBF = DIM == 2 && N == 4 && !DTAB;
    static constexpr int DT = DTAB ? 1 : 0;
    static constexpr int slots = (DBF ? 2 : 1) * Phys::NF + NX + ASL + CS + XB + DT;
};

// One tile of BLK lanes: elements e0 .. e0 + BLK/(N+1)^DIM - 1 of one mesh.
// smem holds LocalShape::slots * BLK values.
// BLEND = false: no blending coefficient can be positive in the tile (no
// limiter, or a flagged-clear tile of the pipelined step); the blending code
// is compiled out, which frees registers for a fourth wavefront per SIMD.
// NCS (MHD): the stage-wise non-conservative interface flux (stage states
// written at the face nodes for the interface phase) instead of the reduced form.
template <typename real, int EQ, int DIM, int N, int FLUX, int S, int BLK, int TAB = 0, bool BLEND = true,
          bool NCS = false>
__device__ __forceinline__ void local_tile(const Tables &t, const StepPtrs &a, long e0, real *smem, int lane = -1)
{
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    using Shape = LocalShape<real, EQ, DIM, N, FLUX, BLEND>;
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int EPB = BLK / NP;
    constexpr int M = Phys::M;
    constexpr int NF = Phys::NF;
    constexpr bool SYM = Shape::SYM;
    constexpr int NPRIM = Shape::NPRIM;
    constexpr int KSELF = Shape::KSELF;
    constexpr bool DBF = Shape::DBF;
    real *lds0 = smem;                               // [NF][BLK] (two sets with DBF)
    real *xch = smem + (DBF ? 2 : 1) * NF * BLK;     // [NX][BLK]
    real *alds = xch + Shape::NX * BLK;   // [EPB][2 DIM + 1]
    real *clds = alds + Shape::ASL * BLK; // [CS][BLK]
    real *xb = clds + Shape::CS * BLK;    // [XB][BLK]
    real *dtab = xb + Shape::XB * BLK;    // DTAB: [DIM][N+1][N+1], dtab[(d n1 + r) n1 + k] = 2 D_{r,(r+k) mod n1}/dx_d
    constexpr bool CSH = Shape::CS > 0;
    constexpr bool DTAB = Shape::DTAB;
    static_assert(!DTAB || DIM * (N + 1) * (N + 1) <= BLK, "the coefficient table fits one slot");
    constexpr bool BAL = Shape::BAL;
    constexpr int NA = 2 * DIM + 1;

    const int tid = lane >= 0 ? lane : (int)threadIdx.x;   // (lane: see the batched local phase)
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = e0 + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;                 // spare lanes read element 0's fields
    const long es = valid ? e : 0;
    const int base = le * NP;
    const int pd[2] = {node % n1, DIM == 2 ? node / n1 : 0};
    const long E = t.nelem;

    const Ctx<real> ctx = make_ctx<real>(t, a.dt);
    const real rdt = real(a.dt[0]);
    constexpr bool stagewise = EQ == EQ_MHD && NCS;

    // per-lane coefficients 2 D_{p,q}/dx_d of rotation k = 1..N, of the diagonal,
    // and 1/(w_p dx_d), read from the tables with the lane's node index
    real Dk[DIM][N], Ddiag[DIM], invw[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int r = pd[d];
        if constexpr (!DTAB) {
#pragma unroll
            for (int k = 1; k <= N; ++k) Dk[d][k - 1] = Tab<real>::dk(t, d, r, k);
            Ddiag[d] = Tab<real>::dk(t, d, r, 0);
        }
        invw[d] = Tab<real>::invw(t, d, r);
    }
    if constexpr (DTAB) {
        // every wavefront writes the whole table (the same values), so that
        // it is visible to the wavefront's own lanes after the first stage's
        // synchronisation also where that is wavefront-scope and the tile
        // spans several wavefronts (the batched tiles)
        static_assert(DIM * (N + 1) * (N + 1) <= 64, "one wavefront writes the table");
        const int wl = tid & 63;
        if (wl < DIM * n1 * n1) {
            const int d = wl / (n1 * n1), r = (wl / n1) % n1, k = wl % n1;
            dtab[wl] = Tab<real>::dk(t, d, r, k);
        }
    }
    // 2 D_{p,q}/dx_d of rotation k = 1..N (k = 0: the diagonal)
    auto dk = [&](int d, int k) -> real {
        if constexpr (DTAB) return dtab[(d * n1 + pd[d]) * n1 + k];
        else return k == 0 ? Ddiag[d] : Dk[d][k - 1];
    };
    // MHD: plain D_pq / dx_d for the non-conservative term, all q
    real Dn[DIM][n1];
    if constexpr (EQ == EQ_MHD) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int q = 0; q < n1; ++q) Dn[d][q] = Tab<real>::dn(t, d, pd[d], q);
    }

    const real *uin = (const real *)a.u_in;
    real un[M];
#pragma unroll
    for (int v = 0; v < M; ++v) un[v] = uin[((long)v * E + es) * NP + node];

    bool onface[DIM];
    int side[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        onface[d] = (pd[d] == 0) || (pd[d] == N);
        side[d] = (pd[d] == N) ? 1 : 0;
    }
    // Rusanov speed of each face through this node: lambda = max of the
    // wave speeds of u^n on both sides (eq:numflux.cons; MHD: and c_h), from
    // the face data, formed here so that the element can add its own share
    // of the interface flux itself.  Meshes without walls (a uniform test)
    // take a copy of this part compiled without the wall cases.
    constexpr int nfn = DIM == 2 ? n1 : 1;
    using FD = FaceData<EQ, M>;
    real lamd[DIM];
    Nbrs nb;
    auto face_speeds = [&](auto walls) {
        constexpr bool W = decltype(walls)::value;
        nb = neighbours<DIM, W>(t, es);
        const real *ts = (const real *)a.traces;
        // every lane loads (an interior lane a face node of its own element,
        // a valid address whose value it drops), so that no branch waits
        // for the loads before the first stage needs them
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int face = 2 * d + side[d], nface = 2 * d + 1 - side[d];
            const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
            // beyond a wall, the mirror image has the element's own wave speed
            const bool wl = W && ((nb.wall >> face) & 1);
            const long en = wl ? es : (side[d] ? nb.n[d][1] : nb.n[d][0]);
            const int fn = wl ? face : nface;
            const real so = ts[((long)(face * FD::NCT + FD::SPEED) * E + es) * nfn + kk];
            const real sn = ts[((long)(fn * FD::NCT + FD::SPEED) * E + en) * nfn + kk];
            real lam = dmax(so, sn);
            if constexpr (EQ == EQ_MHD) lam = dmax(lam, ctx.ch);
            lamd[d] = onface[d] ? lam : real(0);
        }
    };
    if (t.wall[0] | t.wall[1]) face_speeds(std::true_type{});
    else face_speeds(std::false_type{});

    // blending coefficients of the element (slot 0) and of its face
    // neighbours (slot 1 + 2d + side), formed by the first lanes of the
    // element: given (alpha), or in the pipelined step alpha_e =
    // max(alpha_raw_e, max over face neighbours of alpha_raw / 2); read after
    // the first stage's barrier
    const bool smooth = BLEND && a.alpha_raw != nullptr;
    const bool blend = BLEND && (smooth || a.alpha != nullptr);
    real alpha = real(0);
    if constexpr (!BLEND) {
        // pipelined step: the smoothed coefficient of a clear tile is zero
        if (a.alpha_raw != nullptr && valid && node == 0) a.alpha_s[e] = 0.0;
    }
    if (blend && valid) {
#pragma unroll
        for (int r = 0; r < (NA + NP - 1) / NP; ++r) {
            const int j = node + r * NP;
            if (j >= NA) break;
            long tg = es;           // (selects, not a dynamically indexed array: no scratch)
#pragma unroll
            for (int c = 0; c < 2 * DIM; ++c)
                if (j == 1 + c) tg = nb.n[c >> 1][c & 1];
            double am;
            if (!smooth) {
                am = a.alpha[tg];
            } else {
                // the element itself (j = 0) and its face neighbours take the
                // same path, so that the loads of all these lanes are in
                // flight together
                Nbrs nt;
                if (t.wall[0] | t.wall[1]) nt = neighbours<DIM, true>(t, tg);
                else nt = neighbours<DIM, false>(t, tg);
                am = a.alpha_raw[tg];
#pragma unroll
                for (int d = 0; d < DIM; ++d)
#pragma unroll
                    for (int sd = 0; sd < 2; ++sd) am = fmax(am, 0.5 * a.alpha_raw[nt.n[d][sd]]);
                if (j == 0) a.alpha_s[e] = am;
            }
            alds[le * NA + j] = real(am);
        }
    }

    // Interface flux, split by side.  With lambda and the face blending
    // factor a known to both elements, the blended Rusanov flux of
    // eq:numflux.cons is F* = P^- + P^+ with
    //   P^- = (1-a)(F^-/2 + lambda U^-/2) + a(f(u^-)/2 + lambda u^-/2)
    //   P^+ = (1-a)(F^+/2 - lambda U^+/2) + a(f(u^+)/2 - lambda u^+/2)
    // (U = sum_i b_i u^(i), F = sum_i b_i f_d(u^(i)) at the face node, u = u^n).
    // The element applies its own share and its own trace term
    // -(1-alpha_e) F of the lifting itself and publishes P for the neighbour.
    // Nothing needs U or F on their own, so each stage adds its terms
    // straight into P (per face direction) and into W, where
    //   u_out = u^n - dt W,
    //   W = (1-alpha_e) sum_i b_i R^(i) + alpha_e L
    //       - sum_d s_d/(w dx_d) [P_d - (1-alpha_e) F_d]   (s_d = +1 at xi_d = 0, -1 at xi_d = 1)
    // (L: interior subcell FV update).  For MHD the own non-conservative
    // trace term and the own half of 1/2 B(u^n)(g(U^-) + g(U^+)) enter W the
    // same way; the normal field and psi of U are kept and published.
    real Z[S][M];     // Z[k] = sum_{j<k} a_kj R^(j) (TAB 1: Z[k] = R^(k-1), a_{k,k-1} enters with dt)
    real W[M], P[DIM][M];
    real UB[DIM], Upsi = real(0);   // MHD: time averages of B_d and psi
    real hl[DIM], sw[DIM], oaf[DIM], cF[DIM], cU = real(0);
    real ohl[DIM], oafh[DIM];       // oaf hl and oaf / 2, the per-stage factors of P_d
    real oma = real(1);
#pragma unroll
    for (int v = 0; v < M; ++v) {
        W[v] = real(0);
#pragma unroll
        for (int k = 0; k < S; ++k) Z[k][v] = real(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) P[d][v] = real(0);
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        UB[d] = real(0);
        sw[d] = onface[d] ? (side[d] ? -invw[d] : invw[d]) : real(0);
        hl[d] = onface[d] ? (side[d] ? real(0.5) : real(-0.5)) * lamd[d] : real(0);
        oaf[d] = real(1);
        cF[d] = real(0);
        ohl[d] = hl[d];
        oafh[d] = real(0.5);
    }

#pragma unroll
    for (int i = 0; i < S; ++i) {
        real us[M];
        const real cz = (TAB == 1 && i > 0) ? rdt * Tab<real>::A(t, i, i > 0 ? i - 1 : 0) : rdt;
#pragma unroll
        for (int v = 0; v < M; ++v) us[v] = (i == 0) ? un[v] : un[v] - cz * Z[i][v];
        const real bi = Tab<real>::b(t, i);
        if (i > 0) {
            // the u^(i) terms of P_d and W (those of u^(0) = u^n follow the
            // first barrier, where the blending factors are known)
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const real g = bi * ohl[d];
#pragma unroll
                for (int v = 0; v < M; ++v) P[d][v] += g * us[v];
            }
            const real c = bi * cU;
#pragma unroll
            for (int v = 0; v < M; ++v) W[v] -= c * us[v];
        }
        if constexpr (EQ == EQ_MHD) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) UB[d] += bi * us[5 + d];
            Upsi += bi * us[8];
            if (stagewise && valid) {
                // stage-wise interface flux: this stage's state at the face nodes
                real *st = (real *)a.stage_tr;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    if (!onface[d]) continue;
                    const int face = 2 * d + side[d];
                    const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
#pragma unroll
                    for (int v = 0; v < M; ++v)
                        st[(((long)(face * S + i) * M + v) * E + e) * nfn + kk] = us[v];
                }
            }
        }
        real nd[NF];
        Phys::node(us, nd, ctx);
        real *lds = lds0 + ((DBF && (i & 1)) ? NF * BLK : 0);
        if (i > 0 && !DBF) element_sync<NP, BLK>();    // the previous stage has finished reading LDS
#pragma unroll
        for (int f = 0; f < NF; ++f) lds[f * BLK + tid] = nd[f];
        element_sync<NP, BLK>();
        if (i == 0) {
            if (blend && valid) alpha = alds[le * NA];
            oma = real(1) - alpha;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const real af = (blend && valid && onface[d])
                                    ? real(0.5) * (alpha + alds[le * NA + 1 + 2 * d + side[d]]) : real(0);
                oaf[d] = real(1) - af;
                oafh[d] = real(0.5) * oaf[d];
                ohl[d] = oaf[d] * hl[d];
                cF[d] = sw[d] * (oafh[d] - oma);
                cU += sw[d] * ohl[d];
                const real g = bi * ohl[d];
#pragma unroll
                for (int v = 0; v < M; ++v) P[d][v] += g * un[v];
            }
            const real c = bi * cU;
#pragma unroll
            for (int v = 0; v < M; ++v) W[v] -= c * un[v];
        }

        real R[M];
#pragma unroll
        for (int v = 0; v < M; ++v) R[v] = real(0);
        // sound speed of u^n for the subcell fluxes, once per node (the
        // lanes of an element take the same branch)
        real c_own = real(0);
        if constexpr (CSH) {
            if (i == 0 && blend && alpha > real(0)) {
                c_own = Phys::sound(nd, ctx);
                clds[tid] = c_own;
                element_sync<NP, BLK>();
            }
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            // directly evaluated rotations
#pragma unroll
            for (int k = 1; k <= N; ++k) {
                const bool direct = !SYM || k <= NPRIM || (k == KSELF && !BAL);
                if (!direct) continue;
                int qd = pd[d] + k;
                if (qd >= n1) qd -= n1;
                const int q = line_node<N, DIM>(pd, d, qd);
                real ndq[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) ndq[f] = lds[f * BLK + base + q];
                real fs[M];
                Phys::pair(d, nd, ndq, fs, ctx);
                const real ck = dk(d, k);
#pragma unroll
                for (int v = 0; v < M; ++v) R[v] += ck * fs[v];
                if constexpr (SYM) {
                    if (k <= NPRIM) {
#pragma unroll
                        for (int v = 0; v < M; ++v) xch[((d * NPRIM + (k - 1)) * M + v) * BLK + tid] = fs[v];
                    }
                }
            }
            // diagonal term 2 D_pp f_d(u_p) (non-zero only at the two ends of
            // the line) and the face terms in the same branch
            if (onface[d]) {
                real fp[M];
                if constexpr (EQ == EQ_EULER) Phys::phys_cons(d, us, nd, fp, ctx);
                else Phys::phys(d, nd, fp, ctx);
                const real gp = bi * oafh[d], gw = bi * cF[d], c0 = dk(d, 0);
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    R[v] += c0 * fp[v];
                    P[d][v] += gp * fp[v];
                    W[v] -= gw * fp[v];
                }
                if (i == 0 && oaf[d] < real(1)) {
                    // first-order share a (f(u^n)/2 +- lambda u^n/2) of the blended flux
                    const real af = real(1) - oaf[d];
#pragma unroll
                    for (int v = 0; v < M; ++v) {
                        const real lo = af * (real(0.5) * fp[v] + hl[d] * un[v]);
                        P[d][v] += lo;
                        W[v] -= sw[d] * lo;
                    }
                }
                if constexpr (EQ == EQ_MHD) {
                    // own non-conservative trace term, b_i B_d(u^(i)) g_d(u^(i));
                    // the stage-wise interface flux's own half is half of it
                    real o[M];
                    MhdP<real, FLUX>::btimes(d, nd, nd[5 + d], nd[8], o);
                    const real go = stagewise ? real(0.5) * bi * sw[d] : bi * sw[d];
#pragma unroll
                    for (int v = 0; v < M; ++v) W[v] += go * o[v];
                }
            }
            if constexpr (EQ == EQ_MHD) {
                // sum_q D_pq B_d(u_p) g_d(u_q) = B_d(u_p) (sum_q D_pq g_d(u_q))
                real gB = real(0), gpsi = real(0);
#pragma unroll
                for (int q = 0; q < n1; ++q) {
                    const int qq = line_node<N, DIM>(pd, d, q);
                    gB += Dn[d][q] * lds[(5 + d) * BLK + base + qq];
                    gpsi += Dn[d][q] * lds[8 * BLK + base + qq];
                }
                real o[M];
                MhdP<real, FLUX>::btimes(d, nd, gB, gpsi, o);
#pragma unroll
                for (int v = 0; v < M; ++v) R[v] += o[v];
            }
            // first-order subcell fluxes of the blending limiter, from u^n = u^(1)
            if (i == 0 && blend && alpha > real(0)) {
                real fr[M], fl[M], fp[M];
#pragma unroll
                for (int v = 0; v < M; ++v) { fr[v] = real(0); fl[v] = real(0); }
                Phys::phys(d, nd, fp, ctx);
                real lp;
                if constexpr (CSH) lp = Phys::vspeed(d, nd) + c_own;
                else lp = Phys::speed(d, nd, ctx);
#pragma unroll
                for (int sgn = 0; sgn < 2; ++sgn) {
                    const int qd = sgn ? pd[d] + 1 : pd[d] - 1;
                    if (qd < 0 || qd > N) continue;
                    const int q = line_node<N, DIM>(pd, d, qd);
                    real ndq[NF], fq[M], uq[M];
#pragma unroll
                    for (int f = 0; f < NF; ++f) ndq[f] = lds[f * BLK + base + q];
                    Phys::phys(d, ndq, fq, ctx);
                    Phys::cons(ndq, uq, ctx);
                    real lq;
                    if constexpr (CSH) lq = Phys::vspeed(d, ndq) + clds[base + q];
                    else lq = Phys::speed(d, ndq, ctx);
                    const real lam = dmax(lp, lq);
#pragma unroll
                    for (int v = 0; v < M; ++v) {
                        if (sgn) fr[v] = real(0.5) * (fp[v] + fq[v]) - real(0.5) * lam * (uq[v] - un[v]);
                        else fl[v] = real(0.5) * (fq[v] + fp[v]) - real(0.5) * lam * (un[v] - uq[v]);
                    }
                }
#pragma unroll
                for (int v = 0; v < M; ++v) W[v] += alpha * invw[d] * (fr[v] - fl[v]);
            }
        }
        // balanced self-mirrored rotation: the pair of direction dm
        bool xm = false;
        int qx = 0, qy = 0;
        if constexpr (BAL) {
            xm = (pd[0] < KSELF) != (pd[1] < KSELF);
            qx = pd[0] + KSELF < n1 ? pd[0] + KSELF : pd[0] + KSELF - n1;
            qy = pd[1] + KSELF < n1 ? pd[1] + KSELF : pd[1] + KSELF - n1;
            const int q = xm ? line_node<N, DIM>(pd, 0, qx) : line_node<N, DIM>(pd, 1, qy);
            real ndq[NF], fs[M];
#pragma unroll
            for (int f = 0; f < NF; ++f) ndq[f] = lds[f * BLK + base + q];
            Phys::pair_rt(xm ? 0 : 1, nd, ndq, fs, ctx);
            const real c = xm ? dk(0, KSELF) : dk(DIM - 1, KSELF);
#pragma unroll
            for (int v = 0; v < M; ++v) {
                R[v] += c * fs[v];
                xb[v * BLK + tid] = fs[v];
            }
        }
        if constexpr (SYM) {
            element_sync<NP, BLK>();
            if constexpr (BAL) {
                // the pair of the other direction, from the lane that evaluated it
                const int src = base + (xm ? line_node<N, DIM>(pd, 1, qy) : line_node<N, DIM>(pd, 0, qx));
                const real c = xm ? dk(DIM - 1, KSELF) : dk(0, KSELF);
#pragma unroll
                for (int v = 0; v < M; ++v) R[v] += c * xb[v * BLK + src];
            }
#pragma unroll
            for (int d = 0; d < DIM; ++d)
#pragma unroll
                for (int k = 1; k <= NPRIM; ++k) {
                    // mirror rotation n1 - k: the pair (p, p - k) was evaluated by lane p - k
                    int sd = pd[d] - k;
                    if (sd < 0) sd += n1;
                    const int src = base + line_node<N, DIM>(pd, d, sd);
                    const real c = dk(d, n1 - k);
#pragma unroll
                    for (int v = 0; v < M; ++v) R[v] += c * xch[((d * NPRIM + (k - 1)) * M + v) * BLK + src];
                }
        }
        // stage bookkeeping
        if constexpr (TAB == 1) {
            // classical RK4: only a_{i+1,i} is non-zero
            if (i + 1 < S) {
#pragma unroll
                for (int v = 0; v < M; ++v) Z[i + 1][v] = R[v];
            }
        } else {
#pragma unroll
            for (int k = i + 1; k < S; ++k) {
                if (!stage_coupled<TAB>(k, i)) continue;
                const real aki = Tab<real>::A(t, k, i);
#pragma unroll
                for (int v = 0; v < M; ++v) Z[k][v] += aki * R[v];
            }
        }
        const real wbi = oma * bi;
#pragma unroll
        for (int v = 0; v < M; ++v) W[v] += wbi * R[v];
    }

    if (!valid) return;
    if (EQ == EQ_MHD && !stagewise) {
        // own half of 1/2 B(u^n)(g(U^-) + g(U^+))
        real ndo[NF];
        Phys::node_basic(un, ndo, ctx);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (!onface[d]) continue;
            real o[M];
            MhdP<real, FLUX>::btimes(d, ndo, real(0.5) * UB[d], real(0.5) * Upsi, o);
#pragma unroll
            for (int v = 0; v < M; ++v) W[v] -= sw[d] * o[v];
        }
    }
    // face data: P for the neighbours (traces[face][c][e][k], c < M; MHD: c = M, M + 1 the normal field and psi)
    real *tr = (real *)a.traces;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (!onface[d]) continue;
        const int face = 2 * d + side[d];
        const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
        real *tb = tr + ((long)face * FD::NCT * E + e) * nfn + kk;
#pragma unroll
        for (int v = 0; v < M; ++v) tb[((long)v * E) * nfn] = P[d][v];
        if constexpr (EQ == EQ_MHD) {
            tb[((long)M * E) * nfn] = UB[d];
            tb[((long)(M + 1) * E) * nfn] = Upsi;
        }
    }
    real *uout = (real *)a.u_out;
#pragma unroll
    for (int v = 0; v < M; ++v) uout[((long)v * E + e) * NP + node] = un[v] - rdt * W[v];
}

// With tile flags, the BLEND = false instance runs the clear tiles (and
// clears every tile's flag of the next step) and the BLEND = true instance,
// launched after it, the flagged ones; a tile of the other kind is left at
// once.  WPB > 1 (single-wavefront tiles only): each workgroup holds WPB
// wavefronts, each running its own tile with its own LDS slice and never
// waiting for the others, so a launch that skips most tiles dispatches WPB
// times fewer workgroups.
template <int NP, int WPB>
constexpr int local_wpb() { return tile_block<NP>() == 64 ? WPB : 1; }

template <typename real, int EQ, int DIM, int N, int FLUX, int S, int TAB = 0, bool BLEND = true, bool NCS = false,
          int WPB = 1>
__global__ void __launch_bounds__(tile_block<DIM == 2 ? (N + 1) * (N + 1) : N + 1>() * WPB)
k_local(const Tables t, const StepPtrs a)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    constexpr int SL = LocalShape<real, EQ, DIM, N, FLUX, BLEND>::slots * TB;
    static_assert(WPB == 1 || TB == 64, "several tiles per workgroup need single-wavefront tiles");
    __shared__ real smem[SL * WPB];
    const int w = WPB == 1 ? 0 : (int)(threadIdx.x / 64);
    const long tile = (long)xcd_chunk_tile(blockIdx.x, gridDim.x) * WPB + w;
    if constexpr (WPB > 1) {
        if (tile * (TB / NP) >= t.nelem) return;
    }
    if (a.tiles_in != nullptr) {
        const int flagged = a.tiles_in[tile];
        if constexpr (!BLEND) {
            if (threadIdx.x % 64 == 0) a.tiles_out[tile] = 0;
        }
        if (BLEND ? flagged == 0 : flagged != 0) return;
    }
    local_tile<real, EQ, DIM, N, FLUX, S, TB, TAB, BLEND, NCS>(t, a, tile * (TB / NP), smem + w * SL,
                                                               WPB == 1 ? -1 : (int)(threadIdx.x % 64));
}

// ---------------------------------------------------------------- K8 helper: modal indicator
// Blending coefficient of one element from eps = rho*p at its nodes, one lane
// per node: modal coefficients in the orthonormal Legendre basis, energy in
// the highest modes, logistic map (Hennemann-Gassner form), clipping at
// alpha_min and cap at alpha_max.  Every lane of the workgroup must call it.
// sum over the aligned groups of W consecutive lanes of a wavefront (W a
// power of two dividing 64); every lane of a group gets the same bits
template <int W>
__device__ __forceinline__ double group_sum(double x)
{
#pragma unroll
    for (int m = 1; m < W; m <<= 1) x += __shfl_xor(x, m, W);
    return x;
}

// Flag the local-phase tiles (epb elements each) of element e, of its face
// neighbours and of theirs: every tile whose blending coefficients can
// depend on alpha_raw[e] (smoothing over faces, face factor of neighbours).
template <int DIM>
__device__ __forceinline__ void mark_tiles(const Tables &t, long e, int epb, int *tiles)
{
    tiles[e / epb] = 1;
    const Nbrs nb = neighbours<DIM>(t, e);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const long n = nb.n[d][sd];
            tiles[n / epb] = 1;
            const Nbrs n2 = neighbours<DIM>(t, n);
#pragma unroll
            for (int d2 = 0; d2 < DIM; ++d2)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) tiles[n2.n[d2][s2] / epb] = 1;
        }
}

// eps = rho p of a node from its conserved Euler state in FP64, the
// indicator's input.  One function without contraction for the standalone
// indicator and the tail of the pipelined interface phase, so that both give
// the same bits (a pipelined run resumed from its state continues exactly).
template <int DIM>
__device__ __forceinline__ double indicator_eps(const double *us, double gamma)
{
#pragma clang fp contract(off)
    double ke = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) ke += us[1 + k] * us[1 + k];
    const double p = (gamma - 1.0) * (us[DIM + 1] - 0.5 * ke / us[0]);
    return us[0] * p;
}

// a double moved across lanes by a DPP control (CTRL a compile-time control
// word; every source lane exists for the quad permutations and the row
// rotations used here)
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int DIM, int N, int BLK>
__device__ __forceinline__ void indicator_lanes(const Tables &t, int tid, int le, int node, long e, bool valid,
                                                double eps_node, double *eps, double *en, double *alpha_raw,
                                                float *features, int *tiles = nullptr)
{
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    // an element's lanes are one aligned power-of-two group of a wavefront:
    // exchange and sums stay inside the wavefront
    constexpr bool WAVE = (NP & (NP - 1)) == 0 && 64 % NP == 0;
    // degree 3 in 2D: an element is one 16-lane DPP row and each of its node
    // rows (4 lanes) one quad, so the separable transform m = V (V eps)^T
    // moves its values with quad permutations and row rotations, without LDS
    constexpr bool DPP = DIM == 2 && N == 3 && WAVE;
    const int mk = node % n1, ml = DIM == 2 ? node / n1 : 0;
    double m = 0.0;
    if constexpr (DPP) {
        // a(mk, j) = sum_i V[mk][i] eps(i, j): eps of the lane's node row by
        // quad broadcasts (lane 4 j + i holds eps(i, j))
        double a = t.Vinv[mk][0] * dpp_double<0x00>(eps_node);
        a += t.Vinv[mk][1] * dpp_double<0x55>(eps_node);
        a += t.Vinv[mk][2] * dpp_double<0xAA>(eps_node);
        a += t.Vinv[mk][3] * dpp_double<0xFF>(eps_node);
        // m(mk, ml) = sum_j V[ml][j] a(mk, j): rotating the row right by
        // 4 s brings a(mk, (ml - s) mod 4) from lane 4 ((ml - s) mod 4) + mk
        m = t.Vinv[ml][ml] * a;
        m += t.Vinv[ml][(ml + 3) & 3] * dpp_double<0x124>(a);
        m += t.Vinv[ml][(ml + 2) & 3] * dpp_double<0x128>(a);
        m += t.Vinv[ml][(ml + 1) & 3] * dpp_double<0x12C>(a);
    } else {
        eps[tid] = eps_node;
        element_sync<NP, BLK>();
        double rk[n1], rl[n1];
#pragma unroll
        for (int c = 0; c < n1; ++c) {
            rk[c] = t.Vinv[mk][c];
            rl[c] = t.Vinv[ml][c];
        }
        if constexpr (DIM == 1) {
#pragma unroll
            for (int i = 0; i < n1; ++i) m += rk[i] * eps[le * NP + i];
        } else {
#pragma unroll
            for (int j = 0; j < n1; ++j) {
                double sj = 0.0;
#pragma unroll
                for (int i = 0; i < n1; ++i) sj += rk[i] * eps[le * NP + j * n1 + i];
                m += rl[j] * sj;
            }
        }
    }
    const double e2 = m * m;
    const double x1 = (mk <= N - 1 && ml <= N - 1) ? e2 : 0.0;
    const double x2 = (mk <= N - 2 && ml <= N - 2) ? e2 : 0.0;
    double tot, c1, c2;
    if constexpr (WAVE) {
        tot = group_sum<NP>(e2);
        c1 = group_sum<NP>(x1);
        c2 = group_sum<NP>(x2);
    } else {
        en[tid] = e2;
        en[BLK + tid] = x1;
        en[2 * BLK + tid] = x2;
        __syncthreads();
        tot = c1 = c2 = 0.0;
        if (valid) {
            for (int p = 0; p < NP; ++p) {
                tot += en[le * NP + p];
                c1 += en[BLK + le * NP + p];
                c2 += en[2 * BLK + le * NP + p];
            }
        }
    }
    if (valid) {
        // every lane of the element forms the same coefficient
        // both energy fractions from one Newton reciprocal (tot, c1 > 0: they
        // hold the mean's energy)
        const double r = rcp_nr(tot * c1);
        const double E1 = (tot - c1) * (c1 * r), E2 = (c1 - c2) * (tot * r);
        const double En = E1 > E2 ? E1 : E2;
        double al = 0.0;
        if (!(En < t.ind_en_zero)) {   // (a non-finite energy takes the full evaluation)
            al = 1.0 / (1.0 + exp(-t.ind_slope * (En - t.ind_threshold)));
            if (al < t.alpha_min) al = 0.0;
        }
        if (al > 1.0 - t.alpha_min) al = 1.0;
        if (al > t.alpha_max) al = t.alpha_max;
        if (node == 0) alpha_raw[e] = al;
        // tile flags (2D): the lanes of a blending element flag the tiles of
        // the 13 elements within two faces of it (the element, its four face
        // neighbours, the four at distance two along x or y and the four
        // diagonal ones), periodic; target j is taken by lane j mod NP, so
        // elements of fewer than 13 nodes (N = 1, 2) cover all of them too
        if constexpr (DIM == 2) {
            if (tiles != nullptr && al > 0.0) {
                const int nx = t.nx, ny = t.ny, ei = (int)e;
                const int ey = (int)(((unsigned long long)(unsigned)ei * (unsigned long long)t.nx_m) >> t.nx_s), ex = ei - ey * nx;
#pragma unroll
                for (int j0 = 0; j0 < 13; j0 += NP) {
                    const int j = j0 + node;
                    if (j >= 13) break;
                    const int r = j < 9 ? (j - 1) & 3 : j - 9;
                    int dx = 0, dy = 0;
                    if (j >= 1 && j <= 8) {
                        const int s = j <= 4 ? 1 : 2;
                        dx = r == 0 ? s : (r == 1 ? -s : 0);
                        dy = r == 2 ? s : (r == 3 ? -s : 0);
                    } else if (j >= 9) {
                        dx = (r & 1) ? 1 : -1;
                        dy = (r & 2) ? 1 : -1;
                    }
                    // periodic wrap of offsets |dx|, |dy| <= 2 (loops for meshes narrower than that)
                    int x = ex + dx, y = ey + dy;
                    while (x < 0) x += nx;
                    while (x >= nx) x -= nx;
                    while (y < 0) y += ny;
                    while (y >= ny) y -= ny;
                    tiles[(y * nx + x) / (BLK / NP)] = 1;
                }
            }
        }
    }
    // features of the learned indicator: the modal energy fractions
    // f = m_kl^2 / sum m^2 on a log scale, 1 + log10(max(f, 1e-16))/16 in [0, 1]
    if (features != nullptr && valid)
        features[e * NP + node] = (float)(1.0 + log10(fmax(e2 / tot, 1e-16)) / 16.0);
}

// Workgroup maximum of v (all lanes call) into *slot; a one-workgroup kernel
// finishes the reduction after the grid has drained.  With ATOMIC the
// maximum is merged into *slot (which must start at zero) by an integer
// atomic maximum on the bit pattern: for non-negative doubles the integer
// order is the numeric order, so the merged value is exact and does not
// depend on the order of the merges.  A NaN maximum (every lane NaN) counts
// as zero, as fmax would treat it.
template <int BLK, bool ATOMIC = false>
__device__ __forceinline__ void block_max_lanes(double v, double *red, double *slot)
{
    // maximum over the wavefront by butterfly, then over the BLK/64 wavefronts
    static_assert(BLK % 64 == 0, "whole wavefronts");
    const int tid = threadIdx.x;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    if constexpr (BLK > 64) {
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
    }
    if (tid == 0) {
        double r = v;
        if constexpr (BLK > 64) {
            r = red[0];
#pragma unroll
            for (int w = 1; w < BLK / 64; ++w) r = fmax(r, red[w]);
        }
        if constexpr (ATOMIC) {
            const double rr = r >= 0.0 ? r : 0.0;
            atomicMax((unsigned long long *)slot, (unsigned long long)__double_as_longlong(rr));
        } else {
            *slot = r;
        }
    }
}

// Slots of the pipelined step's wave-speed maximum: interface-phase
// workgroup b merges its maximum into slot b mod DT_SLOTS; k_dt_slots, one
// wavefront, reads every slot once (four loads per lane, issued together),
// puts it back to zero for the next step and finishes dt.  Far fewer loads
// than one partial per workgroup.
constexpr int DT_SLOTS = 256;

// ---------------------------------------------------------------- K3: interface + final update
// One lane per node; the face-node lanes apply the interface corrections.
// u^n at the face nodes of both sides is read from the state the step
// started from.  In the pipelined step every lane then holds u^{n+1} of its
// node and the workgroup computes the CFL maximum and the raw indicator.
// One tile of BLK lanes (elements e0 .. e0 + BLK/(N+1)^DIM - 1).  In the
// pipelined step the tile's wave-speed maximum goes to partials[slot] (with
// SLOTS: is merged into partials[slot mod DT_SLOTS]); dsmem holds 5 * BLK
// doubles.
template <typename real, int EQ, int DIM, int N, int FLUX, int BLK, bool SLOTS = false, bool NCS = false>
__device__ __forceinline__ void interface_tile(const Tables &t, const StepPtrs &a, long e0, long slot, double *dsmem)
{
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int EPB = BLK / NP;
    constexpr int M = Phys::M;
    constexpr int NF = Phys::NF;
    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = e0 + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const int pd[2] = {node % n1, DIM == 2 ? node / n1 : 0};
    const bool tail = a.dt_out != nullptr;

    const long E = t.nelem;
    constexpr int nf = DIM == 2 ? n1 : 1;
    using FD = FaceData<EQ, M>;
    const Ctx<real> ctx = make_ctx<real>(t, a.dt);
    const real rdt = real(a.dt[0]);
    const real *tr = (const real *)a.traces;
    real *uo = (real *)a.u_out;

    bool face_lane = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) face_lane |= (pd[d] == 0 || pd[d] == N);
    face_lane &= valid;

    real u[M];
    if (face_lane || (tail && valid)) {
#pragma unroll
        for (int v = 0; v < M; ++v) u[v] = uo[((long)v * E + e) * NP + node];
    } else {
#pragma unroll
        for (int v = 0; v < M; ++v) u[v] = real(v == 0 ? 1 : 0);
    }
    // (meshes without walls, a uniform test, take a copy compiled without the wall cases)
    auto face_update = [&](auto walls) {
        constexpr bool W = decltype(walls)::value;
        // the neighbour's share of the interface flux (the own share and the
        // own trace term were applied by the local phase), lifted with
        // dg_R/dxi = delta_pN/w_N, dg_L/dxi = -delta_p0/w_0
        const Nbrs nb = neighbours<DIM, W>(t, e);
        real ndo[NF];
        if constexpr (EQ == EQ_MHD) {
            const real *uin = (const real *)a.u_in;
            real uno[M];
#pragma unroll
            for (int v = 0; v < M; ++v) uno[v] = uin[((long)v * E + e) * NP + node];
            Phys::node_basic(uno, ndo, ctx);
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (!(pd[d] == 0 || pd[d] == N)) continue;
            const int side = pd[d] == N ? 1 : 0;
            const long en = side ? nb.n[d][1] : nb.n[d][0];
            const int nface = 2 * d + 1 - side;
            const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
            // Beyond a wall lies the mirror image R u of the element (R
            // negates the normal momentum), whose share is -R P of the
            // element's own P: f_d(R u) = -R f_d(u) for every state, so both
            // the time averages and the first-order part mirror that way.
            const bool wl = W && ((nb.wall >> (2 * d + side)) & 1);
            const real *tn = wl ? tr + ((long)(2 * d + side) * FD::NCT * E + e) * nf + kk
                                : tr + ((long)nface * FD::NCT * E + en) * nf + kk;
            real jump[M];
#pragma unroll
            for (int v = 0; v < M; ++v) {
                const real x = tn[((long)v * E) * nf];
                jump[v] = (wl && v != 1 + d) ? -x : x;
            }
            if constexpr (EQ == EQ_MHD) {
                if constexpr (!NCS) {
                    // reduced form: the neighbour's half of 1/2 B(u^n)(g(U^-) + g(U^+))
                    real o[M];
                    MhdP<real, FLUX>::btimes(d, ndo, real(0.5) * tn[((long)M * E) * nf],
                                             real(0.5) * tn[((long)(M + 1) * E) * nf], o);
#pragma unroll
                    for (int v = 0; v < M; ++v) jump[v] += o[v];
                } else {
                    // stage-wise form (eq:bad.numflux.non.cons): the neighbour's half
                    // sum_j b_j 1/2 B(u^(j)_own) g(u^(j)_nb), from the stage states
                    // that both local phases left at the face nodes
                    const real *st = (const real *)a.stage_tr;
                    const int S = t.stages;
                    for (int j = 0; j < S; ++j) {
                        real uj[M], ndj[NF], o[M];
                        const real *so = st + ((long)((2 * d + side) * S + j) * M * E + e) * nf + kk;
                        const real *sn = st + ((long)(nface * S + j) * M * E + en) * nf + kk;
#pragma unroll
                        for (int v = 0; v < M; ++v) uj[v] = so[(long)v * E * nf];
                        Phys::node_basic(uj, ndj, ctx);
                        MhdP<real, FLUX>::btimes(d, ndj, real(0.5) * sn[(long)(5 + d) * E * nf],
                                                 real(0.5) * sn[(long)8 * E * nf], o);
                        const real bj = real(t.b[j]);
#pragma unroll
                        for (int v = 0; v < M; ++v) jump[v] += bj * o[v];
                    }
                }
            }
            const real coef = rdt * real(t.invw_dx[d][side ? N : 0]);
#pragma unroll
            for (int v = 0; v < M; ++v) u[v] += side ? -coef * jump[v] : coef * jump[v];
        }
    };
    if (face_lane) {
        if (t.wall[0] | t.wall[1]) face_update(std::true_type{});
        else face_update(std::false_type{});
    }
    // the pipelined step has every node in registers and writes whole
    // elements (whole cache lines: no read of the lines it only partly
    // writes); otherwise only the face nodes are written
    if (face_lane || (tail && valid)) {
#pragma unroll
        for (int v = 0; v < M; ++v) uo[((long)v * E + e) * NP + node] = u[v];
    }
    if (!tail) return;

    // pipelined tail: CFL maximum, face wave speeds and raw indicator of u^{n+1}
    real nd[NF];
    Phys::node_basic(u, nd, ctx);
    double sp = 0.0;
    if (valid) {
        real *ts = (real *)a.traces;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const real sd = face_speed<real, EQ, DIM, FLUX>(d, nd, ctx);
            if constexpr (EQ == EQ_MHD) sp = fmax(sp, (double)sd);
            else sp += (double)sd * t.invdx[d];
            if (pd[d] == 0 || pd[d] == N) {
                const int face = 2 * d + (pd[d] == N ? 1 : 0);
                const int kk = DIM == 1 ? 0 : (d == 0 ? pd[1] : pd[0]);
                ts[((long)(face * FD::NCT + FD::SPEED) * E + e) * nf + kk] = sd;
            }
        }
    }
    if constexpr (EQ == EQ_EULER) {
        if (a.alpha_raw_out != nullptr) {
            double ud[M];
#pragma unroll
            for (int v = 0; v < M; ++v) ud[v] = (double)u[v];
            indicator_lanes<DIM, N, BLK>(t, tid, le, node, e, valid, indicator_eps<DIM>(ud, t.gamma), dsmem + BLK,
                                         dsmem + 2 * BLK, a.alpha_raw_out, a.features, a.tiles_out);
        }
    }
    if constexpr (SLOTS) block_max_lanes<BLK, true>(sp, dsmem, a.partials + slot % DT_SLOTS);
    else block_max_lanes<BLK>(sp, dsmem, a.partials + slot);
}

template <typename real, int EQ, int DIM, int N, int FLUX, bool NCS = false>
__global__ void __launch_bounds__(tile_block<DIM == 2 ? (N + 1) * (N + 1) : N + 1>()) k_interface(const Tables t, const StepPtrs a)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    __shared__ double dsmem[5 * TB];
    interface_tile<real, EQ, DIM, N, FLUX, TB, true, NCS>(t, a, xcd_tile(blockIdx.x, gridDim.x) * (TB / NP), blockIdx.x, dsmem);
}

// dt = cfl / ((N+1) m) from the global wave-speed maximum m (MHD: m = c_h and
// every lambda_d equals it)
__device__ __forceinline__ void finish_dt(const Tables &t, double m, int is_mhd, double *dt)
{
    if (is_mhd) {
        // every lambda_d = max(|v_d| + c_f, c_h) equals c_h = the global max
        double sdx = 0.0;
        for (int d = 0; d < t.dim; ++d) sdx += t.invdx[d];
        dt[0] = t.cfl / ((t.N + 1) * m * sdx);
        dt[1] = m;
    } else {
        dt[0] = t.cfl / ((t.N + 1) * m);
        dt[1] = 0.0;
    }
}

// ---------------------------------------------------------------- small meshes: every step in one workgroup
// A mesh of up to RUN_BLOCK nodes fits one workgroup: the local phase, the
// interface phase and the dt reduction of each pipelined step run back to
// back inside one launch, separated by workgroup barriers.  The phases
// exchange data through global memory written and read by the waves of one
// CU, which the barriers' workgroup-scope ordering makes visible; dt lives in
// LDS between the steps.  Same device code and arithmetic as the separate
// launches.
constexpr int RUN_BLOCK = 256;   // one wavefront per SIMD: no register cap
template <typename real, int EQ, int DIM, int N, int FLUX, int S, int TAB, bool BLEND>
__global__ void __launch_bounds__(RUN_BLOCK) k_run(const Tables t, const StepPtrs a0, double *dt_io, int nsteps)
{
    constexpr size_t LB = (size_t)LocalShape<real, EQ, DIM, N, FLUX, BLEND>::slots * RUN_BLOCK * sizeof(real);
    constexpr size_t DB = (size_t)5 * RUN_BLOCK * sizeof(double);
    __shared__ double pool[(LB > DB ? LB : DB) / sizeof(double)];   // local phase, then interface phase
    __shared__ double dtl[2];
    const int tid = threadIdx.x;
    StepPtrs ae = a0, ao = a0;         // even and odd steps
    ao.u_in = a0.u_out;
    ao.u_out = const_cast<void *>(a0.u_in);
    ae.dt = ao.dt = dtl;
    ae.dt_out = ao.dt_out = dtl;       // (non-null: the interface phase runs its tail)
    if (tid == 0) { dtl[0] = dt_io[0]; dtl[1] = dt_io[1]; }
    __syncthreads();
    for (int k = 0; k < nsteps; ++k) {
        const StepPtrs &p = (k & 1) ? ao : ae;
        local_tile<real, EQ, DIM, N, FLUX, S, RUN_BLOCK, TAB, BLEND>(t, p, 0, (real *)pool);
        __syncthreads();
        interface_tile<real, EQ, DIM, N, FLUX, RUN_BLOCK>(t, p, 0, 0, pool);
        __syncthreads();
        if (tid == 0) finish_dt(t, p.partials[0], EQ == EQ_MHD ? 1 : 0, dtl);
        __syncthreads();
    }
    if (tid == 0) { dt_io[0] = dtl[0]; dt_io[1] = dtl[1]; }
}

// ---------------------------------------------------------------- K1: time step
// Per node sum_d lambda_d/dx_d (Euler) or max_d (|v_d| + c_f) (MHD); block
// maxima into partials, then one block finishes.  Deterministic, no atomics.
template <typename real, int EQ, int DIM>
__global__ void __launch_bounds__(BLOCK) k_dt_partial(const Tables t, const void *u_, double *partials)
{
    using Phys = typename PhysOf<real, EQ, DIM, (EQ == EQ_MHD ? VOL_DERIGS : VOL_KG)>::type;
    constexpr int M = Phys::M;
    __shared__ double red[BLOCK];
    const real *u = (const real *)u_;
    const long total = (long)t.nelem * t.nnode;
    Ctx<real> ctx = make_ctx<real>(t, nullptr);
    double mx = 0.0;
    for (long idx = (long)blockIdx.x * BLOCK + threadIdx.x; idx < total; idx += (long)gridDim.x * BLOCK) {
        real us[M], nd[Phys::NF];
#pragma unroll
        for (int v = 0; v < M; ++v) us[v] = u[(long)v * total + idx];
        Phys::node_basic(us, nd, ctx);
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if constexpr (EQ == EQ_MHD) s = fmax(s, (double)MhdP<real, VOL_DERIGS>::fast(d, nd, ctx));
            else s += (double)Phys::speed(d, nd, ctx) * t.invdx[d];
        }
        mx = fmax(mx, s);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

constexpr int FINAL_BLOCK = 1024;
static __global__ void __launch_bounds__(FINAL_BLOCK) k_dt_final(const Tables t, const double *partials, int nparts,
                                                                 int is_mhd, double *dt)
{
    // the partials were just written by workgroups on every XCD, so each load
    // is a round trip to memory: issue eight per lane at once rather than one
    // after the other
    __shared__ double red[FINAL_BLOCK / 64];
    const int tid = threadIdx.x;
    double mx = 0.0;
    for (int k0 = 0; k0 < nparts; k0 += 8 * FINAL_BLOCK) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + j * FINAL_BLOCK + tid;
            v[j] = k < nparts ? partials[k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) mx = fmax(mx, v[j]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = red[0];
        for (int w = 1; w < FINAL_BLOCK / 64; ++w) m = fmax(m, red[w]);
        finish_dt(t, m, is_mhd, dt);
    }
}

// dt of the pipelined step from the DT_SLOTS merged maxima, which it leaves
// at zero for the next interface phase
static __global__ void __launch_bounds__(64) k_dt_slots(const Tables t, double *slots, int is_mhd, double *dt)
{
    // one wavefront: DT_SLOTS / 64 loads per lane in flight together, then a butterfly
    const int tid = threadIdx.x;
    double v[DT_SLOTS / 64];
#pragma unroll
    for (int j = 0; j < DT_SLOTS / 64; ++j) v[j] = slots[j * 64 + tid];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < DT_SLOTS / 64; ++j) {
        mx = fmax(mx, v[j]);
        slots[j * 64 + tid] = 0.0;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, 64));
    if (tid == 0) finish_dt(t, mx, is_mhd, dt);
}

static __global__ void k_zero(double *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// tile flags of a state from its raw coefficients (flags zero on entry)
template <int DIM>
__global__ void __launch_bounds__(BLOCK) k_mark_tiles(const Tables t, const double *alpha_raw, int epb, int *tiles)
{
    const long e = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (e < t.nelem && alpha_raw[e] > 0.0) mark_tiles<DIM>(t, e, epb, tiles);
}
static __global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- K8: modal indicator
template <typename real, int DIM, int N>
__global__ void __launch_bounds__(BLOCK) k_indicator(const Tables t, const void *u_, double *alpha_raw, float *features)
{
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int EPB = BLOCK / NP;
    __shared__ double eps[BLOCK];
    __shared__ double en[3 * BLOCK];
    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const long E = t.nelem;
    const real *u = (const real *)u_;
    constexpr int M = DIM + 2;
    double us[M];
#pragma unroll
    for (int v = 0; v < M; ++v) us[v] = (double)u[((long)v * E + es) * NP + node];
    indicator_lanes<DIM, N, BLOCK>(t, tid, le, node, e, valid, indicator_eps<DIM>(us, t.gamma), eps, en, alpha_raw,
                                   features);
}

static __global__ void __launch_bounds__(BLOCK) k_smooth(const Tables t, const double *alpha_raw, double *alpha)
{
    const long e = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= t.nelem) return;
    const Nbrs nb = neighbours_any(t, e);
    double a = alpha_raw[e];
    for (int d = 0; d < t.dim; ++d)
        for (int s = 0; s < 2; ++s) a = fmax(a, 0.5 * alpha_raw[s ? nb.n[d][1] : nb.n[d][0]]);
    alpha[e] = a;
}

// ---------------------------------------------------------------- K5: diagnostics
// partial layout per block: [M totals, entropy, min rho, min p, nonfinite, first bad]
template <typename real, int EQ, int DIM>
__global__ void __launch_bounds__(BLOCK) k_diag_partial(const Tables t, const void *u_, double *partials)
{
    constexpr int M = EQ == EQ_MHD ? 9 : DIM + 2;
    constexpr int K = M + 5;
    __shared__ double red[K][BLOCK];
    const real *u = (const real *)u_;
    const long total = (long)t.nelem * t.nnode;
    const int n1 = t.N + 1;
    double acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = 0.0;
    acc[M + 1] = INFINITY; acc[M + 2] = INFINITY; acc[M + 4] = INFINITY;
    const double vol = (DIM == 2) ? 1.0 / (t.invdx[0] * t.invdx[1]) : 1.0 / t.invdx[0];
    for (long idx = (long)blockIdx.x * BLOCK + threadIdx.x; idx < total; idx += (long)gridDim.x * BLOCK) {
        const long e = idx / t.nnode;
        const int node = (int)(idx - e * t.nnode);
        const int i = node % n1, j = node / n1;
        double wq = t.w[i] * (DIM == 2 ? t.w[j] : 1.0) * vol;
        double us[M];
        bool bad = false;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            us[v] = (double)u[(long)v * total + idx];
            if (!isfinite(us[v])) { acc[M + 3] += 1.0; bad = true; }
            acc[v] += wq * us[v];
        }
        double rho = us[0], p;
        if constexpr (EQ == EQ_MHD) {
            const double vv = (us[1] * us[1] + us[2] * us[2] + us[3] * us[3]) / rho;
            const double BB = us[5] * us[5] + us[6] * us[6] + us[7] * us[7];
            p = (t.gamma - 1.0) * (us[4] - 0.5 * vv - 0.5 * BB - 0.5 * us[8] * us[8]);
        } else {
            double ke = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) ke += us[1 + k] * us[1 + k];
            p = (t.gamma - 1.0) * (us[DIM + 1] - 0.5 * ke / rho);
        }
        if (!(rho > 0.0) || !(p > 0.0)) bad = true;
        acc[M + 1] = fmin(acc[M + 1], rho);
        acc[M + 2] = fmin(acc[M + 2], p);
        if (rho > 0.0 && p > 0.0) acc[M] += wq * (-rho * (log(p) - t.gamma * log(rho)) / (t.gamma - 1.0));
        if (bad) acc[M + 4] = fmin(acc[M + 4], (double)e);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const double x = red[c][threadIdx.x], y = red[c][threadIdx.x + w];
                red[c][threadIdx.x] = (c == M + 1 || c == M + 2 || c == M + 4) ? fmin(x, y) : x + y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c) partials[(long)blockIdx.x * K + c] = red[c][0];
    }
}

static __global__ void k_diag_final(int M, const double *partials, int nparts, double *out)
{
    // one lane per quantity, serial over blocks in index order (deterministic)
    const int c = threadIdx.x;
    const int K = M + 5;
    if (c >= K) return;
    const bool ismin = (c == M + 1 || c == M + 2 || c == M + 4);
    double acc = ismin ? INFINITY : 0.0;
    for (int k = 0; k < nparts; ++k) {
        const double x = partials[(long)k * K + c];
        acc = ismin ? fmin(acc, x) : acc + x;
    }
    if (c == M + 4) acc = isinf(acc) ? -1.0 : acc;
    out[c] = acc;
}

// ---------------------------------------------------------------- launchers
template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_local(const Tables &t, const StepPtrs &p, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    constexpr int EPB = TB / NP;
    const int grid = (t.nelem + EPB - 1) / EPB;
    constexpr int WP = local_wpb<NP, CRK_LOCAL_WPB_PLAIN>(), WB = local_wpb<NP, CRK_LOCAL_WPB_BLEND>();
#define CRK_LOCAL_LAUNCH(BL, W)                                                                                    \
    {                                                                                                              \
        const dim3 g((grid + W - 1) / W), b(TB * W);                                                               \
        switch (t.stages) {                                                                                        \
        case 1: hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 1, 0, BL, false, W>), g, b, 0, s, t, p); break; \
        case 2: hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 2, 0, BL, false, W>), g, b, 0, s, t, p); break; \
        case 3: hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 3, 0, BL, false, W>), g, b, 0, s, t, p); break; \
        case 4:                                                                                                    \
            if (t.tableau == 1) hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 4, 1, BL, false, W>), g, b, 0, s, t, p); \
            else hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 4, 0, BL, false, W>), g, b, 0, s, t, p);  \
            break;                                                                                                 \
        case 5: hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 5, 0, BL, false, W>), g, b, 0, s, t, p); break; \
        case 6:                                                                                                    \
            if (t.tableau == 2) hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 6, 2, BL, false, W>), g, b, 0, s, t, p); \
            else hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 6, 0, BL, false, W>), g, b, 0, s, t, p);  \
            break;                                                                                                 \
        default: return hipErrorInvalidValue;                                                                      \
        }                                                                                                          \
    }
    // without blending coefficients (no limiter) every tile takes the
    // instance without the blending code; with tile flags both run, the
    // blending one second; with given coefficients only the blending one
    if constexpr (EQ == EQ_MHD) {
        if (p.stage_tr != nullptr) {
            // stage-wise non-conservative interface flux: the default tableaus only
            if (!(p.instances == 0 || (p.instances & 1))) return hipSuccess;
            if (t.stages == 4 && t.tableau == 1)
                hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 4, 1, false, true>), dim3(grid), dim3(TB), 0, s, t, p);
            else if (t.stages == 6 && t.tableau == 2)
                hipLaunchKernelGGL((k_local<real, EQ, DIM, N, FLUX, 6, 2, false, true>), dim3(grid), dim3(TB), 0, s, t, p);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        }
    }
    const bool blend = p.alpha != nullptr || p.alpha_raw != nullptr;
    const int which = p.instances ? p.instances : 3;
    if ((which & 1) && (!blend || p.tiles_in != nullptr)) {
        CRK_LOCAL_LAUNCH(false, WP)
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if constexpr (EQ == EQ_EULER) {
        if ((which & 2) && blend) {
            CRK_LOCAL_LAUNCH(true, WB)
        }
    }
#undef CRK_LOCAL_LAUNCH
    return hipGetLastError();
}

inline hipError_t launch_zero_int(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_interface(const Tables &t, const StepPtrs &p, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    constexpr int EPB = TB / NP;
    const int grid = (t.nelem + EPB - 1) / EPB;
    if (EQ == EQ_MHD && p.stage_tr != nullptr)
        hipLaunchKernelGGL((k_interface<real, EQ, DIM, N, FLUX, true>), dim3(grid), dim3(TB), 0, s, t, p);
    else
        hipLaunchKernelGGL((k_interface<real, EQ, DIM, N, FLUX>), dim3(grid), dim3(TB), 0, s, t, p);
    if (p.dt_out != nullptr)
        hipLaunchKernelGGL(k_dt_slots, dim3(1), dim3(64), 0, s, t, p.partials, EQ == EQ_MHD ? 1 : 0, p.dt_out);
    return hipGetLastError();
}

template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_run(const Tables &t, const StepPtrs &p, double *dt, int nsteps, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    if ((long)t.nelem * NP > RUN_BLOCK) return hipErrorInvalidValue;
    // the instance the separate local-phase launches use (no tile flags here)
    const bool blend = p.alpha_raw != nullptr;
#define CRK_RUN(SS, TT)                                                                                              \
    do {                                                                                                             \
        if (blend) hipLaunchKernelGGL((k_run<real, EQ, DIM, N, FLUX, SS, TT, true>), dim3(1), dim3(RUN_BLOCK), 0, s, t, p, dt, nsteps); \
        else hipLaunchKernelGGL((k_run<real, EQ, DIM, N, FLUX, SS, TT, false>), dim3(1), dim3(RUN_BLOCK), 0, s, t, p, dt, nsteps); \
    } while (0)
    switch (t.stages) {
    case 1: CRK_RUN(1, 0); break;
    case 2: CRK_RUN(2, 0); break;
    case 3: CRK_RUN(3, 0); break;
    case 4: if (t.tableau == 1) CRK_RUN(4, 1); else CRK_RUN(4, 0); break;
    case 5: CRK_RUN(5, 0); break;
    case 6: if (t.tableau == 2) CRK_RUN(6, 2); else CRK_RUN(6, 0); break;
    default: return hipErrorInvalidValue;
    }
#undef CRK_RUN
    return hipGetLastError();
}

template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_face_speed(const Tables &t, const StepPtrs &p, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int EPB = BLOCK / NP;
    const int grid = (t.nelem + EPB - 1) / EPB;
    hipLaunchKernelGGL((k_face_speed<real, EQ, DIM, N, FLUX>), dim3(grid), dim3(BLOCK), 0, s, t, p.u_in, p.traces);
    return hipGetLastError();
}

template <typename real, int DIM, int N>
hipError_t launch_indicator(const Tables &t, const void *u, double *araw, double *alpha, float *features, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int EPB = BLOCK / NP;
    const int grid = (t.nelem + EPB - 1) / EPB;
    hipLaunchKernelGGL((k_indicator<real, DIM, N>), dim3(grid), dim3(BLOCK), 0, s, t, u, araw, features);
    if (alpha)
        hipLaunchKernelGGL(k_smooth, dim3((t.nelem + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, t, (const double *)araw, alpha);
    return hipGetLastError();
}

inline hipError_t launch_zero(double *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

inline int reduction_blocks(const Tables &t)
{
    const long total = (long)t.nelem * t.nnode;
    long g = (total + BLOCK - 1) / BLOCK;
    return (int)(g < RED_BLOCKS ? g : RED_BLOCKS);
}

template <typename real, int EQ, int DIM>
hipError_t launch_dt(const Tables &t, const void *u, double *partials, double *dt, hipStream_t s)
{
    const int g = reduction_blocks(t);
    hipLaunchKernelGGL((k_dt_partial<real, EQ, DIM>), dim3(g), dim3(BLOCK), 0, s, t, u, partials);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(FINAL_BLOCK), 0, s, t, (const double *)partials, g, EQ == EQ_MHD ? 1 : 0, dt);
    return hipGetLastError();
}

template <typename real, int EQ, int DIM>
hipError_t launch_diag(const Tables &t, const void *u, double *partials, double *out, hipStream_t s)
{
    const int g = reduction_blocks(t);
    hipLaunchKernelGGL((k_diag_partial<real, EQ, DIM>), dim3(g), dim3(BLOCK), 0, s, t, u, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, t.M, (const double *)partials, g, out);
    return hipGetLastError();
}

} // namespace crk
