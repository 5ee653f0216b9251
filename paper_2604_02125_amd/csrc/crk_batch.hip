// crk_batch.hip -- many independent periodic 2D Euler meshes of uneven size
// and degree (N = 3 with classical RK4, N = 4 with Butcher's RK5) advanced
// together.  A host-built work list of (problem, element tile) items, the
// degree-3 tiles first, is covered per phase by one launch per degree (one
// workgroup per tile, or persistent workgroups walking the tiles); the CFL
// time step is reduced per problem.  Two pipelined steps (u0 -> u1 -> u0)
// can be captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/crk.h"
#include "crk_kernels.hpp"

using namespace crk;

namespace crk {
const char *set_error(crk_status st, const char *msg);   // crk_api.cpp
crk_status fill_tables(const crk_mesh_desc *m, const crk_scheme_desc *sc, Tables *t);
}

namespace {

struct BatchProblem {
    Tables t;
    StepPtrs p[2];   // p[0]: u0 -> u1, p[1]: u1 -> u0
    int tile0, ntiles;
};

struct BatchTile {
    int prob;
    int e0;
};

// Local phase over the tiles [t0, t1) of one degree (the work list holds the
// degree-3 tiles first): one kernel per degree, so that each is compiled and
// scheduled with its own register budget (the six-stage degree-4 path needs
// far more registers than the four-stage degree-3 one).  PERSIST: a fixed
// grid of workgroups walks the tiles; else one workgroup per tile.  In the
// persistent loop the lane index passes through an empty asm statement so
// that the compiler recomputes the lane's per-node constants in every
// iteration instead of keeping them live across the whole loop.
// NDEG = 0: one launch over the whole work list, each tile taking the
// degree-3 or degree-4 path by its problem's degree (the kernel then has the
// degree-4 path's register budget for every tile).
template <typename real, int FLUX, int NDEG>
struct BatchLocalLds {
    static constexpr int s3 = LocalShape<real, EQ_EULER, 2, 3, FLUX, false>::slots;
    static constexpr int s4 = LocalShape<real, EQ_EULER, 2, 4, FLUX, false>::slots;
    static constexpr int slots = NDEG == 3 ? s3 : (NDEG == 4 ? s4 : (s3 > s4 ? s3 : s4));
};

// (three wavefronts per SIMD: the FP64 degree-4 path then holds 168
// registers, spilling a few, which beats two wavefronts)
template <typename real, int FLUX, int BLK, int NDEG, bool PERSIST>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(3))) k_batch_local(const BatchProblem *probs, const BatchTile *tiles, int t0, int t1,
                                                     int dir)
{
    __shared__ real smem[BatchLocalLds<real, FLUX, NDEG>::slots * BLK];
    auto tile = [&](int it, int lane) {
        const BatchTile tl = tiles[it];
        const BatchProblem &bp = probs[tl.prob];
        // batches have no limiter: the instance without the blending code
        if (NDEG == 3 || (NDEG == 0 && bp.t.N == 3))
            local_tile<real, EQ_EULER, 2, 3, FLUX, 4, BLK, 1, false>(bp.t, bp.p[dir], tl.e0, smem, lane);
        else
            local_tile<real, EQ_EULER, 2, 4, FLUX, 6, BLK, 2, false>(bp.t, bp.p[dir], tl.e0, smem, lane);
    };
    if constexpr (PERSIST) {
        for (int it = t0 + blockIdx.x; it < t1; it += gridDim.x) {
            int lane = threadIdx.x;
            asm volatile("" : "+v"(lane));
            tile(it, lane);
            __syncthreads();
        }
    } else {
        tile(t0 + (int)xcd_tile(blockIdx.x, gridDim.x), threadIdx.x);   // the grid is exactly the tile count
    }
}

// Interface phase over the tiles [t0, t1) of one degree, split and
// scheduled as the local phase.  The tile maxima go to partials[tile].
template <typename real, int FLUX, int BLK, int NDEG, bool PERSIST>
__global__ void __launch_bounds__(BLK) k_batch_interface(const BatchProblem *probs, const BatchTile *tiles, int t0,
                                                         int t1, int dir)
{
    __shared__ double dsmem[5 * BLK];
    auto tile = [&](int it) {
        const BatchTile tl = tiles[it];
        const BatchProblem &bp = probs[tl.prob];
        if (NDEG == 3 || (NDEG == 0 && bp.t.N == 3))
            interface_tile<real, EQ_EULER, 2, 3, FLUX, BLK>(bp.t, bp.p[dir], tl.e0, it, dsmem);
        else
            interface_tile<real, EQ_EULER, 2, 4, FLUX, BLK>(bp.t, bp.p[dir], tl.e0, it, dsmem);
    };
    if constexpr (PERSIST) {
        for (int it = t0 + blockIdx.x; it < t1; it += gridDim.x) {
            tile(it);
            __syncthreads();
        }
    } else {
        tile(t0 + (int)xcd_tile(blockIdx.x, gridDim.x));
    }
}

// wave-speed maximum of every tile of state `dir` (0: u0, 1: u1) -> partials[tile]
template <typename real, int BLK>
__device__ __forceinline__ double tile_speed(const Tables &t, const void *u_, long e0, int np)
{
    const int tid = threadIdx.x;
    const int le = tid / np, node = tid - le * np;
    const long e = e0 + le;
    if (le >= BLK / np || e >= t.nelem) return 0.0;
    const real *u = (const real *)u_;
    const long E = t.nelem;
    const double rho = u[((long)0 * E + e) * np + node];
    const double m1 = u[((long)1 * E + e) * np + node];
    const double m2 = u[((long)2 * E + e) * np + node];
    const double En = u[((long)3 * E + e) * np + node];
    const double v1 = m1 / rho, v2 = m2 / rho;
    const double p = (t.gamma - 1.0) * (En - 0.5 * (m1 * v1 + m2 * v2));
    const double c = sqrt(t.gamma * p / rho);
    return (fabs(v1) + c) * t.invdx[0] + (fabs(v2) + c) * t.invdx[1];
}

// wave-speed maximum of every tile of state `dir` -> partials[tile], and the
// face wave speeds of that state into the face data
template <typename real, int FLUX, int BLK>
__global__ void __launch_bounds__(BLK) k_batch_speed(const BatchProblem *probs, const BatchTile *tiles, int ntiles, int dir,
                                                     double *partials)
{
    __shared__ double red[BLK];
    for (int it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const BatchTile tl = tiles[it];
        const BatchProblem &bp = probs[tl.prob];
        const int np = (bp.t.N + 1) * (bp.t.N + 1);
        const void *u = dir == 0 ? bp.p[0].u_in : bp.p[1].u_in;
        const double v = tile_speed<real, BLK>(bp.t, u, tl.e0, np);
        if (bp.t.N == 3) face_speed_tile<real, EQ_EULER, 2, 3, FLUX, BLK>(bp.t, u, bp.p[0].traces, tl.e0);
        else face_speed_tile<real, EQ_EULER, 2, 4, FLUX, BLK>(bp.t, u, bp.p[0].traces, tl.e0);
        block_max_lanes<BLK>(v, red, partials + it);
        __syncthreads();
    }
}

// one workgroup per problem: dt = cfl / ((N+1) max over its tiles)
__global__ void __launch_bounds__(256) k_batch_dt(const BatchProblem *probs, const double *partials, double *dt)
{
    __shared__ double red[256];
    const BatchProblem &bp = probs[blockIdx.x];
    double m = 0.0;
    for (int k0 = 0; k0 < bp.ntiles; k0 += 4 * 256) {
        double v[4];              // independent loads in flight together
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + j * 256 + threadIdx.x;
            v[j] = k < bp.ntiles ? partials[bp.tile0 + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) m = fmax(m, v[j]);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dt[2 * blockIdx.x] = bp.t.cfl / ((bp.t.N + 1) * red[0]);
        dt[2 * blockIdx.x + 1] = 0.0;
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

} // namespace

struct crk_batch {
    int nprob, prec, flux, block, grid, merged;
    std::vector<crk_mesh_desc> mesh;
    std::vector<BatchProblem> probs;     // host copy of the descriptors
    std::vector<BatchTile> tiles;        // degree-3 problems' tiles first, then degree 4
    int ntiles3;                         // number of degree-3 tiles
    std::vector<long> state_off;         // values
    size_t state_bytes;
    std::vector<size_t> trace_off;       // bytes inside the workspace trace area
    size_t off_probs, off_tiles, off_parts, off_traces, ws_bytes;
    char *ws;
    double *dt;
    bool bound, prepared;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

template <typename real, int FLUX, int BLK>
hipError_t launch_phase(const crk_batch *b, int kind, int dir, hipStream_t s)
{
    const BatchProblem *pr = (const BatchProblem *)(b->ws + b->off_probs);
    const BatchTile *tl = (const BatchTile *)(b->ws + b->off_tiles);
    double *parts = (double *)(b->ws + b->off_parts);
    const int nt = (int)b->tiles.size();
    const int g = b->grid > 0 && b->grid < nt ? b->grid : nt;
    const int n3 = b->ntiles3, n4 = nt - n3;
    const bool pers = b->grid > 0;
    auto grid_of = [&](int n) { return dim3(pers && b->grid < n ? b->grid : n); };
    // one launch per degree and phase: the degree-3 tiles [0, n3), then the
    // degree-4 ones [n3, nt); merged: one launch over [0, nt)
#define CRK_BATCH_PHASE(K)                                                                                  \
    do {                                                                                                    \
        if (b->merged) {                                                                                    \
            if (pers) hipLaunchKernelGGL((K<real, FLUX, BLK, 0, true>), grid_of(nt), dim3(BLK), 0, s, pr, tl, 0, nt, dir); \
            else hipLaunchKernelGGL((K<real, FLUX, BLK, 0, false>), dim3(nt), dim3(BLK), 0, s, pr, tl, 0, nt, dir);        \
        } else if (pers) {                                                                                  \
            if (n3 > 0) hipLaunchKernelGGL((K<real, FLUX, BLK, 3, true>), grid_of(n3), dim3(BLK), 0, s, pr, tl, 0, n3, dir);  \
            if (n4 > 0) hipLaunchKernelGGL((K<real, FLUX, BLK, 4, true>), grid_of(n4), dim3(BLK), 0, s, pr, tl, n3, nt, dir); \
        } else {                                                                                            \
            if (n3 > 0) hipLaunchKernelGGL((K<real, FLUX, BLK, 3, false>), dim3(n3), dim3(BLK), 0, s, pr, tl, 0, n3, dir);    \
            if (n4 > 0) hipLaunchKernelGGL((K<real, FLUX, BLK, 4, false>), dim3(n4), dim3(BLK), 0, s, pr, tl, n3, nt, dir);   \
        }                                                                                                   \
    } while (0)
    if (kind == 0) CRK_BATCH_PHASE(k_batch_local);
    else if (kind == 1) CRK_BATCH_PHASE(k_batch_interface);
    else hipLaunchKernelGGL((k_batch_speed<real, FLUX, BLK>), dim3(g), dim3(BLK), 0, s, pr, tl, nt, dir, parts);
#undef CRK_BATCH_PHASE
    if (kind != 0) hipLaunchKernelGGL(k_batch_dt, dim3(b->nprob), dim3(256), 0, s, pr, (const double *)parts, b->dt);
    return hipGetLastError();
}

template <typename real, int FLUX>
hipError_t launch_phase_blk(const crk_batch *b, int kind, int dir, hipStream_t s)
{
    switch (b->block) {
    case 64: return launch_phase<real, FLUX, 64>(b, kind, dir, s);
    case 128: return launch_phase<real, FLUX, 128>(b, kind, dir, s);
    default: return launch_phase<real, FLUX, 256>(b, kind, dir, s);
    }
}

hipError_t run_phase(const crk_batch *b, int kind, int dir, hipStream_t s)
{
    if (b->prec == CRK_FP64)
        return b->flux == CRK_VOL_KG ? launch_phase_blk<double, VOL_KG>(b, kind, dir, s)
                                     : launch_phase_blk<double, VOL_RANOCHA>(b, kind, dir, s);
    return b->flux == CRK_VOL_KG ? launch_phase_blk<float, VOL_KG>(b, kind, dir, s)
                                 : launch_phase_blk<float, VOL_RANOCHA>(b, kind, dir, s);
}

crk_status hip_err(hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    set_error(CRK_ERR_HIP, m.c_str());
    return CRK_ERR_HIP;
}

} // namespace

extern "C" {

crk_status crk_batch_create(const crk_mesh_desc *meshes, int nprob, const crk_scheme_desc *scheme,
                            const crk_batch_tuning *tuning, crk_batch **out)
{
    if (!meshes || !scheme || !out || nprob < 1) {
        set_error(CRK_ERR_ARG, "null argument or empty batch");
        return CRK_ERR_ARG;
    }
    *out = nullptr;
    if (scheme->volume_flux != CRK_VOL_KG && scheme->volume_flux != CRK_VOL_RANOCHA) {
        set_error(CRK_ERR_UNSUPPORTED, "batches support the Kennedy-Gruber and Ranocha fluxes");
        return CRK_ERR_UNSUPPORTED;
    }
    if (scheme->limiter != CRK_LIM_NONE || scheme->A || scheme->b) {
        set_error(CRK_ERR_UNSUPPORTED, "batches use the default tableaus and no limiter");
        return CRK_ERR_UNSUPPORTED;
    }
    const int block = tuning && tuning->block ? tuning->block : 256;
    if (block != 64 && block != 128 && block != 256) {
        set_error(CRK_ERR_ARG, "tuning.block must be 64, 128 or 256");
        return CRK_ERR_ARG;
    }
    crk_batch *b = new (std::nothrow) crk_batch();
    if (!b) {
        set_error(CRK_ERR_ARG, "out of host memory");
        return CRK_ERR_ARG;
    }
    b->nprob = nprob;
    b->prec = meshes[0].precision;
    b->flux = scheme->volume_flux;
    b->block = block;
    b->mesh.assign(meshes, meshes + nprob);
    b->probs.resize(nprob);
    b->state_off.resize(nprob + 1);
    b->trace_off.resize(nprob + 1);
    long off = 0;
    size_t toff = 0;
    const size_t elem = b->prec == CRK_FP64 ? 8 : 4;
    for (int i = 0; i < nprob; ++i) {
        const crk_mesh_desc &m = meshes[i];
        if (m.dim != 2 || m.equation != CRK_EULER || (m.degree != 3 && m.degree != 4) || m.precision != b->prec ||
            m.boundary[0] != CRK_BC_PERIODIC || m.boundary[1] != CRK_BC_PERIODIC) {
            set_error(CRK_ERR_UNSUPPORTED,
                      "batch problems must be periodic 2D Euler of degree 3 or 4 and one precision");
            delete b;
            return CRK_ERR_UNSUPPORTED;
        }
        crk_status st = fill_tables(&m, scheme, &b->probs[i].t);
        if (st) {
            delete b;
            return st;
        }
        const Tables &t = b->probs[i].t;
        b->state_off[i] = off;
        off += (long)t.M * t.nelem * t.nnode;
        b->trace_off[i] = toff;
        // four faces; per face node M flux-share values and the wave speed
        toff = align256(toff + (size_t)2 * 2 * (t.M + 1) * t.nelem * t.nface * elem);
    }
    // work list: the tiles of the degree-3 problems, then those of degree 4;
    // the tiles of one problem stay contiguous
    for (int deg = 3; deg <= 4; ++deg) {
        if (deg == 4) b->ntiles3 = (int)b->tiles.size();
        for (int i = 0; i < nprob; ++i) {
            const Tables &t = b->probs[i].t;
            if (t.N != deg) continue;
            const int epb = block / t.nnode;
            b->probs[i].tile0 = (int)b->tiles.size();
            for (int e0 = 0; e0 < t.nelem; e0 += epb) b->tiles.push_back(BatchTile{i, e0});
            b->probs[i].ntiles = (int)b->tiles.size() - b->probs[i].tile0;
        }
    }
    b->state_off[nprob] = off;
    b->trace_off[nprob] = toff;
    b->state_bytes = (size_t)off * elem;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const int gpc = tuning ? tuning->grid_per_cu : 4;
    b->merged = tuning ? (tuning->merged ? 1 : 0) : 0;
    b->grid = gpc > 0 ? gpc * cus : 0;   // 0: one workgroup per tile
    size_t w = 0;
    b->off_probs = w; w = align256(w + sizeof(BatchProblem) * nprob);
    b->off_tiles = w; w = align256(w + sizeof(BatchTile) * b->tiles.size());
    b->off_parts = w; w = align256(w + sizeof(double) * b->tiles.size());
    b->off_traces = w; w = align256(w + toff);
    b->ws_bytes = w;
    b->ws = nullptr;
    b->dt = nullptr;
    b->bound = b->prepared = false;
    b->graph = nullptr;
    b->exec = nullptr;
    *out = b;
    return CRK_OK;
}

crk_status crk_batch_destroy(crk_batch *b)
{
    if (!b) return CRK_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return CRK_OK;
}

crk_status crk_batch_layout(const crk_batch *b, int64_t *offsets, int *degrees, size_t *state_bytes,
                            size_t *workspace_bytes, int64_t *ntiles)
{
    if (!b) {
        set_error(CRK_ERR_ARG, "null batch");
        return CRK_ERR_ARG;
    }
    for (int i = 0; offsets && i <= b->nprob; ++i) offsets[i] = b->state_off[i];
    for (int i = 0; degrees && i < b->nprob; ++i) degrees[i] = b->mesh[i].degree;
    if (state_bytes) *state_bytes = b->state_bytes;
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    if (ntiles) *ntiles = (int64_t)b->tiles.size();
    return CRK_OK;
}

crk_status crk_batch_bind(crk_batch *b, void *u0, void *u1, double *dt_dev, void *workspace, size_t ws_bytes,
                          crk_stream stream)
{
    if (!b || !u0 || !u1 || !dt_dev || !workspace) {
        set_error(CRK_ERR_ARG, "null argument");
        return CRK_ERR_ARG;
    }
    if (u0 == u1 || (((uintptr_t)u0 | (uintptr_t)u1 | (uintptr_t)workspace) & 255u)) {
        set_error(CRK_ERR_ARG, "u0/u1 must be distinct and 256-byte aligned, as the workspace");
        return CRK_ERR_ARG;
    }
    if (ws_bytes < b->ws_bytes) {
        set_error(CRK_ERR_ARG, "workspace too small");
        return CRK_ERR_ARG;
    }
    const size_t elem = b->prec == CRK_FP64 ? 8 : 4;
    b->ws = (char *)workspace;
    b->dt = dt_dev;
    for (int i = 0; i < b->nprob; ++i) {
        BatchProblem &bp = b->probs[i];
        char *a = (char *)u0 + b->state_off[i] * elem, *c = (char *)u1 + b->state_off[i] * elem;
        void *tr = b->ws + b->off_traces + b->trace_off[i];
        for (int dir = 0; dir < 2; ++dir) {
            StepPtrs &p = bp.p[dir];
            std::memset(&p, 0, sizeof p);
            p.u_in = dir == 0 ? a : c;
            p.u_out = dir == 0 ? c : a;
            p.dt = dt_dev + 2 * i;
            p.traces = tr;
            p.partials = (double *)(b->ws + b->off_parts);
            p.dt_out = dt_dev + 2 * i;   // non-null: the interface phase emits the tile maxima
        }
    }
    hipError_t e = hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(), sizeof(BatchProblem) * b->nprob,
                                  hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->off_tiles, b->tiles.data(), sizeof(BatchTile) * b->tiles.size(),
                           hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "crk_batch_bind");
    b->bound = true;
    b->prepared = false;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    return CRK_OK;
}

crk_status crk_batch_prepare(crk_batch *b, int src, crk_stream stream)
{
    if (!b || !b->bound || (src != 0 && src != 1)) {
        set_error(CRK_ERR_STATE, "batch not bound or bad source index");
        return CRK_ERR_STATE;
    }
    hipError_t e = run_phase(b, 2, src, (hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "crk_batch_prepare");
    b->prepared = true;
    return CRK_OK;
}

crk_status crk_batch_advance(crk_batch *b, int src, int phases, crk_stream stream)
{
    if (!b || !b->bound || !b->prepared || (src != 0 && src != 1)) {
        set_error(CRK_ERR_STATE, "batch not bound/prepared or bad source index");
        return CRK_ERR_STATE;
    }
    if (phases & ~(CRK_PHASE_LOCAL | CRK_PHASE_INTERFACE)) {
        set_error(CRK_ERR_ARG, "unknown phase bits");
        return CRK_ERR_ARG;
    }
    hipError_t e = hipSuccess;
    if (phases & CRK_PHASE_LOCAL) e = run_phase(b, 0, src, (hipStream_t)stream);
    if (e == hipSuccess && (phases & CRK_PHASE_INTERFACE)) e = run_phase(b, 1, src, (hipStream_t)stream);
    return e == hipSuccess ? CRK_OK : hip_err(e, "crk_batch_advance");
}

crk_status crk_batch_graph_capture(crk_batch *b, crk_stream stream)
{
    if (!b || !b->bound || !b->prepared) {
        set_error(CRK_ERR_STATE, "batch not bound/prepared");
        return CRK_ERR_STATE;
    }
    if (!stream) {
        set_error(CRK_ERR_ARG, "graph capture needs a non-default stream");
        return CRK_ERR_ARG;
    }
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "hipStreamBeginCapture");
    hipError_t el = hipSuccess;
    for (int dir = 0; dir < 2 && el == hipSuccess; ++dir) {
        el = run_phase(b, 0, dir, s);
        if (el == hipSuccess) el = run_phase(b, 1, dir, s);
    }
    e = hipStreamEndCapture(s, &b->graph);
    if (el != hipSuccess) return hip_err(el, "graph capture (launch)");
    if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_err(e, "hipGraphInstantiate");
    return CRK_OK;
}

crk_status crk_batch_graph_launch(crk_batch *b, crk_stream stream)
{
    if (!b || !b->exec) {
        set_error(CRK_ERR_STATE, "no captured graph");
        return CRK_ERR_STATE;
    }
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? CRK_OK : hip_err(e, "hipGraphLaunch");
}

} // extern "C"
