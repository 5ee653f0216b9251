// crk_rhs.hpp -- the semi-discrete FR operator du/dt = L(u), a test operator
// beside the time step: the flux-differencing volume term of Section 3 and
// the FR surface correction of eq:general.non.conservative.fr.one with the
// numerical flux of eq:combined.num.flux.fr.  The surface flux is Rusanov,
// or the volume flux itself evaluated on the two traces; with an
// entropy-conservative volume flux the latter makes the semi-discrete
// entropy rate vanish on a periodic mesh, which is what the operator is for.
#pragma once
#include "crk_kernels.hpp"

namespace crk {

enum { SURF_RUSANOV = 0, SURF_EC = 1 };

// LDS of the per-node residual: the node fields, and the symmetric fluxes
// of the rotations whose mirror a line neighbour takes (as in the local
// stages).
template <typename real, int EQ, int DIM, int N, int FLUX>
struct RhsShape {
    using L = LocalShape<real, EQ, DIM, N, FLUX>;
    static constexpr int slots = L::Phys::NF + L::NX;
};

// Semi-discrete FR residual of one node (one lane): R = volume term of
// Section 3 + the g2 surface corrections of eq:general.non.conservative.fr.one,
// so that du/dt = -R.  The correction functions are Huynh's g2 on GLL
// points, whose derivatives are 1/w_N at xi = 1 and -1/w_0 at xi = 0 and
// zero at the other nodes, so only the end nodes of a line are corrected.
// Pairs along a line are visited by rotation as in the local stages: lane p
// evaluates q = p + k (mod N+1) for k < (N+1)/2 and the self-mirrored k, and
// takes the mirrored symmetric fluxes from its line neighbours through LDS.
// Every lane of the workgroup must call it; spare lanes (le set to 0 by the
// caller) compute on element 0 and discard the result.
template <typename real, int EQ, int DIM, int N, int FLUX, int BLK>
__device__ __forceinline__ void rhs_lane(const Tables &t, const real *u, const Ctx<real> &ctx, int surface, int tid,
                                         int le, int node, long es, real *smem, real *R)
{
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    using Shape = LocalShape<real, EQ, DIM, N, FLUX>;
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int M = Phys::M;
    constexpr int NF = Phys::NF;
    constexpr bool SYM = Shape::SYM;
    constexpr int NPRIM = Shape::NPRIM, KSELF = Shape::KSELF;
    real *lds = smem;
    real *xch = smem + NF * BLK;
    const int base = le * NP;
    const int pd[2] = {node % n1, DIM == 2 ? node / n1 : 0};
    const long E = t.nelem;

    real uo[M], nd[NF];
#pragma unroll
    for (int v = 0; v < M; ++v) uo[v] = u[((long)v * E + es) * NP + node];
    Phys::node(uo, nd, ctx);
#pragma unroll
    for (int f = 0; f < NF; ++f) lds[f * BLK + tid] = nd[f];
    element_sync<NP, BLK>();

#pragma unroll
    for (int v = 0; v < M; ++v) R[v] = real(0);
    // volume term: sum_d 1/dx_d sum_q [2 D_pq f_S,d(u_p, u_q) + D_pq B_d(u_p) g_d(u_q)]
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int r = pd[d];
        const bool end = r == 0 || r == N;
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            const bool direct = !SYM || k <= NPRIM || k == KSELF;
            if (!direct) continue;
            const int qd = r + k < n1 ? r + k : r + k - n1;
            const int q = line_node<N, DIM>(pd, d, qd);
            real ndq[NF], fs[M];
#pragma unroll
            for (int f = 0; f < NF; ++f) ndq[f] = lds[f * BLK + base + q];
            Phys::pair(d, nd, ndq, fs, ctx);
            const real c = Tab<real>::dk(t, d, r, k);
#pragma unroll
            for (int v = 0; v < M; ++v) R[v] += c * fs[v];
            if constexpr (SYM) {
                if (k <= NPRIM) {
#pragma unroll
                    for (int v = 0; v < M; ++v) xch[((d * NPRIM + (k - 1)) * M + v) * BLK + tid] = fs[v];
                }
            }
        }
        // diagonal 2 D_pp f_d(u_p): non-zero only at the two ends of a line
        if (end) {
            real fp[M];
            if constexpr (EQ == EQ_EULER) Phys::phys_cons(d, uo, nd, fp, ctx);
            else Phys::phys(d, nd, fp, ctx);
            const real c = Tab<real>::dk(t, d, r, 0);
#pragma unroll
            for (int v = 0; v < M; ++v) R[v] += c * fp[v];
        }
        if constexpr (EQ == EQ_MHD) {
            real gB = real(0), gpsi = real(0);
#pragma unroll
            for (int q = 0; q < n1; ++q) {
                const int qn = line_node<N, DIM>(pd, d, q);
                const real c = Tab<real>::dn(t, d, r, q);
                gB += c * lds[(5 + d) * BLK + base + qn];
                gpsi += c * lds[8 * BLK + base + qn];
            }
            real o[M];
            MhdP<real, FLUX>::btimes(d, nd, gB, gpsi, o);
#pragma unroll
            for (int v = 0; v < M; ++v) R[v] += o[v];
        }
    }
    if constexpr (SYM) {
        element_sync<NP, BLK>();
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int k = 1; k <= NPRIM; ++k) {
                // mirror rotation n1 - k: the pair (p, p - k) was evaluated by lane p - k
                int sd = pd[d] - k;
                if (sd < 0) sd += n1;
                const int src = base + line_node<N, DIM>(pd, d, sd);
                const real c = Tab<real>::dk(t, d, pd[d], n1 - k);
#pragma unroll
                for (int v = 0; v < M; ++v) R[v] += c * xch[((d * NPRIM + (k - 1)) * M + v) * BLK + src];
            }
    }

    // surface correction at the end nodes of each line:
    // s/(w dx_d) (F_num + F_num^nc - f(u_p) - B_d(u_p) g_d(u_p)), s = +1 at
    // xi_d = 1 and -1 at xi_d = 0
    const Nbrs nb = neighbours<DIM>(t, es);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (!(pd[d] == 0 || pd[d] == N)) continue;
        const int side = pd[d] == N ? 1 : 0;
        const long en = nb.n[d][side];
        int pn[2] = {pd[0], pd[1]};
        pn[d] = N - pd[d];
        const int nn = DIM == 2 ? pn[1] * n1 + pn[0] : pn[0];
        real un[M], ndn[NF];
        if ((nb.wall >> (2 * d + side)) & 1) {
            // beyond a wall: the mirror image of this node (normal momentum negated)
#pragma unroll
            for (int v = 0; v < M; ++v) un[v] = v == 1 + d ? -uo[v] : uo[v];
        } else {
#pragma unroll
            for (int v = 0; v < M; ++v) un[v] = u[((long)v * E + en) * NP + nn];
        }
        Phys::node(un, ndn, ctx);
        // left and right traces (selects, no indexing of register arrays by side)
        real aL[NF], aR[NF], uL[M], uR[M];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            aL[f] = side ? nd[f] : ndn[f];
            aR[f] = side ? ndn[f] : nd[f];
        }
#pragma unroll
        for (int v = 0; v < M; ++v) {
            uL[v] = side ? uo[v] : un[v];
            uR[v] = side ? un[v] : uo[v];
        }
        real fnum[M];
        if (surface == SURF_EC) {
            Phys::pair(d, aL, aR, fnum, ctx);
        } else {
            real fL[M], fR[M];
            Phys::phys(d, aL, fL, ctx);
            Phys::phys(d, aR, fR, ctx);
            const real lam = dmax(Phys::speed(d, aL, ctx), Phys::speed(d, aR, ctx));
#pragma unroll
            for (int v = 0; v < M; ++v)
                fnum[v] = real(0.5) * (fL[v] + fR[v]) - real(0.5) * lam * (uR[v] - uL[v]);
        }
        real fo[M];
        Phys::phys(d, nd, fo, ctx);
        real jump[M];
#pragma unroll
        for (int v = 0; v < M; ++v) jump[v] = fnum[v] - fo[v];
        if constexpr (EQ == EQ_MHD) {
            real ncn[M], nco[M];
            MhdP<real, FLUX>::btimes(d, nd, real(0.5) * (aL[5 + d] + aR[5 + d]), real(0.5) * (aL[8] + aR[8]), ncn);
            MhdP<real, FLUX>::btimes(d, nd, nd[5 + d], nd[8], nco);
#pragma unroll
            for (int v = 0; v < M; ++v) jump[v] += ncn[v] - nco[v];
        }
        const real g = side ? Tab<real>::invw(t, d, pd[d]) : -Tab<real>::invw(t, d, pd[d]);
#pragma unroll
        for (int v = 0; v < M; ++v) R[v] += g * jump[v];
    }
}

template <typename real, int EQ, int DIM, int N, int FLUX>
__global__ void __launch_bounds__(tile_block<DIM == 2 ? (N + 1) * (N + 1) : N + 1>())
k_fr_rhs(const Tables t, const void *u_, const double *dtc, int surface, void *rhs_)
{
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int BLK = tile_block<NP>();
    constexpr int EPB = BLK / NP;
    constexpr int M = PhysOf<real, EQ, DIM, FLUX>::type::M;
    __shared__ real smem[RhsShape<real, EQ, DIM, N, FLUX>::slots * BLK];
    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const Ctx<real> ctx = make_ctx<real>(t, dtc);
    real R[M];
    rhs_lane<real, EQ, DIM, N, FLUX, BLK>(t, (const real *)u_, ctx, surface, tid, le, node, es, smem, R);
    if (!valid) return;
    real *rhs = (real *)rhs_;
#pragma unroll
    for (int v = 0; v < M; ++v) rhs[((long)v * t.nelem + e) * NP + node] = -R[v];
}

// ---------------------------------------------------------------- standard multi-stage RKFR
// One stage i of the s-stage RKFR step of eq:rkfr.non.cons: K_i = L(u^(i))
// with the semi-discrete operator above (Rusanov faces: the interface
// exchange of this stage), then u^(i+1) = u^n + dt sum_{m<=i} a_{i+1,m} K_m
// or, after the last stage, u^{n+1} = u^n + dt sum_m b_m K_m.  K_i is kept
// (k[i]) where a later stage or the final sum needs it.  Sums run over m in
// ascending order.
template <typename real, int EQ, int DIM, int N, int FLUX>
__global__ void __launch_bounds__(tile_block<DIM == 2 ? (N + 1) * (N + 1) : N + 1>())
k_rkfr_stage(const Tables t, const RkPtrs a, int i)
{
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int BLK = tile_block<NP>();
    constexpr int EPB = BLK / NP;
    constexpr int M = PhysOf<real, EQ, DIM, FLUX>::type::M;
    __shared__ real smem[RhsShape<real, EQ, DIM, N, FLUX>::slots * BLK];
    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = xcd_tile(blockIdx.x, gridDim.x) * EPB + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const Ctx<real> ctx = make_ctx<real>(t, a.dt);
    real R[M];
    rhs_lane<real, EQ, DIM, N, FLUX, BLK>(t, (const real *)a.x_in, ctx, SURF_RUSANOV, tid, le, node, es, smem, R);
    if (!valid) return;
    const int S = t.stages;
    const real h = real(a.dt[0]);
    const long E = t.nelem, len = (long)M * E * NP;
    const real *un = (const real *)a.u_n;
    real *kb = (real *)a.k;
    real *xo = (real *)a.x_out;
    const bool last = i + 1 == S;
    // is K_i needed by a later stage state or the final sum?
    bool keep = !last && t.b[i] != 0.0;
    for (int j = i + 2; j < S; ++j) keep = keep || t.A[j][i] != 0.0;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        const long idx = ((long)v * E + e) * NP + node;
        const real Ki = -R[v];
        real acc = real(0);
        for (int m = 0; m < i; ++m) {
            const double c = last ? t.b[m] : t.A[i + 1][m];
            if (c != 0.0) acc += real(c) * kb[(long)m * len + idx];
        }
        acc += real(last ? t.b[i] : t.A[i + 1][i]) * Ki;
        xo[idx] = un[idx] + h * acc;
        if (keep) kb[(long)i * len + idx] = Ki;
    }
}

template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_rkfr(const Tables &t, const RkPtrs &p0, void *buf0, void *buf1, void *u_out, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    constexpr int EPB = TB / NP;
    const long grid = (t.nelem + EPB - 1) / EPB;
    RkPtrs p = p0;
    for (int i = 0; i < t.stages; ++i) {
        p.x_in = i == 0 ? p0.u_n : (i % 2 ? buf0 : buf1);
        p.x_out = i + 1 == t.stages ? u_out : (i % 2 ? buf1 : buf0);
        hipLaunchKernelGGL((k_rkfr_stage<real, EQ, DIM, N, FLUX>), dim3((unsigned)grid), dim3(TB), 0, s, t, p, i);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename real, int EQ, int DIM, int N, int FLUX>
hipError_t launch_fr_rhs(const Tables &t, const void *u, const double *dtc, int surface, void *rhs, hipStream_t s)
{
    constexpr int NP = DIM == 2 ? (N + 1) * (N + 1) : N + 1;
    constexpr int TB = tile_block<NP>();
    constexpr int EPB = TB / NP;
    const long grid = (t.nelem + EPB - 1) / EPB;
    hipLaunchKernelGGL((k_fr_rhs<real, EQ, DIM, N, FLUX>), dim3((unsigned)grid), dim3(TB), 0, s, t, u, dtc, surface,
                       rhs);
    return hipGetLastError();
}

} // namespace crk
