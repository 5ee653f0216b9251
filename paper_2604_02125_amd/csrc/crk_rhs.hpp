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

// One lane per node.  The correction functions are Huynh's g2 on GLL
// points, whose derivatives are 1/w_N at xi = 1 and -1/w_0 at xi = 0 and
// zero at the other nodes, so only the end nodes of a line are corrected.
template <typename real, int EQ, int DIM, int N, int FLUX>
__global__ void __launch_bounds__(tile_block<DIM == 2 ? (N + 1) * (N + 1) : N + 1>())
k_fr_rhs(const Tables t, const void *u_, const double *dtc, int surface, void *rhs_)
{
    using Phys = typename PhysOf<real, EQ, DIM, FLUX>::type;
    constexpr int n1 = N + 1;
    constexpr int NP = DIM == 2 ? n1 * n1 : n1;
    constexpr int BLK = tile_block<NP>();
    constexpr int EPB = BLK / NP;
    constexpr int M = Phys::M;
    constexpr int NF = Phys::NF;
    __shared__ real lds[NF * BLK];

    const int tid = threadIdx.x;
    int le = tid / NP;
    const int node = tid - le * NP;
    const long e = (long)blockIdx.x * EPB + le;
    const bool valid = (le < EPB) && (e < t.nelem);
    if (le >= EPB) le = 0;
    const long es = valid ? e : 0;
    const int base = le * NP;
    const int pd[2] = {node % n1, DIM == 2 ? node / n1 : 0};
    const long E = t.nelem;
    const real *u = (const real *)u_;
    const Ctx<real> ctx = make_ctx<real>(t, dtc);

    real uo[M], nd[NF];
#pragma unroll
    for (int v = 0; v < M; ++v) uo[v] = u[((long)v * E + es) * NP + node];
    Phys::node(uo, nd, ctx);
#pragma unroll
    for (int f = 0; f < NF; ++f) lds[f * BLK + tid] = nd[f];
    element_sync<NP>();

    // volume term: sum_d 1/dx_d sum_q [2 D_pq f_S,d(u_p, u_q) + D_pq B_d(u_p) g_d(u_q)]
    real R[M];
#pragma unroll
    for (int v = 0; v < M; ++v) R[v] = real(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        real gB = real(0), gpsi = real(0);
#pragma unroll
        for (int q = 0; q < n1; ++q) {
            const int qn = line_node<N, DIM>(pd, d, q);
            real ndq[NF], fs[M];
#pragma unroll
            for (int f = 0; f < NF; ++f) ndq[f] = lds[f * BLK + base + qn];
            Phys::pair(d, nd, ndq, fs, ctx);
            const real c = real(t.D[pd[d]][q] * t.invdx[d]);
#pragma unroll
            for (int v = 0; v < M; ++v) R[v] += real(2) * c * fs[v];
            if constexpr (EQ == EQ_MHD) {
                gB += c * ndq[5 + d];
                gpsi += c * ndq[8];
            }
        }
        if constexpr (EQ == EQ_MHD) {
            real o[M];
            MhdP<real, FLUX>::btimes(d, nd, gB, gpsi, o);
#pragma unroll
            for (int v = 0; v < M; ++v) R[v] += o[v];
        }
    }

    // surface correction at the end nodes of each line:
    // -s/(w dx_d) (F_num + F_num^nc - f(u_p) - B_d(u_p) g_d(u_p)), s = +1 at
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
#pragma unroll
        for (int v = 0; v < M; ++v) un[v] = u[((long)v * E + en) * NP + nn];
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
        const real g = real(side ? t.invw_dx[d][pd[d]] : -t.invw_dx[d][pd[d]]);
#pragma unroll
        for (int v = 0; v < M; ++v) R[v] += g * jump[v];
    }
    if (!valid) return;
    real *rhs = (real *)rhs_;
#pragma unroll
    for (int v = 0; v < M; ++v) rhs[((long)v * E + e) * NP + node] = -R[v];
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
