// crk_physics.hpp -- device-side physics and two-point fluxes of the cRKFR
// library (gfx950).  Each physics policy describes, for one equation system
// and one volume flux:
//   - M: number of conserved variables;
//   - NF: number of per-node fields staged in LDS for the two-point fluxes
//     (primitive variables plus whatever a flux needs per node, such as the
//     logarithms used by the logarithmic means);
//   - node():  fields from the conserved state;
//   - pair():  symmetric two-point flux f_S,d(u_a, u_b)  (eq:entropy.cons.flux.dev);
//   - phys():  physical flux f_d(u);
//   - speed(): largest |eigenvalue| of f'+Bg' in direction d (eq:combined.wave.speed);
//   - cons():  conserved state from the fields (for the subcell fluxes).
// Systems: compressible Euler (eq:flux.and.non.cons with B = 0) and ideal
// GLM-MHD with the Powell / GLM non-conservative products.
#pragma once
#include <hip/hip_runtime.h>

namespace crk {

enum { VOL_CENTRAL = 0, VOL_KG = 1, VOL_RANOCHA = 2, VOL_DERIGS = 3 };
enum { EQ_EULER = 0, EQ_MHD = 1 };

template <typename real>
struct Ctx {
    real gamma, gm1, inv_gm1, ch;
};

template <typename real> __device__ __forceinline__ real dsqrt(real x) { return sqrt(x); }
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
template <typename real> __device__ __forceinline__ real dlog(real x) { return log(x); }
template <> __device__ __forceinline__ float dlog<float>(float x) { return logf(x); }
template <typename real> __device__ __forceinline__ real dabs(real x) { return fabs(x); }
template <> __device__ __forceinline__ float dabs<float>(float x) { return fabsf(x); }
template <typename real> __device__ __forceinline__ real dmax(real a, real b) { return a > b ? a : b; }

// Switch point of the logarithmic mean between its series and log forms, in
// u = ((x - y)/(x + y))^2: the series truncated after u^3 is accurate to the
// working precision below it, and ln y - ln x loses no more than a few ulps
// of relative accuracy above it.
template <typename real> struct LnMeanSwitch;
template <> struct LnMeanSwitch<double> { static constexpr double value = 1e-4; };
template <> struct LnMeanSwitch<float> { static constexpr float value = 1e-2f; };

// Reciprocal by Newton's iteration r <- r (2 - x r) from the hardware
// estimate: one step (est1) leaves about 1 ulp in FP64, two steps converge.
__device__ __forceinline__ double rcp_est1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_est1(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Logarithmic mean (x - y)/(ln x - ln y) from precomputed logarithms.
// With f = (x - y)/(x + y), u = f^2: ln(x/y) = 2 artanh f =
// 2 f (1 + u/3 + u^2/5 + u^3/7 + ...), so near x = y the mean is
// (x + y) / (2 (1 + u/3 + u^2/5 + u^3/7)).  Both branches are evaluated and
// selected so that a wavefront never diverges here.
//
// Numerator and denominator of the logarithmic mean without a division: u
// only selects the branch and feeds the series (where an error e in u moves
// the mean by about e u / 3), so it takes the one-step reciprocal.
template <typename real>
__device__ __forceinline__ void lnmean_parts_fast(real x, real y, real lx, real ly, real &num, real &den)
{
    const real s = x + y, d = x - y;
    const real u = (d * d) * rcp_est1(s * s);
    const bool series = u < LnMeanSwitch<real>::value;
    const real poly = real(2) * (real(1) + u * (real(1) / real(3) + u * (real(1) / real(5) + u * (real(1) / real(7)))));
    num = series ? s : (y - x);
    den = series ? poly : (ly - lx);
}

// The two means an EC flux needs, ln-mean(x1, y1) and 1/ln-mean(x2, y2), with
// one reciprocal: r = 1/(d1 n2), m1 = n1 n2 r = n1/d1, im2 = d2 d1 r = d2/n2.
// Swapping the states flips the sign of n and d in the log branch and of
// nothing in the series branch, so both results are symmetric bit for bit.
template <typename real>
__device__ __forceinline__ void lnmean_pair(real x1, real y1, real lx1, real ly1, real x2, real y2, real lx2,
                                            real ly2, real &m1, real &im2)
{
    real n1, d1, n2, d2;
    lnmean_parts_fast(x1, y1, lx1, ly1, n1, d1);
    lnmean_parts_fast(x2, y2, lx2, ly2, n2, d2);
    const real r = rcp_nr(d1 * n2);
    m1 = (n1 * n2) * r;
    im2 = (d2 * d1) * r;
}

// ---------------------------------------------------------------- Euler
// u = (rho, rho v_1 [, rho v_2], E), p = (gamma - 1)(E - rho |v|^2 / 2).
// Fields: 0 rho, 1..DIM v, DIM+1 p, then per flux
//   KG:      DIM+2 e = E/rho; all KG fields are stored halved, so that the
//            arithmetic means of the flux are plain sums
//   central: DIM+2 E
//   Ranocha: DIM+2 ln rho, DIM+3 beta = rho/p, DIM+4 ln beta
template <typename real, int DIM, int FLUX>
struct EulerP {
    static constexpr int M = DIM + 2;
    static constexpr int NF = (FLUX == VOL_RANOCHA) ? DIM + 5 : DIM + 3;
    static constexpr int P = DIM + 1;
    static constexpr bool HALF = (FLUX == VOL_KG);

    // fields from the conserved state; with logs = false the logarithms of
    // the Ranocha flux are skipped (enough for phys, speed, cons)
    template <bool LOGS = true>
    __device__ __forceinline__ static void fields(const real *u, real *nd, const Ctx<real> &c)
    {
        const real rho = u[0], irho = rcp_nr(rho);
        if constexpr (HALF) {
            // halved fields straight from u: scaling by 1/2 is exact, so these
            // equal the halves of v, p and E/rho bit for bit
            const real h = real(0.5), ih = h * irho;
            real s = real(0);   // = |m|^2 / (2 rho)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                nd[1 + k] = u[1 + k] * ih;
                s += u[1 + k] * nd[1 + k];
            }
            nd[0] = h * rho;
            nd[P] = (h * c.gm1) * (u[DIM + 1] - s);
            nd[DIM + 2] = u[DIM + 1] * ih;
            return;
        }
        real ke = real(0), v[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            v[k] = u[1 + k] * irho;
            ke += u[1 + k] * v[k];
        }
        const real p = c.gm1 * (u[DIM + 1] - real(0.5) * ke);
        nd[0] = rho;
#pragma unroll
        for (int k = 0; k < DIM; ++k) nd[1 + k] = v[k];
        nd[P] = p;
        if constexpr (FLUX == VOL_CENTRAL) {
            nd[DIM + 2] = u[DIM + 1];
        } else if constexpr (LOGS) {
            const real beta = rho * rcp_nr(p);
            nd[DIM + 2] = dlog(rho);
            nd[DIM + 3] = beta;
            nd[DIM + 4] = dlog(beta);
        }
    }
    __device__ __forceinline__ static void node(const real *u, real *nd, const Ctx<real> &c) { fields<true>(u, nd, c); }
    __device__ __forceinline__ static void node_basic(const real *u, real *nd, const Ctx<real> &c) { fields<false>(u, nd, c); }

    // full primitive values from the fields
    __device__ __forceinline__ static void prim(const real *nd, real &rho, real *v, real &p, real &E, const Ctx<real> &c)
    {
        const real s = HALF ? real(2) : real(1);
        rho = s * nd[0];
        real ke = real(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            v[k] = s * nd[1 + k];
            ke += v[k] * v[k];
        }
        p = s * nd[P];
        if constexpr (HALF) E = rho * (s * nd[DIM + 2]);
        else if constexpr (FLUX == VOL_CENTRAL) E = nd[DIM + 2];
        else E = p * c.inv_gm1 + real(0.5) * rho * ke;
    }

    __device__ __forceinline__ static void cons(const real *nd, real *u, const Ctx<real> &c)
    {
        real rho, v[DIM], p, E;
        prim(nd, rho, v, p, E, c);
        u[0] = rho;
#pragma unroll
        for (int k = 0; k < DIM; ++k) u[1 + k] = rho * v[k];
        u[DIM + 1] = E;
    }

    __device__ __forceinline__ static void phys(int d, const real *nd, real *f, const Ctx<real> &c)
    {
        real rho, v[DIM], p, E;
        prim(nd, rho, v, p, E, c);
        const real m = rho * v[d];
        f[0] = m;
#pragma unroll
        for (int k = 0; k < DIM; ++k) f[1 + k] = m * v[k] + (k == d ? p : real(0));
        f[DIM + 1] = (E + p) * v[d];
    }

    // the same flux from the conserved state u and its fields: the momentum
    // and energy are taken as they are, which saves the products that
    // rebuild them from the fields
    __device__ __forceinline__ static void phys_cons(int d, const real *u, const real *nd, real *f, const Ctx<real> &c)
    {
        const real s = HALF ? real(2) : real(1);
        const real vd = s * nd[1 + d], p = s * nd[P];
        f[0] = u[1 + d];
#pragma unroll
        for (int k = 0; k < DIM; ++k) f[1 + k] = (k == d) ? u[1 + k] * vd + p : u[1 + k] * vd;
        f[DIM + 1] = (u[DIM + 1] + p) * vd;
    }

    __device__ __forceinline__ static real speed(int d, const real *nd, const Ctx<real> &c)
    {
        return vspeed(d, nd) + sound(nd, c);
    }
    // the two parts of speed(): |v_d| and the sound speed ((gamma p / rho)
    // is the same with halved p and rho)
    __device__ __forceinline__ static real vspeed(int d, const real *nd)
    {
        return dabs((HALF ? real(2) : real(1)) * nd[1 + d]);
    }
    __device__ __forceinline__ static real sound(const real *nd, const Ctx<real> &c)
    {
        return dsqrt(c.gamma * nd[P] / nd[0]);
    }

    __device__ __forceinline__ static void pair(int d, const real *a, const real *b, real *f, const Ctx<real> &c)
    {
        if constexpr (FLUX == VOL_CENTRAL) {
            real fa[M], fb[M];
            phys(d, a, fa, c);
            phys(d, b, fb, c);
#pragma unroll
            for (int v = 0; v < M; ++v) f[v] = real(0.5) * (fa[v] + fb[v]);
        } else if constexpr (FLUX == VOL_KG) {
            // fields are halved: every arithmetic mean is a sum
            const real rho = a[0] + b[0];
            const real vd = a[1 + d] + b[1 + d];
            const real p = a[P] + b[P];
            const real e = a[DIM + 2] + b[DIM + 2];
            const real m = rho * vd;
            f[0] = m;
#pragma unroll
            for (int k = 0; k < DIM; ++k) f[1 + k] = (k == d ? m * vd + p : m * (a[1 + k] + b[1 + k]));
            f[DIM + 1] = (rho * e + p) * vd;
        } else {
            real rho_ln, ibeta_ln;
            lnmean_pair(a[0], b[0], a[DIM + 2], b[DIM + 2], a[DIM + 3], b[DIM + 3], a[DIM + 4], b[DIM + 4], rho_ln,
                        ibeta_ln);
            const real vd = real(0.5) * (a[1 + d] + b[1 + d]);
            real vv = real(0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) vv += a[1 + k] * b[1 + k];
            const real m = rho_ln * vd;
            f[0] = m;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                f[1 + k] = (k == d) ? m * vd + real(0.5) * (a[P] + b[P]) : m * (real(0.5) * (a[1 + k] + b[1 + k]));
            f[DIM + 1] = m * (ibeta_ln * c.inv_gm1 + real(0.5) * vv) + real(0.5) * (a[P] * b[1 + d] + b[P] * a[1 + d]);
        }
    }

    // The Ranocha flux of pair() with a direction that varies from lane to
    // lane: the direction enters through selects, not through the index of
    // a field, so that no register array is indexed at run time.
    __device__ __forceinline__ static void pair_rt(int d, const real *a, const real *b, real *f, const Ctx<real> &c)
    {
        static_assert(FLUX == VOL_RANOCHA, "run-time direction: Ranocha flux only");
        real rho_ln, ibeta_ln;
        lnmean_pair(a[0], b[0], a[DIM + 2], b[DIM + 2], a[DIM + 3], b[DIM + 3], a[DIM + 4], b[DIM + 4], rho_ln,
                    ibeta_ln);
        real vk[DIM], vd = real(0), avd = real(0), bvd = real(0), vv = real(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            vk[k] = real(0.5) * (a[1 + k] + b[1 + k]);
            vv += a[1 + k] * b[1 + k];
            if (k == d) {
                vd = vk[k];
                avd = a[1 + k];
                bvd = b[1 + k];
            }
        }
        const real m = rho_ln * vd;
        const real pm = real(0.5) * (a[P] + b[P]);
        f[0] = m;
#pragma unroll
        for (int k = 0; k < DIM; ++k) f[1 + k] = m * vk[k] + (k == d ? pm : real(0));
        f[DIM + 1] = m * (ibeta_ln * c.inv_gm1 + real(0.5) * vv) + real(0.5) * (a[P] * bvd + b[P] * avd);
    }
};

// ---------------------------------------------------------------- GLM-MHD
// u = (rho, rho v (3), E, B (3), psi),
// E = p/(gamma-1) + rho |v|^2/2 + |B|^2/2 + psi^2/2.
// Fields: 0 rho, 1-3 v, 4 p, 5-7 B, 8 psi, 9 ln rho, 10 beta = rho/(2p),
// 11 ln beta, 12 |v|^2, 13 |B|^2, 14 v.B
template <typename real, int FLUX>
struct MhdP {
    static constexpr int M = 9;
    static constexpr int NF = 15;

    __device__ __forceinline__ static void node(const real *u, real *nd, const Ctx<real> &c)
    {
        // Newton reciprocals instead of IEEE divisions, as for Euler
        const real rho = u[0], irho = rcp_nr(rho);
        const real v1 = u[1] * irho, v2 = u[2] * irho, v3 = u[3] * irho;
        const real B1 = u[5], B2 = u[6], B3 = u[7], psi = u[8];
        const real vv = v1 * v1 + v2 * v2 + v3 * v3, BB = B1 * B1 + B2 * B2 + B3 * B3;
        const real p = c.gm1 * (u[4] - real(0.5) * rho * vv - real(0.5) * BB - real(0.5) * psi * psi);
        const real beta = real(0.5) * rho * rcp_nr(p);
        nd[0] = rho; nd[1] = v1; nd[2] = v2; nd[3] = v3; nd[4] = p;
        nd[5] = B1; nd[6] = B2; nd[7] = B3; nd[8] = psi;
        nd[9] = dlog(rho); nd[10] = beta; nd[11] = dlog(beta);
        nd[12] = vv; nd[13] = BB; nd[14] = v1 * B1 + v2 * B2 + v3 * B3;
    }

    // the fields that phys(), speed(), fast(), btimes() and cons() read (no logarithms)
    __device__ __forceinline__ static void node_basic(const real *u, real *nd, const Ctx<real> &c)
    {
        const real rho = u[0], irho = rcp_nr(rho);
        const real v1 = u[1] * irho, v2 = u[2] * irho, v3 = u[3] * irho;
        const real B1 = u[5], B2 = u[6], B3 = u[7], psi = u[8];
        const real vv = v1 * v1 + v2 * v2 + v3 * v3, BB = B1 * B1 + B2 * B2 + B3 * B3;
        nd[0] = rho; nd[1] = v1; nd[2] = v2; nd[3] = v3;
        nd[4] = c.gm1 * (u[4] - real(0.5) * rho * vv - real(0.5) * BB - real(0.5) * psi * psi);
        nd[5] = B1; nd[6] = B2; nd[7] = B3; nd[8] = psi;
        nd[12] = vv; nd[13] = BB; nd[14] = v1 * B1 + v2 * B2 + v3 * B3;
    }

    __device__ __forceinline__ static void cons(const real *nd, real *u, const Ctx<real> &c)
    {
        u[0] = nd[0];
        u[1] = nd[0] * nd[1]; u[2] = nd[0] * nd[2]; u[3] = nd[0] * nd[3];
        u[4] = nd[4] * c.inv_gm1 + real(0.5) * nd[0] * nd[12] + real(0.5) * nd[13] + real(0.5) * nd[8] * nd[8];
        u[5] = nd[5]; u[6] = nd[6]; u[7] = nd[7]; u[8] = nd[8];
    }

    __device__ __forceinline__ static void phys(int d, const real *nd, real *f, const Ctx<real> &c)
    {
        const real rho = nd[0], p = nd[4], psi = nd[8];
        const real vd = nd[1 + d], Bd = nd[5 + d];
        f[0] = rho * vd;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            f[1 + k] = rho * vd * nd[1 + k] - Bd * nd[5 + k] + (k == d ? p + real(0.5) * nd[13] : real(0));
        f[4] = vd * (real(0.5) * rho * nd[12] + c.gamma * c.inv_gm1 * p + nd[13]) - Bd * nd[14] + c.ch * psi * Bd;
#pragma unroll
        for (int k = 0; k < 3; ++k) f[5 + k] = (k == d) ? c.ch * psi : vd * nd[5 + k] - Bd * nd[1 + k];
        f[8] = c.ch * Bd;
    }

    // fast magnetosonic speed + |v_d| (without the cleaning speed)
    __device__ __forceinline__ static real fast(int d, const real *nd, const Ctx<real> &c)
    {
        const real irho = real(1) / nd[0];
        const real a2 = c.gamma * nd[4] * irho;
        const real t = a2 + nd[13] * irho;
        const real Bd = nd[5 + d];
        const real cf = dsqrt(real(0.5) * (t + dsqrt(t * t - real(4) * a2 * Bd * Bd * irho)));
        return dabs(nd[1 + d]) + cf;
    }

    __device__ __forceinline__ static real speed(int d, const real *nd, const Ctx<real> &c)
    {
        return dmax(fast(d, nd, c), c.ch);
    }

    // B_d(u_a) applied to g = (gB, gpsi): Powell phi_P = (0, B, v.B, v, 0),
    // GLM phi_G = (0, 0, v_d psi, 0, v_d)
    __device__ __forceinline__ static void btimes(int d, const real *nd, real gB, real gpsi, real *o)
    {
        o[0] = real(0);
        o[1] = nd[5] * gB; o[2] = nd[6] * gB; o[3] = nd[7] * gB;
        o[4] = nd[14] * gB + nd[1 + d] * nd[8] * gpsi;
        o[5] = nd[1] * gB; o[6] = nd[2] * gB; o[7] = nd[3] * gB;
        o[8] = nd[1 + d] * gpsi;
    }

    __device__ __forceinline__ static void pair(int d, const real *a, const real *b, real *f, const Ctx<real> &c)
    {
        if constexpr (FLUX == VOL_CENTRAL) {
            real fa[M], fb[M];
            phys(d, a, fa, c);
            phys(d, b, fb, c);
#pragma unroll
            for (int v = 0; v < M; ++v) f[v] = real(0.5) * (fa[v] + fb[v]);
            return;
        }
        const real h = real(0.5);
        // both logarithmic means and 1/(2 mean beta) from one reciprocal
        real n1, d1, n2, d2;
        lnmean_parts_fast(a[0], b[0], a[9], b[9], n1, d1);
        lnmean_parts_fast(a[10], b[10], a[11], b[11], n2, d2);
        const real tb = a[10] + b[10];
        const real dn = d1 * n2;
        const real r = rcp_nr(dn * tb);
        const real rho_ln = (n1 * n2) * tb * r, ibeta_ln = (d2 * d1) * tb * r, i2b = dn * r;
        const real rho_a = h * (a[0] + b[0]), psi_a = h * (a[8] + b[8]);
        real va[3], Ba[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) { va[k] = h * (a[1 + k] + b[1 + k]); Ba[k] = h * (a[5 + k] + b[5 + k]); }
        const real f0 = rho_ln * va[d];
        f[0] = f0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            f[1 + k] = f0 * va[k] - Ba[d] * Ba[k] + (k == d ? rho_a * i2b + h * h * (a[13] + b[13]) : real(0));
#pragma unroll
        for (int k = 0; k < 3; ++k) f[5 + k] = (k == d) ? c.ch * psi_a : va[d] * Ba[k] - va[k] * Ba[d];
        f[8] = c.ch * Ba[d];
        f[4] = f0 * (h * c.inv_gm1 * ibeta_ln - h * h * (a[12] + b[12]))
             + f[1] * va[0] + f[2] * va[1] + f[3] * va[2]
             + f[5] * Ba[0] + f[6] * Ba[1] + f[7] * Ba[2] + f[8] * psi_a
             - h * h * (a[1 + d] * a[13] + b[1 + d] * b[13]) + Ba[d] * h * (a[14] + b[14])
             - c.ch * h * (a[5 + d] * a[8] + b[5 + d] * b[8]);
    }
};

} // namespace crk
