// crk_dispatch.hpp -- runtime (degree, volume flux) -> template instance.
// One "family" per (precision, equation, dimension) is compiled in its own
// translation unit (crk_family_*.hip) so that the instances build in parallel.
#pragma once
#include "crk_kernels.hpp"

namespace crk {

template <typename real, int EQ, int DIM>
struct Family {
    static hipError_t local(const Tables &t, int flux, const StepPtrs &p, hipStream_t s);
    static hipError_t interface(const Tables &t, int flux, const StepPtrs &p, hipStream_t s);
    // wave speeds of the face nodes of p.u_in into the face data p.traces
    static hipError_t face_speed(const Tables &t, int flux, const StepPtrs &p, hipStream_t s);
    // nsteps pipelined steps of a one-dimensional mesh of at most RUN_BLOCK
    // nodes in one workgroup (hipErrorNotSupported otherwise)
    static hipError_t run(const Tables &t, int flux, const StepPtrs &p, double *dt, int nsteps, hipStream_t s);
    static hipError_t indicator(const Tables &t, const void *u, double *araw, double *alpha, float *features, hipStream_t s);
    static hipError_t dt(const Tables &t, const void *u, double *partials, double *dt, hipStream_t s);
    static hipError_t diag(const Tables &t, const void *u, double *partials, double *out, hipStream_t s);
    // semi-discrete FR operator du/dt of u into rhs (test operator, crk_rhs.hpp)
    static hipError_t fr_rhs(const Tables &t, int flux, const void *u, const double *dtc, int surface, void *rhs,
                             hipStream_t s);
    // the s stages of a standard RKFR step (crk_rhs.hpp); stage states in b0, b1
    static hipError_t rkfr(const Tables &t, int flux, const RkPtrs &p, void *b0, void *b1, void *u_out,
                           hipStream_t s);
};

// fluxes compiled for an equation system
constexpr bool flux_supported(int eq, int flux)
{
    return eq == EQ_EULER ? (flux == VOL_CENTRAL || flux == VOL_KG || flux == VOL_RANOCHA)
                          : (flux == VOL_CENTRAL || flux == VOL_DERIGS);
}

} // namespace crk
