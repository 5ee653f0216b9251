// crk_family_impl.hpp -- definitions of Family<real, EQ, DIM>; included once
// per family translation unit, followed by an explicit instantiation.
#pragma once
#include "crk_dispatch.hpp"
#include "crk_rhs.hpp"

namespace crk {

#define CRK_FLUX_SWITCH(LAUNCH, N)                                                             \
    switch (flux) {                                                                            \
    case VOL_CENTRAL: return LAUNCH<real, EQ, DIM, N, VOL_CENTRAL>(t, p, s);                   \
    case VOL_KG: if constexpr (EQ == EQ_EULER) return LAUNCH<real, EQ, DIM, N, VOL_KG>(t, p, s); break;          \
    case VOL_RANOCHA: if constexpr (EQ == EQ_EULER) return LAUNCH<real, EQ, DIM, N, VOL_RANOCHA>(t, p, s); break; \
    case VOL_DERIGS: if constexpr (EQ == EQ_MHD) return LAUNCH<real, EQ, DIM, N, VOL_DERIGS>(t, p, s); break;     \
    default: break;                                                                            \
    }                                                                                          \
    return hipErrorInvalidValue;

#define CRK_DEGREE_SWITCH(LAUNCH)                         \
    switch (t.N) {                                        \
    case 1: { CRK_FLUX_SWITCH(LAUNCH, 1) }                \
    case 2: { CRK_FLUX_SWITCH(LAUNCH, 2) }                \
    case 3: { CRK_FLUX_SWITCH(LAUNCH, 3) }                \
    case 4: { CRK_FLUX_SWITCH(LAUNCH, 4) }                \
    default: return hipErrorInvalidValue;                 \
    }

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::local(const Tables &t, int flux, const StepPtrs &p, hipStream_t s)
{
    CRK_DEGREE_SWITCH(launch_local)
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::interface(const Tables &t, int flux, const StepPtrs &p, hipStream_t s)
{
    CRK_DEGREE_SWITCH(launch_interface)
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::fr_rhs(const Tables &t, int flux, const void *u, const double *dtc, int surface,
                                         void *rhs, hipStream_t s)
{
#define CRK_RHS_FLUX(NN)                                                                                        \
    switch (flux) {                                                                                             \
    case VOL_CENTRAL: return launch_fr_rhs<real, EQ, DIM, NN, VOL_CENTRAL>(t, u, dtc, surface, rhs, s);        \
    case VOL_KG: if constexpr (EQ == EQ_EULER) return launch_fr_rhs<real, EQ, DIM, NN, VOL_KG>(t, u, dtc, surface, rhs, s); break;           \
    case VOL_RANOCHA: if constexpr (EQ == EQ_EULER) return launch_fr_rhs<real, EQ, DIM, NN, VOL_RANOCHA>(t, u, dtc, surface, rhs, s); break; \
    case VOL_DERIGS: if constexpr (EQ == EQ_MHD) return launch_fr_rhs<real, EQ, DIM, NN, VOL_DERIGS>(t, u, dtc, surface, rhs, s); break;     \
    default: break;                                                                                             \
    }                                                                                                           \
    return hipErrorInvalidValue;
    switch (t.N) {
    case 1: { CRK_RHS_FLUX(1) }
    case 2: { CRK_RHS_FLUX(2) }
    case 3: { CRK_RHS_FLUX(3) }
    case 4: { CRK_RHS_FLUX(4) }
    default: return hipErrorInvalidValue;
    }
#undef CRK_RHS_FLUX
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::rkfr(const Tables &t, int flux, const RkPtrs &p, void *b0, void *b1, void *uo,
                                       hipStream_t s)
{
#define CRK_RKFR_FLUX(NN)                                                                                       \
    switch (flux) {                                                                                             \
    case VOL_CENTRAL: return launch_rkfr<real, EQ, DIM, NN, VOL_CENTRAL>(t, p, b0, b1, uo, s);                 \
    case VOL_KG: if constexpr (EQ == EQ_EULER) return launch_rkfr<real, EQ, DIM, NN, VOL_KG>(t, p, b0, b1, uo, s); break;           \
    case VOL_RANOCHA: if constexpr (EQ == EQ_EULER) return launch_rkfr<real, EQ, DIM, NN, VOL_RANOCHA>(t, p, b0, b1, uo, s); break; \
    case VOL_DERIGS: if constexpr (EQ == EQ_MHD) return launch_rkfr<real, EQ, DIM, NN, VOL_DERIGS>(t, p, b0, b1, uo, s); break;     \
    default: break;                                                                                             \
    }                                                                                                           \
    return hipErrorInvalidValue;
    switch (t.N) {
    case 1: { CRK_RKFR_FLUX(1) }
    case 2: { CRK_RKFR_FLUX(2) }
    case 3: { CRK_RKFR_FLUX(3) }
    case 4: { CRK_RKFR_FLUX(4) }
    default: return hipErrorInvalidValue;
    }
#undef CRK_RKFR_FLUX
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::face_speed(const Tables &t, int flux, const StepPtrs &p, hipStream_t s)
{
    CRK_DEGREE_SWITCH(launch_face_speed)
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::run(const Tables &t, int flux, const StepPtrs &p, double *dt, int nsteps,
                                      hipStream_t s)
{
    if constexpr (DIM != 1 || EQ != EQ_EULER) {
        return hipErrorNotSupported;
    } else {
#define CRK_RUN_FLUX(NN)                                                                             \
        switch (flux) {                                                                              \
        case VOL_CENTRAL: return launch_run<real, EQ, DIM, NN, VOL_CENTRAL>(t, p, dt, nsteps, s);   \
        case VOL_KG: return launch_run<real, EQ, DIM, NN, VOL_KG>(t, p, dt, nsteps, s);             \
        case VOL_RANOCHA: return launch_run<real, EQ, DIM, NN, VOL_RANOCHA>(t, p, dt, nsteps, s);   \
        default: return hipErrorInvalidValue;                                                        \
        }
        switch (t.N) {
        case 1: CRK_RUN_FLUX(1)
        case 2: CRK_RUN_FLUX(2)
        case 3: CRK_RUN_FLUX(3)
        case 4: CRK_RUN_FLUX(4)
        default: return hipErrorInvalidValue;
        }
#undef CRK_RUN_FLUX
    }
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::indicator(const Tables &t, const void *u, double *araw, double *alpha, float *features,
                                            hipStream_t s)
{
    if constexpr (EQ != EQ_EULER) {
        return hipErrorInvalidValue;
    } else {
        switch (t.N) {
        case 1: return launch_indicator<real, DIM, 1>(t, u, araw, alpha, features, s);
        case 2: return launch_indicator<real, DIM, 2>(t, u, araw, alpha, features, s);
        case 3: return launch_indicator<real, DIM, 3>(t, u, araw, alpha, features, s);
        case 4: return launch_indicator<real, DIM, 4>(t, u, araw, alpha, features, s);
        default: return hipErrorInvalidValue;
        }
    }
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::dt(const Tables &t, const void *u, double *partials, double *dt, hipStream_t s)
{
    return launch_dt<real, EQ, DIM>(t, u, partials, dt, s);
}

template <typename real, int EQ, int DIM>
hipError_t Family<real, EQ, DIM>::diag(const Tables &t, const void *u, double *partials, double *out, hipStream_t s)
{
    return launch_diag<real, EQ, DIM>(t, u, partials, out, s);
}

#undef CRK_DEGREE_SWITCH
#undef CRK_FLUX_SWITCH

} // namespace crk
