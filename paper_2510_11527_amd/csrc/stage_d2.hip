// stage_d2.hip -- instantiations and dispatch of the 2D stage kernels.
#include "stage2o_kernel.hpp"
#include "variants.h"

namespace af4 {

namespace {

constexpr long kLdsCap = 160L * 1024L;

// CV: the variant with the limiter-counting form (p.lact not null)
template <class T, bool LIM, bool SI, bool QF, int TX, int TY, int NT, bool CV>
hipError_t launch_generic(int nblocks, const void *params, hipStream_t s)
{
    const StageParams<T> &p = *(const StageParams<T> *)params;
    if constexpr (stage_lds_bytes<2, T, LIM, SI, TX, TY, 1>() > kLdsCap) {
        return hipErrorInvalidValue;
    } else if (p.lact) {
        if constexpr (CV && LIM) {
            hipLaunchKernelGGL((stage_kernel<2, T, LIM, SI, QF, TX, TY, 1, NT, true>), dim3(nblocks), dim3(NT), 0, s, p);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((stage_kernel<2, T, LIM, SI, QF, TX, TY, 1, NT>), dim3(nblocks), dim3(NT), 0, s, p);
        return hipGetLastError();
    }
}

template <class T, bool LIM, bool QF, bool FT, int TX, int TY, int NT>
hipError_t launch_tuned(int nblocks, const void *params, hipStream_t s)
{
    if constexpr (stage2d_lds_bytes<T, LIM, QF, FT, TX, TY>() > kLdsCap) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((stage2d_kernel<T, LIM, QF, FT, TX, TY, NT>), dim3(nblocks), dim3(NT), 0, s,
                           *(const StageParams<T> *)params);
        return hipGetLastError();
    }
}

template <class T, bool LIM, int FL, int TX, int TY, int NT>
hipError_t launch_own(int nblocks, const void *params, hipStream_t s)
{
    if constexpr (stage2o_lds_bytes<T, LIM, TX, TY>() > kLdsCap) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((stage2o_kernel<T, LIM, FL, TX, TY, NT>), dim3(nblocks), dim3(NT), 0, s,
                           *(const StageParams<T> *)params);
        return hipGetLastError();
    }
}

template <class T, int FL, int TX, int TY, int NT>
hipError_t launch_own_lim(bool lim, int nblocks, const void *params, hipStream_t s)
{
    return lim ? launch_own<T, true, FL, TX, TY, NT>(nblocks, params, s)
               : launch_own<T, false, FL, TX, TY, NT>(nblocks, params, s);
}

template <class T, int TX, int TY, int NT, int KIND, bool CV>
hipError_t launch_kind(bool lim, bool si, unsigned caps, int nblocks, const void *params, hipStream_t s)
{
    const bool qf = (caps & kCapQF) != 0;
    if (KIND != 0 && ((const StageParams<T> *)params)->lact) return hipErrorInvalidValue;  // counting: generic only
    if (KIND != 0 && KIND != 4 && (caps & kCapOpen)) return hipErrorInvalidValue;  // ghosts: generic, own-items
    if constexpr (KIND == 4) {
        if (si || !(caps & kCapI32) || !(qf || (caps & kCapBLF))) return hipErrorInvalidValue;
        const int fl = (!qf ? kOwnGen : 0) | ((caps & kCapPP) ? kOwnPP : 0) | ((qf && (caps & kCapBQ)) ? kOwnBQ : 0) |
                       ((caps & kCapOpen) ? kOwnOpen : 0);
        switch (fl) {
#define AF4_OWN_FL(F) \
    case F: return launch_own_lim<T, F, TX, TY, NT>(lim, nblocks, params, s);
            AF4_OWN_FL(0) AF4_OWN_FL(kOwnPP) AF4_OWN_FL(kOwnBQ) AF4_OWN_FL(kOwnPP | kOwnBQ) AF4_OWN_FL(kOwnGen)
            AF4_OWN_FL(kOwnGen | kOwnPP) AF4_OWN_FL(kOwnOpen) AF4_OWN_FL(kOwnOpen | kOwnPP) AF4_OWN_FL(kOwnOpen | kOwnBQ)
            AF4_OWN_FL(kOwnOpen | kOwnPP | kOwnBQ) AF4_OWN_FL(kOwnOpen | kOwnGen) AF4_OWN_FL(kOwnOpen | kOwnGen | kOwnPP)
#undef AF4_OWN_FL
        }
        return hipErrorInvalidValue;
    } else if constexpr (KIND == 0) {
        if (qf) {
            if (lim) return si ? launch_generic<T, true, true, true, TX, TY, NT, CV>(nblocks, params, s)
                               : launch_generic<T, true, false, true, TX, TY, NT, CV>(nblocks, params, s);
            return si ? launch_generic<T, false, true, true, TX, TY, NT, CV>(nblocks, params, s)
                      : launch_generic<T, false, false, true, TX, TY, NT, CV>(nblocks, params, s);
        }
        if (lim) return si ? launch_generic<T, true, true, false, TX, TY, NT, CV>(nblocks, params, s)
                           : launch_generic<T, true, false, false, TX, TY, NT, CV>(nblocks, params, s);
        return si ? launch_generic<T, false, true, false, TX, TY, NT, CV>(nblocks, params, s)
                  : launch_generic<T, false, false, false, TX, TY, NT, CV>(nblocks, params, s);
    } else {
        constexpr bool FT = KIND == 1;
        if (si) return hipErrorInvalidValue;
        if (qf) return lim ? launch_tuned<T, true, true, FT, TX, TY, NT>(nblocks, params, s)
                           : launch_tuned<T, false, true, FT, TX, TY, NT>(nblocks, params, s);
        if constexpr (!FT) return hipErrorInvalidValue;  // general fluxes need the table
        else
            return lim ? launch_tuned<T, true, false, true, TX, TY, NT>(nblocks, params, s)
                       : launch_tuned<T, false, false, true, TX, TY, NT>(nblocks, params, s);
    }
}

template <class T, int TX, int TY, int KIND>
bool fits_kind(bool lim, bool si, unsigned caps)
{
    const bool qf = (caps & kCapQF) != 0;
    if (KIND != 0 && KIND != 4 && (caps & kCapOpen)) return false;
    if constexpr (KIND == 4) {
        if (si || !(caps & kCapI32) || !(qf || (caps & kCapBLF))) return false;
        return stage2o_lds_bytes<T, true, TX, TY>() <= kLdsCap && stage2o_lds_bytes<T, false, TX, TY>() <= kLdsCap;
    } else if constexpr (KIND == 0) {
        if (lim) return si ? stage_lds_bytes<2, T, true, true, TX, TY, 1>() <= kLdsCap
                           : stage_lds_bytes<2, T, true, false, TX, TY, 1>() <= kLdsCap;
        return si ? stage_lds_bytes<2, T, false, true, TX, TY, 1>() <= kLdsCap
                  : stage_lds_bytes<2, T, false, false, TX, TY, 1>() <= kLdsCap;
    } else {
        constexpr bool FT = KIND == 1;
        if (si) return false;
        if (!qf && !FT) return false;
        // the residual launch uses the unlimited instantiation: both must fit
        const long lim_b = qf ? stage2d_lds_bytes<T, true, true, FT, TX, TY>() : stage2d_lds_bytes<T, true, false, true, TX, TY>();
        const long un_b = qf ? stage2d_lds_bytes<T, false, true, FT, TX, TY>() : stage2d_lds_bytes<T, false, false, true, TX, TY>();
        return (lim ? lim_b : un_b) <= kLdsCap && un_b <= kLdsCap;
    }
}

}  // namespace

bool stage_supported_d2(int prec, bool lim, bool si, unsigned caps, int variant)
{
    switch (variant) {
#define AF4_FITS(V, TX, TY, TZ, NT, KIND, NAME) \
    case V: return prec == 32 ? fits_kind<float, TX, TY, KIND>(lim, si, caps) : fits_kind<double, TX, TY, KIND>(lim, si, caps);
        AF4_VARIANTS_D2(AF4_FITS)
#undef AF4_FITS
    }
    return false;
}

hipError_t stage_launch_d2(int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params,
                           hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    switch (variant) {
#define AF4_CASE(V, TX, TY, TZ, NT, KIND, NAME)                                                            \
    case V:                                                                                                \
        return prec == 32 ? launch_kind<float, TX, TY, NT, KIND, V == count_variant(2)>(lim, si, caps, nblocks, params, s) \
                          : launch_kind<double, TX, TY, NT, KIND, V == count_variant(2)>(lim, si, caps, nblocks, params, s);
        AF4_VARIANTS_D2(AF4_CASE)
#undef AF4_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace af4
