// stage_d3.hip -- instantiations and dispatch of the 3D stage kernels.
#include "stage3m_kernel.hpp"
#include "stage_kernel.hpp"
#include "variants.h"

namespace af4 {

namespace {

constexpr long kLdsCap = 160L * 1024L;

template <class T, bool LIM, bool SI, bool QF, int TX, int TY, int TZ, int NT, bool CV>
hipError_t launch_one(int nblocks, const void *params, hipStream_t s)
{
    const StageParams<T> &p = *(const StageParams<T> *)params;
    if constexpr (stage_lds_bytes<3, T, LIM, SI, TX, TY, TZ>() > kLdsCap) {
        return hipErrorInvalidValue;
    } else if (p.lact) {  // the limiter-counting form: one variant, limiter on
        if constexpr (CV && LIM) {
            hipLaunchKernelGGL((stage_kernel<3, T, LIM, SI, QF, TX, TY, TZ, NT, true>), dim3(nblocks), dim3(NT), 0, s, p);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((stage_kernel<3, T, LIM, SI, QF, TX, TY, TZ, NT>), dim3(nblocks), dim3(NT), 0, s, p);
        return hipGetLastError();
    }
}

// the kernel marching along z (fluxes c1 u + c2 u^2 only)
template <class T, bool LIM, bool SI, int TX, int TY, int TZ, int NT>
hipError_t launch_march(int nblocks, const void *params, hipStream_t s)
{
    const StageParams<T> &p = *(const StageParams<T> *)params;
    if constexpr (stage3m_lds_bytes<T, LIM, SI, TX, TY>() > kLdsCap) {
        return hipErrorInvalidValue;
    } else {
        if (p.lact) return hipErrorInvalidValue;
        hipLaunchKernelGGL((stage3m_kernel<T, LIM, SI, TX, TY, TZ, NT>), dim3(nblocks), dim3(NT), 0, s, p);
        return hipGetLastError();
    }
}

template <class T, bool QF, int TX, int TY, int TZ, int NT, int KIND, bool CV>
hipError_t launch_tq(bool lim, bool si, int nblocks, const void *params, hipStream_t s)
{
    if constexpr (KIND == 1) {
        if constexpr (!QF) {
            return hipErrorInvalidValue;
        } else {
            if (lim) return si ? launch_march<T, true, true, TX, TY, TZ, NT>(nblocks, params, s)
                               : launch_march<T, true, false, TX, TY, TZ, NT>(nblocks, params, s);
            return si ? launch_march<T, false, true, TX, TY, TZ, NT>(nblocks, params, s)
                      : launch_march<T, false, false, TX, TY, TZ, NT>(nblocks, params, s);
        }
    } else {
        if (lim) return si ? launch_one<T, true, true, QF, TX, TY, TZ, NT, CV>(nblocks, params, s)
                           : launch_one<T, true, false, QF, TX, TY, TZ, NT, CV>(nblocks, params, s);
        return si ? launch_one<T, false, true, QF, TX, TY, TZ, NT, CV>(nblocks, params, s)
                  : launch_one<T, false, false, QF, TX, TY, TZ, NT, CV>(nblocks, params, s);
    }
}

// CV: the variant with the limiter-counting form
template <int TX, int TY, int TZ, int NT, int KIND, bool CV>
hipError_t launch_tile(int prec, bool lim, bool si, bool qf, int nblocks, const void *params, hipStream_t s)
{
    if (prec == 32) return qf ? launch_tq<float, true, TX, TY, TZ, NT, KIND, CV>(lim, si, nblocks, params, s)
                              : launch_tq<float, false, TX, TY, TZ, NT, KIND, CV>(lim, si, nblocks, params, s);
    return qf ? launch_tq<double, true, TX, TY, TZ, NT, KIND, CV>(lim, si, nblocks, params, s)
              : launch_tq<double, false, TX, TY, TZ, NT, KIND, CV>(lim, si, nblocks, params, s);
}

template <class T, bool LIM, bool SI, int TX, int TY, int TZ, int KIND>
constexpr bool fits_t()
{
    if constexpr (KIND == 1) return stage3m_lds_bytes<T, LIM, SI, TX, TY>() <= kLdsCap;
    else return stage_lds_bytes<3, T, LIM, SI, TX, TY, TZ>() <= kLdsCap;
}

template <int TX, int TY, int TZ, int KIND>
bool fits(int prec, bool lim, bool si)
{
    if (prec == 32) {
        if (lim) return si ? fits_t<float, true, true, TX, TY, TZ, KIND>() : fits_t<float, true, false, TX, TY, TZ, KIND>();
        return si ? fits_t<float, false, true, TX, TY, TZ, KIND>() : fits_t<float, false, false, TX, TY, TZ, KIND>();
    }
    if (lim) return si ? fits_t<double, true, true, TX, TY, TZ, KIND>() : fits_t<double, true, false, TX, TY, TZ, KIND>();
    return si ? fits_t<double, false, true, TX, TY, TZ, KIND>() : fits_t<double, false, false, TX, TY, TZ, KIND>();
}

}  // namespace

bool stage_supported_d3(int prec, bool lim, bool si, unsigned caps, int variant)
{
    switch (variant) {
#define AF4_FITS(V, TX, TY, TZ, NT, KIND, NAME) \
    case V: return (KIND != 1 || (caps & kCapQF) != 0) && fits<TX, TY, TZ, KIND>(prec, lim, si);
        AF4_VARIANTS_D3(AF4_FITS)
#undef AF4_FITS
    }
    return false;
}

hipError_t stage_launch_d3(int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params,
                           hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    switch (variant) {
#define AF4_CASE(V, TX, TY, TZ, NT, KIND, NAME) \
    case V: return launch_tile<TX, TY, TZ, NT, KIND, V == count_variant(3)>(prec, lim, si, (caps & kCapQF) != 0, nblocks, params, s);
        AF4_VARIANTS_D3(AF4_CASE)
#undef AF4_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace af4
