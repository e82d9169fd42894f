// stage_d3.hip -- instantiations and dispatch of the 3D stage kernels.
#include "stage_kernel.hpp"
#include "variants.h"

namespace af4 {

namespace {

template <class T, bool LIM, bool SI, bool QF, int TX, int TY, int TZ, int NT, bool CV>
hipError_t launch_one(int nblocks, const void *params, hipStream_t s)
{
    const StageParams<T> &p = *(const StageParams<T> *)params;
    if constexpr (stage_lds_bytes<3, T, LIM, SI, TX, TY, TZ>() > 160L * 1024L) {
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

template <class T, bool QF, int TX, int TY, int TZ, int NT, bool CV>
hipError_t launch_tq(bool lim, bool si, int nblocks, const void *params, hipStream_t s)
{
    if (lim) return si ? launch_one<T, true, true, QF, TX, TY, TZ, NT, CV>(nblocks, params, s)
                       : launch_one<T, true, false, QF, TX, TY, TZ, NT, CV>(nblocks, params, s);
    return si ? launch_one<T, false, true, QF, TX, TY, TZ, NT, CV>(nblocks, params, s)
              : launch_one<T, false, false, QF, TX, TY, TZ, NT, CV>(nblocks, params, s);
}

// CV: the variant with the limiter-counting form
template <int TX, int TY, int TZ, int NT, bool CV>
hipError_t launch_tile(int prec, bool lim, bool si, bool qf, int nblocks, const void *params, hipStream_t s)
{
    if (prec == 32) return qf ? launch_tq<float, true, TX, TY, TZ, NT, CV>(lim, si, nblocks, params, s)
                              : launch_tq<float, false, TX, TY, TZ, NT, CV>(lim, si, nblocks, params, s);
    return qf ? launch_tq<double, true, TX, TY, TZ, NT, CV>(lim, si, nblocks, params, s)
              : launch_tq<double, false, TX, TY, TZ, NT, CV>(lim, si, nblocks, params, s);
}

template <int TX, int TY, int TZ>
bool fits(int prec, bool lim, bool si)
{
    constexpr long cap = 160L * 1024L;
    if (prec == 32) {
        if (lim) return si ? stage_lds_bytes<3, float, true, true, TX, TY, TZ>() <= cap
                           : stage_lds_bytes<3, float, true, false, TX, TY, TZ>() <= cap;
        return si ? stage_lds_bytes<3, float, false, true, TX, TY, TZ>() <= cap
                  : stage_lds_bytes<3, float, false, false, TX, TY, TZ>() <= cap;
    }
    if (lim) return si ? stage_lds_bytes<3, double, true, true, TX, TY, TZ>() <= cap
                       : stage_lds_bytes<3, double, true, false, TX, TY, TZ>() <= cap;
    return si ? stage_lds_bytes<3, double, false, true, TX, TY, TZ>() <= cap
              : stage_lds_bytes<3, double, false, false, TX, TY, TZ>() <= cap;
}

}  // namespace

bool stage_supported_d3(int prec, bool lim, bool si, int variant)
{
    switch (variant) {
#define AF4_FITS(V, TX, TY, TZ, NT, NAME) \
    case V: return fits<TX, TY, TZ>(prec, lim, si);
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
#define AF4_CASE(V, TX, TY, TZ, NT, NAME) \
    case V: return launch_tile<TX, TY, TZ, NT, V == count_variant(3)>(prec, lim, si, (caps & kCapQF) != 0, nblocks, params, s);
        AF4_VARIANTS_D3(AF4_CASE)
#undef AF4_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace af4
