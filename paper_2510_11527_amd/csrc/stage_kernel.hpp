// stage_kernel.hpp -- fused forward-Euler / SSP-RK3 stage kernel of the compact
// fourth-order doubly conservative active flux method with monolithic convex
// limiting (J. Duan, arXiv 2510.11527), for gfx950.
//
// One workgroup owns a tile of cells of one instance.  It stages the tile and
// a halo of the input state in LDS as a "half grid": along every axis the
// points x_{i-1/2}, x_i, x_{i+1/2}, ... are spaced dx/2 apart, so that all
// operators of Sec. 2 and their multi-D half-index shifts (Sec. 4) become
// 5-point stencils along one axis.  Cell centres (not DoFs) are reconstructed
// in LDS by inverting the tensor Simpson rule.  The kernel then computes, in
// LDS phases separated by barriers:
//   * point values: the biased 4th-order FVS convection operator with the
//     downwind point, in the exact equivalent form
//       D+ f^+ + D- f^- = [ (f_{-2} - 8 f_{-1} + 8 f_1 - f_2)
//                            + alpha (z_{-2} - 4 z_{-1} + 6 z_0 - 4 z_1 + z_2) ] / (6 dx),
//     plus the compact D^{2,4th} on a(u), then projection onto [umin, umax];
//   * averages: the doubly conservative update with Simpson face fluxes and
//     cell-centred potentials, limited by the monolithic convex limiter
//     against the LLF low-order scheme (Sec. 5.1.1 and 5.2.1);
//   * the SSP-RK3 convex combination with U^n and the bound safeguard;
// and writes the new DoFs of its tile.  Halo values are recomputed, never
// exchanged, so one launch is one stage over all instances.
#pragma once
#include "af_internal.h"

namespace af4 {

// AF kind codes (same numbering as the public header)
enum : int { kFLinear = 0, kFQuad = 1, kFBL = 2, kFBLGrav = 3 };
enum : int { kALinear = 0, kAPower = 1, kADeadzone = 2, kABL = 3, kARamp2 = 4 };

// 1/v within about an ulp, sparing the ten-instruction correctly rounded
// division: in FP64 the hardware estimate refined by two Newton-Raphson
// steps r += r (1 - v r) (v = 0 gives NaN, which the only caller that can
// see it, the limiter's ratio, turns into 1 through fmin); in FP32 the
// hardware reciprocal
template <class T>
__device__ __forceinline__ T fast_rcp(T v)
{
    T r = __builtin_amdgcn_rcp(v);
    T e = fma(-v, r, T(1));
    r = fma(r, e, r);
    e = fma(-v, r, T(1));
    return fma(r, e, r);
}
template <>
__device__ __forceinline__ float fast_rcp<float>(float v)
{
    return __builtin_amdgcn_rcpf(v);
}

// e^x of a blending weight (x <= 0): exp in FP64; in FP32 the hardware 2^y
// of y = x log2(e), whose relative error (about |y| 2^-24 from rounding y,
// plus an ulp) is far inside the FP32 tolerance for the weights' arguments
template <class T>
__device__ __forceinline__ T blend_exp(T x)
{
    return exp(x);
}
template <>
__device__ __forceinline__ float blend_exp<float>(float x)
{
    return __builtin_amdgcn_exp2f(x * 1.44269504f);
}

// p0 * u^p (powers other than 1, 2, 3): kept out of line so that the
// stage kernels do not carry a pow expansion at every evaluation site
template <class T>
__device__ __noinline__ T power_potential(T p0, T p, int m, T u)
{
    if (m > 0) {
        T r = u;
        for (int i = 1; i < m; i++) r *= u;
        return p0 * r;
    }
    return p0 * pow(u, p);
}

template <class T>
struct Phys {
    int fk[3];
    T fc[3], fg[3];
    int ak, am;
    T a0, a1;
    T umin, umax;
    int nc[3];
    const_ptr<InstDev> ip;   // critical points are read from here (scalar loads)
    T pu0, plo, phi, pc1, pc2, pc3;
    bool pabs, ppow;

    // the instance's parameters through the constant address space: scalar
    // loads, whose waits do not hold up the vector loads in flight
    __device__ void load(const InstDev &Iref, int D) { load(as_constant(&Iref), D); }
    __device__ void load(const_ptr<InstDev> I, int D)
    {
        ip = I;
        for (int l = 0; l < 3; l++) {
            fk[l] = I->fk[l];
            fc[l] = (T)I->fp0[l];
            fg[l] = (T)I->fp1[l];
            nc[l] = l < D ? I->ncrit[l] : 0;
        }
        ak = I->ak;
        am = I->am;
        pu0 = (T)I->pu0;
        plo = (T)I->plo;
        phi = (T)I->phi;
        pc1 = (T)I->pc1;
        pc2 = (T)I->pc2;
        pc3 = (T)I->pc3;
        pabs = I->pabs != 0;
        ppow = I->ppow != 0;
        a0 = (T)I->ap0;
        a1 = (T)I->ap1;
        // FP32: the bounds rounded inwards on the host
        if constexpr (sizeof(T) == 4) {
            umin = I->f_umin;
            umax = I->f_umax;
        } else {
            umin = I->umin;
            umax = I->umax;
        }
    }

    // f_l(u)
    __device__ __forceinline__ T f(int l, T u) const
    {
        const int k = fk[l];
        if (k == kFQuad) return fc[l] * u * u;
        if (k == kFLinear) return fc[l] * u;
        T v = T(1) - u;
        T q = u * u * fast_rcp(u * u + v * v);
        if (k == kFBL) return q;
        return q * (T(1) - fg[l] * v * v);
    }

    // |f_l'(u)|
    __device__ __forceinline__ T adf(int l, T u) const
    {
        const int k = fk[l];
        if (k == kFQuad) return fabs(T(2) * fc[l] * u);
        if (k == kFLinear) return fabs(fc[l]);
        T v = T(1) - u;
        T den = u * u + v * v;
        const T r = fast_rcp(den);
        T d1 = T(2) * u * v * (r * r);
        if (k == kFBL) return fabs(d1);
        T q = u * u * r;
        return fabs(d1 * (T(1) - fg[l] * v * v) + q * T(2) * fg[l] * v);
    }

    // a(u): one branch-free form for every supported potential (linear,
    // powers 1..3, dead zone, Buckley-Leverett cubic, squared ramp); other
    // powers take the pow branch
    __device__ __forceinline__ T a(T u) const
    {
        if (ppow) return power_potential<T>(a0, a1, am, u);
        const T v = fmin(fmax((pabs ? fabs(u) : u) - pu0, plo), phi);
        const T g = v * (pc1 + v * (pc2 + v * pc3));
        return pabs ? copysign(g, u) : g;
    }

    // kappa(u) = a'(u) of the same forms (the pow branch: p0 p u^(p-1)); zero
    // where the clamp of the unified form is active
    __device__ __forceinline__ T kappa(T u) const
    {
        if (ppow) return a0 * a1 * power_potential<T>(T(1), a1 - T(1), am - 1, u);
        const T w = (pabs ? fabs(u) : u) - pu0;
        if (!(w > plo && w < phi)) return T(0);
        return pc1 + w * (T(2) * pc2 + w * (T(3) * pc3));
    }

    // max of |f_l'| over [min(x,y), max(x,y)]: end points and interior local
    // maxima of |f_l'|
    __device__ __forceinline__ T alpha_int(int l, T x, T y) const
    {
        T lo = fmin(x, y), hi = fmax(x, y);
        T r = fmax(adf(l, lo), adf(l, hi));
        const int n = nc[l];
        for (int c = 0; c < n; c++) {
            const T cv = (T)ip->crit[l][c];
            if (cv >= lo && cv <= hi) r = fmax(r, adf(l, cv));
        }
        return r;
    }
};

// max / min that propagate NaN (IEEE maximum / minimum): for FP32 they map to
// v_maximum3 / v_minimum3 and, unlike fmax / fmin, need no quieting of
// operands loaded from memory; a NaN operand makes the result NaN, which the
// non-finite check of the update then reports
template <class T>
__device__ __forceinline__ T vmax(T a, T b)
{
    if constexpr (sizeof(T) == 4) return __builtin_elementwise_maximum(a, b);
    else return fmax(a, b);
}
template <class T>
__device__ __forceinline__ T vmin(T a, T b)
{
    if constexpr (sizeof(T) == 4) return __builtin_elementwise_minimum(a, b);
    else return fmin(a, b);
}

// largest t in [0,1] with every low-order state + t * correction in bounds,
// given the common correction magnitude s and the smallest gap to the bound
// the states move towards (selects only; s == 0 gives 0 * inf -> NaN, which
// fmin turns into 1; a gap of s or more may give 1 - ulp, which only
// shortens the correction)
template <class T>
__device__ __forceinline__ T theta_from_gap(T gap, T s)
{
    return fmin(fmax(gap, T(0)) * fast_rcp(s), T(1));
}

// theta d of a limited correction d whose states move by k theta d (k > 0):
// theta = min(1, max(gap, 0) / (k |d|)) gives
//   theta d = sign(d) min(|d|, max(gap, 0) / k),
// evaluated with ik = 1/k of the block, so no reciprocal per item (the gap
// scaled by ik is clamped into [0, |d|], then takes the sign of d).  The
// states then move by at most gap (k ik), i.e. within an ulp of the gap.
// k = 0 (no step) gives 0 or |d|; a stage without a step does not use it.
template <class T>
__device__ __forceinline__ T limited_part(T gap, T d, T ik)
{
    T m;
    if constexpr (sizeof(T) == 4) m = __builtin_amdgcn_fmed3f(gap * ik, 0.0f, __builtin_fabsf(d));
    else m = fmin(fmax(gap * ik, T(0)), fabs(d));
    return copysign(m, d);
}

// smallest distance to the bound that a correction of sign(s) moves the
// states z+ (moved by +s) and z- (moved by -s) towards (only the sign of s
// is used: any positive multiple of the correction will do)
template <class T>
__device__ __forceinline__ T gap2(T s, T zp, T zm, T umin, T umax)
{
    const bool pos = s > T(0);
    const T up = pos ? zp : zm, down = pos ? zm : zp;  // the state moving up, the one moving down
    return fmin(umax - up, down - umin);
}

// same for two states moved by +s (a1, a2) and two moved by -s (b1, b2)
template <class T>
__device__ __forceinline__ T gap4(T s, T a1, T a2, T b1, T b2, T umin, T umax)
{
    const bool pos = s > T(0);
    const T top = pos ? vmax(a1, a2) : vmax(b1, b2), bottom = pos ? vmin(b1, b2) : vmin(a1, a2);
    return fmin(umax - top, bottom - umin);
}

// v clamped to [lo, hi] (lo <= hi); FP32 uses the median of three, one
// instruction that needs no quieting of its operands
template <class T>
__device__ __forceinline__ T clampb(T v, T lo, T hi)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_fmed3f(v, lo, hi);
    else return fmin(fmax(v, lo), hi);
}

// Tile geometry.  Axes beyond D have extent 1 and no halo.
template <int D, int TX, int TY, int TZ, int HL>
struct Geo {
    static constexpr int T0 = TX, T1 = D >= 2 ? TY : 1, T2 = D >= 3 ? TZ : 1;
    static constexpr int H0 = HL, H1 = D >= 2 ? HL : 0, H2 = D >= 3 ? HL : 0;
    static constexpr int R0 = T0 + 2 * H0, R1 = T1 + 2 * H1, R2 = T2 + 2 * H2;
    // the half grid holds, along every axis, the half indices [2h-3, 2h+2t+1]:
    // the tile's points, the reach of their 5-point stencils, the centres of
    // one more cell on each side and the outer face points of those cells
    // (the centre inversion and the potentials of the outermost cells read
    // them); the averages of the region reach further only for the
    // smoothness indicators.  LDS is ample in 1D and 2D: in 2D the held
    // range starts one point earlier, on a cell's first point (even
    // positions keep a cell's two points in one aligned pair), and in 1D the
    // half grid spans the whole region, so that staging needs no checks.
    static constexpr int AL = D == 2 ? 1 : 0;
    static constexpr int HB0 = D == 1 ? 0 : 2 * H0 - 3 - AL, HB1 = D >= 2 ? 2 * H1 - 3 - AL : 0,
                         HB2 = D >= 3 ? 2 * H2 - 3 : 0;
    static constexpr int G0 = D == 1 ? 2 * R0 : 2 * T0 + 5 + AL, G1 = D >= 2 ? 2 * T1 + 5 + AL : 1,
                         G2 = D >= 3 ? 2 * T2 + 5 : 1;
    static constexpr int NCELL = R0 * R1 * R2;
    static constexpr int NHG = G0 * G1 * G2;
    static constexpr int NTILE = T0 * T1 * T2;
    static constexpr int t(int l) { return l == 0 ? T0 : (l == 1 ? T1 : T2); }
    static constexpr int h(int l) { return l == 0 ? H0 : (l == 1 ? H1 : H2); }
    // per-direction line arrays: faces (extent t+3 along l), cells (t+2)
    static constexpr int nface(int l) { return l < D ? (t(l) + 3) * (NTILE / t(l)) : 0; }
    static constexpr int ncl(int l) { return l < D ? (t(l) + 2) * (NTILE / t(l)) : 0; }
    static constexpr int face_off(int l) { return l == 0 ? 0 : (l == 1 ? nface(0) : nface(0) + nface(1)); }
    static constexpr int cell_off(int l) { return l == 0 ? 0 : (l == 1 ? ncl(0) : ncl(0) + ncl(1)); }
    static constexpr int NFACE = nface(0) + nface(1) + nface(2);
    static constexpr int NCL = ncl(0) + ncl(1) + ncl(2);
    // SI boxes of direction l: s_l on [h-1, h+t+1) along l, s~_l on
    // [h-2, h+t+2) along l, both on [h, h+t+1) across (the cells that the
    // tile's points, faces and potentials blend with)
    static constexpr int sbe(int l, int a) { return a >= D ? 1 : (a == l ? t(a) + 2 : t(a) + 1); }
    static constexpr int ste(int l, int a) { return a >= D ? 1 : (a == l ? t(a) + 4 : t(a) + 1); }
    static constexpr int nsb(int l) { return l < D ? sbe(l, 0) * sbe(l, 1) * sbe(l, 2) : 0; }
    static constexpr int nst(int l) { return l < D ? ste(l, 0) * ste(l, 1) * ste(l, 2) : 0; }
    static constexpr int sb_off(int l) { return l == 0 ? 0 : (l == 1 ? nsb(0) : nsb(0) + nsb(1)); }
    static constexpr int st_off(int l) { return l == 0 ? 0 : (l == 1 ? nst(0) : nst(0) + nst(1)); }
    static constexpr int NSB = nsb(0) + nsb(1) + nsb(2);
    static constexpr int NST = nst(0) + nst(1) + nst(2);
    __device__ static __forceinline__ int cidx(int x, int y, int z) { return x + R0 * (y + R1 * z); }
    // half-grid point (x, y, z) in region half indices
    __device__ static __forceinline__ int hidx(int x, int y, int z)
    {
        return (x - HB0) + G0 * ((y - HB1) + G1 * (z - HB2));
    }
    // some half-grid point of region cell (x, y, z) is held
    __device__ static __forceinline__ bool cell_held(int x, int y, int z)
    {
        if (D == 1) return true;
        return (unsigned)(x - (H0 - 2)) <= (unsigned)T0 + 2 && (D < 2 || (unsigned)(y - (H1 - 2)) <= (unsigned)T1 + 2) &&
               (D < 3 || (unsigned)(z - (H2 - 2)) <= (unsigned)T2 + 2);
    }
    // the half-grid point (x, y, z) is held
    __device__ static __forceinline__ bool held(int x, int y, int z)
    {
        if (D == 1) return true;
        return (unsigned)(x - HB0) < (unsigned)G0 && (D < 2 || (unsigned)(y - HB1) < (unsigned)G1) &&
               (D < 3 || (unsigned)(z - HB2) < (unsigned)G2);
    }
};

// Loop over a box of extents E0 x E1 x E2, x fastest, spread over NT threads.
template <int E0, int E1, int E2, int NT, class F>
__device__ __forceinline__ void box_loop(F &&fn)
{
    constexpr int N = E0 * E1 * E2;
    for (int idx = (int)threadIdx.x; idx < N; idx += NT) {
        int x = idx % E0;
        int r = idx / E0;
        int y = r % E1;
        int z = r / E1;
        fn(x, y, z);
    }
}

// box_loop with the thread's round c in [0, ceil(E0 E1 E2 / NT)) passed on
// (unrolled, so that per-round registers are indexed at compile time)
template <int E0, int E1, int E2, int NT, class F>
__device__ __forceinline__ void box_loop_r(F &&fn)
{
    constexpr int N = E0 * E1 * E2, C = (N + NT - 1) / NT;
#pragma unroll
    for (int c = 0; c < C; c++) {
        const int idx = (int)threadIdx.x + c * NT;
        if (N % NT == 0 || idx < N) {
            const int x = idx % E0, r = idx / E0;
            fn(x, r % E1, r / E1, c);
        }
    }
}

__device__ __forceinline__ int wrap_index(int v, int n)
{
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// half-shift mask of the DoF kind z (zeta order of Sec. 4)
template <int D>
__device__ __forceinline__ constexpr int zeta_mask(int z)
{
    return D == 3 ? (z == 3 ? 4 : (z == 4 ? 3 : z)) : z;
}

// The stage's combination of its forward-Euler result v with X0, X1 and the
// stage input vin (kComb*); the blend is written so that its weights sum to
// one exactly.
template <class T>
__device__ __forceinline__ T stage_combine(const StageParams<T> &p, T v, T x0, T x1, T vin)
{
    if (p.mode == kCombBlend) return x0 + p.w * (v - x0);
    if (p.mode == kCombSum) return ((p.c0 * x0 + p.c1 * x1) + p.cin * vin) + p.w * v;
    return v;
}

// Wave-wide maximum of an unsigned value in six DPP steps (shifts within rows
// of 16 lanes, then two row broadcasts), read from the last lane.  Every lane
// of the wave must be active; lanes shifted in from outside a row read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_umax_step(unsigned v)
{
    return max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true));
}
__device__ __forceinline__ unsigned wave_umax(unsigned v)
{
    v = dpp_umax_step<0x111, 0xf>(v);   // row_shr:1
    v = dpp_umax_step<0x112, 0xf>(v);   // row_shr:2
    v = dpp_umax_step<0x114, 0xf>(v);   // row_shr:4
    v = dpp_umax_step<0x118, 0xf>(v);   // row_shr:8
    v = dpp_umax_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v = dpp_umax_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// order-preserving map of floats to unsigned integers (non-NaN values)
__device__ __forceinline__ unsigned ordered_key32(float v)
{
    const unsigned b = __float_as_uint(v);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ordered_value32(unsigned k)
{
    return __uint_as_float((k >> 31) ? (k & 0x7fffffffu) : ~k);
}

// Wave-wide min and max of the averages the threads of a wave wrote, stored
// as ordered keys by the wave's first lane into its slot pair of the block's
// work item (no atomics: the finalize kernel reduces the slots of each
// instance; the CFL wave speed of the next step is evaluated from them when
// every flux has a convex |f'|).  Every lane of the wave must be active.
template <class T>
__device__ __forceinline__ void minmax_slot(unsigned long long *mm, int item, T lo, T hi)
{
    if constexpr (sizeof(T) == 4) {
        const float l = ordered_value32(~wave_umax(~ordered_key32(lo)));
        const float h = ordered_value32(wave_umax(ordered_key32(hi)));
        lo = l;
        hi = h;
    } else {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, o));
            hi = fmax(hi, __shfl_xor(hi, o));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long *slot = mm + 2 * (item * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6));
        slot[0] = ordered_key((double)lo);
        slot[1] = ordered_key((double)hi);
    }
}

// Wave-wide max of a non-negative double, then one atomic per wave; a wave
// whose lanes all hold 0 (the usual case: no safeguard clamp) skips both.
__device__ __forceinline__ void atomic_max_wave(unsigned long long *dst, double v)
{
    if (!__any(v > 0.0)) return;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

// Same for a non-negative value of the kernel's precision (FP32: the bit
// patterns of non-negative floats order like the values).
template <class T>
__device__ __forceinline__ void atomic_max_wave_t(unsigned long long *dst, T v)
{
    if constexpr (sizeof(T) == 4) {
        if (!__any(v > T(0))) return;
        const unsigned m = wave_umax(__float_as_uint(v));
        if ((threadIdx.x & 63) == 0 && m != 0u)
            atomicMax(dst, (unsigned long long)__double_as_longlong((double)__uint_as_float(m)));
    } else {
        atomic_max_wave(dst, (double)v);
    }
}

// a(u) is staged per half-grid point (more LDS, fewer evaluations) in 2D
// and 3D; 1D tiles evaluate it where it is used, which keeps their LDS
// under 32 KB (five workgroups per CU instead of four; the App. A form
// reads kappa, not a, anyway)
template <int D>
constexpr bool stage_staged_a()
{
    return D >= 2;
}

// elements of the shared face arrays (fluxes, and u^{L,+-} when limiting) or
// of the raw smoothness indicators, whichever is larger
template <int D, bool LIM, bool SI, int TX, int TY, int TZ>
constexpr int stage_face_area()
{
    using G = Geo<D, TX, TY, TZ, SI ? 3 : 2>;
    const int f = G::NFACE * (LIM ? 3 : 1), st = SI ? G::NST : 0;
    return f > st ? f : st;
}

// QF: every flux is c1 u + c2 u^2 (evaluated in closed form, no branches on
// the flux kind); CNT (with LIM): the limiter-counting form, which also adds
// the own faces and potentials limited to p.lact
template <int D, class T, bool LIM, bool SI, bool QF, int TX, int TY, int TZ, int NT, bool CNT = false>
__global__ void __launch_bounds__(NT) stage_kernel(StageParams<T> p)
{
    constexpr int HL = SI ? 3 : 2;
    using G = Geo<D, TX, TY, TZ, HL>;
    constexpr int NB = 1 << D;

    __shared__ T ub[G::NCELL];
    __shared__ T hg[G::NHG];
    constexpr bool PA = stage_staged_a<D>();
    __shared__ T ah[PA ? G::NHG : 1];          // a(u) at the half-grid points
    // face arrays of phases D1-D3; the raw indicators s~_l of phase B' share
    // their storage (they are consumed before phase C)
    __shared__ T fla[stage_face_area<D, LIM, SI, TX, TY, TZ>()];
    T *const fl = fla;                         // flux used in the update, per face
    T *const ulp = fla + G::NFACE;             // u^{L,+} of the left cell of a face
    T *const ulm = fla + 2 * G::NFACE;         // u^{L,-} of the right cell of a face
    T *const stl = fla;                        // raw indicator s~_l
    __shared__ T pc[G::NCL];                   // potential used in the update, per cell
    __shared__ T ssm[SI ? G::NSB : 1];         // smoothed indicator s_l

    // block -> (instance, tile); consecutive logical tiles on the same XCD
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int4 wk = p.work[logical];
    // the instance's parameters: scalar loads (see Phys::load)
    const auto I = as_constant(&p.inst[wk.x]);
    const int n0 = I->n[0], n1 = I->n[1], n2 = I->n[2];
    const int tx = wk.y, ty = wk.z, tz = wk.w;
    const int ox = tx * G::T0, oy = ty * G::T1, oz = tz * G::T2;
    const long long kst = I->kstride;
    const T *__restrict__ in = p.in + I->off;
    const T *__restrict__ un = p.un + I->off;
    const T *__restrict__ x1 = p.x1 ? p.x1 + I->off : nullptr;
    T *__restrict__ out = p.out + I->off;
    const bool residual = p.stage == kStageRHS;
    const double dtd = p.st[wk.x].dt;
    // the 1D variant without double conservation (App. A)
    const bool nodc = D == 1 && I->nodc != 0;
    // PA: a(u) at the half-grid points is evaluated once, where the point is
    // staged (App. A's form uses kappa instead)
    const bool pa = PA && !nodc;
    // Non-periodic ends (1D, 2D): a half-grid point on or beyond an open end
    // (global half indices q0, q1) takes a boundary value -- the Dirichlet
    // value of the first Dirichlet end among those it lies on or beyond, else
    // (outflow) the mean average of the domain cells around the point moved
    // onto the boundary; the stored point values on the high ends are not
    // evolved (Dirichlet value, or the input passed through).
    const bool open = D <= 2 && (I->bc[0][0] != 0 || (D == 2 && I->bc[1][0] != 0));
    auto ends = [&](int q0, int q1) -> int {
        int m = 0;
        if (I->bc[0][0] != 0 && (q0 <= -1 || q0 >= 2 * n0 - 1)) m |= 1;
        if (D == 2 && I->bc[1][0] != 0 && (q1 <= -1 || q1 >= 2 * n1 - 1)) m |= 2;
        return m;
    };
    auto bc_point = [&](int q0, int q1, int m) -> T {
#pragma unroll
        for (int l = 0; l < 2; l++) {
            const int q = l == 0 ? q0 : q1, side = q <= -1 ? 0 : 1;
            if ((m >> l & 1) && I->bc[l][side] == 1) return (T)I->bcv[l][side];
        }
        int lo[2], hi[2];
#pragma unroll
        for (int l = 0; l < 2; l++) {
            const int q = l == 0 ? q0 : q1, nl = l == 0 ? n0 : n1;
            if (m >> l & 1) lo[l] = hi[l] = q <= -1 ? 0 : nl - 1;
            else if (q & 1) { lo[l] = (q - 1) >> 1; hi[l] = lo[l] + 1; }
            else lo[l] = hi[l] = q >> 1;
        }
        T sum = T(0);
        int cnt = 0;
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                sum += in[wrap_index(i, n0) + (long long)n0 * wrap_index(j, n1)];
                cnt++;
            }
        return sum / T(cnt);
    };

    const T inf = __builtin_huge_val();
    T vlo = inf, vhi = -inf;  // min / max of the averages written
    if (!residual && dtd == 0.0) {
        // the instance has reached its end time: the stage leaves it unchanged
        box_loop<G::T0, G::T1, G::T2, NT>([&](int i, int j, int k) {
            if (ox + i >= n0 || oy + j >= n1 || oz + k >= n2) return;
            long long gi = (ox + i) + (long long)n0 * ((oy + j) + (long long)n1 * (oz + k));
            for (int z = 0; z < NB; z++) out[z * kst + gi] = in[z * kst + gi];
            vlo = fmin(vlo, in[gi]);
            vhi = fmax(vhi, in[gi]);
        });
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
        return;
    }

    Phys<T> P;
    P.load(I, D);
    // a(u) at half-grid point h holding u
    auto a_at = [&](int h, T u) -> T {
        if constexpr (PA) return ah[h];
        else return P.a(u);
    };
    T qc1[3], qc2[3];  // QF: f_l = qc1 u + qc2 u^2
#pragma unroll
    for (int l = 0; l < 3; l++) {
        qc1[l] = I->fk[l] == kFLinear ? (T)I->fp0[l] : T(0);
        qc2[l] = I->fk[l] == kFQuad ? (T)I->fp0[l] : T(0);
    }
    auto Ff = [&](int l, T u) -> T {
        if constexpr (QF) return u * (qc1[l] + qc2[l] * u);
        else return P.f(l, u);
    };
    auto Fg = [&](int l, T u) -> T {
        if constexpr (QF) return fabs(qc1[l] + T(2) * qc2[l] * u);
        else return P.adf(l, u);
    };
    auto Fint = [&](int l, T x, T y) -> T {  // max |f_l'| over [min(x,y), max(x,y)]
        if constexpr (QF) return fmax(Fg(l, x), Fg(l, y));
        else return P.alpha_int(l, x, y);
    };
    const T dt = (T)dtd * p.dts;
    const T K = T(2 * D);
    T idx1[3], idx2[3], i6dx[3], mu[3], nu[3];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        idx1[l] = (T)I->idx1[l];
        idx2[l] = (T)I->idx2[l];
        i6dx[l] = (T)I->i6dx[l];
        mu[l] = (T)p.st[wk.x].mu[l] * p.dts;
        nu[l] = (T)p.st[wk.x].nu[l] * p.dts;
    }

    // ---- A: stage tile + halo (averages -> ub, point values -> half grid)
    box_loop<G::R0, G::R1, G::R2, NT>([&](int x, int y, int z) {
        if (open) {
            const int c0 = ox + x - G::H0, c1 = D >= 2 ? oy + y - G::H1 : 0;
            const long long gi = wrap_index(c0, n0) + (long long)n0 * (D >= 2 ? wrap_index(c1, n1) : 0);
#pragma unroll
            for (int zk = 0; zk < NB; zk++) {
                const int hx = 2 * x + (zk & 1), hy = 2 * y + ((zk >> 1) & 1);
                if (zk != 0 && !G::held(hx, hy, 0)) continue;
                const int q0 = 2 * c0 + (zk & 1), q1 = 2 * c1 + ((zk >> 1) & 1);
                const int m = ends(q0, q1);
                const T v = m ? bc_point(q0, q1, m) : in[zk * kst + gi];
                if (zk == 0) {
                    ub[G::cidx(x, y, 0)] = v;
                } else {
                    hg[G::hidx(hx, hy, 0)] = v;
                    if (pa) ah[G::hidx(hx, hy, 0)] = P.a(v);
                }
            }
            return;
        }
        int gx = wrap_index(ox + x - G::H0, n0);
        int gy = D >= 2 ? wrap_index(oy + y - G::H1, n1) : 0;
        int gz = D >= 3 ? wrap_index(oz + z - G::H2, n2) : 0;
        long long gi = gx + (long long)n0 * (gy + (long long)n1 * gz);
        ub[G::cidx(x, y, z)] = in[gi];
        if (!G::cell_held(x, y, z)) return;
        // all loads of the cell first (one wait), then the held points
        T v[NB];
#pragma unroll
        for (int zk = 1; zk < NB; zk++) v[zk] = in[zk * kst + gi];
#pragma unroll
        for (int zk = 1; zk < NB; zk++) {
            const int m = zeta_mask<D>(zk);
            const int hx = 2 * x + (m & 1), hy = 2 * y + ((m >> 1) & 1), hz = 2 * z + ((m >> 2) & 1);
            if (!G::held(hx, hy, hz)) continue;
            hg[G::hidx(hx, hy, hz)] = v[zk];
            if (pa) ah[G::hidx(hx, hy, hz)] = P.a(v[zk]);
        }
    });
    // U^n of the own DoFs for the stage's combination, loaded after the
    // stage's own loads and used in phases C and D3: the load latency overlaps
    // phases B to D2 instead of stalling every store (cells outside the grid
    // read cell 0)
    constexpr int NRND = (G::T0 * G::T1 * G::T2 + NT - 1) / NT;
    T unp[NRND][NB];
    box_loop_r<G::T0, G::T1, G::T2, NT>([&](int i, int j, int k, int c) {
        const bool own = ox + i < n0 && oy + j < n1 && oz + k < n2;
        const long long gi = own ? (ox + i) + (long long)n0 * ((oy + j) + (long long)n1 * (oz + k)) : 0;
#pragma unroll
        for (int zk = 0; zk < NB; zk++) unp[c][zk] = un[zk * kst + gi];
    });
    // the stage's combination (stage_combine) with the prefetched U^n; X1,
    // read by summing stages only, is loaded inside their branch
    auto combine_g = [&](T v, T x0, int z, long long g, T vin) -> T {
        if (p.mode == kCombSum) return ((p.c0 * x0 + p.c1 * x1[z * kst + g]) + p.cin * vin) + p.w * v;
        if (p.mode == kCombBlend) return x0 + p.w * (v - x0);
        return v;
    };
    __syncthreads();

    // ---- B: cell centres on [h-1, h+t+1)^D (inverse tensor Simpson)
    {
        constexpr int E0 = G::T0 + 2, E1 = D >= 2 ? G::T1 + 2 : 1, E2 = D >= 3 ? G::T2 + 2 : 1;
        constexpr int L0 = G::H0 - 1, L1 = D >= 2 ? G::H1 - 1 : 0, L2 = D >= 3 ? G::H2 - 1 : 0;
        constexpr T S = D == 1 ? T(6) : (D == 2 ? T(36) : T(216));
        constexpr T iW = D == 1 ? T(0.25) : (D == 2 ? T(0.0625) : T(0.015625));
        box_loop<E0, E1, E2, NT>([&](int i, int j, int k) {
            const int x = i + L0, y = j + L1, z = k + L2;
            if (open) {
                const int q0 = 2 * (ox + x - G::H0), q1 = D >= 2 ? 2 * (oy + y - G::H1) : 0;
                const int m = ends(q0, q1);
                if (m) {  // ghost centre
                    const T v = bc_point(q0, q1, m);
                    hg[G::hidx(2 * x, 2 * y, 0)] = v;
                    if (pa) ah[G::hidx(2 * x, 2 * y, 0)] = P.a(v);
                    return;
                }
            }
            T acc = S * ub[G::cidx(x, y, z)];
#pragma unroll
            for (int oz = (D >= 3 ? -1 : 0); oz <= (D >= 3 ? 1 : 0); oz++)
#pragma unroll
                for (int oy = (D >= 2 ? -1 : 0); oy <= (D >= 2 ? 1 : 0); oy++)
#pragma unroll
                    for (int oxx = -1; oxx <= 1; oxx++) {
                        if (oxx == 0 && oy == 0 && oz == 0) continue;
                        const T w = T((oxx == 0 ? 4 : 1) * (D >= 2 && oy == 0 ? 4 : 1) * (D >= 3 && oz == 0 ? 4 : 1));
                        acc -= w * hg[G::hidx(2 * x + oxx, 2 * y + oy, 2 * z + oz)];
                    }
            const T v = acc * iW;
            hg[G::hidx(2 * x, 2 * y, 2 * z)] = v;
            if (pa) ah[G::hidx(2 * x, 2 * y, 2 * z)] = P.a(v);
        });
    }

    // ---- B': smoothness indicators (Sec. 5.1.3, direction by direction)
    if constexpr (SI) {
#pragma unroll
        for (int l = 0; l < D; l++) {
            const int e0 = G::ste(l, 0), e1 = G::ste(l, 1), ne = G::nst(l);
            for (int id = (int)threadIdx.x; id < ne; id += NT) {
                int i = id % e0, r = id / e0, j = r % e1, k = r / e1;
                int x = i + G::H0 - 2 * (l == 0), y = j + G::H1 - 2 * (l == 1), z = k + G::H2 - 2 * (l == 2);
                const int sx = l == 0, sy = l == 1, sz = l == 2;
                T um = ub[G::cidx(x - sx, y - sy, z - sz)], u0 = ub[G::cidx(x, y, z)], up = ub[G::cidx(x + sx, y + sy, z + sz)];
                stl[G::st_off(l) + id] = fabs(um - T(2) * u0 + up) / (fabs(um) + T(2) * fabs(u0) + fabs(up) + T(1e-13));
            }
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < D; l++) {
            const int e0 = G::ste(l, 0), e1 = G::ste(l, 1);
            const int b0 = G::sbe(l, 0), b1 = G::sbe(l, 1), nb = G::nsb(l);
            for (int id = (int)threadIdx.x; id < nb; id += NT) {
                const int i = id % b0, r = id / b0, j = r % b1, k = r / b1;
                const int si = i + (l == 0), sj = j + (l == 1), sk = k + (l == 2);
                const int st = l == 0 ? 1 : (l == 1 ? e0 : e0 * e1);
                const int c = G::st_off(l) + si + e0 * (sj + e1 * sk);
                ssm[G::sb_off(l) + id] = (stl[c - st] + T(4) * stl[c] + stl[c + st]) * T(1.0 / 6.0);
            }
        }
    }
    __syncthreads();

    // s_l at region cell (x, y, z) (inside the s box of direction l)
    auto s_at = [&](int l, int x, int y, int z) -> T {
        return ssm[G::sb_off(l) + (x - (G::H0 - (l == 0))) +
                   G::sbe(l, 0) * ((y - (G::H1 - (l == 1))) + G::sbe(l, 1) * (z - (G::H2 - (l == 2))))];
    };
    const T gam = (T)I->si_gamma;

    double clamp_mag = 0.0;
    bool bad = false;

    // ---- C: point values of the tile (Eq. 2d_af_dc, projection Sec. 5.1.2)
    box_loop_r<G::T0, G::T1, G::T2, NT>([&](int i, int j, int k, int c) {
        const bool own = ox + i < n0 && oy + j < n1 && oz + k < n2;
        const int x = i + G::H0, y = j + G::H1, z = k + G::H2;
        const long long gi = (ox + i) + (long long)n0 * ((oy + j) + (long long)n1 * (oz + k));
#pragma unroll
        for (int zk = 1; zk < NB; zk++) {
            const int m = zeta_mask<D>(zk);
            const int px = 2 * x + (m & 1), py = 2 * y + ((m >> 1) & 1), pz = 2 * z + ((m >> 2) & 1);
            const T u0 = hg[G::hidx(px, py, pz)];
            T R = T(0);
#pragma unroll
            for (int l = 0; l < D; l++) {
                const int sx = l == 0, sy = l == 1, sz = l == 2;
                T zz[5], ff[5];
                T alpha = T(0);
#pragma unroll
                for (int s = -2; s <= 2; s++) {
                    zz[s + 2] = hg[G::hidx(px + s * sx, py + s * sy, pz + s * sz)];
                    ff[s + 2] = Ff(l, zz[s + 2]);
                    alpha = fmax(alpha, Fg(l, zz[s + 2]));
                }
                T conv = -((ff[0] - T(8) * ff[1] + T(8) * ff[3] - ff[4]) +
                           alpha * (zz[0] - T(4) * zz[1] + T(6) * zz[2] - T(4) * zz[3] + zz[4])) * i6dx[l];
                if constexpr (SI) {
                    if (!residual) {
                        // low-order LLF right-hand side on the half grid; a cell
                        // average replaces a reconstructed centre
                        T nm = zz[1], np = zz[3];
                        if (m == (1 << l)) {
                            nm = ub[G::cidx(x, y, z)];
                            np = ub[G::cidx(x + sx, y + sy, z + sz)];
                        }
                        const T fm = Ff(l, nm), fp = Ff(l, np);
                        const T Fr = T(0.5) * (ff[2] + fp) - T(0.5) * alpha * (np - u0);
                        const T Fl = T(0.5) * (fm + ff[2]) - T(0.5) * alpha * (u0 - nm);
                        const T convL = -T(2) * idx1[l] * (Fr - Fl);
                        // mean of s_l over the cells whose closure contains the point
                        T ssum = T(0);
                        int cnt = 0;
#pragma unroll
                        for (int dz = 0; dz <= ((m >> 2) & 1); dz++)
#pragma unroll
                            for (int dy = 0; dy <= ((m >> 1) & 1); dy++)
#pragma unroll
                                for (int dxx = 0; dxx <= (m & 1); dxx++) {
                                    ssum += s_at(l, x + dxx, y + dy, z + dz);
                                    cnt++;
                                }
                        const T th = blend_exp(-gam * ssum / T(cnt));
                        conv = th * conv + (T(1) - th) * convL;
                    }
                }
                T d2;
                if (nodc) {
                    // App. A: (4/dx^2) sum_m kappa(z_m) (B z)_m, B = [0 0; 0 M] - [M 0; 0 0]
                    // with the 4x4 matrix M printed there (rows of B below)
                    const T b0 = T(-1.0 / 8.0) * zz[0] + T(1.0 / 6.0) * zz[1] - T(1.0 / 24.0) * zz[2];
                    const T b1 = T(1.0 / 6.0) * (zz[0] + zz[3]) + T(0.5) * zz[1] - T(5.0 / 6.0) * zz[2];
                    const T b2 = T(-1.0 / 8.0) * (zz[0] + zz[4]) + T(0.5) * (zz[1] + zz[3]) - T(0.75) * zz[2];
                    const T b3 = T(1.0 / 6.0) * (zz[1] + zz[4]) + T(0.5) * zz[3] - T(5.0 / 6.0) * zz[2];
                    const T b4 = T(-1.0 / 24.0) * zz[2] + T(1.0 / 6.0) * zz[3] - T(1.0 / 8.0) * zz[4];
                    d2 = T(4) * idx2[l] *
                         (((P.kappa(zz[0]) * b0 + P.kappa(zz[1]) * b1) + P.kappa(zz[2]) * b2) +
                          (P.kappa(zz[3]) * b3 + P.kappa(zz[4]) * b4));
                } else {
                    T aa[5];
#pragma unroll
                    for (int s = -2; s <= 2; s++) aa[s + 2] = a_at(G::hidx(px + s * sx, py + s * sy, pz + s * sz), zz[s + 2]);
                    d2 = (-(aa[0] + aa[4]) * T(1.0 / 3.0) + (aa[1] + aa[3]) * T(16.0 / 3.0) - T(10) * aa[2]) * idx2[l];
                }
                R += conv + d2;
            }
            if (!own) continue;
            // stored points on a high open end: right-hand side 0; a stage
            // writes the Dirichlet value or passes the input through
            const int me = open ? ends(2 * (ox + i) + (m & 1), 2 * (oy + j) + ((m >> 1) & 1)) : 0;
            if (residual) {
                out[zk * kst + gi] = me ? T(0) : R;
                continue;
            }
            T v = u0 + dt * R;
            if (me) {
                v = in[zk * kst + gi];
#pragma unroll
                for (int l = 1; l >= 0; l--)
                    if ((me >> l & 1) && I->bc[l][1] == 1) v = (T)I->bcv[l][1];
            }
            if (!isfinite(v)) bad = true;
            if constexpr (LIM) v = clampb(v, P.umin, P.umax);
            // (a stored boundary point combines with its stored input, not the
            // boundary value the stencils see)
            v = combine_g(v, unp[c][zk], zk, gi, me ? in[zk * kst + gi] : u0);
            if constexpr (LIM) v = clampb(v, P.umin, P.umax);
            out[zk * kst + gi] = v;
        }
    });

    unsigned nlf = 0, nlp = 0;  // limited own faces and potentials (p.lact)

    // ---- D1: per direction, faces and cells of the average update.
    // Face array of direction l: index f along l <-> left cell h_l - 2 + f,
    // f in [0, t_l + 3); other axes: own range.  Cell array: index c along l
    // <-> cell h_l - 1 + c, c in [0, t_l + 2).
    const bool use_si = SI && !residual;
#pragma unroll
    for (int l = 0; l < D; l++) {
        const int sx = l == 0, sy = l == 1, sz = l == 2;
        const int E0 = l == 0 ? G::T0 + 3 : G::T0, E1 = l == 1 ? G::T1 + 3 : G::T1, E2 = l == 2 ? G::T2 + 3 : G::T2;
        const int NF = E0 * E1 * E2;
        for (int id = (int)threadIdx.x; id < NF; id += NT) {
            const int i = id % E0, r = id / E0, j = r % E1, k = r / E1;
            const int fidx = l == 0 ? i : (l == 1 ? j : k);
            // left cell of the face in region coordinates
            const int x = i + G::H0 - 2 * sx, y = j + G::H1 - 2 * sy, z = k + G::H2 - 2 * sz;
            const bool need_hi = fidx >= 1 && fidx < G::t(l) + 2;
            if (!LIM && !need_hi) continue;
            const T ua = ub[G::cidx(x, y, z)], ubb = ub[G::cidx(x + sx, y + sy, z + sz)];
            T fL = T(0), up = T(0), um = T(0), dA = T(0);
            if (LIM || use_si) {
                const T fa = Ff(l, ua), fb = Ff(l, ubb);
                const T al = Fint(l, ua, ubb);
                fL = T(0.5) * (fa + fb) - T(0.5) * al * (ubb - ua);
                if constexpr (LIM) {
                    dA = (P.a(ubb) - P.a(ua)) * idx1[l];
                    const T Km = K * mu[l];
                    up = ua - Km * (fL - fa) + Km * dA;   // u^{L,+} of the left cell
                    um = ubb - Km * (fb - fL) - Km * dA;  // u^{L,-} of the right cell
                    const int fo = G::face_off(l) + id;
                    ulp[fo] = up;
                    ulm[fo] = um;
                }
            }
            if (!need_hi) continue;
            // high-order flux: Simpson average of f_l over the face (Sec. 4)
            T fH = T(0);
            {
                const int bx = 2 * x + sx, by = 2 * y + sy, bz = 2 * z + sz;
#pragma unroll
                for (int oz = (D >= 3 && l != 2 ? -1 : 0); oz <= (D >= 3 && l != 2 ? 1 : 0); oz++)
#pragma unroll
                    for (int oy = (D >= 2 && l != 1 ? -1 : 0); oy <= (D >= 2 && l != 1 ? 1 : 0); oy++)
#pragma unroll
                        for (int oxx = (l != 0 ? -1 : 0); oxx <= (l != 0 ? 1 : 0); oxx++) {
                            const T w = T((l != 0 && oxx == 0 ? 4 : 1) * (l != 1 && D >= 2 && oy == 0 ? 4 : 1) *
                                          (l != 2 && D >= 3 && oz == 0 ? 4 : 1));
                            fH += w * Ff(l, hg[G::hidx(bx + oxx, by + oy, bz + oz)]);
                        }
                fH *= D == 1 ? T(1) : (D == 2 ? T(1.0 / 6.0) : T(1.0 / 36.0));
            }
            if (use_si) {
                const T th = blend_exp(-gam * T(0.5) * (s_at(l, x, y, z) + s_at(l, x + sx, y + sy, z + sz)));
                fH = th * fH + (T(1) - th) * fL;
            }
            if (nodc) {
                // App. A: the diffusion flux kappa(u_{i+1/2}) D_c(u)_{i+1/2} joins
                // the convective one, F = fhat - g, with low-order part
                // fhat^L - (a(u_{i+1}) - a(u_i))/dx (the one the u^{L,+-} use)
                const int bx = 2 * x + 1;
                const T z0 = hg[G::hidx(bx - 2, 0, 0)], z1 = hg[G::hidx(bx - 1, 0, 0)], z2 = hg[G::hidx(bx, 0, 0)];
                const T z3 = hg[G::hidx(bx + 1, 0, 0)], z4 = hg[G::hidx(bx + 2, 0, 0)];
                fH -= P.kappa(z2) * ((z0 - z4) + T(8) * (z3 - z1)) * i6dx[l];
                fL -= dA;
            }
            T F = fH;
            if constexpr (LIM) {
                if (!residual) {
                    // each u^{L,+-} carries three corrections (factor 3K); with
                    // the App. A flux it carries one (factor K)
                    const T df = fH - fL;
                    const T s3 = (nodc ? T(1) : T(3)) * K * mu[l] * df;
                    // min(Theta(up, up - s3), Theta(um, um + s3)) with one reciprocal
                    const T gap = gap2<T>(s3, um, up, P.umin, P.umax);
                    const T th = theta_from_gap<T>(gap, (T)fabs(s3));
                    F = fL + th * df;
                    // the face c+1/2 of a tile cell c inside the instance
                    if (CNT && th < T(1) && fidx >= 2 && fidx < G::t(l) + 2 &&
                        ox + i - 2 * sx < n0 && oy + j - 2 * sy < n1 && oz + k - 2 * sz < n2)
                        nlf++;
                }
            }
            fl[G::face_off(l) + id] = F;
        }
    }
    __syncthreads();

    // ---- D2: per direction, cell-centred potentials (Prop. 2.1 and its
    // tensor form), limited with theta^d (Sec. 5.1.1 / 5.2.1)
#pragma unroll
    for (int l = 0; l < D; l++) {
        const int sx = l == 0, sy = l == 1, sz = l == 2;
        const int E0 = l == 0 ? G::T0 + 2 : G::T0, E1 = l == 1 ? G::T1 + 2 : G::T1, E2 = l == 2 ? G::T2 + 2 : G::T2;
        const int FE0 = l == 0 ? G::T0 + 3 : G::T0, FE1 = l == 1 ? G::T1 + 3 : G::T1;
        const int NC = E0 * E1 * E2;
        for (int id = (int)threadIdx.x; id < NC && !nodc; id += NT) {
            const int i = id % E0, r = id / E0, j = r % E1, k = r / E1;
            const int x = i + G::H0 - sx, y = j + G::H1 - sy, z = k + G::H2 - sz;
            T aH = T(0);
#pragma unroll
            for (int oz = (D >= 3 ? -1 : 0); oz <= (D >= 3 ? 1 : 0); oz++)
#pragma unroll
                for (int oy = (D >= 2 ? -1 : 0); oy <= (D >= 2 ? 1 : 0); oy++)
#pragma unroll
                    for (int oxx = -1; oxx <= 1; oxx++) {
                        const int ol = l == 0 ? oxx : (l == 1 ? oy : oz);
                        T w = ol == 0 ? T(8) : T(-1);
                        if (l != 0) w *= oxx == 0 ? T(4) : T(1);
                        if (l != 1 && D >= 2) w *= oy == 0 ? T(4) : T(1);
                        if (l != 2 && D >= 3) w *= oz == 0 ? T(4) : T(1);
                        const int h = G::hidx(2 * x + oxx, 2 * y + oy, 2 * z + oz);
                        aH += w * a_at(h, PA ? T(0) : hg[h]);
                    }
            aH *= D == 1 ? T(1.0 / 6.0) : (D == 2 ? T(1.0 / 36.0) : T(1.0 / 216.0));
            const T aL = P.a(ub[G::cidx(x, y, z)]);
            if (use_si) {
                const T th = blend_exp(-gam * s_at(l, x, y, z));
                aH = th * aH + (T(1) - th) * aL;
            }
            T Pv = aH;
            if constexpr (LIM) {
                if (!residual) {
                    // faces c-1/2 and c+1/2 in the face array of direction l
                    const int f0 = G::face_off(l) + i + FE0 * (j + FE1 * k);
                    const int step = l == 0 ? 1 : (l == 1 ? FE0 : FE0 * FE1);
                    const T pL = ulp[f0], mC = ulm[f0];                  // u^{L,+}_{c-1}, u^{L,-}_c
                    const T pC = ulp[f0 + step], mR = ulm[f0 + step];    // u^{L,+}_c, u^{L,-}_{c+1}
                    const T da = aH - aL;
                    const T s3 = T(3) * K * nu[l] * da;
                    // min of the four Theta's (pL, mR move by +s3; pC, mC by -s3)
                    const T gap = gap4<T>(s3, pL, mR, pC, mC, P.umin, P.umax);
                    const T th = theta_from_gap<T>(gap, (T)fabs(s3));
                    Pv = aL + th * da;
                    // a tile cell inside the instance
                    const int cl = l == 0 ? i : (l == 1 ? j : k);
                    if (CNT && th < T(1) && cl >= 1 && cl <= G::t(l) && ox + i - sx < n0 && oy + j - sy < n1 &&
                        oz + k - sz < n2)
                        nlp++;
                }
            }
            pc[G::cell_off(l) + id] = Pv;
        }
    }
    __syncthreads();

    // ---- D3: averages of the tile (Eq. multid_limited_average; with theta = 1
    // and no blending this is the high-order update of Eq. 2d_af_dc)
    box_loop_r<G::T0, G::T1, G::T2, NT>([&](int i, int j, int k, int c) {
        if (ox + i >= n0 || oy + j >= n1 || oz + k >= n2) return;
        const long long gi = (ox + i) + (long long)n0 * ((oy + j) + (long long)n1 * (oz + k));
        const T u = ub[G::cidx(i + G::H0, j + G::H1, k + G::H2)];
        T dF = T(0), dP = T(0), rF = T(0), rP = T(0);
#pragma unroll
        for (int l = 0; l < D; l++) {
            const int FE0 = l == 0 ? G::T0 + 3 : G::T0, FE1 = l == 1 ? G::T1 + 3 : G::T1;
            const int CE0 = l == 0 ? G::T0 + 2 : G::T0, CE1 = l == 1 ? G::T1 + 2 : G::T1;
            const int fstep = l == 0 ? 1 : (l == 1 ? FE0 : FE0 * FE1);
            const int cstep = l == 0 ? 1 : (l == 1 ? CE0 : CE0 * CE1);
            // face c+1/2 has face index t+2 along l for tile index t; cell c has index t+1
            const int fi = i + (l == 0 ? 2 : 0), fj = j + (l == 1 ? 2 : 0), fk = k + (l == 2 ? 2 : 0);
            const int ci = i + (l == 0 ? 1 : 0), cj = j + (l == 1 ? 1 : 0), ck = k + (l == 2 ? 1 : 0);
            const int fo = G::face_off(l) + fi + FE0 * (fj + FE1 * fk);
            const int co = G::cell_off(l) + ci + CE0 * (cj + CE1 * ck);
            const T Fp = fl[fo], Fm = fl[fo - fstep];
            dF += mu[l] * (Fp - Fm);
            rF += idx1[l] * (Fp - Fm);
            if (nodc) continue;  // the diffusion is part of the face flux
            const T Pm = pc[co - cstep], P0 = pc[co], Pp = pc[co + cstep];
            dP += nu[l] * (Pp - T(2) * P0 + Pm);
            rP += idx2[l] * (Pp - T(2) * P0 + Pm);
        }
        if (residual) {
            out[gi] = rP - rF;
            return;
        }
        T v = u - dF + dP;
        if (!isfinite(v)) bad = true;
        if constexpr (LIM) {
            T c = clampb(v, P.umin, P.umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(c - v));
            v = c;
        }
        v = combine_g(v, unp[c][0], 0, gi, u);
        if constexpr (LIM) {
            T c = clampb(v, P.umin, P.umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(c - v));
            v = c;
        }
        vlo = fmin(vlo, v);
        vhi = fmax(vhi, v);
        out[gi] = v;
    });
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave(&p.st[wk.x].clampmax, clamp_mag);
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
        if constexpr (LIM && CNT) {
            {
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    nlf += __shfl_xor(nlf, o);
                    nlp += __shfl_xor(nlp, o);
                }
                if ((threadIdx.x & 63) == 0) {
                    if (nlf) atomicAdd(&p.lact[2 * wk.x], (unsigned long long)nlf);
                    if (nlp) atomicAdd(&p.lact[2 * wk.x + 1], (unsigned long long)nlp);
                }
            }
        }
    }
}

// LDS bytes of a stage-kernel instantiation (used to skip oversized ones)
template <int D, class T, bool LIM, bool SI, int TX, int TY, int TZ>
constexpr long stage_lds_bytes()
{
    using G = Geo<D, TX, TY, TZ, SI ? 3 : 2>;
    return (long)sizeof(T) *
           (G::NCELL + (stage_staged_a<D>() ? 2 : 1) * G::NHG + stage_face_area<D, LIM, SI, TX, TY, TZ>() + G::NCL + (SI ? G::NSB : 1));
}

}  // namespace af4
