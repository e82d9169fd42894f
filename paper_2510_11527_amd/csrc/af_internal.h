// af_internal.h -- device-side data structures shared by the host runtime and
// the HIP kernels of the AF library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace af4 {

constexpr int kMaxCrit = 6;   // local maxima of |f_l'| kept per axis

// Per-instance parameters, device resident (one array entry per instance).
struct InstDev {
    int n[3];            // cells per axis (1 on unused axes)
    int tiles[3];        // tiles per axis for the selected stage variant
    long long ncell;     // n0*n1*n2
    long long off;       // element offset of the instance's DoF block
    long long kstride;   // elements between consecutive DoF kinds of the block
    double dx[3];
    int fk[3];           // af_flux_kind per axis
    double fp0[3], fp1[3];
    int ak;              // af_diff_kind
    int am;              // integer exponent of a power potential (0: use pow)
    double ap0, ap1;
    double umin, umax;
    double kmax;         // sup of kappa over [umin, umax]
    double cfl;
    int ncrit[3];
    double crit[3][kMaxCrit];  // interior local maxima of |f_l'|
    double adfc[3][kMaxCrit];  // |f_l'| at them
    double vol;          // cell volume
    double si_gamma;     // smoothness-indicator blending strength
    // potential in the unified form a(u) = s * v (pc1 + v (pc2 + v pc3)) with
    // v = min(max((pabs ? |u| : u) - pu0, plo), phi), s = sign(u) if pabs
    // else 1; ppow != 0: p0 * u^p1 by pow (powers other than 1..3)
    double pu0, plo, phi, pc1, pc2, pc3;
    int pabs, ppow;
    int wstart, wcount;  // the instance's range in the work list of the stage kernels
    int cstart, ccount;  // the instance's range of wave-speed chunks (and their slots)
    int nodc, pad0;      // 1: diffusion in the form of App. A (no double conservation; 1D)
    int bc[3][2];        // af_bc of the low / high end of each axis (both periodic or neither)
    double bcv[3][2];    // Dirichlet values
    double idx1[3];      // 1 / dx_l
    double idx2[3];      // 1 / dx_l^2
    double i6dx[3];      // 1 / (6 dx_l)
    // the same parameters rounded to FP32 on the host, for the FP32 kernels
    float f_umin, f_umax;
    float f_fp0[3];
    float f_pc[3];       // pc1, pc2, pc3
    float f_idx1[3], f_idx2[3], f_i6dx[3];
    float f_crit[3][kMaxCrit], f_adfc[3][kMaxCrit];
};

// Control block read by the time-step kernels (uploaded before each af_step).
struct StepCtl {
    double t_end;        // <= 0: no end time
    int prescribed;      // 1: dt from the prescribed array, 0: CFL
    int pad;
};

// Per-instance device scalars.
struct InstState {
    double dt;           // step of the current step
    double t;            // time at the end of the current step
    unsigned long long clampmax;  // bits of the largest average clamp (non-negative)
    unsigned int flags;  // bit 0: non-finite / divergent value produced
    unsigned int pad;
    long long steps;     // steps with dt > 0
    double mu[3];        // dt / dx_l of the current step
    double nu[3];        // dt / dx_l^2 of the current step
    float f_dt;          // dt, mu and nu rounded to FP32
    float f_mu[3], f_nu[3];
    float pad2;
};

// How a stage combines its forward-Euler result v (of step dts * dt) with
// other states (Shu-Osher form of the SSP Runge-Kutta methods):
//   kCombFE:    out = v
//   kCombBlend: out = X0 + w (v - X0)                  (a convex blend)
//   kCombSum:   out = c0 X0 + c1 X1 + cin IN + w v      (IN: the stage input)
enum : int { kCombFE = 0, kCombBlend = 1, kCombSum = 2 };
constexpr int kStageRHS = -1;  // StageParams::stage of a right-hand-side evaluation

template <class T>
struct StageParams {
    const InstDev *inst;
    const int4 *work;    // (instance, tile x, tile y, tile z) per block
    int nwork;
    const T *in;         // stage input U^(s-1)
    const T *un;         // X0 of the combination (U^n)
    const T *x1;         // X1 of a kCombSum stage, else null
    T *out;              // stage output (or right-hand side)
    InstState *st;
    int stage;           // kStageRHS: right-hand side only; else the stage's index in the step (1, 2, ...)
    int mode;            // kComb*
    T w, c0, c1, cin;    // combination weights
    T dts;               // the forward-Euler step of this stage is dts * dt
    // not null: every wave w of the block of work item k stores the ordered
    // keys (see ordered_key) of the min and max average it wrote to
    // mm[2 (k W + w)] and mm[2 (k W + w) + 1], W = waves per block
    unsigned long long *mm;
    // not null: the limiter-counting form of the generic kernel runs (one
    // tile variant per dimension, limiter on); each block adds its own faces
    // and cell potentials whose limiting parameter is below 1 to lact[2 i]
    // and lact[2 i + 1] of its instance i
    unsigned long long *lact;
};

// Read-only per-launch parameters are read through the constant address
// space so that uniform reads become scalar loads into SGPRs (the compiler
// does not prove that on its own once the kernel also writes memory).
template <class T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ const_ptr<T> as_constant(const T *p)
{
    return (const_ptr<T>)p;
}

// Order-preserving map of doubles to unsigned integers: a < b <=> key(a) <
// key(b) for non-NaN values, so that unsigned atomic min / max reduce doubles.
__host__ __device__ inline unsigned long long ordered_key(double v)
{
    unsigned long long b;
    __builtin_memcpy(&b, &v, sizeof b);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double ordered_value(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    __builtin_memcpy(&v, &b, sizeof v);
    return v;
}


}  // namespace af4
