// aux_kernels.hip -- time-step, norm and copy kernels of the AF library.
#include <cfloat>
#include <mutex>
#include "launch.h"
#include "stage_kernel.hpp"

namespace af4 {

// Max over the faces of the MPP CFL quantity alpha_l / dx_l + kappa_max /
// dx_l^2 (Eqs. 1d_av_pp_dt, multid_av_pp_dt), in FP64 from the stored
// averages.  A block covers whole grid rows, or a segment of one long row, of
// one instance (wave_chunk) and writes its maximum to its own slot (the bit
// pattern, ordered as integers for non-negative doubles); the finalize kernel
// reduces the slots of an instance.  No atomics: many small blocks keep the
// loads of the whole grid in flight.
//
// alpha_l of a face is the max of |f_l'| at its two averages and at the
// interior maxima of |f_l'| between them.  Since x -> x / dx_l + kappa_max /
// dx_l^2 is monotone, also after rounding, the max over faces is the max over
// the same |f_l'| values, grouped differently: |f_l'| of every average once
// (every cell is an end of a face along each axis), of every Dirichlet ghost
// value, and of every interior maximum lying inside some face's interval.
// Each value is evaluated exactly as per face, so the step is the same to
// the bit, with half the FP64 evaluations of |f'|.
template <class T, int D>
__global__ void __launch_bounds__(kWaveThreads) wavespeed_kernel(const InstDev *inst, const int2 *chunks, const T *U,
                                                        InstState *st, unsigned long long *slots)
{
    const int2 ch = chunks[blockIdx.x];
    const InstDev &I = inst[ch.x];
    Phys<double> P;
    P.load(I, D);
    double idx[3], kdx2[3];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        idx[l] = I.idx1[l];
        kdx2[l] = I.kmax * I.idx2[l];
    }
    // the interior maxima of |f_l'| and their terms |f_l'(c)| / dx_l +
    // kappa_max / dx_l^2, evaluated once per block
    __shared__ double scv[3][kMaxCrit], scw[3][kMaxCrit];
    if ((int)threadIdx.x < 3 * kMaxCrit) {
        const int l = threadIdx.x / kMaxCrit, c = threadIdx.x % kMaxCrit;
        if (l < D && c < P.nc[l]) {
            const double cv = I.crit[l][c];
            scv[l][c] = cv;
            scw[l][c] = P.adf(l, cv) * idx[l] + kdx2[l];
        }
    }
    __syncthreads();
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const WaveChunk wc = wave_chunk(n0, (long long)n1 * n2, ch.y);
    const T *u = U + I.off;
    const double big = 1e6 * fmax(fmax(fabs(I.umin), fabs(I.umax)), 1.0);
    // non-periodic ends (1D, 2D): the faces at the ends see a ghost cell whose
    // average is the Dirichlet value or (outflow) the boundary cell's average
    const bool open0 = D <= 2 && I.bc[0][0] != 0, open1 = D == 2 && I.bc[1][0] != 0;
    // a face between averages a and b beyond the cell's own term: the other
    // end if it is a ghost value (g), and the interior maxima in [min, max]
    // (the term is monotone in |f_l'|, so this is the per-face maximum)
    auto face = [&](int l, double a, double b, bool ghost, double w) -> double {
        if (ghost) w = fmax(w, P.adf(l, b) * idx[l] + kdx2[l]);
        const double lo = fmin(a, b), hi = fmax(a, b);
        for (int c = 0; c < P.nc[l]; c++)
            if (scv[l][c] >= lo && scv[l][c] <= hi) w = fmax(w, scw[l][c]);
        return w;
    };
    double w = 0.0;
    bool bad = false;
    const int width = wc.i1 - wc.i0;
    const int ncells = width * (wc.r1 - wc.r0);
    // the cell at row r (j, k: its y and z indices), column i
    auto cell = [&](int r, int i, int j, int k) {
        const long long row = (long long)n0 * r;
        // every load of the cell first
        const double uc = (double)u[row + i];
        double ux = (double)u[row + (i + 1 == n0 ? 0 : i + 1)];
        double uy = 0.0, uz = 0.0;
        if constexpr (D >= 2) uy = (double)u[(long long)n0 * ((j + 1 == n1 ? 0 : j + 1) + (long long)n1 * k) + i];
        if constexpr (D >= 3) uz = (double)u[(long long)n0 * (j + (long long)n1 * (k + 1 == n2 ? 0 : k + 1)) + i];
        if (!(fabs(uc) <= big)) bad = true;  // also catches NaN
        // the cell's own |f_l'| (every cell is an end of a face along each axis)
        w = fmax(w, P.adf(0, uc) * idx[0] + kdx2[0]);
        if constexpr (D >= 2) w = fmax(w, P.adf(1, uc) * idx[1] + kdx2[1]);
        if constexpr (D >= 3) w = fmax(w, P.adf(2, uc) * idx[2] + kdx2[2]);
        bool gx = false;
        if (open0 && i + 1 == n0) {
            gx = I.bc[0][1] == 1;
            ux = gx ? (double)(T)I.bcv[0][1] : uc;
        }
        if (open0 && i == 0) {
            const bool g = I.bc[0][0] == 1;
            w = face(0, uc, g ? (double)(T)I.bcv[0][0] : uc, g, w);
        }
        w = face(0, uc, ux, gx, w);
        if constexpr (D >= 2) {
            bool gy = false;
            if (open1 && j + 1 == n1) {
                gy = I.bc[1][1] == 1;
                uy = gy ? (double)(T)I.bcv[1][1] : uc;
            }
            if (open1 && j == 0) {
                const bool g = I.bc[1][0] == 1;
                w = face(1, uc, g ? (double)(T)I.bcv[1][0] : uc, g, w);
            }
            w = face(1, uc, uy, gy, w);
        }
        if constexpr (D >= 3) w = face(2, uc, uz, false, w);
    };
    // a chunk within one row (rows longer than a chunk, the usual case on
    // large grids) takes its row indices once per block, so its loop has no
    // integer division per cell
    if (wc.r1 - wc.r0 == 1) {
        const int j = wc.r0 % n1, k = wc.r0 / n1;
        for (int q = (int)threadIdx.x; q < width; q += kWaveThreads) cell(wc.r0, wc.i0 + q, j, k);
    } else {
        for (int q = (int)threadIdx.x; q < ncells; q += kWaveThreads) {
            const int r = wc.r0 + q / width;
            cell(r, wc.i0 + q % width, r % n1, r / n1);
        }
    }
    // the waves' maxima meet in LDS, then the block's goes to its slot
    constexpr int NW = kWaveThreads / 64;
    __shared__ double wb[NW];
    __shared__ int bb[NW];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) w = fmax(w, __shfl_xor(w, o));
    const bool wbad = __any(bad);
    if ((threadIdx.x & 63) == 0) {
        wb[threadIdx.x >> 6] = w;
        bb[threadIdx.x >> 6] = wbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wb[0];
        int anybad = bb[0];
#pragma unroll
        for (int q = 1; q < NW; q++) {
            m = fmax(m, wb[q]);
            anybad |= bb[q];
        }
        slots[blockIdx.x] = (unsigned long long)__double_as_longlong(m);
        if (anybad) atomicOr(&st[ch.x].flags, 1u);
    }
}

// One block per instance.  wslots != nullptr: the wave speed is the max of
// the instance's slots written by the wave-speed kernel.  mm != nullptr: the wave speed comes from the min /
// max average written by the previous step's last stage, reduced here from
// the per-wave slots of the instance's work items.  Valid when every |f_l'|
// is convex on the bounds interval (linear and quadratic fluxes, no interior
// maxima): then the maximum of alpha_int over all faces is
// max(|f_l'(min)|, |f_l'(max)|), evaluated in FP64 exactly as the wave-speed
// kernel evaluates it per face, so the time step is the same to the bit
// (min and max over the averages and, with open ends, the Dirichlet ghost
// values as stored).
// NT threads per block: 1024 where an instance has many slot pairs (a large
// grid has one pair per wave of 64 cells), else 256.
template <int NT>
__global__ void __launch_bounds__(NT) finalize_kernel(const InstDev *inst, const StepCtl *ctl, const double *dtp,
                                                      InstState *st, int dim, int prec, const unsigned long long *mm,
                                                      const unsigned long long *wslots, int waves_per_block)
{
    const int i = blockIdx.x;
    const InstDev &I = inst[i];
    // what the first lane needs, requested before the reduction so that the
    // load latencies overlap
    const double te = ctl->t_end, dpre = dtp[i], t0 = st[i].t, cfl = I.cfl;
    const int prescribed = ctl->prescribed;
    double w = 0.0;
    double lo = 0.0, hi = 0.0;
    if (wslots) {
        constexpr int NW = NT / 64;
        __shared__ unsigned long long kw[NW];
        unsigned long long b = 0ull;
        const int n = I.ccount;
        const unsigned long long *m = wslots + I.cstart;
        for (int k0 = threadIdx.x; k0 < n; k0 += 4 * NT) {
            unsigned long long v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) v[j] = k0 + NT * j < n ? m[k0 + NT * j] : 0ull;
#pragma unroll
            for (int j = 0; j < 4; j++) b = max(b, v[j]);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) b = max(b, (unsigned long long)__shfl_xor((long long)b, o));
        if ((threadIdx.x & 63) == 0) kw[threadIdx.x >> 6] = b;
        __syncthreads();
        b = kw[0];
#pragma unroll
        for (int q = 1; q < NW; q++) b = max(b, kw[q]);
        w = __longlong_as_double((long long)b);
    }
    if (mm) {
        // slot pairs of the instance: four independent loads in flight per
        // thread, then a wave and a block reduction
        constexpr int NW = NT / 64;
        __shared__ unsigned long long ka[NW], kb[NW];
        unsigned long long a = ~0ull, b = 0ull;
        const int n = I.wcount * waves_per_block;
        const ulonglong2 *m = (const ulonglong2 *)(mm + 2 * (long long)I.wstart * waves_per_block);
        for (int k0 = threadIdx.x; k0 < n; k0 += 4 * NT) {
            ulonglong2 v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) v[j] = k0 + NT * j < n ? m[k0 + NT * j] : make_ulonglong2(~0ull, 0ull);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                a = min(a, v[j].x);
                b = max(b, v[j].y);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            a = min(a, (unsigned long long)__shfl_xor((long long)a, o));
            b = max(b, (unsigned long long)__shfl_xor((long long)b, o));
        }
        if ((threadIdx.x & 63) == 0) {
            ka[threadIdx.x >> 6] = a;
            kb[threadIdx.x >> 6] = b;
        }
        __syncthreads();
        a = ka[0];
        b = kb[0];
#pragma unroll
        for (int q = 1; q < NW; q++) {
            a = min(a, ka[q]);
            b = max(b, kb[q]);
        }
        lo = ordered_value(a);
        hi = ordered_value(b);
    }
    if (threadIdx.x != 0) return;
    if (mm) {
        const double big = 1e6 * fmax(fmax(fabs(I.umin), fabs(I.umax)), 1.0);
        if (!(fabs(lo) <= big && fabs(hi) <= big)) st[i].flags |= 1u;  // divergent or non-finite
        // a Dirichlet end's ghost value (as stored) is an average of the end
        // faces too; outflow ghosts repeat a boundary average
        for (int l = 0; l < 2; l++)
            for (int e = 0; e < 2; e++)
                if (l < dim && I.bc[l][e] == 1) {
                    const double g = prec == 32 ? (double)(float)I.bcv[l][e] : I.bcv[l][e];
                    lo = fmin(lo, g);
                    hi = fmax(hi, g);
                }
        Phys<double> P;
        P.load(I, dim);
        // constant axes: Phys stays in registers
        w = fmax(0.0, P.alpha_int(0, lo, hi) * I.idx1[0] + I.kmax * I.idx2[0]);
        if (dim >= 2) w = fmax(w, P.alpha_int(1, lo, hi) * I.idx1[1] + I.kmax * I.idx2[1]);
        if (dim >= 3) w = fmax(w, P.alpha_int(2, lo, hi) * I.idx1[2] + I.kmax * I.idx2[2]);
    }
    double dt;
    if (prescribed) {
        dt = dpre;
    } else {
        dt = w > 0.0 ? cfl / w : (te > 0.0 ? te - t0 : 0.0);
    }
    if (te > 0.0) {
        const double rem = te - t0;
        if (rem <= 1e-12 * te) dt = 0.0;  // remainder is rounding, not a step
        else if (dt > rem) dt = rem;
    }
    st[i].dt = dt;
    st[i].t = t0 + dt;
    if (dt > 0.0) st[i].steps++;
    st[i].f_dt = (float)dt;
    for (int l = 0; l < 3; l++) {
        const double mu = dt * I.idx1[l], nu = dt * I.idx2[l];
        st[i].mu[l] = mu;
        st[i].nu[l] = nu;
        st[i].f_mu[l] = (float)mu;
        st[i].f_nu[l] = (float)nu;
    }
}

template <class T>
__global__ void copy_kernel(const T *__restrict__ src, T *__restrict__ dst, long long n)
{
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x)
        dst[i] = src[i];
}

// dst = src converted to D (round to nearest) over n values.
template <class S, class D>
__global__ void convert_kernel(const S *__restrict__ src, D *__restrict__ dst, long long n)
{
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x)
        dst[i] = (D)src[i];
}

// Block partials in fixed order, then one block reduces them in fixed order:
// the result is bitwise reproducible.  The three sums are compensated
// (Neumaier) in each thread's loop, in the block's pairwise tree and in the
// final pass over the block partials, so their rounding stays within a few
// units in the last place of the sum of magnitudes whatever the grid size.
__device__ __forceinline__ void neumaier_add(double &s, double &c, double v)
{
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

template <class T>
__global__ void __launch_bounds__(256) norms_kernel(const T *block, long long ncell, long long kstride, int nkinds,
                                                    double *partials)
{
    __shared__ double sh[9][256];
    __shared__ double shc[3][256];  // compensations of the three sums
    double s1 = 0, sa = 0, s2 = 0, c1 = 0, ca = 0, c2 = 0;
    double mx = 0, amin = DBL_MAX, amax = -DBL_MAX, pmin = DBL_MAX, pmax = -DBL_MAX, nbad = 0;
    for (long long c = threadIdx.x + (long long)blockIdx.x * 256; c < ncell; c += (long long)gridDim.x * 256) {
        const double u = (double)block[c];
        if (!isfinite(u)) nbad += 1;
        neumaier_add(s1, c1, u);
        neumaier_add(sa, ca, fabs(u));
        neumaier_add(s2, c2, u * u);
        mx = fmax(mx, fabs(u));
        amin = fmin(amin, u);
        amax = fmax(amax, u);
        for (int z = 1; z < nkinds; z++) {
            const double v = (double)block[z * kstride + c];
            if (!isfinite(v)) nbad += 1;
            pmin = fmin(pmin, v);
            pmax = fmax(pmax, v);
        }
    }
    double vals[9] = {s1, sa, s2, mx, amin, amax, pmin, pmax, nbad};
    for (int q = 0; q < 9; q++) sh[q][threadIdx.x] = vals[q];
    shc[0][threadIdx.x] = c1;
    shc[1][threadIdx.x] = ca;
    shc[2][threadIdx.x] = c2;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int t = threadIdx.x;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                neumaier_add(sh[q][t], shc[q][t], sh[q][t + w]);
                shc[q][t] += shc[q][t + w];
            }
            sh[3][t] = fmax(sh[3][t], sh[3][t + w]);
            sh[4][t] = fmin(sh[4][t], sh[4][t + w]);
            sh[5][t] = fmax(sh[5][t], sh[5][t + w]);
            sh[6][t] = fmin(sh[6][t], sh[6][t + w]);
            sh[7][t] = fmax(sh[7][t], sh[7][t + w]);
            sh[8][t] += sh[8][t + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) partials[blockIdx.x * 9 + threadIdx.x] = sh[threadIdx.x][0] + (threadIdx.x < 3 ? shc[threadIdx.x][0] : 0.0);
}

__global__ void norms_final_kernel(const double *partials, int nblocks, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double r[9] = {0, 0, 0, 0, DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX, 0};
    double c[3] = {0, 0, 0};
    for (int b = 0; b < nblocks; b++) {
        const double *p = partials + 9 * b;
        neumaier_add(r[0], c[0], p[0]);
        neumaier_add(r[1], c[1], p[1]);
        neumaier_add(r[2], c[2], p[2]);
        r[3] = fmax(r[3], p[3]);
        r[4] = fmin(r[4], p[4]);
        r[5] = fmax(r[5], p[5]);
        r[6] = fmin(r[6], p[6]);
        r[7] = fmax(r[7], p[7]);
        r[8] += p[8];
    }
    for (int q = 0; q < 3; q++) r[q] += c[q];
    for (int q = 0; q < 9; q++) out[q] = r[q];
}

hipError_t wavespeed_launch(int dim, int prec, const InstDev *inst, const int2 *chunks, int nchunks, const void *U,
                            InstState *st, unsigned long long *slots, hipStream_t s)
{
    if (nchunks <= 0) return hipSuccess;
    const dim3 g(nchunks), b(kWaveThreads);
    if (prec == 32) {
        const float *u = (const float *)U;
        if (dim == 1) hipLaunchKernelGGL((wavespeed_kernel<float, 1>), g, b, 0, s, inst, chunks, u, st, slots);
        else if (dim == 2) hipLaunchKernelGGL((wavespeed_kernel<float, 2>), g, b, 0, s, inst, chunks, u, st, slots);
        else hipLaunchKernelGGL((wavespeed_kernel<float, 3>), g, b, 0, s, inst, chunks, u, st, slots);
    } else {
        const double *u = (const double *)U;
        if (dim == 1) hipLaunchKernelGGL((wavespeed_kernel<double, 1>), g, b, 0, s, inst, chunks, u, st, slots);
        else if (dim == 2) hipLaunchKernelGGL((wavespeed_kernel<double, 2>), g, b, 0, s, inst, chunks, u, st, slots);
        else hipLaunchKernelGGL((wavespeed_kernel<double, 3>), g, b, 0, s, inst, chunks, u, st, slots);
    }
    return hipGetLastError();
}

hipError_t finalize_launch(int n_inst, const InstDev *inst, const StepCtl *ctl, const double *dtp, InstState *st,
                           int dim, int prec, const unsigned long long *mm, const unsigned long long *wslots,
                           int waves_per_block, long long max_slots, hipStream_t s)
{
    if (max_slots > 4096)
        hipLaunchKernelGGL(finalize_kernel<1024>, dim3(n_inst), dim3(1024), 0, s, inst, ctl, dtp, st, dim, prec, mm,
                           wslots, waves_per_block);
    else
        hipLaunchKernelGGL(finalize_kernel<256>, dim3(n_inst), dim3(256), 0, s, inst, ctl, dtp, st, dim, prec, mm,
                           wslots, waves_per_block);
    return hipGetLastError();
}

// Streaming copy of 16-byte elements: the attainable-bandwidth reference the
// stage kernels are compared with (every byte read once and written once).
// Four independent 16-byte loads per thread are in flight before their
// stores; non-temporal accesses keep the copy from thrashing the caches.
typedef float copy_v4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) copy16_kernel(const copy_v4 *__restrict__ src, copy_v4 *__restrict__ dst,
                                                     long long n)
{
    const long long stride = (long long)gridDim.x * 256;
    long long i = threadIdx.x + (long long)blockIdx.x * 256;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const copy_v4 a = __builtin_nontemporal_load(src + i);
        const copy_v4 b = __builtin_nontemporal_load(src + i + stride);
        const copy_v4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const copy_v4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t copy16_launch(const void *src, void *dst, long long n16, hipStream_t s)
{
    const long long want = (n16 + 1023) / 1024;
    const int blocks = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(copy16_kernel, dim3(blocks), dim3(256), 0, s, (const copy_v4 *)src, (copy_v4 *)dst, n16);
    return hipGetLastError();
}

hipError_t copy_launch(int prec, const void *src, void *dst, long long n, hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (prec == 32)
        hipLaunchKernelGGL(copy_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float *)src, (float *)dst, n);
    else
        hipLaunchKernelGGL(copy_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double *)src,
                           (double *)dst, n);
    return hipGetLastError();
}

hipError_t convert_launch(int prec, bool to_storage, const void *src, void *dst, long long n, hipStream_t s)
{
    if (prec == 64) return copy_launch(64, src, dst, n, s);
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (to_storage)
        hipLaunchKernelGGL((convert_kernel<double, float>), dim3((unsigned)nb), dim3(256), 0, s, (const double *)src,
                           (float *)dst, n);
    else
        hipLaunchKernelGGL((convert_kernel<float, double>), dim3((unsigned)nb), dim3(256), 0, s, (const float *)src,
                           (double *)dst, n);
    return hipGetLastError();
}

hipError_t norms_launch(int prec, const void *block, long long ncell, long long kstride, int nkinds, double *partials,
                        double *out, hipStream_t s)
{
    if (prec == 32)
        hipLaunchKernelGGL(norms_kernel<float>, dim3(kNormBlocks), dim3(256), 0, s, (const float *)block, ncell,
                           kstride, nkinds, partials);
    else
        hipLaunchKernelGGL(norms_kernel<double>, dim3(kNormBlocks), dim3(256), 0, s, (const double *)block, ncell,
                           kstride, nkinds, partials);
    hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(64), 0, s, partials, kNormBlocks, out);
    return hipGetLastError();
}

// Scratch of the norms reduction for callers that cannot allocate
// (af_norms_noalloc): the block partials, then the nine results.  Each GPU
// holds its own copy until the process ends; every call on a GPU shares it.
// In host code `scratch` names a host-side stand-in, never device memory:
// only the address hipGetSymbolAddress returns for the current device is
// passed to kernels.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(double **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (double *)p;
    }
    *ptr = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace af4

#include "variants.h"

namespace af4 {

int stage_num_variants(int dim)
{
    int n = 0;
#define AF4_COUNT(V, TX, TY, TZ, NT, NAME) n++;
#define AF4_COUNT2(V, TX, TY, TZ, NT, KIND, NAME) n++;
    if (dim == 1) { AF4_VARIANTS_D1(AF4_COUNT) }
    if (dim == 2) { AF4_VARIANTS_D2(AF4_COUNT2) }
    if (dim == 3) { AF4_VARIANTS_D3(AF4_COUNT2) }
#undef AF4_COUNT
#undef AF4_COUNT2
    return n;
}

VariantInfo stage_variant(int dim, int v)
{
    VariantInfo r = {{1, 1, 1}, 0, ""};
#define AF4_INFO(V, TX, TY, TZ, NT, NAME) \
    if (v == V) r = VariantInfo{{TX, TY, TZ}, NT, NAME};
#define AF4_INFO2(V, TX, TY, TZ, NT, KIND, NAME) \
    if (v == V) r = VariantInfo{{TX, TY, TZ}, NT, NAME};
    if (dim == 1) { AF4_VARIANTS_D1(AF4_INFO) }
    if (dim == 2) { AF4_VARIANTS_D2(AF4_INFO2) }
    if (dim == 3) { AF4_VARIANTS_D3(AF4_INFO2) }
#undef AF4_INFO
#undef AF4_INFO2
    for (int l = dim; l < 3; l++) r.tile[l] = 1;
    return r;
}

bool stage_supported(int dim, int prec, bool lim, bool si, unsigned caps, int variant)
{
    if (dim == 1) return stage_supported_d1(prec, lim, si, variant);
    if (dim == 2) return stage_supported_d2(prec, lim, si, caps, variant);
    if (dim == 3) return stage_supported_d3(prec, lim, si, caps, variant);
    return false;
}

hipError_t stage_launch(int dim, int prec, bool lim, bool si, unsigned caps, int variant, int nblocks, const void *params,
                        hipStream_t s)
{
    if (dim == 1) return stage_launch_d1(prec, lim, si, caps, variant, nblocks, params, s);
    if (dim == 2) return stage_launch_d2(prec, lim, si, caps, variant, nblocks, params, s);
    if (dim == 3) return stage_launch_d3(prec, lim, si, caps, variant, nblocks, params, s);
    return hipErrorInvalidValue;
}

}  // namespace af4
