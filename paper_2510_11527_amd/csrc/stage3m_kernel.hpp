// stage3m_kernel.hpp -- 3D stage kernel that marches along z.
//
// Same stage as the generic kernel (stage_kernel.hpp): point values by the
// biased fourth-order convection operator with the downwind point plus the
// compact D^{2,4th} on a(u) (Eq. 2d_af_dc, Sec. 4), projected onto the bounds
// (Sec. 5.2.2); averages by the doubly conservative update limited by the
// monolithic convex limiter (Sec. 5.2.1), optional smoothness-indicator
// blending direction by direction (Sec. 5.1.3), the Runge-Kutta combination
// and the bound safeguard.  Fluxes f_l = c1 u + c2 u^2, periodic ends.
//
// A workgroup owns a TX x TY column of cells and a range of LZ cell planes of
// one instance, one thread per (x, y) cell, and walks the column upwards one
// cell plane k per iteration.  Nothing is recomputed across z: every
// quantity that the update of plane k needs from neighbouring planes is
// computed once, when its inputs arrive, and kept in LDS rings indexed by
// plane:
//   * averages of cell planes k .. k+3 (the smoothness indicator of plane
//     k+2 along z needs k+3);
//   * the half-grid planes 2k-2 .. 2k+3 (values and a(u)): the point values
//     of cell planes k-1 .. k+1 and their reconstructed centres;
//   * low-order z-face states of the faces k+1/2, k+3/2; limited z-face
//     fluxes of k-1/2, k+1/2; limited z-potentials of cells k-1 .. k+1;
//   * blending weights (exp(-gamma s_l / 8), see below) of planes k, k+1
//     (x, y) and k-1 .. k+1 (z), raw z-indicators of k .. k+2.
// Per iteration (barriers between the phases):
//   1. load the averages of plane k+3 and the point values of cell plane k+1;
//   2. centres of plane k+1 (inverse tensor Simpson), raw indicators, the
//      low-order states of z-face k+3/2;
//   3. smoothed indicators -> blending weights of planes k+1;
//   4. limited z-potentials of plane k+1, limited z-flux of face k+1/2, x- and
//      y-faces of plane k;
//   5. limited x- and y-potentials of plane k;
//   6. the point values of half planes 2k, 2k+1 and the averages of plane k.
//
// Blending weights: exp(-gamma s) of a mean of s over 1, 2, 4 or 8 cells is
// the product of E = exp(-gamma s / 8) over those cells, raised to the power
// 8, 4, 2 or 1 -- squarings instead of one exponential per point and
// direction (equal to the generic kernel's weights up to rounding).
#pragma once
#include "stage_kernel.hpp"

namespace af4 {

template <int TX, int TY, bool SI>
struct MGeo {
    static constexpr int HZ = SI ? 3 : 2;                    // halo of the averages in x, y (cells)
    static constexpr int RX = TX + 2 * HZ, RY = TY + 2 * HZ;  // averages plane
    static constexpr int NUB = RX * RY;
    static constexpr int HX = 2 * TX + 6, HY = 2 * TY + 6;   // half plane: cells [-2, T] of the tile
    static constexpr int NHP = HX * HY;
    // blending-weight boxes (tile-local cells): x: u in [-1, TX], v in [0, TY];
    // y: u in [0, TX], v in [-1, TY]; z: u in [0, TX], v in [0, TY]
    static constexpr int EXW = TX + 2, EXN = (TX + 2) * (TY + 1);
    static constexpr int EYW = TX + 1, EYN = (TX + 1) * (TY + 2);
    static constexpr int EZW = TX + 1, EZN = (TX + 1) * (TY + 1);
    // raw indicators of plane k+1: x: u in [-2, TX+1], v in [0, TY]; y: u in [0, TX], v in [-2, TY+1]
    static constexpr int TXW = TX + 4, TXN = (TX + 4) * (TY + 1);
    static constexpr int TYW = TX + 1, TYN = (TX + 1) * (TY + 4);
    // x-faces (left cell u in [-2, TX], v in [0, TY)), y-faces likewise
    static constexpr int FXW = TX + 3, FXN = (TX + 3) * TY;
    static constexpr int FYW = TX, FYN = TX * (TY + 3);
    // x-potentials (u in [-1, TX]), y-potentials (v in [-1, TY])
    static constexpr int PXW = TX + 2, PXN = (TX + 2) * TY;
    static constexpr int PYW = TX, PYN = TX * (TY + 2);
    static constexpr int NOWN = TX * TY;

    __device__ static __forceinline__ int ub(int u, int v) { return (u + HZ) + RX * (v + HZ); }
    // half-plane point at tile-local half indices p = 2u + bx, q = 2v + by
    // (p, q >= -4), stored in the cell-indexed sub-grid of its parity (bx,
    // by): the points that a wave reads at one stencil offset are then
    // consecutive words, not every other one (LDS bank conflicts)
    static constexpr int SW = TX + 3, SUB = SW * (TY + 3);
    __device__ static __forceinline__ int hp(int p, int q)
    {
        return ((p & 1) + 2 * (q & 1)) * SUB + ((p + 4) >> 1) + SW * ((q + 4) >> 1);
    }
};

// LDS bytes of a marching-kernel instantiation
template <class T, bool LIM, bool SI, int TX, int TY>
constexpr long stage3m_lds_bytes()
{
    using G = MGeo<TX, TY, SI>;
    long n = 8L * G::NUB + 12L * G::NHP;
    n += 3L * 2 * G::NOWN + 3L * G::NOWN + 2L * G::NOWN;                   // z-faces, P_z, F_z
    n += (long)G::FXN * (LIM ? 3 : 1) + (long)G::FYN * (LIM ? 3 : 1) + G::PXN + G::PYN;
    if (SI) n += 2L * G::EXN + 2L * G::EYN + 3L * G::EZN + 3L * G::EZN + G::TXN + G::TYN;
    return n * (long)sizeof(T);
}

// Phase 6 work of a column split among NH threads (twice the waves on the
// same LDS with NH = 2): the part of the thread that updates point value zk
// (zk = 0: the average) -- NH = 2: the even half plane's three point values
// and the average, the odd half plane's four.
template <int NH>
__device__ __forceinline__ constexpr int m3_part(int zk)
{
    return NH == 1 ? 0 : (zeta_mask<3>(zk) >> 2) & 1;
}
// position of DoF kind zk among the 8 / NH kinds of its part (in zk order),
// and the kind at position j of part h
template <int NH>
__device__ __forceinline__ constexpr int m3_slot(int zk)
{
    int s = 0;
    for (int j = 0; j < zk; j++) s += m3_part<NH>(j) == m3_part<NH>(zk) ? 1 : 0;
    return s;
}
template <int NH>
__device__ __forceinline__ int m3_kind(int h, int j)
{
    int r = 0;
#pragma unroll
    for (int zk = 7; zk >= 0; zk--)
        if (m3_part<NH>(zk) == h && m3_slot<NH>(zk) == j) r = zk;
    return r;
}

// One loop over the items of several boxes of a phase, for boxes smaller
// than the workgroup: box b takes a segment of one index space, each segment
// starting at a wave boundary, so that a wave works on one box and the
// boxes are spread over all the waves (a loop per box would give each box's
// items to the first waves only and leave the last idle).  A segment that is
// off takes its place in the index space but does nothing.
template <int W_, int H_, class F>
struct MSeg {
    static constexpr int W = W_, N = W_ * H_, PAD = (N + 63) / 64 * 64;
    bool on;
    F f;
};
template <int W, int H, class F>
__device__ __forceinline__ MSeg<W, H, F> mseg(bool on, F f)
{
    return MSeg<W, H, F>{on, f};
}
template <int OFF>
__device__ __forceinline__ void mseg_run(int)
{
}
template <int OFF, class S, class... R>
__device__ __forceinline__ void mseg_run(int idx, const S &s, const R &...rest)
{
    if (idx < OFF + S::PAD) {
        const int li = idx - OFF;
        if (s.on && li < S::N) s.f(li % S::W, li / S::W);
        return;
    }
    mseg_run<OFF + S::PAD>(idx, rest...);
}
template <int NT, class S>
__device__ __forceinline__ void mseg_alone(const S &s)
{
    if (!s.on) return;
    for (int li = (int)threadIdx.x; li < S::N; li += NT) s.f(li % S::W, li / S::W);
}
template <int NT, class... S>
__device__ __forceinline__ void box_merge(const S &...segs)
{
    if constexpr (NT >= 256) {
        constexpr int TOT = (S::PAD + ... + 0);
#pragma unroll
        for (int r = 0; r < (TOT + NT - 1) / NT; r++) mseg_run<0>((int)threadIdx.x + r * NT, segs...);
    } else {
        // two waves take every box of these phases in one round each anyway,
        // and the merged loop cost them registers (one wave per SIMD): a loop
        // per box
        (mseg_alone<NT>(segs), ...);
    }
}

// NT = NH TX TY threads, NH in {1, 2} per column
template <class T, bool LIM, bool SI, int TX, int TY, int LZ, int NT>
__global__ void __launch_bounds__(NT) stage3m_kernel(StageParams<T> p)
{
    using G = MGeo<TX, TY, SI>;
    constexpr int NH = NT / (TX * TY);
    static_assert(NT == NH * TX * TY && (NH == 1 || NH == 2), "one or two threads per column");
    constexpr int HZ = G::HZ;

    __shared__ T sUB[4][G::NUB];   // averages of planes k .. k+3 (slot: plane & 3)
    __shared__ T sAU[4][G::NUB];   // a(u) of those averages (evaluated once, at the commit)
    __shared__ T sH[6][G::NHP];    // half planes 2k-2 .. 2k+3 (slot: half plane % 6)
    __shared__ T sA[6][G::NHP];    // a(u) at the same points
    __shared__ T sZL[2][G::NOWN], sZP[2][G::NOWN], sZM[2][G::NOWN];  // z-faces (slot: face index & 1)
    __shared__ T sPZ[3][G::NOWN];  // limited z-potential of planes k-1 .. k+1 (slot: plane % 3)
    __shared__ T sFZ[2][G::NOWN];  // limited z-flux of faces k-1/2, k+1/2 (slot: face index & 1)
    __shared__ T sXF[G::FXN], sYF[G::FYN];                         // limited x-, y-fluxes of plane k
    __shared__ T sXP[LIM ? G::FXN : 1], sXM[LIM ? G::FXN : 1];    // u^{L,+} (left), u^{L,-} (right) per x-face
    __shared__ T sYP[LIM ? G::FYN : 1], sYM[LIM ? G::FYN : 1];
    __shared__ T sPX[G::PXN], sPY[G::PYN];                         // limited x-, y-potentials of plane k
    __shared__ T sEX[SI ? 2 : 1][SI ? G::EXN : 1];                 // blending weights (slot: plane & 1)
    __shared__ T sEY[SI ? 2 : 1][SI ? G::EYN : 1];
    __shared__ T sEZ[SI ? 3 : 1][SI ? G::EZN : 1];                 // (slot: plane % 3)
    __shared__ T sTZ[SI ? 3 : 1][SI ? G::EZN : 1];                 // raw z-indicators (slot: plane % 3)
    __shared__ T sTX[SI ? G::TXN : 1], sTY[SI ? G::TYN : 1];      // raw x-, y-indicators of plane k+1

    // block -> (instance, column tile, z chunk); consecutive logical tiles on one XCD
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int4 wk = p.work[logical];
    const InstDev &I = p.inst[wk.x];
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const int ox = wk.y * TX, oy = wk.z * TY, z0 = wk.w * LZ;
    const int zend = z0 + LZ < n2 ? z0 + LZ : n2;
    const long long kst = I.kstride;
    const long long plane = (long long)n0 * n1;
    const T *__restrict__ in = p.in + I.off;
    const T *__restrict__ un = p.un + I.off;
    const T *__restrict__ x1 = p.x1 ? p.x1 + I.off : nullptr;
    T *__restrict__ out = p.out + I.off;
    const bool residual = p.stage == kStageRHS;
    const double dtd = p.st[wk.x].dt;
    const T inf = __builtin_huge_val();
    T vlo = inf, vhi = -inf;

    // global index of tile-local cell (u, v) in plane k (periodic)
    auto gidx = [&](int u, int v, int k) -> long long {
        return (long long)wrap_index(ox + u, n0) + (long long)n0 * wrap_index(oy + v, n1) + plane * wrap_index(k, n2);
    };

    if (!residual && dtd == 0.0) {
        // the instance has reached its end time: the stage leaves it unchanged
        for (int k = z0; k < zend; k++)
            box_loop<TX, TY, 1, NT>([&](int u, int v, int) {
                if (ox + u >= n0 || oy + v >= n1) return;
                const long long gi = (ox + u) + (long long)n0 * (oy + v) + plane * k;
                for (int z = 0; z < 8; z++) out[z * kst + gi] = in[z * kst + gi];
                vlo = fmin(vlo, in[gi]);
                vhi = fmax(vhi, in[gi]);
            });
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
        return;
    }

    Phys<T> P;
    P.load(I, 3);
    {
        // the bounds as scalar loads: a vector load of them stayed pending
        // into the loop, where the first clamp waited for every load in flight
        const auto Ic = as_constant(&p.inst[wk.x]);
        if constexpr (sizeof(T) == 4) {
            P.umin = Ic->f_umin;
            P.umax = Ic->f_umax;
        } else {
            P.umin = Ic->umin;
            P.umax = Ic->umax;
        }
    }
    T qc1[3], qc2[3];  // f_l = qc1 u + qc2 u^2
#pragma unroll
    for (int l = 0; l < 3; l++) {
        qc1[l] = I.fk[l] == kFLinear ? (T)I.fp0[l] : T(0);
        qc2[l] = I.fk[l] == kFQuad ? (T)I.fp0[l] : T(0);
    }
    auto Ff = [&](int l, T u) -> T { return u * (qc1[l] + qc2[l] * u); };
    auto Fg = [&](int l, T u) -> T { return fabs(qc1[l] + T(2) * qc2[l] * u); };
    const T dt = (T)dtd * p.dts;
    const T K = T(6);
    T idx1[3], idx2[3], i6dx[3], mu[3], nu[3];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        idx1[l] = (T)I.idx1[l];
        idx2[l] = (T)I.idx2[l];
        i6dx[l] = (T)I.i6dx[l];
        mu[l] = (T)p.st[wk.x].mu[l] * p.dts;
        nu[l] = (T)p.st[wk.x].nu[l] * p.dts;
    }
    // theta^c and theta^d move their states by 3 K mu and 3 K nu times the
    // correction; their reciprocals scale the gaps
    T ik3mu[3], ik3nu[3];
#pragma unroll
    for (int l = 0; l < 3; l++) {
        ik3mu[l] = fast_rcp(T(3) * K * mu[l]);
        ik3nu[l] = fast_rcp(T(3) * K * nu[l]);
    }
    const bool use_si = SI && !residual;
    const bool lim = LIM && !residual;
    const T gam8 = (T)I.si_gamma * T(0.125);
    double clamp_mag = 0.0;
    bool bad = false;

    // ring slots (offsets keep the dividends non-negative: k >= -6)
    auto s4 = [](int k) { return (k + 24) & 3; };
    auto s3 = [](int k) { return (k + 24) % 3; };
    auto s2 = [](int k) { return (k + 24) & 1; };
    auto s6 = [](int h) { return (h + 48) % 6; };

    const int kbeg = z0 - 3 - HZ;
    // Global loads of an iteration (averages of plane k+3, point values of
    // cell plane k+1) are issued one iteration ahead into registers, so that
    // their latency overlaps the previous iteration's compute phases.
    constexpr int NU = (G::NUB + NT - 1) / NT;
    constexpr int NPC = (TX + 3) * (TY + 3);
    constexpr int NP = (NPC + NT - 1) / NT;
    const int tid = (int)threadIdx.x;
    T pu[NU], pv[NP][8];
    // U^n of the DoFs this thread updates in phase 6 (its column and part of
    // the column's kinds), loaded with the other loads of the iteration
    // before: a load issued in phase 6 itself made the wait for it also wait
    // for those prefetches (the memory counter is in order)
    constexpr int NK = 8 / NH;
    const int pu6 = tid % TX, pv6 = (tid / TX) % TY, ph6 = tid / (TX * TY);
    const bool own6 = ox + pu6 < n0 && oy + pv6 < n1;
    T unn[NK], unc[NK];
#pragma unroll
    for (int j = 0; j < NK; j++) unn[j] = unc[j] = T(0);
    auto issue = [&](int k) {
        if (k >= z0) {
            const long long g6 = own6 ? (ox + pu6) + (long long)n0 * (oy + pv6) + plane * k : 0;
#pragma unroll
            for (int j = 0; j < NK; j++) unn[j] = un[m3_kind<NH>(ph6, j) * kst + g6];
        }
#pragma unroll
        for (int i = 0; i < NU; i++) {
            const int idx = tid + i * NT;
            if (idx < G::NUB) pu[i] = in[gidx(idx % G::RX - HZ, idx / G::RX - HZ, k + 3)];
        }
#pragma unroll
        for (int j = 0; j < NP; j++) {
            const int idx = tid + j * NT;
            if (idx < NPC) {
                const long long gi = gidx(idx % (TX + 3) - 2, idx / (TX + 3) - 2, k + 1);
#pragma unroll
                for (int z = 1; z < 8; z++) pv[j][z] = in[z * kst + gi];
            }
        }
    };
    // the stage's combination (stage_combine) with the prefetched U^n; X1,
    // read by summing stages only, is loaded and used inside their branch, so
    // that the other stages wait for no load in phase 6
    auto combine6 = [&](T v, T x0, int z, long long g, T vin) -> T {
        if (p.mode == kCombSum) return ((p.c0 * x0 + p.c1 * x1[z * kst + g]) + p.cin * vin) + p.w * v;
        if (p.mode == kCombBlend) return x0 + p.w * (v - x0);
        return v;
    };
    auto commit = [&](int k) {
        // the empty asm reads each loaded value here, where the loads of the
        // iteration before are waited for anyway; a first read in phase 6,
        // behind the next iteration's loads, would wait for those too
#pragma unroll
        for (int j = 0; j < NK; j++) {
            T v = unn[j];
            asm volatile("" : "+v"(v));
            unc[j] = v;
        }
        T *ubk = sUB[s4(k + 3)], *auk = sAU[s4(k + 3)];
#pragma unroll
        for (int i = 0; i < NU; i++) {
            const int idx = tid + i * NT;
            if (idx < G::NUB) {
                ubk[idx] = pu[i];
                auk[idx] = P.a(pu[i]);
            }
        }
        T *he = sH[s6(2 * k + 2)], *ho = sH[s6(2 * k + 3)];
        T *ae = sA[s6(2 * k + 2)], *ao = sA[s6(2 * k + 3)];
#pragma unroll
        for (int j = 0; j < NP; j++) {
            const int idx = tid + j * NT;
            if (idx < NPC) {
                const T *w = pv[j];
                // zeta order: 1 x-face, 2 y-face, 3 z-face, 4 xy-edge, 5 xz-edge, 6 yz-edge, 7 corner
                const int pe = 2 * (idx % (TX + 3) - 2), qe = 2 * (idx / (TX + 3) - 2);
                he[G::hp(pe + 1, qe)] = w[1];
                he[G::hp(pe, qe + 1)] = w[2];
                he[G::hp(pe + 1, qe + 1)] = w[4];
                ho[G::hp(pe, qe)] = w[3];
                ho[G::hp(pe + 1, qe)] = w[5];
                ho[G::hp(pe, qe + 1)] = w[6];
                ho[G::hp(pe + 1, qe + 1)] = w[7];
                ae[G::hp(pe + 1, qe)] = P.a(w[1]);
                ae[G::hp(pe, qe + 1)] = P.a(w[2]);
                ae[G::hp(pe + 1, qe + 1)] = P.a(w[4]);
                ao[G::hp(pe, qe)] = P.a(w[3]);
                ao[G::hp(pe + 1, qe)] = P.a(w[5]);
                ao[G::hp(pe, qe + 1)] = P.a(w[6]);
                ao[G::hp(pe + 1, qe + 1)] = P.a(w[7]);
            }
        }
    };
    issue(kbeg);
    for (int k = kbeg; k < zend; k++) {
        // ---- 1: averages of plane k+3, point values of cell plane k+1 (loaded
        // during the previous iteration); the next iteration's loads go out
        commit(k);
        if (k + 1 < zend) issue(k + 1);
        __syncthreads();

        // ---- 2: centres of plane k+1, raw indicators, low-order z-face k+3/2
        // (one merged loop over the five boxes: see box_merge)
        {
            const T *hm = sH[s6(2 * k + 1)], *hp1 = sH[s6(2 * k + 3)];
            T *hc = sH[s6(2 * k + 2)], *ac = sA[s6(2 * k + 2)];
            const T *ub1 = sUB[s4(k + 1)], *ub2 = sUB[s4(k + 2)], *ub3 = sUB[s4(k + 3)];
            const T *au1 = sAU[s4(k + 1)], *au2 = sAU[s4(k + 2)];
            T *tz = sTZ[s3(k + 2)];
            const int sl = s2(k + 1);
            // the indicator boxes are empty without blending
            constexpr int SIH = SI ? 1 : 0;
            box_merge<NT>(
                mseg<TX + 2, TY + 2>(k >= z0 - 2, [&](int x, int y) {
                    const int u = x - 1, v = y - 1;
                    const int pc = 2 * u, qc = 2 * v;
                    T acc = T(216) * ub1[G::ub(u, v)];
#pragma unroll
                    for (int oy = -1; oy <= 1; oy++)
#pragma unroll
                        for (int oxx = -1; oxx <= 1; oxx++) {
                            const int i = G::hp(pc + oxx, qc + oy);
                            const T wxy = T((oxx == 0 ? 4 : 1) * (oy == 0 ? 4 : 1));
                            acc -= wxy * (hm[i] + hp1[i]);                        // oz = -1, +1
                            if (oxx != 0 || oy != 0) acc -= T(4) * wxy * hc[i];  // oz = 0
                        }
                    const T c = acc * T(0.015625);
                    hc[G::hp(pc, qc)] = c;
                    ac[G::hp(pc, qc)] = P.a(c);
                }),
                mseg<G::TXW, (TY + 1) * SIH>(use_si && k >= z0 - 1, [&](int x, int y) {
                    const int u = x - 2, v = y;
                    const T um = ub1[G::ub(u - 1, v)], u0 = ub1[G::ub(u, v)], up = ub1[G::ub(u + 1, v)];
                    sTX[x + G::TXW * y] = fabs(um - T(2) * u0 + up) * fast_rcp(fabs(um) + T(2) * fabs(u0) + fabs(up) + T(1e-13));
                }),
                mseg<TX + 1, (TY + 4) * SIH>(use_si && k >= z0 - 1, [&](int x, int y) {
                    const int u = x, v = y - 2;
                    const T um = ub1[G::ub(u, v - 1)], u0 = ub1[G::ub(u, v)], up = ub1[G::ub(u, v + 1)];
                    sTY[x + G::TYW * y] = fabs(um - T(2) * u0 + up) * fast_rcp(fabs(um) + T(2) * fabs(u0) + fabs(up) + T(1e-13));
                }),
                mseg<TX + 1, (TY + 1) * SIH>(use_si && k >= z0 - 4, [&](int u, int v) {
                    const int i = G::ub(u, v);
                    const T um = ub1[i], u0 = ub2[i], up = ub3[i];
                    tz[u + G::EZW * v] = fabs(um - T(2) * u0 + up) * fast_rcp(fabs(um) + T(2) * fabs(u0) + fabs(up) + T(1e-13));
                }),
                // z-face (k+1)+1/2 between planes k+1 and k+2: LLF flux, and with the
                // limiter u^{L,+} of the lower cell and u^{L,-} of the upper one
                mseg<TX, TY>(k >= z0 - 3, [&](int u, int v) {
                    const int i = G::ub(u, v), o = u + TX * v;
                    const T ua = ub1[i], ubb = ub2[i];
                    const T fa = Ff(2, ua), fb = Ff(2, ubb);
                    const T al = fmax(Fg(2, ua), Fg(2, ubb));
                    const T fL = T(0.5) * (fa + fb) - T(0.5) * al * (ubb - ua);
                    sZL[sl][o] = fL;
                    if constexpr (LIM) {
                        const T dA = (au2[i] - au1[i]) * idx1[2];
                        const T Km = K * mu[2];
                        sZP[sl][o] = ua - Km * (fL - fa) + Km * dA;
                        sZM[sl][o] = ubb - Km * (fb - fL) - Km * dA;
                    }
                }));
        }
        __syncthreads();

        // ---- 3: blending weights E = exp(-gamma s / 8) of plane k+1
        if (use_si) {
            if (k >= z0 - 1) {
                T *ex = sEX[s2(k + 1)], *ey = sEY[s2(k + 1)];
                box_loop<G::EXW, TY + 1, 1, NT>([&](int x, int y, int) {
                    const int c = (x + 1) + G::TXW * y;  // s~ index of cell u = x - 1
                    const T s = (sTX[c - 1] + T(4) * sTX[c] + sTX[c + 1]) * T(1.0 / 6.0);
                    ex[x + G::EXW * y] = blend_exp(-gam8 * s);
                });
                box_loop<TX + 1, TY + 2, 1, NT>([&](int x, int y, int) {
                    const int c = x + G::TYW * (y + 1);  // s~ index of cell v = y - 1
                    const T s = (sTY[c - G::TYW] + T(4) * sTY[c] + sTY[c + G::TYW]) * T(1.0 / 6.0);
                    ey[x + G::EYW * y] = blend_exp(-gam8 * s);
                });
            }
            if (k >= z0 - 2) {
                const T *t0 = sTZ[s3(k)], *t1 = sTZ[s3(k + 1)], *t2 = sTZ[s3(k + 2)];
                T *ez = sEZ[s3(k + 1)];
                box_loop<TX + 1, TY + 1, 1, NT>([&](int u, int v, int) {
                    const int i = u + G::EZW * v;
                    ez[i] = blend_exp(-gam8 * ((t0[i] + T(4) * t1[i] + t2[i]) * T(1.0 / 6.0)));
                });
            }
            __syncthreads();
        }

        // ---- 4: z-potential of plane k+1, z-flux of face k+1/2, x/y-faces of plane k
        // (the two z boxes in one merged loop, see box_merge; merging the x-
        // and y-faces too took more registers than two waves per SIMD allow)
        {
            const T *a0 = sA[s6(2 * k + 1)], *a1 = sA[s6(2 * k + 2)], *a2 = sA[s6(2 * k + 3)];
            const T *ubz = sUB[s4(k + 1)], *auz = sAU[s4(k + 1)];
            const int fl = s2(k), fu = s2(k + 1);  // faces (k+1) -+ 1/2
            const T *h = sH[s6(2 * k + 1)];
            const int fs = s2(k);
            const T *ubk = sUB[s4(k)], *auk = sAU[s4(k)];
            const T *hm = sH[s6(2 * k - 1)], *h0 = sH[s6(2 * k)], *hq = sH[s6(2 * k + 1)];
            box_merge<NT>(
                mseg<TX, TY>(k >= z0 - 2, [&](int u, int v) {
                    const int o = u + TX * v;
                    // (1/216) sum of v_z (x) w (x) w a over the cell's 27 points
                    T sl[3];
                    const T *ap[3] = {a0, a1, a2};
#pragma unroll
                    for (int oz = 0; oz < 3; oz++) {
                        T acc = T(0);
#pragma unroll
                        for (int oy = -1; oy <= 1; oy++)
#pragma unroll
                            for (int oxx = -1; oxx <= 1; oxx++)
                                acc += T((oxx == 0 ? 4 : 1) * (oy == 0 ? 4 : 1)) * ap[oz][G::hp(2 * u + oxx, 2 * v + oy)];
                        sl[oz] = acc;
                    }
                    T aH = (T(8) * sl[1] - sl[0] - sl[2]) * T(1.0 / 216.0);
                    const T aL = auz[G::ub(u, v)];
                    if (use_si) {
                        T e = sEZ[s3(k + 1)][u + G::EZW * v];
                        e *= e;
                        e *= e;
                        const T th = e * e;
                        aH = th * aH + (T(1) - th) * aL;
                    }
                    T Pv = aH;
                    if (lim) {
                        const T da = aH - aL;
                        const T gap = gap4<T>(da, sZP[fl][o], sZM[fu][o], sZP[fu][o], sZM[fl][o], P.umin, P.umax);
                        Pv = aL + limited_part<T>(gap, da, ik3nu[2]);
                    }
                    sPZ[s3(k + 1)][o] = Pv;
                }),
                mseg<TX, TY>(k >= z0 - 1, [&](int u, int v) {
                    const int o = u + TX * v;
                    T fH = T(0);
#pragma unroll
                    for (int oy = -1; oy <= 1; oy++)
#pragma unroll
                        for (int oxx = -1; oxx <= 1; oxx++)
                            fH += T((oxx == 0 ? 4 : 1) * (oy == 0 ? 4 : 1)) * Ff(2, h[G::hp(2 * u + oxx, 2 * v + oy)]);
                    fH *= T(1.0 / 36.0);
                    const T fL = sZL[fs][o];
                    if (use_si) {
                        T e = sEZ[s3(k)][u + G::EZW * v] * sEZ[s3(k + 1)][u + G::EZW * v];
                        e *= e;
                        const T th = e * e;
                        fH = th * fH + (T(1) - th) * fL;
                    }
                    T F = fH;
                    if (lim) {
                        const T df = fH - fL;
                        const T gap = gap2<T>(df, sZM[fs][o], sZP[fs][o], P.umin, P.umax);
                        F = fL + limited_part<T>(gap, df, ik3mu[2]);
                    }
                    sFZ[fs][o] = F;
                }));
            box_merge<NT>(
                // x-faces: left cell u in [-2, TX], v in [0, TY)
                mseg<G::FXW, TY>(k >= z0, [&](int x, int v) {
                    const int u = x - 2, fi = x + G::FXW * v;
                    const T ua = ubk[G::ub(u, v)], ubb = ubk[G::ub(u + 1, v)];
                    const T fa = Ff(0, ua), fb = Ff(0, ubb);
                    const T al = fmax(Fg(0, ua), Fg(0, ubb));
                    const T fL = T(0.5) * (fa + fb) - T(0.5) * al * (ubb - ua);
                    T up = T(0), um = T(0);
                    if constexpr (LIM) {
                        const T dA = (auk[G::ub(u + 1, v)] - auk[G::ub(u, v)]) * idx1[0];
                        const T Km = K * mu[0];
                        up = ua - Km * (fL - fa) + Km * dA;
                        um = ubb - Km * (fb - fL) - Km * dA;
                        sXP[fi] = up;
                        sXM[fi] = um;
                    }
                    if (u < -1 || u > TX - 1) return;
                    // Simpson average of f_x over the face (points 2u+1, 2v + oy, 2k + oz)
                    const int pf = 2 * u + 1;
                    T fH = T(0);
#pragma unroll
                    for (int oy = -1; oy <= 1; oy++) {
                        const int i = G::hp(pf, 2 * v + oy);
                        const T wy = T(oy == 0 ? 4 : 1);
                        fH += wy * (Ff(0, hm[i]) + T(4) * Ff(0, h0[i]) + Ff(0, hq[i]));
                    }
                    fH *= T(1.0 / 36.0);
                    if (use_si) {
                        const T *ex = sEX[s2(k)];
                        T e = ex[(u + 1) + G::EXW * v] * ex[(u + 2) + G::EXW * v];
                        e *= e;
                        const T th = e * e;
                        fH = th * fH + (T(1) - th) * fL;
                    }
                    T F = fH;
                    if (lim) {
                        const T df = fH - fL;
                        F = fL + limited_part<T>(gap2<T>(df, um, up, P.umin, P.umax), df, ik3mu[0]);
                    }
                    sXF[fi] = F;
                }));
            box_merge<NT>(
                // y-faces: lower cell v in [-2, TY], u in [0, TX)
                mseg<TX, TY + 3>(k >= z0, [&](int u, int y) {
                    const int v = y - 2, fi = u + G::FYW * y;
                    const T ua = ubk[G::ub(u, v)], ubb = ubk[G::ub(u, v + 1)];
                    const T fa = Ff(1, ua), fb = Ff(1, ubb);
                    const T al = fmax(Fg(1, ua), Fg(1, ubb));
                    const T fL = T(0.5) * (fa + fb) - T(0.5) * al * (ubb - ua);
                    T up = T(0), um = T(0);
                    if constexpr (LIM) {
                        const T dA = (auk[G::ub(u, v + 1)] - auk[G::ub(u, v)]) * idx1[1];
                        const T Km = K * mu[1];
                        up = ua - Km * (fL - fa) + Km * dA;
                        um = ubb - Km * (fb - fL) - Km * dA;
                        sYP[fi] = up;
                        sYM[fi] = um;
                    }
                    if (v < -1 || v > TY - 1) return;
                    const int qf = 2 * v + 1;
                    T fH = T(0);
#pragma unroll
                    for (int oxx = -1; oxx <= 1; oxx++) {
                        const int i = G::hp(2 * u + oxx, qf);
                        const T wx = T(oxx == 0 ? 4 : 1);
                        fH += wx * (Ff(1, hm[i]) + T(4) * Ff(1, h0[i]) + Ff(1, hq[i]));
                    }
                    fH *= T(1.0 / 36.0);
                    if (use_si) {
                        const T *ey = sEY[s2(k)];
                        T e = ey[u + G::EYW * (v + 1)] * ey[u + G::EYW * (v + 2)];
                        e *= e;
                        const T th = e * e;
                        fH = th * fH + (T(1) - th) * fL;
                    }
                    T F = fH;
                    if (lim) {
                        const T df = fH - fL;
                        F = fL + limited_part<T>(gap2<T>(df, um, up, P.umin, P.umax), df, ik3mu[1]);
                    }
                    sYF[fi] = F;
                }));
        }
        __syncthreads();

        // ---- 5: x- and y-potentials of plane k
        if (k >= z0) {
            const T *auk = sAU[s4(k)];
            const T *am = sA[s6(2 * k - 1)], *a0 = sA[s6(2 * k)], *aq = sA[s6(2 * k + 1)];
            // x: cells u in [-1, TX], v in [0, TY)
            box_loop<G::PXW, TY, 1, NT>([&](int x, int v, int) {
                const int u = x - 1;
                T aH = T(0);
#pragma unroll
                for (int oy = -1; oy <= 1; oy++)
#pragma unroll
                    for (int oxx = -1; oxx <= 1; oxx++) {
                        const int i = G::hp(2 * u + oxx, 2 * v + oy);
                        const T w = T((oxx == 0 ? 8 : -1) * (oy == 0 ? 4 : 1));
                        aH += w * (am[i] + T(4) * a0[i] + aq[i]);
                    }
                aH *= T(1.0 / 216.0);
                const T aL = auk[G::ub(u, v)];
                if (use_si) {
                    T e = sEX[s2(k)][x + G::EXW * v];
                    e *= e;
                    e *= e;
                    const T th = e * e;
                    aH = th * aH + (T(1) - th) * aL;
                }
                T Pv = aH;
                if (lim) {
                    // faces u -+ 1/2 (left cells u-1, u)
                    const int f0 = (u + 1) + G::FXW * v;
                    const T da = aH - aL;
                    const T gap = gap4<T>(da, sXP[f0], sXM[f0 + 1], sXP[f0 + 1], sXM[f0], P.umin, P.umax);
                    Pv = aL + limited_part<T>(gap, da, ik3nu[0]);
                }
                sPX[x + G::PXW * v] = Pv;
            });
            // y: cells v in [-1, TY], u in [0, TX)
            box_loop<TX, TY + 2, 1, NT>([&](int u, int y, int) {
                const int v = y - 1;
                T aH = T(0);
#pragma unroll
                for (int oy = -1; oy <= 1; oy++)
#pragma unroll
                    for (int oxx = -1; oxx <= 1; oxx++) {
                        const int i = G::hp(2 * u + oxx, 2 * v + oy);
                        const T w = T((oy == 0 ? 8 : -1) * (oxx == 0 ? 4 : 1));
                        aH += w * (am[i] + T(4) * a0[i] + aq[i]);
                    }
                aH *= T(1.0 / 216.0);
                const T aL = auk[G::ub(u, v)];
                if (use_si) {
                    T e = sEY[s2(k)][u + G::EYW * y];
                    e *= e;
                    e *= e;
                    const T th = e * e;
                    aH = th * aH + (T(1) - th) * aL;
                }
                T Pv = aH;
                if (lim) {
                    const int f0 = u + G::FYW * (v + 1);
                    const T da = aH - aL;
                    const T gap = gap4<T>(da, sYP[f0], sYM[f0 + G::FYW], sYP[f0 + G::FYW], sYM[f0], P.umin, P.umax);
                    Pv = aL + limited_part<T>(gap, da, ik3nu[1]);
                }
                sPY[u + G::PYW * y] = Pv;
            });
        }
        __syncthreads();

        // ---- 6: point values of half planes 2k, 2k+1 and averages of plane k
        if (k >= z0) {
            const T *ub0 = sUB[s4(k)], *ub1 = sUB[s4(k + 1)];
            box_loop<TX, TY, NH, NT>([&](int u, int v, int half) {
                const bool own = ox + u < n0 && oy + v < n1;
                const long long gi = own ? (ox + u) + (long long)n0 * (oy + v) + plane * k : 0;
                // the seven point values: mask bits (x, y, z) and zeta index
#pragma unroll
                for (int zk = 1; zk < 8; zk++) {
                    const int m = zeta_mask<3>(zk);
                    const int bx = m & 1, by = (m >> 1) & 1, bz = (m >> 2) & 1;
                    if (m3_part<NH>(zk) != half) continue;
                    const int pp = 2 * u + bx, qq = 2 * v + by, hh = 2 * k + bz;
                    const T *hrow = sH[s6(hh)];
                    const T u0 = hrow[G::hp(pp, qq)];
                    T R = T(0);
#pragma unroll
                    for (int l = 0; l < 3; l++) {
                        T zz[5], aa[5];
#pragma unroll
                        for (int s = -2; s <= 2; s++) {
                            if (l == 0) {
                                zz[s + 2] = hrow[G::hp(pp + s, qq)];
                                aa[s + 2] = sA[s6(hh)][G::hp(pp + s, qq)];
                            } else if (l == 1) {
                                zz[s + 2] = hrow[G::hp(pp, qq + s)];
                                aa[s + 2] = sA[s6(hh)][G::hp(pp, qq + s)];
                            } else {
                                zz[s + 2] = sH[s6(hh + s)][G::hp(pp, qq)];
                                aa[s + 2] = sA[s6(hh + s)][G::hp(pp, qq)];
                            }
                        }
                        T ff[5], alpha = T(0);
#pragma unroll
                        for (int s = 0; s < 5; s++) {
                            ff[s] = Ff(l, zz[s]);
                            alpha = fmax(alpha, Fg(l, zz[s]));
                        }
                        T conv = -((ff[0] - T(8) * ff[1] + T(8) * ff[3] - ff[4]) +
                                   alpha * (zz[0] - T(4) * zz[1] + T(6) * zz[2] - T(4) * zz[3] + zz[4])) * i6dx[l];
                        if (use_si) {
                            // low-order LLF right-hand side on the half grid; the
                            // averages of the two cells replace reconstructed centres
                            T nm = zz[1], np = zz[3];
                            if (m == (1 << l)) {
                                if (l == 0) {
                                    nm = ub0[G::ub(u, v)];
                                    np = ub0[G::ub(u + 1, v)];
                                } else if (l == 1) {
                                    nm = ub0[G::ub(u, v)];
                                    np = ub0[G::ub(u, v + 1)];
                                } else {
                                    nm = ub0[G::ub(u, v)];
                                    np = ub1[G::ub(u, v)];
                                }
                            }
                            const T fm = Ff(l, nm), fp = Ff(l, np);
                            const T Fr = T(0.5) * (ff[2] + fp) - T(0.5) * alpha * (np - u0);
                            const T Fl = T(0.5) * (fm + ff[2]) - T(0.5) * alpha * (u0 - nm);
                            const T convL = -T(2) * idx1[l] * (Fr - Fl);
                            // exp(-gamma mean of s_l over the cells containing the point)
                            T e = T(1);
                            const int cnt = (1 << (bx + by + bz));
#pragma unroll
                            for (int dz = 0; dz <= 1; dz++)
#pragma unroll
                                for (int dy = 0; dy <= 1; dy++)
#pragma unroll
                                    for (int dx = 0; dx <= 1; dx++) {
                                        if (dx > bx || dy > by || dz > bz) continue;
                                        if (l == 0) e *= sEX[s2(k + dz)][(u + dx + 1) + G::EXW * (v + dy)];
                                        else if (l == 1) e *= sEY[s2(k + dz)][(u + dx) + G::EYW * (v + dy + 1)];
                                        else e *= sEZ[s3(k + dz)][(u + dx) + G::EZW * (v + dy)];
                                    }
                            // raise to the power 8 / cnt
                            if (cnt <= 4) e *= e;
                            if (cnt <= 2) e *= e;
                            if (cnt <= 1) e *= e;
                            conv = e * conv + (T(1) - e) * convL;
                        }
                        const T d2 = (-(aa[0] + aa[4]) * T(1.0 / 3.0) + (aa[1] + aa[3]) * T(16.0 / 3.0) - T(10) * aa[2]) * idx2[l];
                        R += conv + d2;
                    }
                    if (!own) continue;
                    if (residual) {
                        out[zk * kst + gi] = R;
                        continue;
                    }
                    T val = u0 + dt * R;
                    if (!isfinite(val)) bad = true;
                    if constexpr (LIM) val = clampb(val, P.umin, P.umax);
                    val = combine6(val, unc[m3_slot<NH>(zk)], zk, gi, u0);
                    if constexpr (LIM) val = clampb(val, P.umin, P.umax);
                    out[zk * kst + gi] = val;
                }
                if (!own || half != m3_part<NH>(0)) return;
                // the average
                const T uc = ub0[G::ub(u, v)];
                const T Fxp = sXF[(u + 2) + G::FXW * v], Fxm = sXF[(u + 1) + G::FXW * v];
                const T Fyp = sYF[u + G::FYW * (v + 2)], Fym = sYF[u + G::FYW * (v + 1)];
                const T Fzp = sFZ[s2(k)][u + TX * v], Fzm = sFZ[s2(k - 1)][u + TX * v];
                const T Pxm = sPX[u + G::PXW * v], Px0 = sPX[(u + 1) + G::PXW * v], Pxp = sPX[(u + 2) + G::PXW * v];
                const T Pym = sPY[u + G::PYW * v], Py0 = sPY[u + G::PYW * (v + 1)], Pyp = sPY[u + G::PYW * (v + 2)];
                const int o = u + TX * v;
                const T Pzm = sPZ[s3(k - 1)][o], Pz0 = sPZ[s3(k)][o], Pzp = sPZ[s3(k + 1)][o];
                if (residual) {
                    const T rF = idx1[0] * (Fxp - Fxm) + idx1[1] * (Fyp - Fym) + idx1[2] * (Fzp - Fzm);
                    const T rP = idx2[0] * (Pxp - T(2) * Px0 + Pxm) + idx2[1] * (Pyp - T(2) * Py0 + Pym) +
                                 idx2[2] * (Pzp - T(2) * Pz0 + Pzm);
                    out[gi] = rP - rF;
                    return;
                }
                const T dF = mu[0] * (Fxp - Fxm) + mu[1] * (Fyp - Fym) + mu[2] * (Fzp - Fzm);
                const T dP = nu[0] * (Pxp - T(2) * Px0 + Pxm) + nu[1] * (Pyp - T(2) * Py0 + Pym) +
                             nu[2] * (Pzp - T(2) * Pz0 + Pzm);
                T val = uc - dF + dP;
                if (!isfinite(val)) bad = true;
                if constexpr (LIM) {
                    const T c = clampb(val, P.umin, P.umax);
                    clamp_mag = fmax(clamp_mag, (double)fabs(c - val));
                    val = c;
                }
                val = combine6(val, unc[m3_slot<NH>(0)], 0, gi, uc);
                if constexpr (LIM) {
                    const T c = clampb(val, P.umin, P.umax);
                    clamp_mag = fmax(clamp_mag, (double)fabs(c - val));
                    val = c;
                }
                vlo = fmin(vlo, val);
                vhi = fmax(vhi, val);
                out[gi] = val;
            });
        }
        __syncthreads();
    }
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave(&p.st[wk.x].clampmax, clamp_mag);
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
    }
}

}  // namespace af4
