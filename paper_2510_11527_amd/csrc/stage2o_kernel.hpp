// stage2o_kernel.hpp -- 2D stage kernel for fluxes f_l = c1 u + c2 u^2 (linear
// advection, Burgers) and Buckley-Leverett fluxes, organised around
// thread-owned work items.
//
// Same arithmetic as the generic kernel of stage_kernel.hpp (the compact
// fourth-order AF scheme with monolithic convex limiting, J. Duan, arXiv
// 2510.11527, Secs. 2, 4, 5).  The instruction count is what bounds a stage,
// so the work is laid out to spend as few vector instructions per cell as
// possible:
//   * each thread owns a vertical pair of cells and does every per-cell item
//     of them itself -- loads, centres, the six point values, the two x- and
//     two y-faces to their right/top, the four cell-centred potentials and the
//     two average updates;
//   * the items of the halo (cells, centres, faces and potentials outside the
//     tile that the tile's items read) are short wave-aligned extra passes;
//   * every LDS array shares one row stride, so each item (own or halo)
//     reaches all its operands at constant offsets of one cell index;
//   * the half grid is split by parity into four cell-indexed sub-grids of
//     {u, a(u)}: centres C (x_i, y_j), x-faces X (x_{i+1/2}, y_j), y-faces
//     Y (x_i, y_{j+1/2}) and corners K (x_{i+1/2}, y_{j+1/2}); every 5-point
//     half-grid stencil alternates between two of them;
//   * f is recomputed from u (two instructions) instead of stored, which keeps
//     the LDS footprint at four workgroups per CU;
//   * the polynomial potentials without clamps (linear, u^2, u^3) take a
//     three-instruction path (flag kOwnPP);
//   * for pure quadratic fluxes f_l = c2 u^2 (flag kOwnBQ) the point-value
//     stencil works on u^2 and max|u|: |f_l'| = 2|c2| |u|, and the constant
//     c2 moves into the per-direction scale; the LLF face states use the
//     factored differences f(a) - f^L and f^L - f(b);
//   * the scales 1/(6 dx), 1/dx^2 and dt are folded into one multiply-add
//     per term of the point-value update;
//   * Buckley-Leverett fluxes (flag kOwnGen) take one branch-free rational
//     form with the hardware reciprocal in FP32, recomputed per use, and the
//     interval maximum of |f'| from host-tabulated values at the interior
//     maxima;
//   * non-periodic ends (flag kOwnOpen, separate instantiations) replace the
//     values on or beyond an open end by the boundary rule after the loads;
//   * global memory is addressed with 32-bit byte offsets from per-DoF-kind
//     base pointers (a plane holds fewer than 2^32 bytes; the host checks).
#pragma once
#include "stage2d_kernel.hpp"

namespace af4 {

// Buffer-resource word 3 of the gfx9 family (untyped 32-bit data format);
// raw buffer accesses then range-check byte offsets against num_records:
// loads beyond it return 0, stores beyond it are dropped.
constexpr int kBufWord3 = 0x00020000;

template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <class T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T v)
{
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
    else {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
    }
}

// kernel variant flags
enum : int { kOwnPP = 1, kOwnBQ = 2, kOwnGen = 4, kOwnOpen = 8 };

// LDS geometry.  Every array is indexed by the same cell index b = xx + SX yy
// of the tile region (RX x RY cells: the tile and a halo of 2), so that all
// accesses of one work item are constant offsets of one base:
//   * five {u, a} grids of RX x RY cells (row stride SX = RX + 1): the cells
//     {ubar, a(ubar)}, then the half-grid sub-grids C, X, Y, K;
//   * face values: x-face (xx, yy) (between cells (xx, yy) and (xx+1, yy);
//     xx in [0, TX+2], yy in [2, TY+2)) at b - 2 SX; y-face (xx, yy) (between
//     (xx, yy) and (xx, yy+1); xx in [2, TX+2), yy in [0, TY+2]) at
//     NXF + b - 2;
//   * potentials: x (xx in [1, TX+2], yy in [2, TY+2)) at b - 1 - 2 SX, y (xx
//     in [2, TX+2), yy in [1, TY+2]) at NXC + b - 2 - SX.
template <int TX, int TY>
struct Own2Geo {
    static constexpr int RX = TX + 4, RY = TY + 4, SX = RX + 1, SG = SX * RY;
    static constexpr int NXF = (TY - 1) * SX + TX + 3, NYF = (TY + 2) * SX + TX, NF = NXF + NYF;
    static constexpr int NXC = (TY - 1) * SX + TX + 2, NYC = (TY + 1) * SX + TX, NC = NXC + NYC;
    __device__ static __forceinline__ int fx(int b) { return b - 2 * SX; }
    __device__ static __forceinline__ int fy(int b) { return NXF + b - 2; }
    __device__ static __forceinline__ int px(int b) { return b - 1 - 2 * SX; }
    __device__ static __forceinline__ int py(int b) { return NXC + b - 2 - SX; }
};

template <class T, bool LIM, int FL, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stage2o_kernel(StageParams<T> p)
{
    // GEN: Buckley-Leverett fluxes f_l = q (1 - g_l (1-u)^2), q = u^2 / (u^2 +
    // (1-u)^2) (g_l = 0 without gravity), one branch-free form with the
    // hardware reciprocal in FP32, f and |f'| recomputed per use; alpha^L
    // from the host's table of |f'| at the interior maxima
    constexpr bool PP = (FL & kOwnPP) != 0, BQ = (FL & kOwnBQ) != 0, GEN = (FL & kOwnGen) != 0;
    constexpr bool OPEN = (FL & kOwnOpen) != 0;
    static_assert(!(GEN && BQ), "a general flux is not purely quadratic");
    static_assert(TX * TY == 2 * NT && TY % 2 == 0, "two cells per thread");
    static_assert(NT % TX == 0 && NT % 64 == 0, "threads cover whole columns and waves");
    using FG = Own2Geo<TX, TY>;
    constexpr int RX = FG::RX, SX = FG::SX, SG = FG::SG;
    constexpr int SC = 1, SXF = 2, SYF = 3, SK = 4;  // grids 1..4: the half-grid sub-grids

    // One LDS block: the five {u, a} grids (grid 0: the cells), then the face
    // and potential arrays.  With the limiter, u^{L,+} (of the left cell of a
    // face) and u^{L,-} (of the right cell) live there until the potentials
    // have read them; the flux and the potential used in the update are kept
    // in registers until then and take their place.
    static_assert(FG::NC <= FG::NF, "potentials fit in a face array");
    constexpr int NFB = LIM ? 2 * FG::NF : FG::NF + FG::NC;
    __shared__ V2<T> smem[5 * SG + (NFB + 1) / 2];
    T *const fbuf = (T *)(smem + 5 * SG);
    T *const ulp = fbuf, *const ulm = fbuf + FG::NF;
    T *const fl = fbuf, *const pc = fbuf + FG::NF;

    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int4 wk = p.work[logical];
    const InstDev &I = p.inst[wk.x];
    const auto Ic = as_constant(&p.inst[wk.x]);   // scalar reads of the parameters
    const auto Sc = as_constant(&p.st[wk.x]);     // (fields this kernel does not write)
    const int n0 = Ic->n[0], n1 = Ic->n[1];
    const int tx0 = wk.y, ty0 = wk.z;
    const int ox = tx0 * TX, oy = ty0 * TY;
    // the right-hand side is evaluated by the unlimited instantiation
    const bool residual = !LIM && p.stage == kStageRHS;
    const double dtd = Sc->dt;
    const int tid = (int)threadIdx.x;
    // the instance's DoF blocks of the three state buffers as buffer
    // resources (32-bit offsets, hardware range check); plane z at byte
    // offset z * kstride * sizeof(T)
    const unsigned kb = (unsigned)Ic->kstride * (unsigned)sizeof(T);
    const unsigned blk = 4u * kb;
    const auto rin = __builtin_amdgcn_make_buffer_rsrc((void *)(p.in + Ic->off), 0, (int)blk, kBufWord3);
    // X0 (U^n) of the combination; a forward-Euler stage reads it from an
    // empty range (zeros), so that one blend X0 + w (v - X0) with w = 1 serves
    // every stage but the summing ones
    const auto run = __builtin_amdgcn_make_buffer_rsrc((void *)(p.un + Ic->off), 0,
                                                       p.mode == kCombFE ? 0 : (int)blk, kBufWord3);
    const auto rout = __builtin_amdgcn_make_buffer_rsrc((void *)(p.out + Ic->off), 0, (int)blk, kBufWord3);
    // X1 of a kCombSum stage (an empty range otherwise)
    const auto rx1 = __builtin_amdgcn_make_buffer_rsrc((void *)(p.x1 ? p.x1 + Ic->off : p.in + Ic->off), 0,
                                                       p.x1 ? (int)blk : 0, kBufWord3);
    auto ld = [&](const __amdgpu_buffer_rsrc_t &r, int z, unsigned gi) -> T {
        return buf_load<T>(r, gi * (unsigned)sizeof(T), (unsigned)z * kb);
    };
    auto st = [&](int z, unsigned gi, T v) { buf_store<T>(rout, gi * (unsigned)sizeof(T), (unsigned)z * kb, v); };
    // periodic indices: one fold when the grid is wider than a tile plus its
    // halo (the usual case); narrower grids fold on in a loop behind a
    // uniform branch (no integer division: its expansion, if-converted, cost
    // every thread some 25 instructions per index)
    const bool fold0 = n0 >= TX + 4, fold1 = n1 >= TY + 4;
    // a tile whose halo lies inside the grid needs no wrap at all (most
    // tiles of large grids; uniform, so a scalar branch)
    const bool inner = ox >= 2 && oy >= 2 && ox + TX + 2 <= n0 && oy + TY + 2 <= n1;
    auto wrap = [&](int v, int n, bool fold) -> int {
        if (inner) return v;
        int r = v < 0 ? v + n : (v >= n ? v - n : v);
        if (!fold) {
            while (r < 0) r += n;
            while (r >= n) r -= n;
        }
        return r;
    };
    // own cells: region column x, rows y and y + 1
    const int ci = tid % TX, cj = 2 * (tid / TX);
    const int x = ci + 2, y = cj + 2;
    const bool ownx = ox + ci < n0;
    const bool own0 = ownx && oy + cj < n1, own1 = ownx && oy + cj + 1 < n1;
    const int gxo = wrap(ox + ci, n0, fold0);
    const unsigned g0 = (unsigned)(gxo + n0 * wrap(oy + cj, n1, fold1));
    const unsigned g1 = (unsigned)(gxo + n0 * wrap(oy + cj + 1, n1, fold1));

    const T inf = __builtin_huge_val();
    T vlo = inf, vhi = -inf;  // min / max of the averages written
    if (!residual && dtd == 0.0) {
        // the instance has reached its end time: the stage leaves it unchanged
#pragma unroll
        for (int z = 0; z < 4; z++) {
            const T a = ld(rin, z, g0), b = ld(rin, z, g1);
            if (own0) st(z, g0, a);
            if (own1) st(z, g1, b);
            if (z == 0) {
                if (own0) vlo = vhi = a;
                if (own1) {
                    vlo = fmin(vlo, b);
                    vhi = fmax(vhi, b);
                }
            }
        }
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
        return;
    }

    // parameters in the kernel's precision (FP32 copies rounded on the host)
    auto prm = [&](double d, float f) -> T {
        if constexpr (sizeof(T) == 4) return f;
        else return (T)d;
    };
    Phys<T> P;
    if constexpr (!PP) P.load(I, 2);
    T gg[2], gg2[2];  // g_l and 2 g_l of the Buckley-Leverett fluxes
#pragma unroll
    for (int l = 0; l < 2; l++) {
        gg[l] = Ic->fk[l] == kFBLGrav ? prm(Ic->fp1[l], (float)Ic->fp1[l]) : T(0);
        gg2[l] = T(2) * gg[l];
    }
    T c1[2], c2[2], c2x2[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        const T c = prm(Ic->fp0[l], Ic->f_fp0[l]);
        c1[l] = Ic->fk[l] == kFLinear ? c : T(0);
        c2[l] = Ic->fk[l] == kFQuad ? c : T(0);
        c2x2[l] = T(2) * c2[l];
    }
    // pure quadratic fluxes: |c2|, c2 / 2 and c2 / 6 for the faces
    T cabs[2], chalf[2], csix[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        cabs[l] = fabs(c2[l]);
        chalf[l] = T(0.5) * c2[l];
        csix[l] = c2[l] * T(1.0 / 6.0);
    }
    const T dt = prm(dtd, Sc->f_dt) * p.dts;
    const T umin = prm(Ic->umin, Ic->f_umin), umax = prm(Ic->umax, Ic->f_umax);
    // umax once in a vector register for the FP32 clamps: a median of three
    // reads at most one scalar register, so umin (scalar) and umax (vector)
    T umaxv = umax;
    if constexpr (sizeof(T) == 4) asm volatile("" : "+v"(umaxv));
    const T pc1 = prm(Ic->pc1, Ic->f_pc[0]), pc2 = prm(Ic->pc2, Ic->f_pc[1]), pc3 = prm(Ic->pc3, Ic->f_pc[2]);
    T idx1[2], idx2[2], i6dx[2], mu[2], nu[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        idx1[l] = prm(Ic->idx1[l], Ic->f_idx1[l]);
        idx2[l] = prm(Ic->idx2[l], Ic->f_idx2[l]);
        i6dx[l] = prm(Ic->i6dx[l], Ic->f_i6dx[l]);
        mu[l] = prm(Sc->mu[l], Sc->f_mu[l]) * p.dts;
        nu[l] = prm(Sc->nu[l], Sc->f_nu[l]) * p.dts;
    }
    // K = 2 d = 4: the LLF states use K mu; theta^c and theta^d move their
    // states by 3 K mu and 3 K nu times the correction (their reciprocals,
    // once per thread, scale the gaps)
    T kmu[2], ik3mu[2], ik3nu[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        kmu[l] = T(4) * mu[l];
        ik3mu[l] = fast_rcp(T(12) * mu[l]);
        ik3nu[l] = fast_rcp(T(12) * nu[l]);
    }

    // the stage's combination (stage_combine): a forward-Euler stage is the
    // blend with X0 = 0 (empty range above) and w = 1, exactly v
    const T wb = p.mode == kCombFE ? T(1) : p.w;
    const bool summing = p.mode == kCombSum;
    // a forward-Euler stage stores its (clamped) result as it is: the blend
    // and the second clamp are skipped (a uniform branch)
    const bool fe = p.mode == kCombFE;
    // (X1 of DoF kind z at global cell gi is read here, by summing stages)
    auto combine = [&](T v, T x0, int z, unsigned gi, T vin) -> T {
        if (summing) return ((p.c0 * x0 + p.c1 * ld(rx1, z, gi)) + p.cin * vin) + p.w * v;
        return x0 + wb * (v - x0);
    };

    auto pot = [&](T u) -> T {
        if constexpr (PP) return u * (pc1 + u * (pc2 + u * pc3));
        else return P.a(u);
    };
    auto fq = [&](int l, T u) -> T {
        if constexpr (GEN) {
            const T v = T(1) - u, u2 = u * u;
            const T q = u2 * fast_rcp(u2 + v * v);
            return q * (T(1) - gg[l] * v * v);
        } else {
            return u * (c1[l] + c2[l] * u);
        }
    };
    auto gq = [&](int l, T u) -> T {
        if constexpr (GEN) {
            const T v = T(1) - u, u2 = u * u;
            const T r = fast_rcp(u2 + v * v);
            const T d1 = T(2) * (u * v) * (r * r);
            return fabs(d1 * (T(1) - gg[l] * v * v) + (u2 * r) * (gg2[l] * v));
        } else {
            return fabs(c1[l] + c2x2[l] * u);
        }
    };
    // max of |f_l'| over [min(a,b), max(a,b)]: the end points and the interior
    // maxima inside (their |f_l'| tabulated on the host)
    auto alpha_iv = [&](int l, T a, T b) -> T {
        const T lo = vmin(a, b), hi = vmax(a, b);
        T r = vmax(gq(l, a), gq(l, b));
        const int nc = Ic->ncrit[l];
        for (int k = 0; k < nc; k++) {
            const T cv = prm(Ic->crit[l][k], Ic->f_crit[l][k]);
            const T av = prm(Ic->adfc[l][k], Ic->f_adfc[l][k]);
            r = (cv >= lo && cv <= hi) ? vmax(r, av) : r;
        }
        return r;
    };
    // grid s at cell index b (the neighbours of b are b +- 1 and b +- SX)
    auto S = [&](int s, int b) -> V2<T> { return smem[s * SG + b]; };
    auto Su = [&](int s, int b) -> T { return smem[s * SG + b].x; };
    auto Sa = [&](int s, int b) -> T { return smem[s * SG + b].y; };
    auto bix = [](int xx, int yy) -> int { return xx + SX * yy; };

    // Non-periodic ends: a half-grid point on or beyond an open end (global
    // half indices q0, q1) takes the Dirichlet value of the first Dirichlet
    // end among those it lies on or beyond, else (outflow) the mean average of
    // the domain cells around the point moved onto the boundary; the stored
    // point values on the high ends are not evolved.
    // (OPEN: instances may have non-periodic ends; a separate instantiation
    // keeps this code out of the periodic kernels)
    const bool open = OPEN && (Ic->bc[0][0] != 0 || Ic->bc[1][0] != 0);
    auto ends = [&](int q0, int q1) -> int {
        return ((Ic->bc[0][0] != 0 && (q0 <= -1 || q0 >= 2 * n0 - 1)) ? 1 : 0) |
               ((Ic->bc[1][0] != 0 && (q1 <= -1 || q1 >= 2 * n1 - 1)) ? 2 : 0);
    };
    auto bc_point = [&](int q0, int q1, int m) -> T {
#pragma unroll
        for (int l = 0; l < 2; l++) {
            const int q = l == 0 ? q0 : q1, side = q <= -1 ? 0 : 1;
            if ((m >> l & 1) && Ic->bc[l][side] == 1) return prm(Ic->bcv[l][side], (float)Ic->bcv[l][side]);
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
                sum += ld(rin, 0, (unsigned)(wrap(i, n0, false) + n0 * wrap(j, n1, false)));
                cnt++;
            }
        return sum / T(cnt);
    };

    // ---- A: cells of the tile and its halo -> LDS with their potentials.
    // Loads are issued in the order they are consumed (own cells, halo cells,
    // then U^n, which is needed only by the updates): the memory counter the
    // waits use is in order.
    constexpr int NHR = 4 * RX, NH = NHR + 4 * TY;   // halo: 4 rows, then 4 columns
    constexpr int NHI = (NH + NT - 1) / NT;          // halo cells per thread
    T own[2][4], halo[NHI][4];
    int hb[NHI];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        own[0][z] = ld(rin, z, g0);
        own[1][z] = ld(rin, z, g1);
    }
#pragma unroll
    for (int k = 0; k < NHI; k++) {
        // halo cell h: rows 0, 1, TY+2, TY+3 over all columns, then columns
        // 0, 1, TX+2, TX+3 over rows [2, TY+2); threads past the end redo the
        // last one (same value to the same place: no branch, and the loads
        // stay ahead of the U^n loads)
        const int h = min(tid + k * NT, NH - 1);
        int xx, yy;
        if (h < NHR) {
            const int r = h / RX;
            xx = h - r * RX;
            yy = r < 2 ? r : r + TY;
        } else {
            const int h2 = h - NHR, q = h2 & 3;
            yy = 2 + (h2 >> 2);
            xx = q < 2 ? q : q + TX;
        }
        hb[k] = bix(xx, yy);
        const unsigned gi = (unsigned)(wrap(ox + xx - 2, n0, fold0) + n0 * wrap(oy + yy - 2, n1, fold1));
#pragma unroll
        for (int z = 0; z < 4; z++) halo[k][z] = ld(rin, z, gi);
    }
    // X0 (U^n) of the own cells for the stage's combination (a stage that
    // does not combine reads X0 too, from cache: the load sequence up to here
    // stays free of branches, so the waits above stay exact).  X1, needed by
    // summing stages only, is loaded where it is combined, so that no
    // registers hold it through the point-value phase.
    T unv[2][4];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        unv[0][z] = ld(run, z, g0);
        unv[1][z] = ld(run, z, g1);
    }
    if (open) {
        // values on or beyond open ends (own cells past a partial tile's
        // domain edge included) take the boundary rule
        auto fix = [&](int xx, int yy, T *u) {
            const int c0 = ox + xx - 2, c1 = oy + yy - 2;
#pragma unroll
            for (int z = 0; z < 4; z++) {
                const int q0 = 2 * c0 + (z & 1), q1 = 2 * c1 + (z >> 1);
                const int m = ends(q0, q1);
                if (m) u[z] = bc_point(q0, q1, m);
            }
        };
        fix(x, y, own[0]);
        fix(x, y + 1, own[1]);
#pragma unroll
        for (int k = 0; k < NHI; k++) fix(hb[k] % SX, hb[k] / SX, halo[k]);
    }
    auto put_cell = [&](int b, const T *u) {
        smem[b] = V2<T>{u[0], pot(u[0])};
        smem[SXF * SG + b] = V2<T>{u[1], pot(u[1])};
        smem[SYF * SG + b] = V2<T>{u[2], pot(u[2])};
        smem[SK * SG + b] = V2<T>{u[3], pot(u[3])};
    };
    const int b0 = bix(x, y), b1 = b0 + SX;  // the own cells
    put_cell(b0, own[0]);
    put_cell(b1, own[1]);
#pragma unroll
    for (int k = 0; k < NHI; k++) put_cell(hb[k], halo[k]);
    __syncthreads();

    // ---- B: cell centres by inverting the tensor Simpson rule
    auto centre = [&](int b) {
        if (open) {
            const int c0 = ox + b % SX - 2, c1 = oy + b / SX - 2;
            const int m = ends(2 * c0, 2 * c1);
            if (m) {  // a ghost cell's centre
                const T u = bc_point(2 * c0, 2 * c1, m);
                smem[SC * SG + b] = V2<T>{u, pot(u)};
                return;
            }
        }
        const T faces = Su(SXF, b - 1) + Su(SXF, b) + Su(SYF, b - SX) + Su(SYF, b);
        const T corners = Su(SK, b - 1 - SX) + Su(SK, b - SX) + Su(SK, b - 1) + Su(SK, b);
        const T u = (T(36) * Su(0, b) - T(4) * faces - corners) * T(0.0625);
        smem[SC * SG + b] = V2<T>{u, pot(u)};
    };
    centre(b0);
    centre(b1);
    {
        // halo centres: rows 1 and TY+2 over columns [1, TX+3), columns 1
        // and TX+2 over rows [2, TY+2)
        constexpr int NR = 2 * (TX + 2), NH = NR + 2 * TY;
        for (int h = tid; h < NH; h += NT) {
            int xx, yy;
            if (h < NR) {
                const int r = h >= TX + 2;
                xx = 1 + h - r * (TX + 2);
                yy = r ? TY + 2 : 1;
            } else {
                const int h2 = h - NR;
                yy = 2 + (h2 >> 1);
                xx = (h2 & 1) ? TX + 2 : 1;
            }
            centre(bix(xx, yy));
        }
    }
    __syncthreads();

    T clamp_mag = T(0);  // largest safeguard clamp of an average
    bool bad = false;

    // ---- C: the six point values of the two own cells
    {
        // Per direction l, the point-value update adds kc_l t + kd_l d with
        //   t = (f_{-2} - 8 f_{-1} + 8 f_1 - f_2) + alpha d4,  d4 = 4th difference of u,
        //   d = 16 (a_{-1} + a_1) - (a_{-2} + a_2) - 30 a_0,
        // kc_l = -sc / (6 dx_l) and kd_l = sc / (3 dx_l^2), sc = dt (sc = 1 for
        // the residual); for pure quadratic fluxes t is c2 times
        //   (u_{-2}^2 - 8 u_{-1}^2 + 8 u_1^2 - u_2^2) + 2 sgn(c2) max|u| d4.
        const T sc = residual ? T(1) : dt;
        T kc[2], kd[2], sg2[2], kd30 = T(0);
#pragma unroll
        for (int l = 0; l < 2; l++) {
            kc[l] = -(BQ ? c2[l] : T(1)) * i6dx[l] * sc;
            kd[l] = idx2[l] * T(1.0 / 3.0) * sc;
            kd30 -= T(30) * kd[l];
            sg2[l] = c2[l] > T(0) ? T(2) : (c2[l] < T(0) ? T(-2) : T(0));
        }
        auto pv_dir = [&](int l, V2<T> w0, V2<T> w1, V2<T> w2, V2<T> w3, V2<T> w4, T acc) -> T {
            const T d4 = (w0.x + w4.x) - T(4) * (w1.x + w3.x) + T(6) * w2.x;
            T t;
            if constexpr (BQ) {
                const T m = vmax(vmax(vmax(T(fabs(w0.x)), T(fabs(w1.x))), T(fabs(w2.x))),
                                 vmax(T(fabs(w3.x)), T(fabs(w4.x))));
                const T e = (w0.x * w0.x - w4.x * w4.x) + T(8) * (w3.x * w3.x - w1.x * w1.x);
                t = e + (sg2[l] * m) * d4;
            } else {
                const T al = fmax(fmax(fmax(gq(l, w0.x), gq(l, w1.x)), fmax(gq(l, w2.x), gq(l, w3.x))), gq(l, w4.x));
                const T dcf = (fq(l, w0.x) - fq(l, w4.x)) + T(8) * (fq(l, w3.x) - fq(l, w1.x));
                t = dcf + al * d4;
            }
            // the centre term -30 a_0 of both directions is added once per point
            const T d = T(16) * (w1.y + w3.y) - (w0.y + w4.y);
            return (acc + kc[l] * t) + kd[l] * d;
        };
        T R[2][3];  // per own cell: x-face, y-face, corner point value (or du/dt)
        auto store_cell = [&](int c) {
            const bool own = c == 0 ? own0 : own1;
            const unsigned gi = c == 0 ? g0 : g1;
            if (!own) return;
#pragma unroll
            for (int z = 1; z < 4; z++) {
                // stored points on a high open end: right-hand side 0; a stage
                // writes the Dirichlet value or passes the input through, and
                // combines with the stored input
                const int me = open ? ends(2 * (ox + ci) + (z & 1), 2 * (oy + cj + c) + (z >> 1)) : 0;
                if (residual) {
                    st(z, gi, me ? T(0) : R[c][z - 1]);
                    continue;
                }
                T v = R[c][z - 1];
                T vin = Su(z == 1 ? SXF : (z == 2 ? SYF : SK), c == 0 ? b0 : b1);
                if (me) {
                    vin = v = ld(rin, z, gi);
#pragma unroll
                    for (int l = 1; l >= 0; l--)
                        if ((me >> l & 1) && Ic->bc[l][1] == 1) v = prm(Ic->bcv[l][1], (float)Ic->bcv[l][1]);
                }
                if (!isfinite(v)) bad = true;
                if constexpr (LIM) v = clampb(v, umin, umaxv);
                if (!fe) {
                    v = combine(v, unv[c][z], z, gi, vin);
                    if constexpr (LIM) v = clampb(v, umin, umaxv);
                }
                st(z, gi, v);
            }
        };
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int b = c == 0 ? b0 : b1;
            const bool z0 = residual;
            // x-face point (x+1/2, y)
            T r = kd30 * Sa(SXF, b) + (z0 ? T(0) : Su(SXF, b));
            r = pv_dir(0, S(SXF, b - 1), S(SC, b), S(SXF, b), S(SC, b + 1), S(SXF, b + 1), r);
            R[c][0] = pv_dir(1, S(SXF, b - SX), S(SK, b - SX), S(SXF, b), S(SK, b), S(SXF, b + SX), r);
            // y-face point (x, y+1/2)
            r = kd30 * Sa(SYF, b) + (z0 ? T(0) : Su(SYF, b));
            r = pv_dir(0, S(SYF, b - 1), S(SK, b - 1), S(SYF, b), S(SK, b), S(SYF, b + 1), r);
            R[c][1] = pv_dir(1, S(SYF, b - SX), S(SC, b), S(SYF, b), S(SC, b + SX), S(SYF, b + SX), r);
            // corner point (x+1/2, y+1/2)
            r = kd30 * Sa(SK, b) + (z0 ? T(0) : Su(SK, b));
            r = pv_dir(0, S(SK, b - 1), S(SYF, b), S(SK, b), S(SYF, b + 1), S(SK, b + 1), r);
            R[c][2] = pv_dir(1, S(SK, b - SX), S(SXF, b), S(SK, b), S(SXF, b + SX), S(SK, b + SX), r);
            // Buckley-Leverett fluxes store each cell before computing the
            // next: the two cells share stencil points, but holding both
            // cells' results and the shared flux terms at once costs more
            // registers than recomputing them (the kernels spilled, or ran at
            // one wave per SIMD in FP64)
            if constexpr (GEN) store_cell(c);
        }
        if constexpr (!GEN) {
            store_cell(0);
            store_cell(1);
        }
    }

    // ---- D1: faces.  The low-order (LLF) quantities on every face the
    // potentials' theta^d reads; the Simpson flux and theta^c on the faces
    // of the tile's cells (HI).
    struct Item {
        T v;
        int id;
    };
    auto face = [&](int l, int b, bool hi) -> Item {
        const V2<T> A = S(0, b);
        const V2<T> B = S(0, l == 0 ? b + 1 : b + SX);
        const int id = l == 0 ? FG::fx(b) : FG::fy(b);
        T fL = T(0), up = T(0), um = T(0), D = T(0), gmh = T(0);
        if constexpr (LIM) {
            const T Km = kmu[l];
            const T dA = (B.y - A.y) * idx1[l];
            if constexpr (BQ) {
                // f_l = c2 u^2: with D = b - a, g = |c2| max(|a|, |b|) (half the
                // LLF speed) and h = c2 (a + b) / 2, f(a) - f^L = D (g - h) and
                // f^L - f(b) = -D (g + h)
                D = B.x - A.x;
                const T g = cabs[l] * vmax(T(fabs(A.x)), T(fabs(B.x))), s2 = A.x + B.x;
                gmh = g - chalf[l] * s2;
                const T gph = g + chalf[l] * s2;
                up = A.x + Km * (dA + D * gmh);
                um = B.x - Km * (dA + D * gph);
            } else {
                const T fa = fq(l, A.x), fb = fq(l, B.x);
                const T al = GEN ? alpha_iv(l, A.x, B.x) : fmax(gq(l, A.x), gq(l, B.x));
                fL = T(0.5) * (fa + fb) - T(0.5) * al * (B.x - A.x);
                up = A.x + Km * (dA - fL + fa);
                um = B.x + Km * (fL - fb - dA);
            }
            ulp[id] = up;
            ulm[id] = um;
        }
        if (!hi) return Item{T(0), -1};
        // Simpson average of f_l over the three points of the face
        T fH;
        {
            const T k1 = l == 0 ? Su(SK, b - SX) : Su(SK, b - 1), k2 = Su(SK, b);
            const T m = l == 0 ? Su(SXF, b) : Su(SYF, b);
            if constexpr (BQ) fH = csix[l] * ((k1 * k1 + k2 * k2) + T(4) * (m * m));
            else fH = (fq(l, k1) + T(4) * fq(l, m) + fq(l, k2)) * T(1.0 / 6.0);
        }
        T F = fH;
        if constexpr (LIM) {
            if (!residual) {
                if constexpr (BQ) fL = c2[l] * (A.x * A.x) - D * gmh;
                const T df = fH - fL;
                // up moves by -3 K mu theta df, um by +3 K mu theta df
                const T gap = gap2<T>(df, um, up, umin, umax);
                F = fL + limited_part<T>(gap, df, ik3mu[l]);
            }
        }
        if constexpr (!LIM) fl[id] = F;
        return Item{F, id};
    };
    Item fo[4] = {face(0, b0, true), face(0, b1, true), face(1, b0, true), face(1, b1, true)};
    // halo faces: x-faces at columns 0, 1 (HI), TX+2 over the tile rows;
    // y-faces at rows 0, 1 (HI), TY+2 over the tile columns (from the next
    // wave boundary on, so no wave mixes the two)
    constexpr int NXHF = 3 * TY, Y0F = (NXHF + 63) / 64 * 64, NHF = Y0F + 3 * TX, NHFI = (NHF + NT - 1) / NT;
    Item fh[NHFI];
#pragma unroll
    for (int k = 0; k < NHFI; k++) {
        const int h = tid + k * NT;
        fh[k] = Item{T(0), -1};
        if (h < NXHF) {
            const int q = h / TY;
            fh[k] = face(0, bix(q < 2 ? q : TX + 2, 2 + h - q * TY), q == 1);
        } else if (h >= Y0F && h < NHF) {
            const int h2 = h - Y0F, q = h2 / TX;
            fh[k] = face(1, bix(2 + h2 - q * TX, q < 2 ? q : TY + 2), q == 1);
        }
    }
    __syncthreads();

    // ---- D2: cell-centred potentials a^H of Prop. 2.1 and their limited blend
    auto potential = [&](int l, int b) -> Item {
        const T corners = Sa(SK, b - 1 - SX) + Sa(SK, b - SX) + Sa(SK, b - 1) + Sa(SK, b);
        T aH;
        if (l == 0)
            aH = (T(8) * (Sa(SYF, b - SX) + Sa(SYF, b)) + T(32) * Sa(SC, b) - corners -
                  T(4) * (Sa(SXF, b - 1) + Sa(SXF, b))) *
                 T(1.0 / 36.0);
        else
            aH = (T(8) * (Sa(SXF, b - 1) + Sa(SXF, b)) + T(32) * Sa(SC, b) - corners -
                  T(4) * (Sa(SYF, b - SX) + Sa(SYF, b))) *
                 T(1.0 / 36.0);
        T Pv = aH;
        if constexpr (LIM) {
            if (!residual) {
                const T aL = Sa(0, b);
                // faces c-1/2 (f0) and c+1/2 (f1) of the cell
                const int f0 = l == 0 ? FG::fx(b - 1) : FG::fy(b - SX);
                const int f1 = l == 0 ? FG::fx(b) : FG::fy(b);
                const T pL = ulp[f0], mC = ulm[f0], pC = ulp[f1], mR = ulm[f1];
                const T da = aH - aL;
                // pL, mR move by +3 K nu theta da; pC, mC by -3 K nu theta da
                const T gap = gap4<T>(da, pL, mR, pC, mC, umin, umax);
                Pv = aL + limited_part<T>(gap, da, ik3nu[l]);
            }
        }
        const int id = l == 0 ? FG::px(b) : FG::py(b);
        if constexpr (!LIM) pc[id] = Pv;
        return Item{Pv, id};
    };
    Item po[4] = {potential(0, b0), potential(0, b1), potential(1, b0), potential(1, b1)};
    // halo potentials: x at columns 1, TX+2; y at rows 1, TY+2
    constexpr int NXHP = 2 * TY, Y0P = (NXHP + 63) / 64 * 64, NHP = Y0P + 2 * TX, NHPI = (NHP + NT - 1) / NT;
    Item ph[NHPI];
#pragma unroll
    for (int k = 0; k < NHPI; k++) {
        const int h = tid + k * NT;
        ph[k] = Item{T(0), -1};
        if (h < NXHP) {
            const int q = h / TY;
            ph[k] = potential(0, bix(q ? TX + 2 : 1, 2 + h - q * TY));
        } else if (h >= Y0P && h < NHP) {
            const int h2 = h - Y0P, q = h2 / TX;
            ph[k] = potential(1, bix(2 + h2 - q * TX, q ? TY + 2 : 1));
        }
    }
    if constexpr (LIM) {
        // every theta^d has read u^{L,+-}: the fluxes and potentials of the
        // update take their place
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; k++) {
            fl[fo[k].id] = fo[k].v;
            pc[po[k].id] = po[k].v;
        }
#pragma unroll
        for (int k = 0; k < NHFI; k++)
            if (fh[k].id >= 0) fl[fh[k].id] = fh[k].v;
#pragma unroll
        for (int k = 0; k < NHPI; k++)
            if (ph[k].id >= 0) pc[ph[k].id] = ph[k].v;
    }
    __syncthreads();

    // ---- D3: averages of the two own cells
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const bool own = c == 0 ? own0 : own1;
        if (!own) continue;
        const unsigned gi = c == 0 ? g0 : g1;
        const int b = c == 0 ? b0 : b1;
        const T dFx = fl[FG::fx(b)] - fl[FG::fx(b - 1)];
        const T dFy = fl[FG::fy(b)] - fl[FG::fy(b - SX)];
        const T dPx = pc[FG::px(b + 1)] - T(2) * pc[FG::px(b)] + pc[FG::px(b - 1)];
        const T dPy = pc[FG::py(b + SX)] - T(2) * pc[FG::py(b)] + pc[FG::py(b - SX)];
        if (residual) {
            st(0, gi, (dPx * idx2[0] + dPy * idx2[1]) - (dFx * idx1[0] + dFy * idx1[1]));
            continue;
        }
        const T u = Su(0, b);
        T v = u - (mu[0] * dFx + mu[1] * dFy) + (nu[0] * dPx + nu[1] * dPy);
        if (!isfinite(v)) bad = true;
        if constexpr (LIM) {
            const T cl = clampb(v, umin, umaxv);
            clamp_mag = fmax(clamp_mag, (T)fabs(cl - v));
            v = cl;
        }
        if (!fe) {
            v = combine(v, unv[c][0], 0, gi, u);
            if constexpr (LIM) {
                const T cl = clampb(v, umin, umaxv);
                clamp_mag = fmax(clamp_mag, (T)fabs(cl - v));
                v = cl;
            }
        }
        vlo = fmin(vlo, v);
        vhi = fmax(vhi, v);
        st(0, gi, v);
    }
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave_t<T>(&p.st[wk.x].clampmax, clamp_mag);
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
    }
}

template <class T, bool LIM, int TX, int TY>
constexpr long stage2o_lds_bytes()
{
    using FG = Own2Geo<TX, TY>;
    constexpr long NFB = LIM ? 2L * FG::NF : (long)FG::NF + FG::NC;
    return (long)sizeof(T) * (10L * FG::SG + 2 * ((NFB + 1) / 2));
}

}  // namespace af4
