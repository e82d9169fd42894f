// stage2q_kernel.hpp -- 2D stage kernel for fluxes f_l = c1_l u + c2_l u^2
// (linear advection, Burgers), no SI blending; gfx950.
//
// Arithmetic of the compact fourth-order AF scheme with monolithic convex
// limiting (J. Duan, arXiv 2510.11527, Secs. 2, 4, 5), as in the generic
// kernel, with this organisation:
//   * LDS holds the half grid of the tile + halo split by parity into four
//     cell-indexed sub-grids: centres, x-face, y-face and corner point values
//     (each entry {u, a(u)}).  Every stencil then reads consecutive entries
//     across consecutive lanes (no stride-2 bank conflicts), and every
//     half-index shift of Sec. 4 is a fixed (sub-grid, cell offset) pair.
//   * Each thread owns a vertical pair of cells.  Every phase first does the
//     thread's own items (its six point values, the four faces on the right
//     and top of its cells, the four cell potentials) and then a short list
//     of halo items, so no per-item index division is needed.
//   * f, |f'| are recomputed from u (one fma, one mul); the LLF interval
//     maximum of |f'| is the end-point maximum because |c1 + 2 c2 u| is
//     convex in u.
//   * theta^c / theta^d take one reciprocal each (shared denominators).
#pragma once
#include "stage2d_kernel.hpp"

namespace af4 {

template <class T, bool LIM, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stage2q_kernel(StageParams<T> p)
{
    static_assert(TX == 32 && TX * TY == 2 * NT && TY % 2 == 0, "32-wide tile, two cells per thread");
    constexpr int RX = TX + 4, RY = TY + 4;  // tile + halo 2
    constexpr int SX = RX + 1;               // padded row stride of a sub-grid
    constexpr int SG = SX * RY;              // entries per sub-grid
    constexpr int FXE = TX + 3, FYE = TY + 3;
    constexpr int NXF = FXE * TY, NYF = TX * FYE;
    constexpr int CXE = TX + 2, CYE = TY + 2;
    constexpr int NXC = CXE * TY, NYC = TX * CYE;
    // sub-grid kinds
    constexpr int KC = 0, KX = 1, KY = 2, KR = 3;  // centre, x-face, y-face, corner

    __shared__ V2<T> hs[4 * SG];              // {u, a(u)} of the four sub-grids
    __shared__ V2<T> cs[SG];                  // {ubar, a(ubar)}
    __shared__ T fl[NXF + NYF];               // flux used in the update
    __shared__ T ulp[LIM ? NXF + NYF : 1];    // u^{L,+} of the left/lower cell of a face
    __shared__ T ulm[LIM ? NXF + NYF : 1];    // u^{L,-} of the right/upper cell
    __shared__ T pc[NXC + NYC];               // potential used in the update

    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int2 wk = p.work[logical];
    const InstDev &I = p.inst[wk.x];
    const int n0 = I.n[0], n1 = I.n[1];
    const int tx0 = wk.y % I.tiles[0], ty0 = wk.y / I.tiles[0];
    const int ox = tx0 * TX, oy = ty0 * TY;
    const long long kst = I.kstride;
    const T *__restrict__ in = p.in + I.off;
    const T *__restrict__ un = p.un + I.off;
    T *__restrict__ out = p.out + I.off;
    const bool residual = p.stage == 4;
    const InstState &S = p.st[wk.x];
    const double dtd = S.dt;
    const int tid = (int)threadIdx.x;
    const int ci = tid % TX, cj = 2 * (tid / TX);       // own cells (ci, cj), (ci, cj + 1)
    const int X0 = ci + 2, Y0 = cj + 2;                 // their region coordinates
    const bool ownx = ox + ci < n0;
    const bool own0 = ownx && oy + cj < n1, own1 = ownx && oy + cj + 1 < n1;
    const long long g0 = (ox + ci) + (long long)n0 * (oy + cj), g1 = g0 + n0;

    if (!residual && dtd == 0.0) {
        for (int z = 0; z < 4; z++) {
            if (own0) out[z * kst + g0] = in[z * kst + g0];
            if (own1) out[z * kst + g1] = in[z * kst + g1];
        }
        return;
    }

    Phys<T> P;
    P.load(I, 2);
    T c1[2], c2[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        c1[l] = P.fk[l] == kFLinear ? P.fc[l] : T(0);
        c2[l] = P.fk[l] == kFQuad ? P.fc[l] : T(0);
    }
    const T dt = (T)dtd;
    const T umin = P.umin, umax = P.umax;
    T idx1[2], idx2[2], i6dx[2], mu[2], nu[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        idx1[l] = (T)I.idx1[l];
        idx2[l] = (T)I.idx2[l];
        i6dx[l] = (T)I.i6dx[l];
        mu[l] = (T)S.mu[l];
        nu[l] = (T)S.nu[l];
    }
    constexpr T K = T(4);

    auto fq = [&](int l, T u) -> T { return u * (c1[l] + c2[l] * u); };
    auto gq = [&](int l, T u) -> T { return fabs(c1[l] + T(2) * c2[l] * u); };
    auto at = [&](int k, int x, int y) -> V2<T> { return hs[k * SG + x + SX * y]; };
    auto put = [&](int k, int x, int y, T u) { hs[k * SG + x + SX * y] = V2<T>{u, P.a(u)}; };

    // U^n of the own cells, fetched before the barriers
    T unv[2][4];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        unv[0][z] = (!residual && p.stage >= 2 && own0) ? un[z * kst + g0] : T(0);
        unv[1][z] = (!residual && p.stage >= 2 && own1) ? un[z * kst + g1] : T(0);
    }

    // ---- A: tile + halo -> LDS
    auto load_cell = [&](int x, int y) {
        const int gx = wrap_index(ox + x - 2, n0), gy = wrap_index(oy + y - 2, n1);
        const long long gi = gx + (long long)n0 * gy;
        const T ub = in[gi];
        cs[x + SX * y] = V2<T>{ub, P.a(ub)};
        put(KX, x, y, in[kst + gi]);
        put(KY, x, y, in[2 * kst + gi]);
        put(KR, x, y, in[3 * kst + gi]);
    };
    // region cells in row-major order: each load instruction covers whole
    // rows of the tile + halo (coalesced)
    for (int t = tid; t < RX * RY; t += NT) load_cell(t % RX, t / RX);
    __syncthreads();

    // ---- B: centres on [1, TX+3) x [1, TY+3): own cells, then 100 halo cells
    auto centre = [&](int x, int y) {
        const T faces = at(KX, x - 1, y).x + at(KX, x, y).x + at(KY, x, y - 1).x + at(KY, x, y).x;
        const T corners = at(KR, x - 1, y - 1).x + at(KR, x, y - 1).x + at(KR, x - 1, y).x + at(KR, x, y).x;
        put(KC, x, y, (T(36) * cs[x + SX * y].x - T(4) * faces - corners) * T(0.0625));
    };
    {
        constexpr int NS = 2 * (TY + 2), NR = 2 * TX;
        for (int t = tid; t < 2 * NT + NS + NR; t += NT) {
            int x, y;
            if (t < 2 * NT) {
                x = X0;
                y = Y0 + t / NT;
            } else if (t < 2 * NT + NS) {
                const int u = t - 2 * NT;
                x = (u & 1) ? TX + 2 : 1;
                y = 1 + (u >> 1);
            } else {
                const int u = t - 2 * NT - NS;
                x = 2 + u % TX;
                y = (u / TX) ? TY + 2 : 1;
            }
            centre(x, y);
        }
    }
    __syncthreads();

    double clamp_mag = 0.0;
    bool bad = false;

    // ---- C: the six point values of the two own cells
    {
        // du/dt contribution of direction l from a 5-point window
        auto pv_dir = [&](int l, const V2<T> (&w)[5]) -> T {
            const T al = fmax(fmax(fmax(gq(l, w[0].x), gq(l, w[1].x)), fmax(gq(l, w[2].x), gq(l, w[3].x))),
                              gq(l, w[4].x));
            const T dcf = (fq(l, w[0].x) - fq(l, w[4].x)) + T(8) * (fq(l, w[3].x) - fq(l, w[1].x));
            const T d4 = (w[0].x + w[4].x) - T(4) * (w[1].x + w[3].x) + T(6) * w[2].x;
            const T conv = -(dcf + al * d4) * i6dx[l];
            const T d2 = ((w[1].y + w[3].y) * T(16.0 / 3.0) - (w[0].y + w[4].y) * T(1.0 / 3.0) - T(10) * w[2].y) * idx2[l];
            return conv + d2;
        };
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int x = X0, y = Y0 + c;
            T R[3];
            T U0[3];
            {   // x-face point (x+1/2, y)
                const V2<T> wx[5] = {at(KX, x - 1, y), at(KC, x, y), at(KX, x, y), at(KC, x + 1, y), at(KX, x + 1, y)};
                const V2<T> wy[5] = {at(KX, x, y - 1), at(KR, x, y - 1), at(KX, x, y), at(KR, x, y), at(KX, x, y + 1)};
                R[0] = pv_dir(0, wx) + pv_dir(1, wy);
                U0[0] = wx[2].x;
            }
            {   // y-face point (x, y+1/2)
                const V2<T> wx[5] = {at(KY, x - 1, y), at(KR, x - 1, y), at(KY, x, y), at(KR, x, y), at(KY, x + 1, y)};
                const V2<T> wy[5] = {at(KY, x, y - 1), at(KC, x, y), at(KY, x, y), at(KC, x, y + 1), at(KY, x, y + 1)};
                R[1] = pv_dir(0, wx) + pv_dir(1, wy);
                U0[1] = wx[2].x;
            }
            {   // corner point (x+1/2, y+1/2)
                const V2<T> wx[5] = {at(KR, x - 1, y), at(KY, x, y), at(KR, x, y), at(KY, x + 1, y), at(KR, x + 1, y)};
                const V2<T> wy[5] = {at(KR, x, y - 1), at(KX, x, y), at(KR, x, y), at(KX, x, y + 1), at(KR, x, y + 1)};
                R[2] = pv_dir(0, wx) + pv_dir(1, wy);
                U0[2] = wx[2].x;
            }
            const bool own = c == 0 ? own0 : own1;
            const long long gi = c == 0 ? g0 : g1;
            if (!own) continue;
#pragma unroll
            for (int z = 1; z < 4; z++) {
                if (residual) {
                    out[z * kst + gi] = R[z - 1];
                    continue;
                }
                T v = U0[z - 1] + dt * R[z - 1];
                if (!isfinite(v)) bad = true;
                if constexpr (LIM) v = clampb(v, umin, umax);
                v = rk_combine(p.stage, v, unv[c][z]);
                if constexpr (LIM) v = clampb(v, umin, umax);
                out[z * kst + gi] = v;
            }
        }
    }

    // ---- D1: faces.  x-face array: left cell x in [0, TX+3), row y-2;
    // y-face array: column x-2, lower cell y in [0, TY+3).
    auto face = [&](bool xd, int x, int y) {
        const int l = xd ? 0 : 1;
        const int id = xd ? x + FXE * (y - 2) : NXF + (x - 2) + TX * y;
        const bool need_hi = xd ? (x >= 1 && x < TX + 2) : (y >= 1 && y < TY + 2);
        const V2<T> A = cs[x + SX * y];
        const V2<T> B = xd ? cs[x + 1 + SX * y] : cs[x + SX * (y + 1)];
        const T fa = fq(l, A.x), fb = fq(l, B.x);
        T fL = T(0), up = T(0), um = T(0);
        if constexpr (LIM) {
            const T al = fmax(gq(l, A.x), gq(l, B.x));
            fL = T(0.5) * (fa + fb) - T(0.5) * al * (B.x - A.x);
            const T Km = K * mu[l];
            const T dA = (B.y - A.y) * idx1[l];
            up = A.x + Km * (dA - fL + fa);
            um = B.x + Km * (fL - fb - dA);
            ulp[id] = up;
            ulm[id] = um;
        }
        if (!need_hi) return;
        const T fH = xd ? (fq(0, at(KR, x, y - 1).x) + T(4) * fq(0, at(KX, x, y).x) + fq(0, at(KR, x, y).x)) * T(1.0 / 6.0)
                        : (fq(1, at(KR, x - 1, y).x) + T(4) * fq(1, at(KY, x, y).x) + fq(1, at(KR, x, y).x)) * T(1.0 / 6.0);
        T F = fH;
        if constexpr (LIM) {
            if (!residual) {
                const T df = fH - fL;
                const T s3 = T(3) * K * mu[l] * df;
                const T gap = gap2<T>(s3, um, up, umin, umax);
                F = fL + theta_from_gap<T>(gap, (T)fabs(s3)) * df;
            }
        }
        fl[id] = F;
    };
    {
        // own: x-faces right of the two cells, then y-faces above them; halo:
        // x-faces with left cell x in {0, 1, TX+2}, y-faces with lower cell
        // y in {0, 1, TY+2}
        constexpr int NXH = 3 * TY, NYH = 3 * TX;
        for (int t = tid; t < 4 * NT + NXH + NYH; t += NT) {
            bool xd;
            int x, y;
            if (t < 4 * NT) {
                const int k = t / NT;
                xd = k < 2;
                x = X0;
                y = Y0 + (k & 1);
            } else if (t < 4 * NT + NXH) {
                const int u = t - 4 * NT, sx = u / TY;
                xd = true;
                x = sx < 2 ? sx : TX + 2;
                y = 2 + u % TY;
            } else {
                const int u = t - 4 * NT - NXH, sy = u / TX;
                xd = false;
                x = 2 + u % TX;
                y = sy < 2 ? sy : TY + 2;
            }
            face(xd, x, y);
        }
    }
    __syncthreads();

    // ---- D2: cell-centred potentials, limited with theta^d.
    // x-cell array: x-1 in [0, TX+2), row y-2; y-cell array: column x-2, y-1.
    auto cellp = [&](bool xd, int x, int y) {
        const int id = xd ? (x - 1) + CXE * (y - 2) : NXC + (x - 2) + TX * (y - 1);
        const T a4 = at(KR, x - 1, y - 1).y + at(KR, x, y - 1).y + at(KR, x - 1, y).y + at(KR, x, y).y;
        const T ax = at(KX, x - 1, y).y + at(KX, x, y).y, ay = at(KY, x, y - 1).y + at(KY, x, y).y;
        const T ac = at(KC, x, y).y;
        // (-1, 8, -1) along the direction, (1, 4, 1) across, / 36 (Prop. 2.1)
        const T aH = xd ? (T(8) * ay + T(32) * ac - a4 - T(4) * ax) * T(1.0 / 36.0)
                        : (T(8) * ax + T(32) * ac - a4 - T(4) * ay) * T(1.0 / 36.0);
        T Pv = aH;
        if constexpr (LIM) {
            if (!residual) {
                const T aL = cs[x + SX * y].y;
                // faces below / above the cell in its direction
                const int f0 = xd ? (x - 1) + FXE * (y - 2) : NXF + (x - 2) + TX * (y - 1);
                const int f1 = xd ? f0 + 1 : f0 + TX;
                const T pL = ulp[f0], mC = ulm[f0], pC = ulp[f1], mR = ulm[f1];
                const T da = aH - aL;
                const T s = T(3) * K * nu[xd ? 0 : 1] * da;
                const T gap = gap4<T>(s, pL, mR, pC, mC, umin, umax);
                Pv = aL + theta_from_gap<T>(gap, (T)fabs(s)) * da;
            }
        }
        pc[id] = Pv;
    };
    {
        constexpr int NXH = 2 * TY, NYH = 2 * TX;
        for (int t = tid; t < 4 * NT + NXH + NYH; t += NT) {
            bool xd;
            int x, y;
            if (t < 4 * NT) {
                const int k = t / NT;
                xd = k < 2;
                x = X0;
                y = Y0 + (k & 1);
            } else if (t < 4 * NT + NXH) {
                const int u = t - 4 * NT;
                xd = true;
                x = (u / TY) ? TX + 2 : 1;
                y = 2 + u % TY;
            } else {
                const int u = t - 4 * NT - NXH;
                xd = false;
                x = 2 + u % TX;
                y = (u / TX) ? TY + 2 : 1;
            }
            cellp(xd, x, y);
        }
    }
    __syncthreads();

    // ---- D3: averages of the two own cells
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const bool own = c == 0 ? own0 : own1;
        if (!own) continue;
        const long long gi = c == 0 ? g0 : g1;
        const int x = X0, y = Y0 + c;
        const int fx = x + FXE * (y - 2), fy = NXF + (x - 2) + TX * y;
        const int cx = (x - 1) + CXE * (y - 2), cy = NXC + (x - 2) + TX * (y - 1);
        const T dFx = fl[fx] - fl[fx - 1], dFy = fl[fy] - fl[fy - TX];
        const T dPx = pc[cx + 1] - T(2) * pc[cx] + pc[cx - 1];
        const T dPy = pc[cy + TX] - T(2) * pc[cy] + pc[cy - TX];
        if (residual) {
            out[gi] = (dPx * idx2[0] + dPy * idx2[1]) - (dFx * idx1[0] + dFy * idx1[1]);
            continue;
        }
        const T u = cs[x + SX * y].x;
        T v = u - (mu[0] * dFx + mu[1] * dFy) + (nu[0] * dPx + nu[1] * dPy);
        if (!isfinite(v)) bad = true;
        if constexpr (LIM) {
            const T cl = clampb(v, umin, umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(cl - v));
            v = cl;
        }
        v = rk_combine(p.stage, v, unv[c][0]);
        if constexpr (LIM) {
            const T cl = clampb(v, umin, umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(cl - v));
            v = cl;
        }
        out[gi] = v;
    }
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave(&p.st[wk.x].clampmax, clamp_mag);
    }
}

template <class T, bool LIM, int TX, int TY>
constexpr long stage2q_lds_bytes()
{
    constexpr long SG = (TX + 5) * (TY + 4);
    constexpr long NF = (TX + 3) * TY + TX * (TY + 3), NC = (TX + 2) * TY + TX * (TY + 2);
    return (long)sizeof(T) * (2 * 4 * SG + 2 * SG + NF * (LIM ? 3 : 1) + NC);
}

}  // namespace af4
