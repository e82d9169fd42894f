// stage2o_kernel.hpp -- 2D stage kernel for fluxes f_l = c1 u + c2 u^2 (linear
// advection, Burgers), organised around thread-owned work items.
//
// Same arithmetic as the generic kernel of stage_kernel.hpp (the compact
// fourth-order AF scheme with monolithic convex limiting, J. Duan, arXiv
// 2510.11527, Secs. 2, 4, 5).  The instruction count is what bounds a stage,
// so the work is laid out to spend as few vector instructions per cell as
// possible:
//   * each thread owns a vertical pair of cells and does every per-cell item
//     of them itself -- loads, centres, the six point values, the two x- and
//     two y-faces to their right/top, the four cell-centred potentials and the
//     two average updates -- with all LDS addresses fixed offsets of one base;
//   * the items of the halo (cells, centres, faces and potentials outside the
//     tile that the tile's items read) are short wave-aligned extra passes;
//   * the half grid is split by parity into four cell-indexed sub-grids of
//     {u, a(u)}: centres C (x_i, y_j), x-faces X (x_{i+1/2}, y_j), y-faces
//     Y (x_i, y_{j+1/2}) and corners K (x_{i+1/2}, y_{j+1/2}); every 5-point
//     half-grid stencil alternates between two of them;
//   * f is recomputed from u (two instructions) instead of stored, which keeps
//     the LDS footprint at three workgroups per CU;
//   * the polynomial potentials without clamps (linear, u^2, u^3) take a
//     three-instruction path (template flag PP);
//   * global memory is addressed with 32-bit byte offsets from per-DoF-kind
//     base pointers (a plane holds fewer than 2^32 bytes; the host checks).
#pragma once
#include "stage2d_kernel.hpp"

namespace af4 {

template <class T>
__device__ __forceinline__ T ld_plane(const T *base, unsigned i)
{
    return *(const T *)((const char *)base + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st_plane(T *base, unsigned i, T v)
{
    *(T *)((char *)base + i * (unsigned)sizeof(T)) = v;
}

template <class T, bool LIM, bool PP, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stage2o_kernel(StageParams<T> p)
{
    static_assert(TX * TY == 2 * NT && TY % 2 == 0, "two cells per thread");
    static_assert(NT % TX == 0 && NT % 64 == 0, "threads cover whole columns and waves");
    constexpr int RX = TX + 4, RY = TY + 4;     // tile + halo 2
    constexpr int SX = RX + 1, SG = SX * RY;    // sub-grid row stride (padded) and size
    constexpr int FXE = TX + 3, FYE = TY + 3;   // faces along the normal
    constexpr int NXF = FXE * TY, NYF = TX * FYE;
    constexpr int CXE = TX + 2, CYE = TY + 2;   // potentials along the direction
    constexpr int NXC = CXE * TY, NYC = TX * CYE;
    constexpr int SC = 0, SXF = 1, SYF = 2, SK = 3;  // sub-grids

    __shared__ V2<T> hs[4 * SG];                // {u, a} of the four sub-grids
    __shared__ V2<T> cg[RX * RY];               // {ubar, a(ubar)} of the cells
    __shared__ T fl[NXF + NYF];                 // flux used in the update
    __shared__ T ulp[LIM ? NXF + NYF : 1];      // u^{L,+} of the left cell of a face
    __shared__ T ulm[LIM ? NXF + NYF : 1];      // u^{L,-} of the right cell
    __shared__ T pc[NXC + NYC];                 // potential used in the update

    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int2 wk = p.work[logical];
    const InstDev &I = p.inst[wk.x];
    const int n0 = I.n[0], n1 = I.n[1];
    const int tx0 = wk.y % I.tiles[0], ty0 = wk.y / I.tiles[0];
    const int ox = tx0 * TX, oy = ty0 * TY;
    const long long kst = I.kstride;
    const T *inz[4], *unz[4];
    T *outz[4];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        inz[z] = p.in + I.off + z * kst;
        unz[z] = p.un + I.off + z * kst;
        outz[z] = p.out + I.off + z * kst;
    }
    const bool residual = p.stage == 4;
    const double dtd = p.st[wk.x].dt;
    const int tid = (int)threadIdx.x;
    // own cells: region column x, rows y and y + 1
    const int ci = tid % TX, cj = 2 * (tid / TX);
    const int x = ci + 2, y = cj + 2;
    const bool ownx = ox + ci < n0;
    const bool own0 = ownx && oy + cj < n1, own1 = ownx && oy + cj + 1 < n1;
    const int gxo = wrap_index(ox + ci, n0);
    const unsigned g0 = (unsigned)(gxo + n0 * wrap_index(oy + cj, n1));
    const unsigned g1 = (unsigned)(gxo + n0 * wrap_index(oy + cj + 1, n1));

    const T inf = __builtin_huge_val();
    T vlo = inf, vhi = -inf;  // min / max of the averages written
    if (!residual && dtd == 0.0) {
        // the instance has reached its end time: the stage leaves it unchanged
#pragma unroll
        for (int z = 0; z < 4; z++) {
            if (own0) st_plane(outz[z], g0, ld_plane(inz[z], g0));
            if (own1) st_plane(outz[z], g1, ld_plane(inz[z], g1));
        }
        if (p.minmax) {
            if (own0) vlo = vhi = ld_plane(inz[0], g0);
            if (own1) {
                const T v = ld_plane(inz[0], g1);
                vlo = fmin(vlo, v);
                vhi = fmax(vhi, v);
            }
            minmax_wave(&p.st[wk.x], vlo, vhi);
        }
        return;
    }

    Phys<T> P;
    P.load(I, 2);
    T c1[2], c2[2], c2x2[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        c1[l] = P.fk[l] == kFLinear ? P.fc[l] : T(0);
        c2[l] = P.fk[l] == kFQuad ? P.fc[l] : T(0);
        c2x2[l] = T(2) * c2[l];
    }
    const T dt = (T)dtd;
    const T umin = P.umin, umax = P.umax;
    T idx1[2], idx2[2], i6dx[2], mu[2], nu[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        idx1[l] = (T)I.idx1[l];
        idx2[l] = (T)I.idx2[l];
        i6dx[l] = (T)I.i6dx[l];
        mu[l] = (T)p.st[wk.x].mu[l];
        nu[l] = (T)p.st[wk.x].nu[l];
    }
    const T K = T(4);

    auto pot = [&](T u) -> T {
        if constexpr (PP) return u * (P.pc1 + u * (P.pc2 + u * P.pc3));
        else return P.a(u);
    };
    auto fq = [&](int l, T u) -> T { return u * (c1[l] + c2[l] * u); };
    auto gq = [&](int l, T u) -> T { return fabs(c1[l] + c2x2[l] * u); };
    auto sg = [&](int s, int xx, int yy) -> int { return s * SG + xx + SX * yy; };
    auto S = [&](int s, int xx, int yy) -> V2<T> { return hs[sg(s, xx, yy)]; };
    auto Su = [&](int s, int xx, int yy) -> T { return hs[sg(s, xx, yy)].x; };
    auto Sa = [&](int s, int xx, int yy) -> T { return hs[sg(s, xx, yy)].y; };
    auto cgi = [&](int xx, int yy) -> int { return xx + RX * yy; };
    // face and potential slots: x-face between cells (xx, yy) and (xx+1, yy);
    // y-face between (xx, yy) and (xx, yy+1); potentials of cell (xx, yy)
    auto fxi = [&](int xx, int yy) -> int { return xx + FXE * (yy - 2); };
    auto fyi = [&](int xx, int yy) -> int { return NXF + (xx - 2) + TX * yy; };
    auto pxi = [&](int xx, int yy) -> int { return (xx - 1) + CXE * (yy - 2); };
    auto pyi = [&](int xx, int yy) -> int { return NXC + (xx - 2) + TX * (yy - 1); };

    // U^n of the own cells (used by the RK combination), fetched first
    const bool rk = !residual && p.stage >= 2;
    T unv[2][4];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        unv[0][z] = (rk && own0) ? ld_plane(unz[z], g0) : T(0);
        unv[1][z] = (rk && own1) ? ld_plane(unz[z], g1) : T(0);
    }

    // ---- A: cells of the tile and its halo -> LDS with their potentials
    auto load_cell = [&](int xx, int yy, unsigned gi) {
        const T ub = ld_plane(inz[0], gi), ux = ld_plane(inz[1], gi);
        const T uy = ld_plane(inz[2], gi), uc = ld_plane(inz[3], gi);
        cg[cgi(xx, yy)] = V2<T>{ub, pot(ub)};
        hs[sg(SXF, xx, yy)] = V2<T>{ux, pot(ux)};
        hs[sg(SYF, xx, yy)] = V2<T>{uy, pot(uy)};
        hs[sg(SK, xx, yy)] = V2<T>{uc, pot(uc)};
    };
    load_cell(x, y, g0);
    load_cell(x, y + 1, g1);
    {
        // halo: rows 0, 1, TY+2, TY+3 (all columns), then columns 0, 1,
        // TX+2, TX+3 of rows [2, TY+2)
        constexpr int NR = 4 * RX, NH = NR + 4 * TY;
        for (int h = tid; h < NH; h += NT) {
            int xx, yy;
            if (h < NR) {
                const int r = h / RX;
                xx = h - r * RX;
                yy = r < 2 ? r : r + TY;
            } else {
                const int h2 = h - NR, k = h2 & 3;
                yy = 2 + (h2 >> 2);
                xx = k < 2 ? k : k + TX;
            }
            const int gx = wrap_index(ox + xx - 2, n0), gy = wrap_index(oy + yy - 2, n1);
            load_cell(xx, yy, (unsigned)(gx + n0 * gy));
        }
    }
    __syncthreads();

    // ---- B: cell centres by inverting the tensor Simpson rule
    auto centre = [&](int xx, int yy) {
        const T faces = Su(SXF, xx - 1, yy) + Su(SXF, xx, yy) + Su(SYF, xx, yy - 1) + Su(SYF, xx, yy);
        const T corners = Su(SK, xx - 1, yy - 1) + Su(SK, xx, yy - 1) + Su(SK, xx - 1, yy) + Su(SK, xx, yy);
        const T u = (T(36) * cg[cgi(xx, yy)].x - T(4) * faces - corners) * T(0.0625);
        hs[sg(SC, xx, yy)] = V2<T>{u, pot(u)};
    };
    centre(x, y);
    centre(x, y + 1);
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
            centre(xx, yy);
        }
    }
    __syncthreads();

    double clamp_mag = 0.0;
    bool bad = false;

    // ---- C: the six point values of the two own cells
    {
        // one direction of du/dt at a point from its 5-point window
        auto pv_dir = [&](int l, V2<T> w0, V2<T> w1, V2<T> w2, V2<T> w3, V2<T> w4) -> T {
            const T al = fmax(fmax(fmax(gq(l, w0.x), gq(l, w1.x)), fmax(gq(l, w2.x), gq(l, w3.x))), gq(l, w4.x));
            const T dcf = (fq(l, w0.x) - fq(l, w4.x)) + T(8) * (fq(l, w3.x) - fq(l, w1.x));
            const T d4 = (w0.x + w4.x) - T(4) * (w1.x + w3.x) + T(6) * w2.x;
            const T conv = -(dcf + al * d4) * i6dx[l];
            const T d2 = ((w1.y + w3.y) * T(16.0 / 3.0) - (w0.y + w4.y) * T(1.0 / 3.0) - T(10) * w2.y) * idx2[l];
            return conv + d2;
        };
        T R[2][3];  // per own cell: x-face, y-face, corner point value
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int yy = y + c;
            // x-face point (x+1/2, yy)
            R[c][0] = pv_dir(0, S(SXF, x - 1, yy), S(SC, x, yy), S(SXF, x, yy), S(SC, x + 1, yy), S(SXF, x + 1, yy)) +
                      pv_dir(1, S(SXF, x, yy - 1), S(SK, x, yy - 1), S(SXF, x, yy), S(SK, x, yy), S(SXF, x, yy + 1));
            // y-face point (x, yy+1/2)
            R[c][1] = pv_dir(0, S(SYF, x - 1, yy), S(SK, x - 1, yy), S(SYF, x, yy), S(SK, x, yy), S(SYF, x + 1, yy)) +
                      pv_dir(1, S(SYF, x, yy - 1), S(SC, x, yy), S(SYF, x, yy), S(SC, x, yy + 1), S(SYF, x, yy + 1));
            // corner point (x+1/2, yy+1/2)
            R[c][2] = pv_dir(0, S(SK, x - 1, yy), S(SYF, x, yy), S(SK, x, yy), S(SYF, x + 1, yy), S(SK, x + 1, yy)) +
                      pv_dir(1, S(SK, x, yy - 1), S(SXF, x, yy), S(SK, x, yy), S(SXF, x, yy + 1), S(SK, x, yy + 1));
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const bool own = c == 0 ? own0 : own1;
            const unsigned gi = c == 0 ? g0 : g1;
            if (!own) continue;
#pragma unroll
            for (int z = 1; z < 4; z++) {
                if (residual) {
                    st_plane(outz[z], gi, R[c][z - 1]);
                    continue;
                }
                const int s = z == 1 ? SXF : (z == 2 ? SYF : SK);
                T v = Su(s, x, y + c) + dt * R[c][z - 1];
                if (!isfinite(v)) bad = true;
                if constexpr (LIM) v = clampb(v, umin, umax);
                v = rk_combine(p.stage, v, unv[c][z]);
                if constexpr (LIM) v = clampb(v, umin, umax);
                st_plane(outz[z], gi, v);
            }
        }
    }

    // ---- D1: faces.  The low-order (LLF) quantities on every face the
    // potentials' theta^d reads; the Simpson flux and theta^c on the faces
    // of the tile's cells (HI).
    auto face = [&](int l, int xx, int yy, bool hi) {
        const V2<T> A = cg[cgi(xx, yy)];
        const V2<T> B = l == 0 ? cg[cgi(xx + 1, yy)] : cg[cgi(xx, yy + 1)];
        const int id = l == 0 ? fxi(xx, yy) : fyi(xx, yy);
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
        if (!hi) return;
        // Simpson average of f_l over the three points of the face
        T fH;
        if (l == 0)
            fH = (fq(0, Su(SK, xx, yy - 1)) + T(4) * fq(0, Su(SXF, xx, yy)) + fq(0, Su(SK, xx, yy))) * T(1.0 / 6.0);
        else
            fH = (fq(1, Su(SK, xx - 1, yy)) + T(4) * fq(1, Su(SYF, xx, yy)) + fq(1, Su(SK, xx, yy))) * T(1.0 / 6.0);
        T F = fH;
        if constexpr (LIM) {
            if (!residual) {
                const T df = fH - fL;
                const T s3 = T(3) * K * mu[l] * df;
                // up moves by -s3, um by +s3
                const T gap = gap2<T>(s3, um, up, umin, umax);
                F = fL + theta_from_gap<T>(gap, (T)fabs(s3)) * df;
            }
        }
        fl[id] = F;
    };
    face(0, x, y, true);
    face(0, x, y + 1, true);
    face(1, x, y, true);
    face(1, x, y + 1, true);
    {
        // halo faces: x-faces at columns 0, 1 (HI), TX+2 over the tile rows;
        // y-faces at rows 0, 1 (HI), TY+2 over the tile columns (from the
        // next wave boundary on, so no wave mixes the two)
        constexpr int NXH = 3 * TY, Y0 = (NXH + 63) / 64 * 64, NH = Y0 + 3 * TX;
        for (int h = tid; h < NH; h += NT) {
            if (h < NXH) {
                const int k = h / TY;
                face(0, k < 2 ? k : TX + 2, 2 + h - k * TY, k == 1);
            } else if (h >= Y0) {
                const int h2 = h - Y0, k = h2 / TX;
                face(1, 2 + h2 - k * TX, k < 2 ? k : TY + 2, k == 1);
            }
        }
    }
    __syncthreads();

    // ---- D2: cell-centred potentials a^H of Prop. 2.1 and their limited blend
    auto potential = [&](int l, int xx, int yy) {
        const T corners = Sa(SK, xx - 1, yy - 1) + Sa(SK, xx, yy - 1) + Sa(SK, xx - 1, yy) + Sa(SK, xx, yy);
        T aH;
        if (l == 0)
            aH = (T(8) * (Sa(SYF, xx, yy - 1) + Sa(SYF, xx, yy)) + T(32) * Sa(SC, xx, yy) - corners -
                  T(4) * (Sa(SXF, xx - 1, yy) + Sa(SXF, xx, yy))) *
                 T(1.0 / 36.0);
        else
            aH = (T(8) * (Sa(SXF, xx - 1, yy) + Sa(SXF, xx, yy)) + T(32) * Sa(SC, xx, yy) - corners -
                  T(4) * (Sa(SYF, xx, yy - 1) + Sa(SYF, xx, yy))) *
                 T(1.0 / 36.0);
        T Pv = aH;
        if constexpr (LIM) {
            if (!residual) {
                const T aL = cg[cgi(xx, yy)].y;
                // faces c-1/2 (f0) and c+1/2 (f1) of the cell
                const int f0 = l == 0 ? fxi(xx - 1, yy) : fyi(xx, yy - 1);
                const int f1 = l == 0 ? fxi(xx, yy) : fyi(xx, yy);
                const T pL = ulp[f0], mC = ulm[f0], pC = ulp[f1], mR = ulm[f1];
                const T da = aH - aL;
                const T s = T(3) * K * nu[l] * da;
                // pL, mR move by +s; pC, mC by -s
                const T gap = gap4<T>(s, pL, mR, pC, mC, umin, umax);
                Pv = aL + theta_from_gap<T>(gap, (T)fabs(s)) * da;
            }
        }
        pc[l == 0 ? pxi(xx, yy) : pyi(xx, yy)] = Pv;
    };
    potential(0, x, y);
    potential(0, x, y + 1);
    potential(1, x, y);
    potential(1, x, y + 1);
    {
        // halo potentials: x at columns 1, TX+2; y at rows 1, TY+2
        constexpr int NXH = 2 * TY, Y0 = (NXH + 63) / 64 * 64, NH = Y0 + 2 * TX;
        for (int h = tid; h < NH; h += NT) {
            if (h < NXH) {
                const int k = h / TY;
                potential(0, k ? TX + 2 : 1, 2 + h - k * TY);
            } else if (h >= Y0) {
                const int h2 = h - Y0, k = h2 / TX;
                potential(1, 2 + h2 - k * TX, k ? TY + 2 : 1);
            }
        }
    }
    __syncthreads();

    // ---- D3: averages of the two own cells
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const bool own = c == 0 ? own0 : own1;
        if (!own) continue;
        const unsigned gi = c == 0 ? g0 : g1;
        const int yy = y + c;
        const T dFx = fl[fxi(x, yy)] - fl[fxi(x - 1, yy)];
        const T dFy = fl[fyi(x, yy)] - fl[fyi(x, yy - 1)];
        const T dPx = pc[pxi(x + 1, yy)] - T(2) * pc[pxi(x, yy)] + pc[pxi(x - 1, yy)];
        const T dPy = pc[pyi(x, yy + 1)] - T(2) * pc[pyi(x, yy)] + pc[pyi(x, yy - 1)];
        if (residual) {
            st_plane(outz[0], gi, (dPx * idx2[0] + dPy * idx2[1]) - (dFx * idx1[0] + dFy * idx1[1]));
            continue;
        }
        const T u = cg[cgi(x, yy)].x;
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
        vlo = fmin(vlo, v);
        vhi = fmax(vhi, v);
        st_plane(outz[0], gi, v);
    }
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave(&p.st[wk.x].clampmax, clamp_mag);
        if (p.minmax) minmax_wave(&p.st[wk.x], vlo, vhi);
    }
}

template <class T, bool LIM, int TX, int TY>
constexpr long stage2o_lds_bytes()
{
    constexpr long RX = TX + 4, RY = TY + 4;
    constexpr long NF = (TX + 3) * TY + TX * (TY + 3), NC = (TX + 2) * TY + TX * (TY + 2);
    return (long)sizeof(T) * (8 * (RX + 1) * RY + 2 * RX * RY + NF * (LIM ? 3 : 1) + NC);
}

}  // namespace af4
