// stage2d_kernel.hpp -- 2D stage kernel tuned for gfx950 (no SI blending).
//
// Same arithmetic as the generic kernel of stage_kernel.hpp (the compact
// fourth-order AF scheme with monolithic convex limiting, J. Duan, arXiv
// 2510.11527, Secs. 2, 4, 5), reorganised to cut instructions:
//   * every half-grid point of the tile+halo gets {u, a(u), f_x(u), f_y(u)}
//     once, in LDS, so stencils read values instead of re-evaluating f and a;
//   * for fluxes c1 u + c2 u^2 (linear, Burgers) |f'| is one fused multiply-add
//     and the LLF interval maximum is the end-point maximum (|f'| is convex);
//   * each thread owns a vertical pair of cells, so the twelve 5-point
//     stencils of its six point values share their LDS reads;
//   * theta^c and theta^d take one reciprocal each: the Theta's of one theta
//     share the denominator |3 K mu Delta f| (or |3 K nu Delta a|), and the
//     largest admissible blend is min(1, gap / denominator) with gap the
//     distance of the low-order states to the bound they move towards;
//   * U^n of the own cells is fetched with the tile, before any barrier.
#pragma once
#include "stage_kernel.hpp"

namespace af4 {

template <class T>
struct V4 {
    T x, y, z, w;
};
template <class T>
struct V2 {
    T x, y;
};

// FT: keep f_x, f_y in the half-grid table (else recomputed from u; only
// for quadratic fluxes)
template <class T, bool LIM, bool QF, bool FT, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stage2d_kernel(StageParams<T> p)
{
    static_assert(TX * TY == 2 * NT && TY % 2 == 0, "two cells per thread");
    static_assert(NT % TX == 0, "threads cover whole columns");
    constexpr int RX = TX + 4, RY = TY + 4;     // tile + halo 2
    constexpr int GX = 2 * RX, GY = 2 * RY;     // half grid
    constexpr int FXE = TX + 3, FYE = TY + 3;   // face extents along the normal
    constexpr int NXF = FXE * TY, NYF = TX * FYE;
    constexpr int CXE = TX + 2, CYE = TY + 2;   // cell extents along the direction
    constexpr int NXC = CXE * TY, NYC = TX * CYE;

    constexpr bool TAB = FT || !QF;
    // {u, a} table: the half grid split by parity into four cell-indexed
    // sub-grids (centres, x-faces, y-faces, corners), rows padded by one
    constexpr int SX = RX + 1, SG = SX * RY;
    __shared__ V4<T> hg[TAB ? GX * GY : 1];     // {u, a, f_x, f_y} on the half grid
    __shared__ V2<T> hs[TAB ? 1 : 4 * SG];      // {u, a} on the split half grid
    __shared__ V4<T> cg[RX * RY];               // {ubar, a, f_x, f_y} of the cells
    __shared__ T gq[QF ? 1 : 2 * GX * GY];      // |f_x'|, |f_y'| (general fluxes)
    __shared__ T fl[NXF + NYF];                 // flux used in the update
    __shared__ T ulp[LIM ? NXF + NYF : 1];      // u^{L,+} of the left cell of a face
    __shared__ T ulm[LIM ? NXF + NYF : 1];      // u^{L,-} of the right cell
    __shared__ T pc[NXC + NYC];                 // potential used in the update

    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int4 wk = p.work[logical];
    const InstDev &I = p.inst[wk.x];
    const int n0 = I.n[0], n1 = I.n[1];
    const int tx0 = wk.y, ty0 = wk.z;
    const int ox = tx0 * TX, oy = ty0 * TY;
    const long long kst = I.kstride;
    const T *__restrict__ in = p.in + I.off;
    const T *__restrict__ un = p.un + I.off;
    const T *__restrict__ x1 = p.x1 ? p.x1 + I.off : nullptr;
    T *__restrict__ out = p.out + I.off;
    const bool residual = p.stage == kStageRHS;
    const double dtd = p.st[wk.x].dt;
    const int tid = (int)threadIdx.x;
    // own cells of this thread: column i, rows j and j+1
    const int ci = tid % TX, cj = 2 * (tid / TX);
    const bool ownx = ox + ci < n0;
    const bool own0 = ownx && oy + cj < n1, own1 = ownx && oy + cj + 1 < n1;
    const long long g0 = (ox + ci) + (long long)n0 * (oy + cj), g1 = g0 + n0;

    const T inf = __builtin_huge_val();
    T vlo = inf, vhi = -inf;  // min / max of the averages written
    if (!residual && dtd == 0.0) {
        // the instance has reached its end time: the stage leaves it unchanged
        for (int z = 0; z < 4; z++) {
            if (own0) out[z * kst + g0] = in[z * kst + g0];
            if (own1) out[z * kst + g1] = in[z * kst + g1];
        }
        if (p.mm) {
            if (own0) vlo = vhi = in[g0];
            if (own1) {
                vlo = fmin(vlo, in[g1]);
                vhi = fmax(vhi, in[g1]);
            }
            minmax_slot(p.mm, logical, vlo, vhi);
        }
        return;
    }

    Phys<T> P;
    P.load(I, 2);
    // quadratic fluxes f_l = c1 u + c2 u^2
    T c1[2], c2[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        c1[l] = P.fk[l] == kFLinear ? P.fc[l] : T(0);
        c2[l] = P.fk[l] == kFQuad ? P.fc[l] : T(0);
    }
    const T dt = (T)dtd * p.dts;
    const T umin = P.umin, umax = P.umax;
    T idx1[2], idx2[2], i6dx[2], mu[2], nu[2];
#pragma unroll
    for (int l = 0; l < 2; l++) {
        idx1[l] = (T)I.idx1[l];
        idx2[l] = (T)I.idx2[l];
        i6dx[l] = (T)I.i6dx[l];
        mu[l] = (T)p.st[wk.x].mu[l] * p.dts;
        nu[l] = (T)p.st[wk.x].nu[l] * p.dts;
    }
    const T K = T(4);

    auto fq = [&](int l, T u) -> T { return QF ? u * (c1[l] + c2[l] * u) : P.f(l, u); };
    auto gq_of = [&](int l, T u) -> T { return QF ? fabs(c1[l] + T(2) * c2[l] * u) : P.adf(l, u); };
    auto tab = [&](T u) -> V4<T> { return V4<T>{u, P.a(u), fq(0, u), fq(1, u)}; };
    // index of half-grid point (x, y) in the split table
    auto sidx = [&](int x, int y) -> int { return ((x & 1) + 2 * (y & 1)) * SG + (x >> 1) + SX * (y >> 1); };
    auto put = [&](int x, int y, T u) {
        if constexpr (TAB) hg[x + GX * y] = tab(u);
        else hs[sidx(x, y)] = V2<T>{u, P.a(u)};
    };
    auto H = [&](int x, int y) -> V4<T> {
        if constexpr (TAB) {
            return hg[x + GX * y];
        } else {
            const V2<T> v = hs[sidx(x, y)];
            return V4<T>{v.x, v.y, fq(0, v.x), fq(1, v.x)};
        }
    };
    auto Hu = [&](int x, int y) -> T {
        if constexpr (TAB) return hg[x + GX * y].x;
        else return hs[sidx(x, y)].x;
    };
    auto Ha = [&](int x, int y) -> T {
        if constexpr (TAB) return hg[x + GX * y].y;
        else return hs[sidx(x, y)].y;
    };

    // U^n of the own cells (used by the RK combination), fetched early
    T unv[2][4];
#pragma unroll
    for (int z = 0; z < 4; z++) {
        unv[0][z] = (!residual && p.mode != kCombFE && own0) ? un[z * kst + g0] : T(0);
        unv[1][z] = (!residual && p.mode != kCombFE && own1) ? un[z * kst + g1] : T(0);
    }

    // ---- A: tile + halo -> LDS, with the pointwise tables
    for (int id = tid; id < RX * RY; id += NT) {
        const int x = id % RX, y = id / RX;
        const int gx = wrap_index(ox + x - 2, n0), gy = wrap_index(oy + y - 2, n1);
        const long long gi = gx + (long long)n0 * gy;
        const T ub = in[gi], ux = in[kst + gi], uy = in[2 * kst + gi], uc = in[3 * kst + gi];
        cg[id] = tab(ub);
        put(2 * x + 1, 2 * y, ux);
        put(2 * x, 2 * y + 1, uy);
        put(2 * x + 1, 2 * y + 1, uc);
        if constexpr (!QF) {
            const int px = (2 * x + 1) + GX * (2 * y), py = (2 * x) + GX * (2 * y + 1), pc_ = (2 * x + 1) + GX * (2 * y + 1);
            gq[2 * px] = gq_of(0, ux);
            gq[2 * px + 1] = gq_of(1, ux);
            gq[2 * py] = gq_of(0, uy);
            gq[2 * py + 1] = gq_of(1, uy);
            gq[2 * pc_] = gq_of(0, uc);
            gq[2 * pc_ + 1] = gq_of(1, uc);
        }
    }
    __syncthreads();

    // ---- B: cell centres on region cells [1, RX-1) x [1, RY-1)
    for (int id = tid; id < CXE * CYE; id += NT) {
        const int x = id % CXE + 1, y = id / CXE + 1;
        const int hx = 2 * x, hy = 2 * y;
        const T faces = Hu(hx - 1, hy) + Hu(hx + 1, hy) + Hu(hx, hy - 1) + Hu(hx, hy + 1);
        const T corners = Hu(hx - 1, hy - 1) + Hu(hx + 1, hy - 1) + Hu(hx - 1, hy + 1) + Hu(hx + 1, hy + 1);
        const T u = (T(36) * cg[x + RX * y].x - T(4) * faces - corners) * T(0.0625);
        put(hx, hy, u);
        if constexpr (!QF) {
            gq[2 * (hx + GX * hy)] = gq_of(0, u);
            gq[2 * (hx + GX * hy) + 1] = gq_of(1, u);
        }
    }
    __syncthreads();

    double clamp_mag = 0.0;
    bool bad = false;

    // ---- C: the six point values of the thread's two cells
    {
        const int x = ci + 2, y = cj + 2;         // region coordinates of the first cell
        const int hx = 2 * x, hy = 2 * y;
        // one direction of du/dt at a point from its 5-point window w[0..4]
        auto pv_dir = [&](int l, const V4<T> *w, const T *g) -> T {
            const T f0 = l == 0 ? w[0].z : w[0].w, f1 = l == 0 ? w[1].z : w[1].w;
            const T f3 = l == 0 ? w[3].z : w[3].w, f4 = l == 0 ? w[4].z : w[4].w;
            T al;
            if constexpr (QF) {
                al = fmax(fmax(fmax(gq_of(l, w[0].x), gq_of(l, w[1].x)), fmax(gq_of(l, w[2].x), gq_of(l, w[3].x))),
                          gq_of(l, w[4].x));
            } else {
                al = fmax(fmax(fmax(g[0], g[1]), fmax(g[2], g[3])), g[4]);
            }
            const T dcf = (f0 - f4) + T(8) * (f3 - f1);
            const T d4 = (w[0].x + w[4].x) - T(4) * (w[1].x + w[3].x) + T(6) * w[2].x;
            const T conv = -(dcf + al * d4) * i6dx[l];
            const T d2 = ((w[1].y + w[3].y) * T(16.0 / 3.0) - (w[0].y + w[4].y) * T(1.0 / 3.0) - T(10) * w[2].y) * idx2[l];
            return conv + d2;
        };
        auto gwin = [&](int l, int px, int py, int sx, int sy, T *g) {
            if constexpr (!QF) {
#pragma unroll
                for (int s = 0; s < 5; s++) g[s] = gq[2 * ((px + (s - 2) * sx) + GX * (py + (s - 2) * sy)) + l];
            }
        };
        // rows hy..hy+3 around columns hx-2..hx+3; columns hx, hx+1 rows hy-2..hy+5
        V4<T> w[5];
        T gw[5];
        T R[6];  // X0, Y0, C0, X1, Y1, C1
        const int px[6] = {hx + 1, hx, hx + 1, hx + 1, hx, hx + 1};
        const int py[6] = {hy, hy + 1, hy + 1, hy + 2, hy + 3, hy + 3};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            // x direction
#pragma unroll
            for (int s = 0; s < 5; s++) w[s] = H(px[k] + s - 2, py[k]);
            gwin(0, px[k], py[k], 1, 0, gw);
            T r = pv_dir(0, w, gw);
            // y direction
#pragma unroll
            for (int s = 0; s < 5; s++) w[s] = H(px[k], py[k] + s - 2);
            gwin(1, px[k], py[k], 0, 1, gw);
            r += pv_dir(1, w, gw);
            R[k] = r;
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const bool own = c == 0 ? own0 : own1;
            const long long gi = c == 0 ? g0 : g1;
            if (!own) continue;
#pragma unroll
            for (int z = 1; z < 4; z++) {
                const int k = 3 * c + z - 1;
                if (residual) {
                    out[z * kst + gi] = R[k];
                    continue;
                }
                const T vin = Hu(px[k], py[k]);
                T v = vin + dt * R[k];
                if (!isfinite(v)) bad = true;
                if constexpr (LIM) v = clampb(v, umin, umax);
                v = stage_combine(p, v, unv[c][z], x1 ? x1[z * kst + gi] : T(0), vin);
                if constexpr (LIM) v = clampb(v, umin, umax);
                out[z * kst + gi] = v;
            }
        }
    }

    // ---- D1: faces.  x-faces: index f in [0, TX+3) <-> left cell region x = f,
    // rows region y in [2, TY+2); y-faces: columns [2, TX+2), f <-> lower cell y = f.
    for (int id = tid; id < NXF + NYF; id += NT) {
        const bool xd = id < NXF;
        const int rem = xd ? id : id - NXF;
        int f, x, y;
        if (xd) {
            f = rem % FXE;
            x = f;
            y = rem / FXE + 2;
        } else {
            f = rem / TX;
            x = rem % TX + 2;
            y = f;
        }
        const int l = xd ? 0 : 1;
        const int fe = xd ? FXE : FYE;
        const bool need_hi = f >= 1 && f < fe - 1;
        if (!LIM && !need_hi) continue;
        const V4<T> A = cg[x + RX * y];
        const V4<T> B = xd ? cg[x + 1 + RX * y] : cg[x + RX * (y + 1)];
        const T fa = xd ? A.z : A.w, fb = xd ? B.z : B.w;
        T fL = T(0), up = T(0), um = T(0);
        if constexpr (LIM) {
            T al;
            if constexpr (QF) al = fmax(gq_of(l, A.x), gq_of(l, B.x));
            else al = P.alpha_int(l, A.x, B.x);
            fL = T(0.5) * (fa + fb) - T(0.5) * al * (B.x - A.x);
            const T Km = K * mu[l];
            const T dA = (B.y - A.y) * idx1[l];
            up = A.x + Km * (dA - fL + fa);
            um = B.x + Km * (fL - fb - dA);
            ulp[id] = up;
            ulm[id] = um;
        }
        if (!need_hi) continue;
        // Simpson face average of f_l over the three face points
        T fH;
        if (xd) fH = (H(2 * x + 1, 2 * y - 1).z + T(4) * H(2 * x + 1, 2 * y).z + H(2 * x + 1, 2 * y + 1).z) * T(1.0 / 6.0);
        else fH = (H(2 * x - 1, 2 * y + 1).w + T(4) * H(2 * x, 2 * y + 1).w + H(2 * x + 1, 2 * y + 1).w) * T(1.0 / 6.0);
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
    }
    __syncthreads();

    // ---- D2: cell-centred potentials.  x-cells: index c in [0, TX+2) <-> region
    // x = c + 1, rows [2, TY+2); y-cells: columns [2, TX+2), c <-> y = c + 1.
    for (int id = tid; id < NXC + NYC; id += NT) {
        const bool xd = id < NXC;
        const int rem = xd ? id : id - NXC;
        int c, x, y;
        if (xd) {
            c = rem % CXE;
            x = c + 1;
            y = rem / CXE + 2;
        } else {
            c = rem / TX;
            x = rem % TX + 2;
            y = c + 1;
        }
        const int hx = 2 * x, hy = 2 * y;
        T aH;
        if (xd)
            aH = (T(8) * (Ha(hx, hy - 1) + Ha(hx, hy + 1)) + T(32) * Ha(hx, hy) -
                  (Ha(hx - 1, hy - 1) + Ha(hx + 1, hy - 1) + Ha(hx - 1, hy + 1) + Ha(hx + 1, hy + 1)) -
                  T(4) * (Ha(hx - 1, hy) + Ha(hx + 1, hy))) *
                 T(1.0 / 36.0);
        else
            aH = (T(8) * (Ha(hx - 1, hy) + Ha(hx + 1, hy)) + T(32) * Ha(hx, hy) -
                  (Ha(hx - 1, hy - 1) + Ha(hx + 1, hy - 1) + Ha(hx - 1, hy + 1) + Ha(hx + 1, hy + 1)) -
                  T(4) * (Ha(hx, hy - 1) + Ha(hx, hy + 1))) *
                 T(1.0 / 36.0);
        T Pv = aH;
        if constexpr (LIM) {
            if (!residual) {
                const T aL = cg[x + RX * y].y;
                // faces c-1/2 and c+1/2 of this cell in the face arrays
                int f0, f1;
                if (xd) {
                    f0 = c + FXE * (y - 2);
                    f1 = f0 + 1;
                } else {
                    f0 = NXF + (x - 2) + TX * c;
                    f1 = f0 + TX;
                }
                const T pL = ulp[f0], mC = ulm[f0], pC = ulp[f1], mR = ulm[f1];
                const T da = aH - aL;
                const T s = T(3) * K * nu[xd ? 0 : 1] * da;
                // pL, mR move by +s; pC, mC by -s
                const T gap = gap4<T>(s, pL, mR, pC, mC, umin, umax);
                Pv = aL + theta_from_gap<T>(gap, (T)fabs(s)) * da;
            }
        }
        pc[id] = Pv;
    }
    __syncthreads();

    // ---- D3: averages of the two own cells
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const bool own = c == 0 ? own0 : own1;
        if (!own) continue;
        const long long gi = c == 0 ? g0 : g1;
        const int i = ci, j = cj + c;
        // x: faces i+1 (c-1/2) and i+2 (c+1/2); cells i, i+1, i+2
        const int fx = (i + 2) + FXE * j, cx = (i + 1) + CXE * j;
        const int fy = NXF + i + TX * (j + 2), cy = NXC + i + TX * (j + 1);
        const T dFx = fl[fx] - fl[fx - 1], dFy = fl[fy] - fl[fy - TX];
        const T dPx = pc[cx + 1] - T(2) * pc[cx] + pc[cx - 1];
        const T dPy = pc[cy + TX] - T(2) * pc[cy] + pc[cy - TX];
        if (residual) {
            out[gi] = (dPx * idx2[0] + dPy * idx2[1]) - (dFx * idx1[0] + dFy * idx1[1]);
            continue;
        }
        const T u = cg[(i + 2) + RX * (j + 2)].x;
        T v = u - (mu[0] * dFx + mu[1] * dFy) + (nu[0] * dPx + nu[1] * dPy);
        if (!isfinite(v)) bad = true;
        if constexpr (LIM) {
            const T cl = clampb(v, umin, umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(cl - v));
            v = cl;
        }
        v = stage_combine(p, v, unv[c][0], x1 ? x1[gi] : T(0), u);
        if constexpr (LIM) {
            const T cl = clampb(v, umin, umax);
            clamp_mag = fmax(clamp_mag, (double)fabs(cl - v));
            v = cl;
        }
        vlo = fmin(vlo, v);
        vhi = fmax(vhi, v);
        out[gi] = v;
    }
    if (!residual) {
        if (bad) atomicOr(&p.st[wk.x].flags, 1u);
        if constexpr (LIM) atomic_max_wave(&p.st[wk.x].clampmax, clamp_mag);
        if (p.mm) minmax_slot(p.mm, logical, vlo, vhi);
    }
}

template <class T, bool LIM, bool QF, bool FT, int TX, int TY>
constexpr long stage2d_lds_bytes()
{
    constexpr long RX = TX + 4, RY = TY + 4, G = 4 * RX * RY;
    constexpr long NF = (TX + 3) * TY + TX * (TY + 3), NC = (TX + 2) * TY + TX * (TY + 2);
    constexpr bool TAB = FT || !QF;
    return (long)sizeof(T) * ((TAB ? 4 * G : 8 * (RX + 1) * RY) + 4 * RX * RY + (QF ? 1 : 2 * G) + NF * (LIM ? 3 : 1) + NC);
}

}  // namespace af4
