/*
 * af_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the compact fourth-order doubly
 * conservative active flux (AF) method with monolithic convex limiting for
 * u_t + div f(u) = Lap a(u) on Cartesian meshes (periodic ends; Dirichlet or
 * outflow ends in 1D and 2D by the ghost rule of ends_of / bc_point)
 * (J. Duan, "A compact fourth-order doubly conservative active flux method
 * with maximum-principle-preserving limiting for degenerate
 * convection-diffusion equations", arXiv 2510.11527).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  The GPU library neither links nor calls it, and the two share
 * no code, header, table or constant.
 *
 * Style: every quantity of the paper is a function of its grid position and
 * is recomputed on demand from the DoF arrays, with periodic wrap-around of
 * indices.  Nothing is blocked, fused or reordered beyond what the formulas
 * state; the point is that a reader can check each function against the
 * paper by eye.  It is deliberately slow.
 *
 * With nodc set (1D only) the diffusion follows the variant of App. A without
 * double conservation: kappa(u) D_c(u) face fluxes in the average, the
 * compact B-matrix operator in the point value; its limiting is a reading
 * (see F_nodc_lim).
 *
 * Smoothness-indicator blending (Sec. 5.1.3) of the point values defers its
 * low-order scheme to other work; the one here is a reading (LLF on the
 * half grid, a cell average for a cell centre).  Its gamma -> inf limit, its
 * 1D weight and, by reduction to 1D, the weights of the face points in 2D
 * and 3D are pinned by the tests; the edge and corner point weights at
 * finite gamma > 0 (means of s over 4 to 8 cells) are parity unpinned.
 *
 * Half-grid reading (used by the paper's "half-index shifts", Sec. 4): along
 * axis l, the points x_{i-1/2}, x_i, x_{i+1/2}, x_{i+1}, ... form a uniform
 * grid of spacing dx_l/2.  A half-grid point has integer coordinates p; an
 * odd p_l means a half index in axis l.  Cell (i,j,k) owns the points
 * (2i+b0, 2j+b1, 2k+b2) for b in {0,1}^d; b = 0 is the cell centre, which is
 * not a DoF and is reconstructed by inverting the tensor Simpson rule; every
 * other b is a point-value DoF.  All 1D operators of Sec. 2 become 5-point
 * stencils along an axis of this grid.
 *
 * DoF arrays follow the zeta order of Sec. 4:
 *   1D: avg, x-face
 *   2D: avg, x-face, y-face, corner
 *   3D: avg, x-, y-, z-face, (i+1/2,j+1/2,k), (i+1/2,j,k+1/2),
 *       (i,j+1/2,k+1/2), corner
 * each of n0*n1*n2 values, x fastest; the point value at i+1/2 is stored at
 * index i.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 3
#define ORC_MAXCRIT 16

enum { ORC_F_LINEAR = 0, ORC_F_QUAD = 1, ORC_F_BL = 2, ORC_F_BL_GRAV = 3 };
enum { ORC_A_LINEAR = 0, ORC_A_POWER = 1, ORC_A_DEADZONE = 2, ORC_A_BL = 3, ORC_A_RAMP2 = 4 };
enum { ORC_THETA_COMPUTED = 0, ORC_THETA_ONE = 1, ORC_THETA_ZERO = 2 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_DIRICHLET = 1, ORC_BC_OUTFLOW = 2 };

typedef struct {
    /* problem (filled by the caller) */
    int dim;
    int n[3];
    double lo[3], hi[3];
    int fkind[3];
    double fpar[3][2];
    int akind;
    double apar[3];
    double umin, umax;
    int limiter;      /* monolithic convex limiting of averages + PV projection */
    int si;           /* smoothness-indicator blending */
    double si_gamma;
    int theta_mode;   /* ORC_THETA_*: computed, forced to 1, forced to 0 */
    int nodc;         /* 1: the variant of App. A without double conservation (1D) */
    int bc[3][2];        /* ORC_BC_* of the low and high end of each axis (both periodic or neither) */
    double bcval[3][2];  /* Dirichlet values */
    /* derived (filled by orc_setup) */
    double dx[3];
    double kappa_max;
    int ncrit[3];
    double crit[3][ORC_MAXCRIT];
} orc_problem;

typedef struct {
    long long uL_out_of_bounds;  /* intermediate states outside [umin,umax] */
    long long n_theta;           /* theta values computed */
    long long n_theta_lt1;       /* of which < 1 */
    double max_avg_clamp;        /* largest safeguard clamp on an average */
    double max_pv_clamp;
} orc_diag;

/* ------------------------------------------------------------------ */
/* Flux f_l and its derivatives.                                      */
/* ------------------------------------------------------------------ */

/* Buckley-Leverett fractional flow u^2/(u^2+(1-u)^2)  (Examples 6.6, 6.7) */
static double bl_f(double u) { double D = u * u + (1 - u) * (1 - u); return u * u / D; }
static double bl_df(double u) { double D = u * u + (1 - u) * (1 - u); return 2 * u * (1 - u) / (D * D); }
static double bl_ddf(double u)
{
    /* quotient rule on 2u(1-u)/D^2 with D' = 4u-2 */
    double D = u * u + (1 - u) * (1 - u);
    double N = 2 * u * (1 - u), dN = 2 - 4 * u, dD = 4 * u - 2;
    return (dN * D - 2 * N * dD) / (D * D * D);
}

static double flux(const orc_problem *P, int l, double u)
{
    double c = P->fpar[l][0], g = P->fpar[l][1];
    switch (P->fkind[l]) {
    case ORC_F_LINEAR: return c * u;
    case ORC_F_QUAD: return c * u * u;
    case ORC_F_BL: return bl_f(u);
    case ORC_F_BL_GRAV: return bl_f(u) * (1 - g * (1 - u) * (1 - u));
    }
    return 0;
}

static double dflux(const orc_problem *P, int l, double u)
{
    double c = P->fpar[l][0], g = P->fpar[l][1];
    switch (P->fkind[l]) {
    case ORC_F_LINEAR: return c;
    case ORC_F_QUAD: return 2 * c * u;
    case ORC_F_BL: return bl_df(u);
    case ORC_F_BL_GRAV: return bl_df(u) * (1 - g * (1 - u) * (1 - u)) + bl_f(u) * 2 * g * (1 - u);
    }
    return 0;
}

static double ddflux(const orc_problem *P, int l, double u)
{
    double c = P->fpar[l][0], g = P->fpar[l][1];
    switch (P->fkind[l]) {
    case ORC_F_LINEAR: return 0;
    case ORC_F_QUAD: return 2 * c;
    case ORC_F_BL: return bl_ddf(u);
    case ORC_F_BL_GRAV:
        return bl_ddf(u) * (1 - g * (1 - u) * (1 - u)) + 4 * g * (1 - u) * bl_df(u) - 2 * g * bl_f(u);
    }
    return 0;
}

/* Diffusion potential a(u) = int kappa, and kappa = a'. */
static double pot(const orc_problem *P, double u)
{
    double p0 = P->apar[0], p1 = P->apar[1];
    switch (P->akind) {
    case ORC_A_LINEAR: return p0 * u;
    case ORC_A_POWER: return p0 * pow(u, p1);                        /* PME u^m, Eq. (pme) */
    case ORC_A_DEADZONE: {                                            /* Examples 6.8, 6.9 */
        double m = fabs(u) - p1;
        if (m <= 0) return 0;
        return u > 0 ? p0 * m : -p0 * m;
    }
    case ORC_A_BL:                                                    /* Example 6.6 */
        if (u < 0) return 0;
        if (u > 1) return p0 * 2.0 / 3.0;
        return p0 * (2 * u * u - 4.0 / 3.0 * u * u * u);
    case ORC_A_RAMP2: {
        double m = u - p1;
        return m > 0 ? 0.5 * p0 * m * m : 0;
    }
    }
    return 0;
}

static double kappa(const orc_problem *P, double u)
{
    double p0 = P->apar[0], p1 = P->apar[1];
    switch (P->akind) {
    case ORC_A_LINEAR: return p0;
    case ORC_A_POWER: return p0 * p1 * pow(u, p1 - 1);
    case ORC_A_DEADZONE: return fabs(u) > p1 ? p0 : 0;
    case ORC_A_BL: return (u < 0 || u > 1) ? 0 : p0 * (4 * u - 4 * u * u);
    case ORC_A_RAMP2: return u > p1 ? p0 * (u - p1) : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Setup: dx, kappa_max (Sec. 5.1), critical points of f_l' for the    */
/* interval maximum of |f_l'| in the LLF viscosity (Eq. 1d_local_wave_speed). */
/* ------------------------------------------------------------------ */

/* sup of kappa over [umin, umax].  kappa is piecewise monotone for every
 * supported potential; its supremum is attained at an end point, at a kink
 * (approached from the side where kappa is positive) or at an interior
 * stationary point, so those candidates are evaluated. */
static double kappa_max_over(const orc_problem *P, double lo, double hi)
{
    double cand[8];
    int nc = 0;
    cand[nc++] = lo;
    cand[nc++] = hi;
    if (P->akind == ORC_A_BL && lo <= 0.5 && 0.5 <= hi) cand[nc++] = 0.5;
    double best = 0;
    for (int i = 0; i < nc; i++) {
        double k = kappa(P, cand[i]);
        if (k > best) best = k;
    }
    if (P->akind == ORC_A_DEADZONE && (hi > P->apar[1] || lo < -P->apar[1]) && P->apar[0] > best)
        best = P->apar[0];
    return best;
}

/* roots of f_l'' in [a,b], found by a sign scan and bisection */
static int find_crit(const orc_problem *P, int l, double a, double b, double *out, int maxout)
{
    const int M = 20000;
    int nr = 0;
    double h = (b - a) / M;
    double x0 = a, g0 = ddflux(P, l, x0);
    for (int s = 1; s <= M && nr < maxout; s++) {
        double x1 = a + s * h, g1 = ddflux(P, l, x1);
        if (g0 == 0) {
            out[nr++] = x0;
        } else if (g0 * g1 < 0) {
            double L = x0, R = x1, gL = g0;
            for (int it = 0; it < 200; it++) {
                double m = 0.5 * (L + R), gm = ddflux(P, l, m);
                if (gm == 0 || m == L || m == R) { L = R = m; break; }
                if ((gm < 0) == (gL < 0)) { L = m; gL = gm; } else R = m;
            }
            out[nr++] = 0.5 * (L + R);
        }
        x0 = x1;
        g0 = g1;
    }
    return nr;
}

int orc_setup(orc_problem *P)
{
    if (P->dim < 1 || P->dim > 3) return -1;
    if (P->nodc && (P->dim != 1 || P->si)) return -1;  /* App. A is a 1D scheme */
    for (int l = 0; l < 3; l++) {
        for (int s = 0; s < 2; s++)
            if (P->bc[l][s] < ORC_BC_PERIODIC || P->bc[l][s] > ORC_BC_OUTFLOW) return -1;
        if ((P->bc[l][0] == ORC_BC_PERIODIC) != (P->bc[l][1] == ORC_BC_PERIODIC)) return -1;
        if (P->bc[l][0] != ORC_BC_PERIODIC && (l >= P->dim || P->dim == 3 || P->si)) return -1;
    }
    for (int l = 0; l < 3; l++) {
        if (l >= P->dim) { P->n[l] = 1; P->dx[l] = 1; P->ncrit[l] = 0; continue; }
        if (P->n[l] < 4) return -1;
        P->dx[l] = (P->hi[l] - P->lo[l]) / P->n[l];
        P->ncrit[l] = 0;
        if (P->fkind[l] == ORC_F_BL || P->fkind[l] == ORC_F_BL_GRAV) {
            double w = P->umax - P->umin;
            P->ncrit[l] = find_crit(P, l, P->umin - w - 1, P->umax + w + 1, P->crit[l], ORC_MAXCRIT);
        }
    }
    P->kappa_max = kappa_max_over(P, P->umin, P->umax);
    return 0;
}

double orc_kappa_max(const orc_problem *P) { return P->kappa_max; }

int orc_crit(const orc_problem *P, int l, double *out)
{
    for (int i = 0; i < P->ncrit[l]; i++) out[i] = P->crit[l][i];
    return P->ncrit[l];
}

/* ------------------------------------------------------------------ */
/* Index helpers.                                                     */
/* ------------------------------------------------------------------ */

/* zeta-order index of the point value with half-shift mask b (bit l = half
 * index in axis l), following the DoF list of Sec. 4 */
static int zeta_of_mask(int d, int b)
{
    static const int z3[8] = {0, 1, 2, 4, 3, 5, 6, 7};
    if (d == 3) return z3[b];
    return b;
}

static int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

static long cell_index(const orc_problem *P, const int c[3])
{
    int i = wrapi(c[0], P->n[0]), j = wrapi(c[1], P->n[1]), k = wrapi(c[2], P->n[2]);
    return (long)i + (long)P->n[0] * ((long)j + (long)P->n[1] * k);
}

/* Non-periodic ends (1D and 2D).  The paper runs Examples 6.5-6.9 with
 * Dirichlet or outflow boundaries but states no ghost treatment; the reading
 * taken here: a half-grid point on or beyond an open end -- the boundary
 * points x_{-1/2}, x_{N-1/2} included -- takes a boundary value, and so does
 * a ghost cell's average (the value at its centre):
 *   * if one of the ends it lies on or beyond is Dirichlet, the Dirichlet
 *     value (the lowest such axis first);
 *   * else (outflow) the mean average of the domain cells whose closure
 *     contains the point moved onto the boundary (the point clamped to the
 *     domain along the axes it leaves): one cell in 1D, one or two along an
 *     edge in 2D, the corner cell at a corner.
 * The stored point values on the high ends are not unknowns: their input is
 * ignored, a stage writes the Dirichlet value (Dirichlet) or passes the
 * input through (outflow), and the right-hand side there is 0. */
static int axis_open(const orc_problem *P, int l) { return l < P->dim && P->bc[l][0] != ORC_BC_PERIODIC; }
static int bc_open(const orc_problem *P) { return axis_open(P, 0) || axis_open(P, 1) || axis_open(P, 2); }

/* bit l set: p lies on or beyond an open end of axis l */
static int ends_of(const orc_problem *P, const int p[3])
{
    int m = 0;
    for (int l = 0; l < 3; l++)
        if (axis_open(P, l) && (p[l] <= -1 || p[l] >= 2 * P->n[l] - 1)) m |= 1 << l;
    return m;
}

static double bc_point(const orc_problem *P, const double *const *U, const int p[3], int m)
{
    for (int l = 0; l < 3; l++)
        if ((m >> l & 1) && P->bc[l][p[l] <= -1 ? 0 : 1] == ORC_BC_DIRICHLET) return P->bcval[l][p[l] <= -1 ? 0 : 1];
    /* outflow: mean over the cells containing the clamped point */
    int lo[3], hi[3];
    for (int l = 0; l < 3; l++) {
        if (m >> l & 1) {
            lo[l] = hi[l] = p[l] <= -1 ? 0 : P->n[l] - 1;
        } else if (p[l] & 1) {
            lo[l] = (p[l] - 1) >> 1;  /* floor, also for negative (periodic) indices */
            hi[l] = lo[l] + 1;
        } else {
            lo[l] = hi[l] = p[l] >> 1;
        }
    }
    double sum = 0;
    int cnt = 0;
    for (int k = lo[2]; k <= hi[2]; k++)
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                const int c[3] = {i, j, k};
                sum += U[0][cell_index(P, c)];
                cnt++;
            }
    return sum / cnt;
}

static double avg(const orc_problem *P, const double *const *U, const int c[3])
{
    const int p[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
    const int m = ends_of(P, p);
    if (m) return bc_point(P, U, p, m);
    return U[0][cell_index(P, c)];
}

static double H(const orc_problem *P, const double *const *U, const int p[3]);

/* Cell-centre value from the average and the surrounding point values by
 * inverting the tensor-product Simpson rule: 1D (Sec. 2), 2D (Sec. 4); the
 * 3D form is the same inversion with weights (1,4,1)^3 / 216. */
static double centre(const orc_problem *P, const double *const *U, const int c[3])
{
    int d = P->dim;
    double S = 1, wc = 1;
    for (int l = 0; l < d; l++) { S *= 6; wc *= 4; }
    double acc = S * avg(P, U, c);
    int o[3] = {0, 0, 0};
    int lim[3] = {1, d > 1 ? 1 : 0, d > 2 ? 1 : 0};
    for (o[2] = -lim[2]; o[2] <= lim[2]; o[2]++)
        for (o[1] = -lim[1]; o[1] <= lim[1]; o[1]++)
            for (o[0] = -lim[0]; o[0] <= lim[0]; o[0]++) {
                if (o[0] == 0 && o[1] == 0 && o[2] == 0) continue;
                double w = 1;
                for (int l = 0; l < d; l++) w *= (o[l] == 0) ? 4 : 1;
                int p[3] = {2 * c[0] + o[0], 2 * c[1] + o[1], 2 * c[2] + o[2]};
                acc -= w * H(P, U, p);
            }
    return acc / wc;
}

/* value at half-grid point p: a point-value DoF, or a reconstructed centre */
static double H(const orc_problem *P, const double *const *U, const int p[3])
{
    const int m = ends_of(P, p);
    if (m) return bc_point(P, U, p, m);
    int q[3], c[3], b = 0;
    for (int l = 0; l < 3; l++) {
        q[l] = wrapi(p[l], 2 * P->n[l]);
        c[l] = q[l] >> 1;
        if (q[l] & 1) b |= 1 << l;
    }
    if (b == 0) return centre(P, U, c);
    return U[zeta_of_mask(P->dim, b)][cell_index(P, c)];
}

/* ------------------------------------------------------------------ */
/* Smoothness indicator (Sec. 5.1.3), applied direction by direction.  */
/* ------------------------------------------------------------------ */

static double s_tilde(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int m[3] = {c[0], c[1], c[2]}, p[3] = {c[0], c[1], c[2]};
    m[l] -= 1;
    p[l] += 1;
    double um = avg(P, U, m), u0 = avg(P, U, c), up = avg(P, U, p);
    return fabs(um - 2 * u0 + up) / (fabs(um) + 2 * fabs(u0) + fabs(up) + 1e-13);
}

static double s_smooth(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int m[3] = {c[0], c[1], c[2]}, p[3] = {c[0], c[1], c[2]};
    m[l] -= 1;
    p[l] += 1;
    return (s_tilde(P, U, l, m) + 4 * s_tilde(P, U, l, c) + s_tilde(P, U, l, p)) / 6;
}

/* ------------------------------------------------------------------ */
/* Point-value right-hand side (Eqs. 1d_af_dc, 2d_af_dc).              */
/* ------------------------------------------------------------------ */

/* LLF flux between two states with a given viscosity (used by the low-order
 * point-value right-hand side under SI blending) */
static double llf(const orc_problem *P, int l, double a, double b, double alpha)
{
    return 0.5 * (flux(P, l, a) + flux(P, l, b)) - 0.5 * alpha * (b - a);
}

/* App. A: the compact fourth-order operator for (kappa(u) u_x)_x at a point
 * value (Eq. 1d_diff_compact_kappa_u),
 *   (4/dx^2) sum_{m,n=-2..2} b_mn kappa(z_m) z_n,
 * on the 5-point half-grid line z_{-2..2} = u_{i-1/2}, u_i, u_{i+1/2},
 * u_{i+1}, u_{i+3/2}, where the 5x5 matrix B is the 4x4 matrix M printed
 * there placed in the lower-right corner minus M placed in the upper-left
 * corner. */
static const double M_nodc[4][4] = {
    {1.0 / 8, -1.0 / 6, 1.0 / 24, 0.0},
    {-1.0 / 6, -3.0 / 8, 2.0 / 3, -1.0 / 8},
    {1.0 / 8, -2.0 / 3, 3.0 / 8, 1.0 / 6},
    {0.0, -1.0 / 24, 1.0 / 6, -1.0 / 8},
};
static double b_nodc(int m, int n)  /* m, n in 0..4 for -2..2 */
{
    double b = 0;
    if (m >= 1 && n >= 1) b += M_nodc[m - 1][n - 1];
    if (m <= 3 && n <= 3) b -= M_nodc[m][n];
    return b;
}
static double dtilde2(const orc_problem *P, const double z[5], double dx)
{
    double s = 0;
    for (int m = 0; m < 5; m++)
        for (int n = 0; n < 5; n++) s += b_nodc(m, n) * kappa(P, z[m]) * z[n];
    return 4 * s / (dx * dx);
}

/* contribution of direction l to du/dt at the point value p:
 *   -( D+^{4th} f^+ + D-^{4th} f^- ) + D^{2,4th} a(u)
 * with D+ (Eq. 1d_upwind_ops_4p), D- (Eq. 1d_upwind_ops_4m), the local LF
 * flux-vector splitting f^{+-} = (f +- alpha u)/2 whose alpha is the largest
 * |f_l'| over the 5-point stencil (Sec. 2.1), and D^{2,4th}
 * (Eq. 1d_diff_compact_a).  With SI on, the convection part is blended with
 * a first-order LLF right-hand side on the half grid. */
static double pv_rhs_dir(const orc_problem *P, const double *const *U, const int p[3], int l)
{
    double z[5], f[5], a[5], alpha = 0;
    for (int m = -2; m <= 2; m++) {
        int q[3] = {p[0], p[1], p[2]};
        q[l] += m;
        z[m + 2] = H(P, U, q);
        f[m + 2] = flux(P, l, z[m + 2]);
        a[m + 2] = pot(P, z[m + 2]);
        double s = fabs(dflux(P, l, z[m + 2]));
        if (s > alpha) alpha = s;
    }
    double fp[5], fm[5];
    for (int m = 0; m < 5; m++) {
        fp[m] = 0.5 * (f[m] + alpha * z[m]);
        fm[m] = 0.5 * (f[m] - alpha * z[m]);
    }
    double dx = P->dx[l];
    double Dp = (fp[0] - 6 * fp[1] + 3 * fp[2] + 2 * fp[3]) / (3 * dx);
    double Dm = (-2 * fm[1] - 3 * fm[2] + 6 * fm[3] - fm[4]) / (3 * dx);
    double D2 = P->nodc ? dtilde2(P, z, dx)
                        : (-a[0] / 3 + 16 * a[1] / 3 - 10 * a[2] + 16 * a[3] / 3 - a[4] / 3) / (dx * dx);
    double conv = -(Dp + Dm);
    if (P->si) {
        /* low-order LLF right-hand side: neighbours at +-dx/2, a cell
         * average replacing a reconstructed centre */
        double nb[2];
        for (int s = 0; s < 2; s++) {
            int q[3] = {p[0], p[1], p[2]};
            q[l] += s ? 1 : -1;
            int qw[3], allEven = 1;
            for (int k = 0; k < 3; k++) { qw[k] = wrapi(q[k], 2 * P->n[k]); if (qw[k] & 1) allEven = 0; }
            if (allEven) {
                int c[3] = {qw[0] >> 1, qw[1] >> 1, qw[2] >> 1};
                nb[s] = avg(P, U, c);
            } else {
                nb[s] = H(P, U, q);
            }
        }
        double convL = -(2 / dx) * (llf(P, l, z[2], nb[1], alpha) - llf(P, l, nb[0], z[2], alpha));
        /* blending weight: exp(-gamma * mean s_l over the cells whose
         * closure contains p) */
        double ssum = 0;
        int cnt = 0;
        int qw[3];
        for (int k = 0; k < 3; k++) qw[k] = wrapi(p[k], 2 * P->n[k]);
        int lo[3], hi[3];
        for (int k = 0; k < 3; k++) {
            if (qw[k] & 1) { lo[k] = (qw[k] - 1) / 2; hi[k] = lo[k] + 1; }
            else { lo[k] = hi[k] = qw[k] / 2; }
        }
        for (int k2 = lo[2]; k2 <= hi[2]; k2++)
            for (int k1 = lo[1]; k1 <= hi[1]; k1++)
                for (int k0 = lo[0]; k0 <= hi[0]; k0++) {
                    int c[3] = {k0, k1, k2};
                    ssum += s_smooth(P, U, l, c);
                    cnt++;
                }
        double th = exp(-P->si_gamma * ssum / cnt);
        conv = th * conv + (1 - th) * convL;
    }
    return conv + D2;
}

static double pv_rhs(const orc_problem *P, const double *const *U, const int p[3])
{
    double r = 0;
    for (int l = 0; l < P->dim; l++) r += pv_rhs_dir(P, U, p, l);
    return r;
}

/* ------------------------------------------------------------------ */
/* Cell-average quantities.                                           */
/* ------------------------------------------------------------------ */

static double wS(int o) { return o == 0 ? 4.0 : 1.0; }     /* Simpson (1,4,1) */
static double vC(int o) { return o == 0 ? 8.0 : -1.0; }    /* (-1,8,-1) of Prop. 2.1 */

/* transverse offsets of a face / cell in direction l: loops over the axes
 * other than l with o in {-1,0,1}, leaving o[l] = 0 */
#define FOR_TRANSVERSE(P, l, o)                                                      \
    for (o[2] = ((l) == 2 || (P)->dim < 3) ? 0 : -1; o[2] <= (((l) == 2 || (P)->dim < 3) ? 0 : 1); o[2]++) \
        for (o[1] = ((l) == 1 || (P)->dim < 2) ? 0 : -1; o[1] <= (((l) == 1 || (P)->dim < 2) ? 0 : 1); o[1]++) \
            for (o[0] = ((l) == 0) ? 0 : -1; o[0] <= (((l) == 0) ? 0 : 1); o[0]++)

static double transverse_weight(const orc_problem *P, int l, const int o[3])
{
    double w = 1;
    for (int m = 0; m < P->dim; m++)
        if (m != l) w *= wS(o[m]) / 6.0;
    return w;
}

/* high-order convection flux at the face c + e_l/2: the tensor Simpson face
 * average of f_l(u) (Sec. 4; in 1D simply f(u_{i+1/2}), Sec. 2.1) */
static double fhat_H(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int o[3];
    double s = 0;
    FOR_TRANSVERSE(P, l, o) {
        int p[3] = {2 * c[0] + o[0], 2 * c[1] + o[1], 2 * c[2] + o[2]};
        p[l] += 1;
        s += transverse_weight(P, l, o) * flux(P, l, H(P, U, p));
    }
    return s;
}

/* face average at c + e_l/2 of the central difference D_c^{(l),4th} a(u)
 * (Eqs. 1d_diff_central_4th, 2d_af_dc) */
static double dca_face(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int o[3];
    double s = 0, dx = P->dx[l];
    FOR_TRANSVERSE(P, l, o) {
        int p[3] = {2 * c[0] + o[0], 2 * c[1] + o[1], 2 * c[2] + o[2]};
        p[l] += 1;
        double a[5];
        for (int m = -2; m <= 2; m++) {
            int q[3] = {p[0], p[1], p[2]};
            q[l] += m;
            a[m + 2] = pot(P, H(P, U, q));
        }
        double Dc = (a[0] - 8 * a[1] + 8 * a[3] - a[4]) / (6 * dx);
        s += transverse_weight(P, l, o) * Dc;
    }
    return s;
}

/* high-order cell-centred numerical potential of direction l (Prop. 2.1 in
 * 1D; its face-averaged form in multi-D): the (-1,8,-1)/6 combination along
 * l, Simpson-averaged over the transverse directions */
static double ahat_H(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int o[3];
    double s = 0;
    FOR_TRANSVERSE(P, l, o) {
        double wt = transverse_weight(P, l, o);
        for (int m = -1; m <= 1; m++) {
            int p[3] = {2 * c[0] + o[0], 2 * c[1] + o[1], 2 * c[2] + o[2]};
            p[l] += m;
            s += wt * vC(m) / 6.0 * pot(P, H(P, U, p));
        }
    }
    return s;
}

/* interval maximum of |f_l'| over [min(ua,ub), max(ua,ub)]
 * (Eq. 1d_local_wave_speed and its multi-D form): end points and the
 * interior stationary points of f_l' */
static double alpha_L(const orc_problem *P, int l, double ua, double ub)
{
    double lo = ua < ub ? ua : ub, hi = ua < ub ? ub : ua;
    double r = fabs(dflux(P, l, lo)), t = fabs(dflux(P, l, hi));
    if (t > r) r = t;
    for (int i = 0; i < P->ncrit[l]; i++) {
        double x = P->crit[l][i];
        if (x >= lo && x <= hi) {
            t = fabs(dflux(P, l, x));
            if (t > r) r = t;
        }
    }
    return r;
}

static void shift(const int c[3], int l, int s, int out[3])
{
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
    out[l] += s;
}

/* low-order LLF flux at the face c + e_l/2 (Eq. 1d_av_pp / multid_av_pp) */
static double fhat_L(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int cp[3];
    shift(c, l, 1, cp);
    double ua = avg(P, U, c), ub = avg(P, U, cp);
    return 0.5 * (flux(P, l, ua) + flux(P, l, ub)) - 0.5 * alpha_L(P, l, ua, ub) * (ub - ua);
}

/* low-order diffusion flux at the face c + e_l/2: (a(u_{c+e}) - a(u_c))/dx_l */
static double ahat_L_face(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int cp[3];
    shift(c, l, 1, cp);
    return (pot(P, avg(P, U, cp)) - pot(P, avg(P, U, c))) / P->dx[l];
}

/* App. A: the diffusion flux at the face c + e_l/2 of the variant without
 * double conservation (Eqs. 1d_diff_nodc_av_u, 1d_diff_nodc_pnt_p):
 * kappa(u_{i+1/2}) times the central difference D_c^{4th}(u)_{i+1/2}
 * (Eq. 1d_diff_central_4th) on the 5-point half-grid line around the face */
static double g_nodc(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    int p[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
    p[l] += 1;
    double z[5];
    for (int m = -2; m <= 2; m++) {
        int q[3] = {p[0], p[1], p[2]};
        q[l] += m;
        z[m + 2] = H(P, U, q);
    }
    double Dc = (z[0] - 8 * z[1] + 8 * z[3] - z[4]) / (6 * P->dx[l]);
    return kappa(P, z[2]) * Dc;
}

/* directional low-order intermediate states
 * (Eqs. 1d_low_directional_plus/minus, multid_low_directional_plus/minus)
 * with the factor K = 2d (2 in 1D, 6 in 3D; 4 in 2D by the same argument) */
static double uL_plus(const orc_problem *P, const double *const *U, int l, const int c[3], double dt)
{
    double K = 2.0 * P->dim, mu = dt / P->dx[l], u = avg(P, U, c);
    return u - K * mu * (fhat_L(P, U, l, c) - flux(P, l, u)) + K * mu * ahat_L_face(P, U, l, c);
}

static double uL_minus(const orc_problem *P, const double *const *U, int l, const int c[3], double dt)
{
    double K = 2.0 * P->dim, mu = dt / P->dx[l], u = avg(P, U, c);
    int cm[3];
    shift(c, l, -1, cm);
    return u - K * mu * (flux(P, l, u) - fhat_L(P, U, l, cm)) - K * mu * ahat_L_face(P, U, l, cm);
}

/* SI-blended (when enabled) high-order flux and potential, Sec. 5.1.3 */
static double fhat_H_used(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    double fH = fhat_H(P, U, l, c);
    if (!P->si) return fH;
    int cp[3];
    shift(c, l, 1, cp);
    double th = exp(-P->si_gamma * 0.5 * (s_smooth(P, U, l, c) + s_smooth(P, U, l, cp)));
    return th * fH + (1 - th) * fhat_L(P, U, l, c);
}

static double ahat_H_used(const orc_problem *P, const double *const *U, int l, const int c[3])
{
    double aH = ahat_H(P, U, l, c);
    if (!P->si) return aH;
    double th = exp(-P->si_gamma * s_smooth(P, U, l, c));
    return th * aH + (1 - th) * pot(P, avg(P, U, c));
}

/* Theta(zL, zH): the largest blend keeping (1-t) zL + t zH in the bounds
 * (Sec. 5.1.1).  zH inside the bounds gives 1 (so zH == zL gives 1);
 * a zL outside the bounds, possible only after a CFL or rounding
 * violation, is clamped into [0,1]. */
static double Theta(const orc_problem *P, double zL, double zH)
{
    double t;
    if (zH < P->umin) t = (zL - P->umin) / (zL - zH);
    else if (zH > P->umax) t = (zL - P->umax) / (zL - zH);
    else return 1.0;
    if (!(t > 0)) return 0.0;
    return t > 1 ? 1.0 : t;
}

static double min2(double a, double b) { return a < b ? a : b; }

/* convection limiting parameter at the face c + e_l/2
 * (Eqs. 1d_convection_limiting_parameter, multid_convection_limiting_parameter),
 * factor 3K */
static double theta_c(const orc_problem *P, const double *const *U, int l, const int c[3], double dt, orc_diag *dg)
{
    if (P->theta_mode == ORC_THETA_ONE) return 1;
    if (P->theta_mode == ORC_THETA_ZERO) return 0;
    double K = 2.0 * P->dim, mu = dt / P->dx[l];
    int cp[3];
    shift(c, l, 1, cp);
    double df = fhat_H_used(P, U, l, c) - fhat_L(P, U, l, c);
    double up = uL_plus(P, U, l, c, dt), um = uL_minus(P, U, l, cp, dt);
    double t = min2(Theta(P, up, up - 3 * K * mu * df), Theta(P, um, um + 3 * K * mu * df));
    if (dg) {
        dg->n_theta++;
        if (t < 1) dg->n_theta_lt1++;
    }
    return t;
}

/* diffusion limiting parameter of cell c, direction l
 * (Eqs. 1d_diffusion_limiting_parameter, multid_diffusion_limiting_parameter) */
static double theta_d(const orc_problem *P, const double *const *U, int l, const int c[3], double dt, orc_diag *dg)
{
    if (P->theta_mode == ORC_THETA_ONE) return 1;
    if (P->theta_mode == ORC_THETA_ZERO) return 0;
    double K = 2.0 * P->dim, nu = dt / (P->dx[l] * P->dx[l]);
    int cm[3], cp[3];
    shift(c, l, -1, cm);
    shift(c, l, 1, cp);
    double da = ahat_H_used(P, U, l, c) - pot(P, avg(P, U, c));
    double a = uL_plus(P, U, l, cm, dt), b = uL_plus(P, U, l, c, dt);
    double e = uL_minus(P, U, l, c, dt), g = uL_minus(P, U, l, cp, dt);
    double s = 3 * K * nu * da;
    double t = min2(min2(Theta(P, a, a + s), Theta(P, b, b - s)), min2(Theta(P, e, e - s), Theta(P, g, g + s)));
    if (dg) {
        dg->n_theta++;
        if (t < 1) dg->n_theta_lt1++;
    }
    return t;
}

/* limited flux and potential (Sec. 5.1.1 / 5.2.1) */
static double F_lim(const orc_problem *P, const double *const *U, int l, const int c[3], double dt, orc_diag *dg)
{
    double fL = fhat_L(P, U, l, c);
    return fL + theta_c(P, U, l, c, dt, dg) * (fhat_H_used(P, U, l, c) - fL);
}

static double P_lim(const orc_problem *P, const double *const *U, int l, const int c[3], double dt, orc_diag *dg)
{
    double aL = pot(P, avg(P, U, c));
    return aL + theta_d(P, U, l, c, dt, dg) * (ahat_H_used(P, U, l, c) - aL);
}

/* App. A with limiting.  The paper limits this variant too but gives no
 * formula; the reading taken here: the diffusion flux g joins the convective
 * flux, F = fhat - g, whose low-order part F^L = fhat^L - (a(ubar_{i+1}) -
 * a(ubar_i))/dx is the one the low-order states u^{L,+-} of Sec. 5.1 are
 * built from.  The limited average is ubar - mu (F^Lim_{i+1/2} -
 * F^Lim_{i-1/2}) = (u^{Lim,+} + u^{Lim,-})/2 with u^{Lim,+}_i = u^{L,+}_i -
 * K mu theta_{i+1/2} dF_{i+1/2} and u^{Lim,-}_{i+1} = u^{L,-}_{i+1} + K mu
 * theta_{i+1/2} dF_{i+1/2} (one correction per state, so the factor is K,
 * not 3K); theta is the largest value keeping both in the bounds. */
static double F_nodc_lim(const orc_problem *P, const double *const *U, int l, const int c[3], double dt, orc_diag *dg)
{
    double FL = fhat_L(P, U, l, c) - ahat_L_face(P, U, l, c);
    double dF = (fhat_H(P, U, l, c) - g_nodc(P, U, l, c)) - FL;
    double t;
    if (P->theta_mode == ORC_THETA_ONE) t = 1;
    else if (P->theta_mode == ORC_THETA_ZERO) t = 0;
    else {
        double K = 2.0 * P->dim, mu = dt / P->dx[l];
        int cp[3];
        shift(c, l, 1, cp);
        double up = uL_plus(P, U, l, c, dt), um = uL_minus(P, U, l, cp, dt);
        t = min2(Theta(P, up, up - K * mu * dF), Theta(P, um, um + K * mu * dF));
        if (dg) {
            dg->n_theta++;
            if (t < 1) dg->n_theta_lt1++;
        }
    }
    return FL + t * dF;
}

/* ------------------------------------------------------------------ */
/* Public per-cell evaluations.                                       */
/* ------------------------------------------------------------------ */

static void cell_of(const orc_problem *P, long idx, int c[3])
{
    c[0] = (int)(idx % P->n[0]);
    c[1] = (int)((idx / P->n[0]) % P->n[1]);
    c[2] = (int)(idx / ((long)P->n[0] * P->n[1]));
}

/* semi-discrete right-hand side (Eq. 2d_af_dc, no limiting, no blending) of
 * the 2^d DoFs of one cell, in zeta order (average first) */
static void rhs_cell(const orc_problem *P, const double *const *U, const int c[3], double *out)
{
    double r = 0;
    for (int l = 0; l < P->dim; l++) {
        int cm[3];
        shift(c, l, -1, cm);
        r -= (fhat_H(P, U, l, c) - fhat_H(P, U, l, cm)) / P->dx[l];
        if (P->nodc) r += (g_nodc(P, U, l, c) - g_nodc(P, U, l, cm)) / P->dx[l];
        else r += (dca_face(P, U, l, c) - dca_face(P, U, l, cm)) / P->dx[l];
    }
    out[0] = r;
    int nb = 1 << P->dim;
    orc_problem Q = *P;
    Q.si = 0;
    for (int b = 1; b < nb; b++) {
        int p[3] = {2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), 2 * c[2] + ((b >> 2) & 1)};
        out[zeta_of_mask(P->dim, b)] = pv_rhs(&Q, U, p);
    }
    if (bc_open(P))
        for (int b = 1; b < nb; b++) {  /* boundary points are not unknowns */
            const int p[3] = {2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), 2 * c[2] + ((b >> 2) & 1)};
            if (ends_of(P, p)) out[zeta_of_mask(P->dim, b)] = 0;
        }
}

/* one forward-Euler stage of the (limited) scheme for one cell */
static void fe_cell(const orc_problem *P, const double *const *U, double dt, const int c[3], double *out, orc_diag *dg)
{
    double u = avg(P, U, c);
    double un;
    if (P->limiter) {
        /* Eq. multid_limited_average */
        un = u;
        for (int l = 0; l < P->dim; l++) {
            double mu = dt / P->dx[l], nu = dt / (P->dx[l] * P->dx[l]);
            int cm[3], cp[3];
            shift(c, l, -1, cm);
            shift(c, l, 1, cp);
            if (P->nodc) {
                un -= mu * (F_nodc_lim(P, U, l, c, dt, dg) - F_nodc_lim(P, U, l, cm, dt, dg));
                continue;
            }
            un -= mu * (F_lim(P, U, l, c, dt, dg) - F_lim(P, U, l, cm, dt, dg));
            un += nu * (P_lim(P, U, l, cp, dt, dg) - 2 * P_lim(P, U, l, c, dt, dg) + P_lim(P, U, l, cm, dt, dg));
        }
        if (dg) {
            for (int l = 0; l < P->dim; l++) {
                double a = uL_plus(P, U, l, c, dt), b = uL_minus(P, U, l, c, dt);
                if (a < P->umin || a > P->umax || b < P->umin || b > P->umax) dg->uL_out_of_bounds++;
            }
        }
        double cl = un < P->umin ? P->umin : (un > P->umax ? P->umax : un);
        if (dg && fabs(cl - un) > dg->max_avg_clamp) dg->max_avg_clamp = fabs(cl - un);
        un = cl;
    } else if (P->si) {
        /* blended high-order update without limiting */
        un = u;
        for (int l = 0; l < P->dim; l++) {
            double mu = dt / P->dx[l], nu = dt / (P->dx[l] * P->dx[l]);
            int cm[3], cp[3];
            shift(c, l, -1, cm);
            shift(c, l, 1, cp);
            un -= mu * (fhat_H_used(P, U, l, c) - fhat_H_used(P, U, l, cm));
            un += nu * (ahat_H_used(P, U, l, cp) - 2 * ahat_H_used(P, U, l, c) + ahat_H_used(P, U, l, cm));
        }
    } else {
        double r[8];
        rhs_cell(P, U, c, r);
        un = u + dt * r[0];
    }
    out[0] = un;
    int nb = 1 << P->dim;
    for (int b = 1; b < nb; b++) {
        int p[3] = {2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), 2 * c[2] + ((b >> 2) & 1)};
        double v = H(P, U, p) + dt * pv_rhs(P, U, p);
        if (P->limiter) {
            /* projection of point values (Sec. 5.1.2) */
            double cl = v < P->umin ? P->umin : (v > P->umax ? P->umax : v);
            v = cl;
        }
        out[zeta_of_mask(P->dim, b)] = v;
    }
    if (bc_open(P))
        for (int b = 1; b < nb; b++) {
            const int p[3] = {2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), 2 * c[2] + ((b >> 2) & 1)};
            const int m = ends_of(P, p);
            if (!m) continue;
            int dir = 0;  /* a Dirichlet end among those the point lies on */
            double g = 0;
            for (int l = 0; l < 3 && !dir; l++)
                if ((m >> l & 1) && P->bc[l][1] == ORC_BC_DIRICHLET) { dir = 1; g = P->bcval[l][1]; }
            out[zeta_of_mask(P->dim, b)] = dir ? g : U[zeta_of_mask(P->dim, b)][cell_index(P, c)];
        }
}

static long ncells(const orc_problem *P) { return (long)P->n[0] * P->n[1] * P->n[2]; }

/* full semi-discrete RHS: rhs[z][cell] */
void orc_rhs(const orc_problem *P, const double *const *U, double *const *R)
{
    long N = ncells(P);
    int nb = 1 << P->dim;
#pragma omp parallel for schedule(dynamic, 64)
    for (long idx = 0; idx < N; idx++) {
        int c[3];
        double r[8];
        cell_of(P, idx, c);
        rhs_cell(P, U, c, r);
        for (int z = 0; z < nb; z++) R[z][idx] = r[z];
    }
}

/* RHS of selected cells: out[k*2^d + z] */
void orc_rhs_cells(const orc_problem *P, const double *const *U, const long *cells, long nc, double *out)
{
    int nb = 1 << P->dim;
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < nc; k++) {
        int c[3];
        cell_of(P, cells[k], c);
        rhs_cell(P, U, c, out + k * nb);
    }
}

/* one forward-Euler stage over the whole grid: V = FE(U) */
/* diagnostics are gathered per thread and merged once */
static void diag_merge(orc_diag *dst, const orc_diag *src)
{
    dst->uL_out_of_bounds += src->uL_out_of_bounds;
    dst->n_theta += src->n_theta;
    dst->n_theta_lt1 += src->n_theta_lt1;
    if (src->max_avg_clamp > dst->max_avg_clamp) dst->max_avg_clamp = src->max_avg_clamp;
    if (src->max_pv_clamp > dst->max_pv_clamp) dst->max_pv_clamp = src->max_pv_clamp;
}

void orc_fe(const orc_problem *P, const double *const *U, double dt, double *const *V, orc_diag *dg)
{
    long N = ncells(P);
    int nb = 1 << P->dim;
#pragma omp parallel
    {
        orc_diag local;
        memset(&local, 0, sizeof local);
#pragma omp for schedule(dynamic, 64)
        for (long idx = 0; idx < N; idx++) {
            int c[3];
            double r[8];
            cell_of(P, idx, c);
            fe_cell(P, U, dt, c, r, dg ? &local : NULL);
            for (int z = 0; z < nb; z++) V[z][idx] = r[z];
        }
        if (dg) {
#pragma omp critical
            diag_merge(dg, &local);
        }
    }
}

/* forward-Euler stage of selected cells: out[k*2^d + z] */
void orc_fe_cells(const orc_problem *P, const double *const *U, double dt, const long *cells, long nc, double *out,
                  orc_diag *dg)
{
    int nb = 1 << P->dim;
#pragma omp parallel
    {
        orc_diag local;
        memset(&local, 0, sizeof local);
#pragma omp for schedule(dynamic, 16)
        for (long k = 0; k < nc; k++) {
            int c[3];
            cell_of(P, cells[k], c);
            fe_cell(P, U, dt, c, out + k * nb, dg ? &local : NULL);
        }
        if (dg) {
#pragma omp critical
            diag_merge(dg, &local);
        }
    }
}

/* safeguard: clamp every DoF into [umin, umax] after an RK combination */
static void clamp_all(const orc_problem *P, double *const *V, orc_diag *dg)
{
    long N = ncells(P);
    int nb = 1 << P->dim;
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) {
            double v = V[z][i], cl = v < P->umin ? P->umin : (v > P->umax ? P->umax : v);
            if (dg && cl != v) {
                double m = fabs(cl - v);
                if (z == 0 && m > dg->max_avg_clamp) dg->max_avg_clamp = m;
                if (z != 0 && m > dg->max_pv_clamp) dg->max_pv_clamp = m;
            }
            V[z][i] = cl;
        }
}

/* one SSP-RK3 step in Shu-Osher form (the stability polynomial of Sec. 3.2):
 *   U1 = FE(U), U2 = 3/4 U + 1/4 FE(U1), U <- 1/3 U + 2/3 FE(U2),
 * all three stages with the same dt.  W1, W2 are work arrays. */
void orc_ssprk3_step(const orc_problem *P, double *const *U, double dt, double *const *W1, double *const *W2,
                     orc_diag *dg)
{
    long N = ncells(P);
    int nb = 1 << P->dim;
    orc_fe(P, (const double *const *)U, dt, W1, dg);
    orc_fe(P, (const double *const *)W1, dt, W2, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) W2[z][i] = 0.75 * U[z][i] + 0.25 * W2[z][i];
    if (P->limiter) clamp_all(P, W2, dg);
    orc_fe(P, (const double *const *)W2, dt, W1, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) U[z][i] = (1.0 / 3.0) * U[z][i] + (2.0 / 3.0) * W1[z][i];
    if (P->limiter) clamp_all(P, U, dg);
}

/* SSP-RK(5,4) of Spiteri and Ruuth (2002), the paper's time integrator (Sec. 1;
 * its stability polynomial is printed in Sec. 3.2 with the z^5 coefficient
 * eta = 0.004477718303076), in Shu-Osher form:
 *   U1 = U + b10 dt L(U)
 *   U2 = a20 U + a21 U1 + b21 dt L(U1)
 *   U3 = a30 U + a32 U2 + b32 dt L(U2)
 *   U4 = a40 U + a43 U3 + b43 dt L(U3)
 *   U5 = a52 U2 + a53 U3 + b53 dt L(U3) + a54 U4 + b54 dt L(U4)
 * Every term a U_k + b dt L(U_k) is a times one limited forward-Euler stage
 * of step (b / a) dt, so the step is a convex combination of such stages.
 * W1..W4 are work arrays; U is overwritten with U5. */
static const double RK54_B10 = 0.391752226571890;
static const double RK54_A20 = 0.444370493651235, RK54_A21 = 0.555629506348765, RK54_B21 = 0.368410593050371;
static const double RK54_A30 = 0.620101851488403, RK54_A32 = 0.379898148511597, RK54_B32 = 0.251891774271694;
static const double RK54_A40 = 0.178079954393132, RK54_A43 = 0.821920045606868, RK54_B43 = 0.544974750228521;
static const double RK54_A52 = 0.517231671970585, RK54_A53 = 0.096059710526147, RK54_B53 = 0.063692468666290;
static const double RK54_A54 = 0.386708617503269, RK54_B54 = 0.226007483236906;

void orc_ssprk54_step(const orc_problem *P, double *const *U, double dt, double *const *W1, double *const *W2,
                      double *const *W3, double *const *W4, orc_diag *dg)
{
    long N = ncells(P);
    int nb = 1 << P->dim;
    /* W1 = U1 */
    orc_fe(P, (const double *const *)U, RK54_B10 * dt, W1, dg);
    /* W2 = U2 = a20 U + a21 FE_{(b21/a21) dt}(U1) */
    orc_fe(P, (const double *const *)W1, (RK54_B21 / RK54_A21) * dt, W2, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) W2[z][i] = RK54_A20 * U[z][i] + RK54_A21 * W2[z][i];
    if (P->limiter) clamp_all(P, W2, dg);
    /* W3 = U3 = a30 U + a32 FE_{(b32/a32) dt}(U2) */
    orc_fe(P, (const double *const *)W2, (RK54_B32 / RK54_A32) * dt, W3, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) W3[z][i] = RK54_A30 * U[z][i] + RK54_A32 * W3[z][i];
    if (P->limiter) clamp_all(P, W3, dg);
    /* W4 = U4 = a40 U + a43 FE_{(b43/a43) dt}(U3) */
    orc_fe(P, (const double *const *)W3, (RK54_B43 / RK54_A43) * dt, W4, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) W4[z][i] = RK54_A40 * U[z][i] + RK54_A43 * W4[z][i];
    if (P->limiter) clamp_all(P, W4, dg);
    /* W1 = FE_{(b53/a53) dt}(U3) (the ratio equals b43/a43 to the printed digits),
     * W3 = FE_{(b54/a54) dt}(U4); U5 = a52 U2 + a53 W1 + a54 W3 */
    orc_fe(P, (const double *const *)W3, (RK54_B53 / RK54_A53) * dt, W1, dg);
    orc_fe(P, (const double *const *)W4, (RK54_B54 / RK54_A54) * dt, W3, dg);
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) U[z][i] = RK54_A52 * W2[z][i] + RK54_A53 * W1[z][i] + RK54_A54 * W3[z][i];
    if (P->limiter) clamp_all(P, U, dg);
}

/* time step from the MPP CFL condition (Eqs. 1d_av_pp_dt, multid_av_pp_dt):
 * dt = C / max_{l, faces} (alpha_L / dx_l + kappa_max / dx_l^2) */
double orc_dt(const orc_problem *P, const double *const *U, double cfl)
{
    long N = ncells(P);
    double m = 0;
#pragma omp parallel for reduction(max : m)
    for (long idx = 0; idx < N; idx++) {
        int c[3];
        cell_of(P, idx, c);
        for (int l = 0; l < P->dim; l++) {
            int cp[3];
            shift(c, l, 1, cp);
            double v = alpha_L(P, l, avg(P, U, c), avg(P, U, cp)) / P->dx[l] + P->kappa_max / (P->dx[l] * P->dx[l]);
            if (v > m) m = v;
            if (axis_open(P, l) && c[l] == 0) {  /* the face at the low end with the ghost cell */
                int cm[3];
                shift(c, l, -1, cm);
                v = alpha_L(P, l, avg(P, U, cm), avg(P, U, c)) / P->dx[l] + P->kappa_max / (P->dx[l] * P->dx[l]);
                if (v > m) m = v;
            }
        }
    }
    return cfl / m;
}

/* Limiter internals of one cell and direction, for tests:
 * out = { uL+, uL-, fhat_H (face c+e/2, SI-blended), fhat_L, ahat_H
 *         (SI-blended), a(avg), theta_c, theta_d } */
void orc_limiter_probe(const orc_problem *P, const double *const *U, double dt, int l, long idx, double *out)
{
    int c[3];
    cell_of(P, idx, c);
    out[0] = uL_plus(P, U, l, c, dt);
    out[1] = uL_minus(P, U, l, c, dt);
    out[2] = fhat_H_used(P, U, l, c);
    out[3] = fhat_L(P, U, l, c);
    out[4] = ahat_H_used(P, U, l, c);
    out[5] = pot(P, avg(P, U, c));
    out[6] = theta_c(P, U, l, c, dt, NULL);
    out[7] = theta_d(P, U, l, c, dt, NULL);
}

/* values of the pointwise functions, for tests */
void orc_eval(const orc_problem *P, int l, const double *u, long n, double *f, double *df, double *a, double *k)
{
    for (long i = 0; i < n; i++) {
        if (f) f[i] = flux(P, l, u[i]);
        if (df) df[i] = dflux(P, l, u[i]);
        if (a) a[i] = pot(P, u[i]);
        if (k) k[i] = kappa(P, u[i]);
    }
}

double orc_alpha_L(const orc_problem *P, int l, double ua, double ub) { return alpha_L(P, l, ua, ub); }

/* half-grid values of a whole grid (centres reconstructed): out has
 * prod(2 n_l) entries, first axis fastest */
void orc_halfgrid(const orc_problem *P, const double *const *U, double *out)
{
    long m0 = 2L * P->n[0], m1 = P->dim > 1 ? 2L * P->n[1] : 1, m2 = P->dim > 2 ? 2L * P->n[2] : 1;
#pragma omp parallel for
    for (long k = 0; k < m2; k++)
        for (long j = 0; j < m1; j++)
            for (long i = 0; i < m0; i++) {
                int p[3] = {(int)i, (int)j, (int)k};
                out[i + m0 * (j + m1 * k)] = H(P, U, p);
            }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following oracle calls (n >= 1; timing only) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_sizeof_problem(void) { return (int)sizeof(orc_problem); }
int orc_sizeof_diag(void) { return (int)sizeof(orc_diag); }
