/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Runs the oracle (compiled into this program as one translation unit) under
 * AddressSanitizer and UndefinedBehaviorSanitizer on small problems: every
 * dimension, both diffusion forms (1D), limiter and blending on and off,
 * periodic and open ends, the right-hand side, forward-Euler stages, SSP-RK3
 * and SSP-RK(5,4) steps and the CFL step.  It exits 1 if a check of what the
 * paper fixes fails (finite values, the MPP bounds of Def. 5.1 with the
 * limiter, mass conservation on periodic meshes), and the sanitizers abort it
 * on any out-of-bounds access or undefined behaviour.
 */
#include "af_oracle.c"

#include <stdio.h>

static double lcg(unsigned long long *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int dim, int n, int fk, int ak, int lim, int si, int nodc, int open, int integ, unsigned long long seed)
{
    orc_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    for (int l = 0; l < 3; l++) {
        P.n[l] = l < dim ? n + l : 1;
        P.lo[l] = 0.0;
        P.hi[l] = 1.0 + 0.1 * l;
        P.fkind[l] = fk;
        P.fpar[l][0] = fk == ORC_F_QUAD ? 0.5 : (fk == ORC_F_LINEAR ? -0.7 : 0.0);
        P.fpar[l][1] = fk == ORC_F_BL_GRAV ? 5.0 : 0.0;
    }
    P.akind = ak;
    P.apar[0] = 0.05;
    P.apar[1] = ak == ORC_A_POWER ? 2.0 : 0.3;
    P.umin = 0.0;
    P.umax = 1.0;
    P.limiter = lim;
    P.si = si;
    P.si_gamma = 1.0;
    P.nodc = nodc;
    if (open && dim <= 2) {
        P.bc[0][0] = ORC_BC_DIRICHLET;
        P.bcval[0][0] = 0.8;
        P.bc[0][1] = ORC_BC_OUTFLOW;
    }
    if (orc_setup(&P) != 0) return 1;
    long N = 1;
    for (int l = 0; l < dim; l++) N *= P.n[l];
    int nb = 1 << dim;
    double *buf = malloc(sizeof(double) * (size_t)N * nb * 7);
    double *U[8], *V[8], *W1[8], *W2[8], *W3[8], *W4[8], *R[8];
    for (int z = 0; z < nb; z++) {
        U[z] = buf + (size_t)N * z;
        V[z] = buf + (size_t)N * (nb + z);
        W1[z] = buf + (size_t)N * (2 * nb + z);
        W2[z] = buf + (size_t)N * (3 * nb + z);
        W3[z] = buf + (size_t)N * (4 * nb + z);
        W4[z] = buf + (size_t)N * (5 * nb + z);
        R[z] = buf + (size_t)N * (6 * nb + z);
        for (long i = 0; i < N; i++) U[z][i] = lcg(&seed) < 0.3 ? (lcg(&seed) < 0.5 ? 0.0 : 1.0) : lcg(&seed);
    }
    double vol = 1.0;
    for (int l = 0; l < dim; l++) vol *= P.dx[l];
    double m0 = 0.0;
    for (long i = 0; i < N; i++) m0 += U[0][i] * vol;
    orc_diag dg;
    memset(&dg, 0, sizeof dg);
    orc_rhs(&P, (const double *const *)U, R);
    double dt = orc_dt(&P, (const double *const *)U, 0.3 / (2 * dim));
    orc_fe(&P, (const double *const *)U, dt, V, &dg);
    for (int s = 0; s < 2; s++) {
        dt = orc_dt(&P, (const double *const *)U, 0.3 / (2 * dim));
        if (integ == 0) orc_ssprk3_step(&P, U, dt, W1, W2, &dg);
        else orc_ssprk54_step(&P, U, dt, W1, W2, W3, W4, &dg);
    }
    int bad = 0;
    double m1 = 0.0;
    for (int z = 0; z < nb; z++)
        for (long i = 0; i < N; i++) {
            if (!isfinite(U[z][i]) || !isfinite(R[z][i]) || !isfinite(V[z][i])) bad = 1;
            if (lim && (U[z][i] < P.umin || U[z][i] > P.umax || V[z][i] < P.umin || V[z][i] > P.umax)) bad = 1;
        }
    for (long i = 0; i < N; i++) m1 += U[0][i] * vol;
    if (!open && fabs(m1 - m0) > 1e-12 * (fabs(m0) + 1.0)) bad = 1;
    free(buf);
    if (bad) fprintf(stderr, "check failed: dim %d fk %d ak %d lim %d si %d nodc %d open %d integ %d\n", dim, fk, ak,
                     lim, si, nodc, open, integ);
    return bad;
}

int main(void)
{
    int fails = 0;
    unsigned long long seed = 2510;
    for (int dim = 1; dim <= 3; dim++)
        for (int fk = 0; fk < 4; fk++)
            for (int lim = 0; lim <= 1; lim++)
                for (int si = 0; si <= 1; si++) {
                    const int n = dim == 3 ? 5 : (dim == 2 ? 7 : 13);
                    const int ak = (fk + dim) % 5;
                    fails += run_case(dim, n, fk, ak, lim, si, 0, 0, (fk + si) & 1, seed++);
                    if (dim <= 2 && !si) fails += run_case(dim, n, fk, ak, lim, 0, 0, 1, fk & 1, seed++);
                    if (dim == 1 && !si) fails += run_case(dim, n, fk, ak, lim, 0, 1, 0, 0, seed++);
                }
    printf("sanitized oracle cases done, %d failed\n", fails);
    return fails ? 1 : 0;
}
