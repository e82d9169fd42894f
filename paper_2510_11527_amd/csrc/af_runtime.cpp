// af_runtime.cpp -- host runtime behind the C ABI of include/af.h: contexts,
// instance table, device buffers, work lists, time stepping (eager and as one
// HIP graph per af_step), residuals and norms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "af.h"
#include "af_internal.h"
#include "launch.h"
#include "variants.h"

using af4::InstDev;
using af4::InstState;
using af4::StageParams;
using af4::StepCtl;

struct af_ctx {
    int n_inst = 0, dim = 0, prec = 64, lim = 0, si = 0, integ = 0;
    unsigned caps = 0;  // af4::kCap* properties of all instances
    std::vector<af_problem> prob;
    std::vector<InstDev> ih;
    std::vector<int> have_state;
    InstDev *d_inst = nullptr;
    InstState *d_st = nullptr;
    StepCtl *d_ctl = nullptr;
    double *d_dtp = nullptr;
    int4 *d_work = nullptr;
    int nwork = 0;
    std::vector<int> work_start, work_count;
    int2 *d_chunks = nullptr;
    unsigned long long *d_mm = nullptr;  // per-wave min / max slots of the last stage
    int waves_per_block = 1;
    long long max_slots = 0;  // most min / max slot pairs of one instance
    unsigned long long *d_lact = nullptr;  // limiter-activity counters (2 per instance), on demand
    bool lact_on = false;                  // stage launches count limited faces / potentials
    int nchunks = 0;
    unsigned long long *d_wslot = nullptr;  // one wave-speed slot per chunk
    long long max_chunks = 0;               // most chunks of one instance
    void *buf[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // state buffers (A = U^n)
    long long total = 0;     // elements per state buffer
    double *d_npart = nullptr, *d_nout = nullptr;
    hipStream_t own_stream = nullptr, stream = nullptr;
    int variant = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_steps = 0;
    bool graph_ws = true;   // the cached graph's first step runs the wave-speed kernel
    // the last stage of the previous step reduced the min / max averages of
    // every instance, so the next step's CFL needs no wave-speed pass
    bool keys_fresh = false;
    bool open = false;   // some instance has non-periodic ends
    std::string err;
};

static thread_local std::string g_create_err;

namespace {

size_t vbytes(const af_ctx *c) { return c->prec == 32 ? 4 : 8; }

af_status fail(af_ctx *c, af_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_err = msg;
    return s;
}

#define HIPOK(ctx, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), AF_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- physics (host)

// |f_l'(u)| for the local-maximum search of the LLF wave speed
double host_adf(int kind, double c, double g, double u)
{
    switch (kind) {
    case AF_F_LINEAR: return std::fabs(c);
    case AF_F_QUAD: return std::fabs(2 * c * u);
    default: {
        double v = 1 - u, den = u * u + v * v;
        double d1 = 2 * u * v / (den * den);
        if (kind == AF_F_BL) return std::fabs(d1);
        double q = u * u / den;
        return std::fabs(d1 * (1 - g * v * v) + q * 2 * g * v);
    }
    }
}

// Interior local maxima of |f_l'| over [a, b]: dense sampling, then golden
// section refinement of every sampled local maximum.
int host_local_maxima(int kind, double c, double g, double a, double b, double *out, int maxout)
{
    if (kind == AF_F_LINEAR || kind == AF_F_QUAD) return 0;  // |f'| convex or constant
    const int M = 8192;
    std::vector<double> x(M + 1), y(M + 1);
    for (int i = 0; i <= M; i++) {
        x[i] = a + (b - a) * i / M;
        y[i] = host_adf(kind, c, g, x[i]);
    }
    int n = 0;
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int i = 1; i < M && n < maxout; i++) {
        if (!(y[i] > y[i - 1] && y[i] >= y[i + 1])) continue;
        double lo = x[i - 1], hi = x[i + 1];
        double p = hi - gr * (hi - lo), q = lo + gr * (hi - lo);
        double fp = host_adf(kind, c, g, p), fq = host_adf(kind, c, g, q);
        for (int it = 0; it < 200 && hi - lo > 1e-15 * (1 + std::fabs(lo)); it++) {
            if (fp < fq) {
                lo = p; p = q; fp = fq;
                q = lo + gr * (hi - lo); fq = host_adf(kind, c, g, q);
            } else {
                hi = q; q = p; fq = fp;
                p = hi - gr * (hi - lo); fp = host_adf(kind, c, g, p);
            }
        }
        out[n++] = 0.5 * (lo + hi);
    }
    return n;
}

// sup of kappa = a' over [lo, hi], closed forms per potential
double host_kappa_max(int kind, double p0, double p1, double lo, double hi)
{
    switch (kind) {
    case AF_A_LINEAR: return std::max(p0, 0.0);
    case AF_A_POWER: {
        auto k = [&](double u) { return p0 * p1 * std::pow(u, p1 - 1); };
        return std::max(0.0, std::max(k(lo), k(hi)));
    }
    case AF_A_DEADZONE: return (hi > p1 || lo < -p1) ? std::max(p0, 0.0) : 0.0;
    case AF_A_BL: {
        double a = std::max(lo, 0.0), b = std::min(hi, 1.0);
        if (a > b) return 0.0;
        double u = std::min(std::max(0.5, a), b);
        return std::max(0.0, 4 * p0 * u * (1 - u));
    }
    case AF_A_RAMP2: return std::max(0.0, p0 * std::max(0.0, hi - p1));
    }
    return 0.0;
}

// Bounds as FP32 values inside [umin, umax]: the nearest float at or above
// umin, at or below umax, so that FP32 clamps and limiter gaps never admit a
// value outside the FP64 bounds (a bound without an exact FP32 value would
// otherwise round outwards half the time).
float f32_at_least(double v)
{
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    return f;
}
float f32_at_most(double v)
{
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    return f;
}

// FP32 copies of the parameters the FP32 kernels read (rounded to nearest,
// as a device-side conversion would; the bounds rounded inwards).
void set_f32_params(InstDev &I)
{
    I.f_umin = f32_at_least(I.umin);
    I.f_umax = f32_at_most(I.umax);
    I.f_pc[0] = (float)I.pc1;
    I.f_pc[1] = (float)I.pc2;
    I.f_pc[2] = (float)I.pc3;
    for (int l = 0; l < 3; l++) {
        I.f_fp0[l] = (float)I.fp0[l];
        I.f_idx1[l] = (float)I.idx1[l];
        I.f_idx2[l] = (float)I.idx2[l];
        I.f_i6dx[l] = (float)I.i6dx[l];
        for (int k = 0; k < af4::kMaxCrit; k++) {
            I.f_crit[l][k] = (float)I.crit[l][k];
            I.f_adfc[l][k] = (float)I.adfc[l][k];
        }
    }
}

void derive_bounds_params(InstDev &I, const af_problem &P, int dim)
{
    I.kmax = host_kappa_max(P.diff, P.diff_par[0], P.diff_par[1], I.umin, I.umax);
    const double w = I.umax - I.umin;
    for (int l = 0; l < 3; l++) {
        I.ncrit[l] = 0;
        for (int k = 0; k < af4::kMaxCrit; k++) I.crit[l][k] = 0;
        if (l < dim)
            I.ncrit[l] = host_local_maxima(P.flux[l], P.flux_par[l][0], P.flux_par[l][1], I.umin - w - 1,
                                           I.umax + w + 1, I.crit[l], af4::kMaxCrit);
        for (int k = 0; k < af4::kMaxCrit; k++)
            I.adfc[l][k] = k < I.ncrit[l] ? host_adf(P.flux[l], P.flux_par[l][0], P.flux_par[l][1], I.crit[l][k]) : 0.0;
    }
}

// Coefficients of the unified potential evaluation used by the kernels:
// a(u) = s * v (c1 + v (c2 + v c3)), v = clamp((abs ? |u| : u) - u0, lo, hi).
void set_unified_potential(InstDev &I, const af_problem &P)
{
    const double p0 = P.diff_par[0], p1 = P.diff_par[1];
    const double inf = std::numeric_limits<double>::infinity();
    I.pu0 = 0;
    I.plo = -inf;
    I.phi = inf;
    I.pc1 = I.pc2 = I.pc3 = 0;
    I.pabs = 0;
    I.ppow = 0;
    switch (P.diff) {
    case AF_A_LINEAR: I.pc1 = p0; break;
    case AF_A_POWER:
        if (p1 == 1.0) I.pc1 = p0;
        else if (p1 == 2.0) I.pc2 = p0;
        else if (p1 == 3.0) I.pc3 = p0;
        else I.ppow = 1;
        break;
    case AF_A_DEADZONE:
        I.pabs = 1;
        I.pu0 = p1;
        I.plo = 0;
        I.pc1 = p0;
        break;
    case AF_A_BL:
        I.plo = 0;
        I.phi = 1;
        I.pc2 = 2 * p0;
        I.pc3 = -4.0 / 3.0 * p0;
        break;
    case AF_A_RAMP2:
        I.pu0 = p1;
        I.plo = 0;
        I.pc2 = 0.5 * p0;
        break;
    }
}

// One stage of a time step in Shu-Osher form: the forward-Euler stage of
// step dts * dt on buffer `in`, combined (af4::kComb*) with X0 = U^n (buffer
// 0), X1 (buffer x1) and the stage input, into buffer `out`.
struct StageSpec {
    int in, out, x1;  // buffer indices; x1 < 0: none
    int mode;
    double w, c0, c1, cin, dts;
    bool last;        // the step's last stage: stores the min / max slots
};

// SSP-RK3 (Shu-Osher form; stability polynomial of Sec. 3.2)
const StageSpec kSSP3[3] = {
    {0, 1, -1, af4::kCombFE, 1.0, 0, 0, 0, 1.0, false},
    {1, 2, -1, af4::kCombBlend, 0.25, 0, 0, 0, 1.0, false},
    {2, 0, -1, af4::kCombBlend, 2.0 / 3.0, 0, 0, 0, 1.0, true},
};

// SSP-RK(5,4) of Spiteri and Ruuth (2002), the paper's integrator (its
// stability polynomial, with the z^5 coefficient 0.004477718303076, is printed
// in Sec. 3.2), in Shu-Osher form:
//   U1 = U + b10 dt L(U),  Uk = ak0 U + ak,k-1 U(k-1) + bk,k-1 dt L(U(k-1)), k = 2..4,
//   U5 = a52 U2 + a53 U3 + b53 dt L(U3) + a54 U4 + b54 dt L(U4).
// Each "a V + b dt L(V)" is a times a forward-Euler stage of step (b/a) dt.
// b53/a53 equals b43/a43, so a53 (U3 + (b53/a53) dt L(U3)) is recovered from
// U4 as (a53/a43)(U4 - a40 U), which spares a sixth stage: the last stage
// sums a52 U2 - (a53 a40 / a43) U + (a53 / a43) U4 + a54 FE(U4).
constexpr double kB10 = 0.391752226571890;
constexpr double kA21 = 0.555629506348765, kB21 = 0.368410593050371;
constexpr double kA32 = 0.379898148511597, kB32 = 0.251891774271694;
constexpr double kA40 = 0.178079954393132, kA43 = 0.821920045606868, kB43 = 0.544974750228521;
constexpr double kA52 = 0.517231671970585, kA53 = 0.096059710526147;
constexpr double kA54 = 0.386708617503269, kB54 = 0.226007483236906;
const StageSpec kSSP54[5] = {
    {0, 1, -1, af4::kCombFE, 1.0, 0, 0, 0, kB10, false},
    {1, 2, -1, af4::kCombBlend, kA21, 0, 0, 0, kB21 / kA21, false},
    {2, 3, -1, af4::kCombBlend, kA32, 0, 0, 0, kB32 / kA32, false},
    {3, 4, -1, af4::kCombBlend, kA43, 0, 0, 0, kB43 / kA43, false},
    {4, 0, 2, af4::kCombSum, kA54, -kA53 * kA40 / kA43, kA52, kA53 / kA43, kB54 / kA54, true},
};
// largest forward-Euler step of a stage, in units of dt
constexpr double kSSP54MaxStage = kB21 / kA21;

const StageSpec kEuler[1] = {{0, 1, -1, af4::kCombFE, 1.0, 0, 0, 0, 1.0, true}};

int num_stages(int integ) { return integ == AF_RK_SSP3 ? 3 : (integ == AF_RK_SSP54 ? 5 : 1); }
const StageSpec *stages_of(int integ) { return integ == AF_RK_SSP3 ? kSSP3 : (integ == AF_RK_SSP54 ? kSSP54 : kEuler); }
int num_buffers(int integ) { return integ == AF_RK_SSP54 ? 5 : 3; }

bool is_int_exponent(double p, int *m)
{
    double r = std::round(p);
    if (r >= 1 && r <= 16 && r == p) {
        *m = (int)r;
        return true;
    }
    return false;
}

af_status validate(const af_problem &P, int idx)
{
    char buf[256];
    auto bad = [&](af_status s, const char *what) {
        std::snprintf(buf, sizeof buf, "instance %d: %s", idx, what);
        return fail(nullptr, s, buf);
    };
    if (P.dim < 1 || P.dim > 3) return bad(AF_ERR_ARG, "dim must be 1, 2 or 3");
    for (int l = 0; l < P.dim; l++) {
        if (P.n[l] < 4) return bad(AF_ERR_ARG, "need at least 4 cells per axis");
        if (!(P.hi[l] > P.lo[l])) return bad(AF_ERR_ARG, "hi must exceed lo");
        if (P.flux[l] < AF_F_LINEAR || P.flux[l] > AF_F_BL_GRAV) return bad(AF_ERR_ARG, "unknown flux kind");
    }
    if (P.diff < AF_A_LINEAR || P.diff > AF_A_RAMP2) return bad(AF_ERR_ARG, "unknown potential kind");
    if (P.precision != 32 && P.precision != 64) return bad(AF_ERR_ARG, "precision must be 32 or 64");
    if (P.integrator != AF_RK_SSP3 && P.integrator != AF_RK_EULER && P.integrator != AF_RK_SSP54)
        return bad(AF_ERR_ARG, "unknown integrator");
    if (!(P.cfl > 0)) return bad(AF_ERR_CFL, "cfl must be positive");
    // every forward-Euler stage must satisfy the MPP condition C <= 1/(2 dim)
    const double stage_max = P.integrator == AF_RK_SSP54 ? kSSP54MaxStage : 1.0;
    if (P.limiter && P.cfl * stage_max > 1.0 / (2 * P.dim) * (1 + 1e-12))
        return bad(AF_ERR_CFL, "with the limiter cfl times the largest stage step must not exceed 1/(2 dim)");
    if (!std::isnan(P.umin) && !std::isnan(P.umax) && !(P.umax >= P.umin)) return bad(AF_ERR_ARG, "umax < umin");
    if (P.si_blend && !(P.si_gamma >= 0)) return bad(AF_ERR_ARG, "si_gamma must be >= 0");
    if (P.diffusion_form != AF_DIFF_DC && P.diffusion_form != AF_DIFF_NODC)
        return bad(AF_ERR_ARG, "unknown diffusion form");
    if (P.diffusion_form == AF_DIFF_NODC && (P.dim != 1 || P.si_blend))
        return bad(AF_ERR_UNSUPPORTED, "the diffusion form of App. A is one-dimensional and unblended");
    for (int l = 0; l < 3; l++) {
        for (int e = 0; e < 2; e++)
            if (P.bc[l][e] < AF_BC_PERIODIC || P.bc[l][e] > AF_BC_OUTFLOW)
                return bad(AF_ERR_ARG, "unknown boundary kind");
        if ((P.bc[l][0] == AF_BC_PERIODIC) != (P.bc[l][1] == AF_BC_PERIODIC))
            return bad(AF_ERR_ARG, "both ends of an axis periodic or neither");
        if (P.bc[l][0] == AF_BC_PERIODIC) continue;
        if (l >= P.dim) return bad(AF_ERR_ARG, "ends of an unused axis must be periodic");
        if (P.dim > 2 || P.si_blend)
            return bad(AF_ERR_UNSUPPORTED, "non-periodic ends are supported for unblended 1D and 2D problems");
        for (int e = 0; e < 2; e++) {
            if (P.bc[l][e] != AF_BC_DIRICHLET) continue;
            if (!std::isfinite(P.bc_value[l][e])) return bad(AF_ERR_ARG, "Dirichlet value must be finite");
            if (P.limiter && !std::isnan(P.umin) && !std::isnan(P.umax) &&
                !(P.bc_value[l][e] >= P.umin && P.bc_value[l][e] <= P.umax))
                return bad(AF_ERR_BOUNDS, "Dirichlet value outside [umin, umax]");
        }
    }
    return AF_OK;
}

int nkinds(const af_ctx *c) { return 1 << c->dim; }

void drop_graph(af_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_steps = 0;
    c->graph_ws = true;
}

// Fluxes with convex |f'| (linear, quadratic): the CFL wave speed is a
// function of the min / max average, which the last stage of a step reduces
// (with open ends, together with the Dirichlet ghost values).
bool cfl_from_keys(const af_ctx *c) { return (c->caps & af4::kCapQF) != 0; }

// Work list (instance, tile) for the current variant; instances are kept
// contiguous so that one instance can be launched alone.
af_status build_work(af_ctx *c)
{
    af4::VariantInfo vi = af4::stage_variant(c->dim, c->variant);
    std::vector<int4> work;
    c->work_start.assign(c->n_inst, 0);
    c->work_count.assign(c->n_inst, 0);
    for (int i = 0; i < c->n_inst; i++) {
        InstDev &I = c->ih[i];
        long long nt = 1;
        for (int l = 0; l < 3; l++) {
            I.tiles[l] = (I.n[l] + vi.tile[l] - 1) / vi.tile[l];
            nt *= I.tiles[l];
        }
        c->work_start[i] = (int)work.size();
        c->work_count[i] = (int)nt;
        I.wstart = c->work_start[i];
        I.wcount = c->work_count[i];
        for (int tz = 0; tz < I.tiles[2]; tz++)
            for (int ty = 0; ty < I.tiles[1]; ty++)
                for (int tx = 0; tx < I.tiles[0]; tx++) work.push_back(make_int4(i, tx, ty, tz));
    }
    if (c->d_work) (void)hipFree(c->d_work);
    c->d_work = nullptr;
    c->nwork = (int)work.size();
    HIPOK(c, hipMalloc(&c->d_work, sizeof(int4) * work.size()));
    if (c->d_mm) (void)hipFree(c->d_mm);
    c->d_mm = nullptr;
    // one slot pair per wave of every work item
    c->waves_per_block = (vi.nt + 63) / 64;
    c->max_slots = 0;
    for (int i = 0; i < c->n_inst; i++)
        c->max_slots = std::max(c->max_slots, (long long)c->work_count[i] * c->waves_per_block);
    HIPOK(c, hipMalloc(&c->d_mm, sizeof(unsigned long long) * 2 * c->waves_per_block * work.size()));
    c->keys_fresh = false;
    HIPOK(c, hipMemcpy(c->d_work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
    HIPOK(c, hipMemcpy(c->d_inst, c->ih.data(), sizeof(InstDev) * c->n_inst, hipMemcpyHostToDevice));
    return AF_OK;
}

template <class T>
StageParams<T> stage_params(af_ctx *c, const StageSpec &sp, int stage)
{
    StageParams<T> p;
    p.inst = c->d_inst;
    p.work = c->d_work;
    p.nwork = c->nwork;
    p.in = (const T *)c->buf[sp.in];
    p.un = (const T *)c->buf[0];
    p.x1 = sp.x1 >= 0 ? (const T *)c->buf[sp.x1] : nullptr;
    p.out = (T *)c->buf[sp.out];
    p.st = c->d_st;
    p.stage = stage;
    p.mode = sp.mode;
    p.w = (T)sp.w;
    p.c0 = (T)sp.c0;
    p.c1 = (T)sp.c1;
    p.cin = (T)sp.cin;
    p.dts = (T)sp.dts;
    p.mm = nullptr;
    p.lact = c->lact_on ? c->d_lact : nullptr;
    return p;
}

hipError_t launch_stage(af_ctx *c, const StageSpec &sp, int stage, bool lim, bool si, int wstart, int wcount,
                        bool minmax = false)
{
    if (c->prec == 32) {
        StageParams<float> p = stage_params<float>(c, sp, stage);
        p.work += wstart;
        p.nwork = wcount;
        p.mm = minmax ? c->d_mm + (size_t)2 * c->waves_per_block * wstart : nullptr;
        return af4::stage_launch(c->dim, 32, lim, si, c->caps, c->variant, wcount, &p, c->stream);
    }
    StageParams<double> p = stage_params<double>(c, sp, stage);
    p.work += wstart;
    p.nwork = wcount;
    p.mm = minmax ? c->d_mm + (size_t)2 * c->waves_per_block * wstart : nullptr;
    return af4::stage_launch(c->dim, 64, lim, si, c->caps, c->variant, wcount, &p, c->stream);
}

// One time step over all instances, enqueued on the context stream.  With
// events != nullptr, records an event pair around every stage launch.  The
// wave-speed pass runs unless the previous step's last stage reduced the
// min / max averages (ws == false).
hipError_t enqueue_step(af_ctx *c, bool ws, std::vector<hipEvent_t> *events, size_t *ev_next)
{
    hipError_t e;
    if (ws) {
        e = af4::wavespeed_launch(c->dim, c->prec, c->d_inst, c->d_chunks, c->nchunks, c->buf[0], c->d_st, c->d_wslot,
                                  c->stream);
        if (e != hipSuccess) return e;
    }
    e = af4::finalize_launch(c->n_inst, c->d_inst, c->d_ctl, c->d_dtp, c->d_st, c->dim, c->prec,
                             ws ? nullptr : c->d_mm, ws ? c->d_wslot : nullptr, c->waves_per_block,
                             ws ? c->max_chunks : c->max_slots, c->stream);
    if (e != hipSuccess) return e;
    const bool mm = cfl_from_keys(c);
    const StageSpec *sp = stages_of(c->integ);
    for (int k = 0; k < num_stages(c->integ); k++) {
        if (events) (void)hipEventRecord((*events)[(*ev_next)++], c->stream);
        e = launch_stage(c, sp[k], k + 1, c->lim, c->si, 0, c->nwork, sp[k].last && mm);
        if (events) (void)hipEventRecord((*events)[(*ev_next)++], c->stream);
        if (e != hipSuccess) return e;
    }
    if (c->integ == AF_RK_EULER) e = af4::copy_launch(c->prec, c->buf[1], c->buf[0], c->total, c->stream);
    return e;
}

af_status upload_ctl(af_ctx *c, double t_end, const double *dtp)
{
    StepCtl ctl;
    ctl.t_end = t_end > 0 ? t_end : 0.0;
    ctl.prescribed = dtp ? 1 : 0;
    ctl.pad = 0;
    HIPOK(c, hipMemcpyAsync(c->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, c->stream));
    if (dtp) HIPOK(c, hipMemcpyAsync(c->d_dtp, dtp, sizeof(double) * c->n_inst, hipMemcpyHostToDevice, c->stream));
    // the host buffers may go away after return: finish the copies now
    HIPOK(c, hipStreamSynchronize(c->stream));
    return AF_OK;
}

af_status check_ready(af_ctx *c)
{
    for (int i = 0; i < c->n_inst; i++)
        if (!c->have_state[i]) return fail(c, AF_ERR_STATE, "af_set_state has not been called for every instance");
    return AF_OK;
}

af_status finish_step(af_ctx *c, double *dt_used)
{
    std::vector<InstState> st(c->n_inst);
    HIPOK(c, hipMemcpyAsync(st.data(), c->d_st, sizeof(InstState) * c->n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    bool bad = false;
    for (int i = 0; i < c->n_inst; i++) {
        if (dt_used) dt_used[i] = st[i].dt;
        if (st[i].flags & 1u) bad = true;
    }
    if (bad) return fail(c, AF_ERR_NONFINITE, "non-finite or divergent state produced");
    return AF_OK;
}

template <class T>
void to_device_layout(const double *src, void *dst, long long n)
{
    T *d = (T *)dst;
    for (long long i = 0; i < n; i++) d[i] = (T)src[i];
}

template <class T>
void from_device_layout(const void *src, double *dst, long long n)
{
    const T *s = (const T *)src;
    for (long long i = 0; i < n; i++) dst[i] = (double)s[i];
}

}  // namespace

extern "C" {

af_status af_create(int n_inst, const af_problem *probs, af_ctx **out)
{
    if (!out || !probs || n_inst < 1) return fail(nullptr, AF_ERR_ARG, "af_create: bad arguments");
    *out = nullptr;
    for (int i = 0; i < n_inst; i++) {
        af_status s = validate(probs[i], i);
        if (s != AF_OK) return s;
        const af_problem &a = probs[0], &b = probs[i];
        if (b.dim != a.dim || b.precision != a.precision || !!b.limiter != !!a.limiter ||
            !!b.si_blend != !!a.si_blend || b.integrator != a.integrator)
            return fail(nullptr, AF_ERR_UNSUPPORTED,
                        "instances of one context must share dim, precision, limiter, si_blend and integrator");
    }
    af_ctx *c = new af_ctx();
    c->n_inst = n_inst;
    c->dim = probs[0].dim;
    c->prec = probs[0].precision;
    c->lim = !!probs[0].limiter;
    c->si = !!probs[0].si_blend;
    for (int i = 0; i < n_inst; i++)
        for (int l = 0; l < 3; l++)
            if (probs[i].bc[l][0] != AF_BC_PERIODIC) c->open = true;
    c->integ = probs[0].integrator;
    c->prob.assign(probs, probs + n_inst);
    c->ih.resize(n_inst);
    c->have_state.assign(n_inst, 0);
    long long off = 0;
    for (int i = 0; i < n_inst; i++) {
        const af_problem &P = probs[i];
        InstDev &I = c->ih[i];
        std::memset(&I, 0, sizeof I);
        I.vol = 1.0;
        for (int l = 0; l < 3; l++) {
            I.n[l] = l < P.dim ? P.n[l] : 1;
            I.dx[l] = l < P.dim ? (P.hi[l] - P.lo[l]) / P.n[l] : 1.0;
            I.fk[l] = l < P.dim ? P.flux[l] : AF_F_LINEAR;
            I.fp0[l] = l < P.dim ? P.flux_par[l][0] : 0.0;
            I.fp1[l] = l < P.dim ? P.flux_par[l][1] : 0.0;
            if (l < P.dim) I.vol *= I.dx[l];
            I.idx1[l] = 1.0 / I.dx[l];
            I.idx2[l] = 1.0 / (I.dx[l] * I.dx[l]);
            I.i6dx[l] = 1.0 / (6.0 * I.dx[l]);
        }
        I.ncell = (long long)I.n[0] * I.n[1] * I.n[2];
        I.kstride = (I.ncell + 63) / 64 * 64;
        I.off = off;
        off += I.kstride * (1 << P.dim);
        I.ak = P.diff;
        I.ap0 = P.diff_par[0];
        I.ap1 = P.diff_par[1];
        int m = 0;
        I.am = (P.diff == AF_A_POWER && is_int_exponent(P.diff_par[1], &m)) ? m : 0;
        set_unified_potential(I, P);
        I.umin = P.umin;
        I.umax = P.umax;
        I.cfl = P.cfl;
        I.si_gamma = P.si_blend ? P.si_gamma : 0.0;
        I.nodc = P.diffusion_form == AF_DIFF_NODC;
        for (int l = 0; l < 3; l++)
            for (int e = 0; e < 2; e++) {
                I.bc[l][e] = P.bc[l][e];
                I.bcv[l][e] = P.bc[l][e] == AF_BC_DIRICHLET ? P.bc_value[l][e] : 0.0;
            }
        if (!std::isnan(P.umin) && !std::isnan(P.umax)) derive_bounds_params(I, P, P.dim);
        set_f32_params(I);
    }
    c->total = off;
    c->caps = af4::kCapQF | af4::kCapPP | af4::kCapI32 | af4::kCapBQ | af4::kCapBLF | (c->open ? af4::kCapOpen : 0u);
    for (int i = 0; i < n_inst; i++) {
        const InstDev &I = c->ih[i];
        for (int l = 0; l < c->dim; l++) {
            if (probs[i].flux[l] != AF_F_LINEAR && probs[i].flux[l] != AF_F_QUAD) c->caps &= ~af4::kCapQF;
            if (probs[i].flux[l] != AF_F_BL && probs[i].flux[l] != AF_F_BL_GRAV) c->caps &= ~af4::kCapBLF;
            if (probs[i].flux[l] != AF_F_QUAD && !(probs[i].flux[l] == AF_F_LINEAR && probs[i].flux_par[l][0] == 0.0))
                c->caps &= ~af4::kCapBQ;
        }
        const bool pure_poly = !I.ppow && !I.pabs && I.pu0 == 0.0 && std::isinf(I.plo) && I.plo < 0 &&
                               std::isinf(I.phi) && I.phi > 0;
        if (!pure_poly) c->caps &= ~af4::kCapPP;
        if ((double)(1 << c->dim) * (double)I.kstride * (double)vbytes(c) >= 4294967296.0) c->caps &= ~af4::kCapI32;
    }
    // default tile variant: the first one built for this combination (the
    // residual kernel, unlimited and unblended, fits wherever the stage does)
    c->variant = -1;
    for (int v = 0; v < af4::stage_num_variants(c->dim); v++)
        if (af4::stage_supported(c->dim, c->prec, c->lim, c->si, c->caps, v)) {
            c->variant = v;
            break;
        }
    if (c->variant < 0) {
        delete c;
        return fail(nullptr, AF_ERR_UNSUPPORTED, "no stage kernel fits this dimension/precision/flag combination");
    }
    hipError_t e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        fail(nullptr, AF_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        delete c;
        return AF_ERR_DEVICE;
    }
    c->stream = c->own_stream;
    auto alloc = [&](void **p, size_t bytes) -> bool {
        hipError_t r = hipMalloc(p, bytes);
        if (r != hipSuccess) {
            fail(nullptr, AF_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(r));
            return false;
        }
        return true;
    };
    bool ok = true;
    for (int b = 0; b < num_buffers(c->integ) && ok; b++) ok = alloc(&c->buf[b], (size_t)c->total * vbytes(c));
    ok = ok && alloc((void **)&c->d_inst, sizeof(InstDev) * n_inst);
    ok = ok && alloc((void **)&c->d_st, sizeof(InstState) * n_inst);
    ok = ok && alloc((void **)&c->d_ctl, sizeof(StepCtl));
    ok = ok && alloc((void **)&c->d_dtp, sizeof(double) * n_inst);
    ok = ok && alloc((void **)&c->d_npart, sizeof(double) * 9 * af4::kNormBlocks);
    ok = ok && alloc((void **)&c->d_nout, sizeof(double) * 16);
    if (!ok) {
        af_destroy(c);
        return AF_ERR_ALLOC;
    }
    if (hipMemset(c->d_st, 0, sizeof(InstState) * n_inst) != hipSuccess ||
        hipMemset(c->d_dtp, 0, sizeof(double) * n_inst) != hipSuccess) {
        af_destroy(c);
        return fail(nullptr, AF_ERR_DEVICE, "hipMemset failed");
    }
    // wave-speed chunks
    std::vector<int2> chunks;
    for (int i = 0; i < n_inst; i++) {
        // rows, or segments of long rows, per chunk (af4::wave_chunk)
        InstDev &I = c->ih[i];
        const long long nch = af4::wave_chunk_count(I.n[0], (long long)I.n[1] * I.n[2]);
        if ((long long)chunks.size() + nch > (1ll << 30)) {
            af_destroy(c);
            return fail(nullptr, AF_ERR_ARG, "af_create: too many cells");
        }
        I.cstart = (int)chunks.size();
        I.ccount = (int)nch;
        c->max_chunks = std::max(c->max_chunks, nch);
        for (long long k = 0; k < nch; k++) chunks.push_back(make_int2(i, (int)k));
    }
    c->nchunks = (int)chunks.size();
    if (!alloc((void **)&c->d_wslot, sizeof(unsigned long long) * chunks.size()) ||
        !alloc((void **)&c->d_chunks, sizeof(int2) * chunks.size()) ||
        hipMemcpy(c->d_chunks, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice) != hipSuccess) {
        af_destroy(c);
        return AF_ERR_DEVICE;
    }
    af_status s = build_work(c);
    if (s != AF_OK) {
        g_create_err = c->err;
        af_destroy(c);
        return s;
    }
    *out = c;
    return AF_OK;
}

af_status af_destroy(af_ctx *c)
{
    if (!c) return AF_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    for (int b = 0; b < 5; b++)  // SSP-RK(5,4) contexts hold five state buffers
        if (c->buf[b]) (void)hipFree(c->buf[b]);
    void *ptrs[] = {c->d_inst, c->d_st,     c->d_ctl,  c->d_dtp, c->d_work,
                    c->d_chunks, c->d_npart, c->d_nout, c->d_mm,  c->d_lact, c->d_wslot};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
    return AF_OK;
}

const char *af_last_error(const af_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

af_status af_set_stream(af_ctx *c, void *stream)
{
    if (!c) return AF_ERR_ARG;
    HIPOK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->stream = stream ? (hipStream_t)stream : c->own_stream;
    return AF_OK;
}

int af_num_variants(const af_ctx *c) { return c ? af4::stage_num_variants(c->dim) : 0; }

int af_get_variant(const af_ctx *c) { return c ? c->variant : -1; }

const char *af_variant_name(const af_ctx *c, int v)
{
    if (!c || v < 0 || v >= af4::stage_num_variants(c->dim)) return "";
    return af4::stage_variant(c->dim, v).name;
}

af_status af_set_variant(af_ctx *c, int v)
{
    if (!c) return AF_ERR_ARG;
    if (v < 0 || v >= af4::stage_num_variants(c->dim)) return fail(c, AF_ERR_ARG, "variant out of range");
    if (!af4::stage_supported(c->dim, c->prec, c->lim, c->si, c->caps, v))
        return fail(c, AF_ERR_UNSUPPORTED, "tile variant not built for this combination");
    HIPOK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->variant = v;
    return build_work(c);
}

}  // extern "C"

namespace {

// The bounds part of setting a state, shared by the host and the device
// setters: lo / hi are the min / max of the DoFs rounded to the storage
// precision.  Derives [umin, umax] on the first call when they were NaN at
// creation, then checks the DoFs and the Dirichlet values against them when
// the limiter is on.  Mutates nothing before every check has passed.
af_status accept_bounds(af_ctx *c, int inst, double lo, double hi, const char *who)
{
    InstDev &I = c->ih[inst];
    const af_problem &P = c->prob[inst];
    double umin = I.umin, umax = I.umax;
    const bool derive = (std::isnan(P.umin) || std::isnan(P.umax)) && !c->have_state[inst];
    if (derive) {
        umin = lo;
        umax = hi;
        for (int l = 0; l < 3; l++)  // Dirichlet data bound the solution too
            for (int e = 0; e < 2; e++)
                if (P.bc[l][e] == AF_BC_DIRICHLET) {
                    const double g = c->prec == 32 ? (double)(float)P.bc_value[l][e] : P.bc_value[l][e];
                    umin = std::min(umin, g);
                    umax = std::max(umax, g);
                }
    }
    if (c->lim) {
        if (lo < umin || hi > umax) return fail(c, AF_ERR_BOUNDS, std::string(who) + ": DoF outside [umin, umax]");
        for (int l = 0; l < 3; l++)
            for (int e = 0; e < 2; e++) {
                const double g = c->prec == 32 ? (double)(float)P.bc_value[l][e] : P.bc_value[l][e];
                if (P.bc[l][e] == AF_BC_DIRICHLET && !(g >= umin && g <= umax))
                    return fail(c, AF_ERR_BOUNDS, std::string(who) + ": Dirichlet value outside [umin, umax]");
            }
    }
    if (derive) {
        I.umin = umin;
        I.umax = umax;
        derive_bounds_params(I, P, c->dim);
        set_f32_params(I);
        HIPOK(c, hipMemcpy(c->d_inst + inst, &I, sizeof I, hipMemcpyHostToDevice));
    }
    return AF_OK;
}

// The last part of setting a state: time t, step count and flags cleared.
af_status commit_state(af_ctx *c, int inst, double t)
{
    InstState st;
    std::memset(&st, 0, sizeof st);
    st.t = t;
    HIPOK(c, hipMemcpyAsync(c->d_st + inst, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    c->have_state[inst] = 1;
    c->keys_fresh = false;  // the new state's min / max are not reduced yet
    return AF_OK;
}

// Orders the context's work after the caller's: the caller's arrays are
// ready (and free to overwrite) once the work queued on `stream` is done.
af_status after_caller(af_ctx *c, void *stream)
{
    if ((hipStream_t)stream != c->stream) HIPOK(c, hipStreamSynchronize((hipStream_t)stream));
    return AF_OK;
}

}  // namespace

extern "C" {

af_status af_set_state(af_ctx *c, int inst, const double *const *dofs, double t)
{
    if (!c || inst < 0 || inst >= c->n_inst || !dofs) return fail(c, AF_ERR_ARG, "af_set_state: bad arguments");
    const InstDev &I = c->ih[inst];
    const int nk = nkinds(c);
    const long long n = I.ncell;
    // round to the storage precision first: bounds and checks see what is stored
    std::vector<double> r((size_t)n * nk);
    for (int z = 0; z < nk; z++) {
        if (!dofs[z]) return fail(c, AF_ERR_ARG, "af_set_state: null DoF array");
        for (long long k = 0; k < n; k++) {
            const double v = c->prec == 32 ? (double)(float)dofs[z][k] : dofs[z][k];
            if (!std::isfinite(v)) return fail(c, AF_ERR_NONFINITE, "af_set_state: non-finite DoF");
            r[(size_t)z * n + k] = v;
        }
    }
    const auto mm = std::minmax_element(r.begin(), r.end());
    const af_status bs = accept_bounds(c, inst, *mm.first, *mm.second, "af_set_state");
    if (bs != AF_OK) return bs;
    std::vector<char> stage((size_t)n * vbytes(c));
    char *base = (char *)c->buf[0] + (size_t)I.off * vbytes(c);
    for (int z = 0; z < nk; z++) {
        if (c->prec == 32) to_device_layout<float>(&r[(size_t)z * n], stage.data(), n);
        else to_device_layout<double>(&r[(size_t)z * n], stage.data(), n);
        HIPOK(c, hipMemcpyAsync(base + (size_t)z * I.kstride * vbytes(c), stage.data(), stage.size(),
                                hipMemcpyHostToDevice, c->stream));
        HIPOK(c, hipStreamSynchronize(c->stream));
    }
    return commit_state(c, inst, t);
}

af_status af_set_state_dev(af_ctx *c, int inst, const double *const *dofs, double t, void *stream)
{
    if (!c || inst < 0 || inst >= c->n_inst || !dofs) return fail(c, AF_ERR_ARG, "af_set_state_dev: bad arguments");
    const InstDev &I = c->ih[inst];
    const int nk = nkinds(c);
    const size_t vb = vbytes(c);
    for (int z = 0; z < nk; z++)
        if (!dofs[z]) return fail(c, AF_ERR_ARG, "af_set_state_dev: null DoF array");
    const af_status os = after_caller(c, stream);
    if (os != AF_OK) return os;
    // the rounded DoFs go to the instance's part of state buffer 1 (free
    // between steps) and are checked there, so a rejected state leaves the
    // context's state as it was
    char *stg = (char *)c->buf[1] + (size_t)I.off * vb;
    for (int z = 0; z < nk; z++)
        HIPOK(c, af4::convert_launch(c->prec, true, dofs[z], stg + (size_t)z * I.kstride * vb, I.ncell, c->stream));
    HIPOK(c, af4::norms_launch(c->prec, stg, I.ncell, I.kstride, nk, c->d_npart, c->d_nout, c->stream));
    double r[9];
    HIPOK(c, hipMemcpyAsync(r, c->d_nout, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    if (r[8] > 0) return fail(c, AF_ERR_NONFINITE, "af_set_state_dev: non-finite DoF");
    const af_status bs = accept_bounds(c, inst, std::min(r[4], r[6]), std::max(r[5], r[7]), "af_set_state_dev");
    if (bs != AF_OK) return bs;
    char *base = (char *)c->buf[0] + (size_t)I.off * vb;
    for (int z = 0; z < nk; z++)
        HIPOK(c, af4::copy_launch(c->prec, stg + (size_t)z * I.kstride * vb, base + (size_t)z * I.kstride * vb, I.ncell,
                                  c->stream));
    return commit_state(c, inst, t);
}

af_status af_get_state(af_ctx *c, int inst, double *const *dofs, double *t)
{
    if (!c || inst < 0 || inst >= c->n_inst || !dofs) return fail(c, AF_ERR_ARG, "af_get_state: bad arguments");
    const InstDev &I = c->ih[inst];
    const long long n = I.ncell;
    std::vector<char> stage((size_t)n * vbytes(c));
    const char *base = (const char *)c->buf[0] + (size_t)I.off * vbytes(c);
    for (int z = 0; z < nkinds(c); z++) {
        if (!dofs[z]) return fail(c, AF_ERR_ARG, "af_get_state: null DoF array");
        HIPOK(c, hipMemcpyAsync(stage.data(), base + (size_t)z * I.kstride * vbytes(c), stage.size(),
                                hipMemcpyDeviceToHost, c->stream));
        HIPOK(c, hipStreamSynchronize(c->stream));
        if (c->prec == 32) from_device_layout<float>(stage.data(), dofs[z], n);
        else from_device_layout<double>(stage.data(), dofs[z], n);
    }
    if (t) {
        InstState st;
        HIPOK(c, hipMemcpyAsync(&st, c->d_st + inst, sizeof st, hipMemcpyDeviceToHost, c->stream));
        HIPOK(c, hipStreamSynchronize(c->stream));
        *t = st.t;
    }
    return AF_OK;
}

af_status af_get_state_dev(af_ctx *c, int inst, double *const *dofs, double *t, void *stream)
{
    if (!c || inst < 0 || inst >= c->n_inst || !dofs) return fail(c, AF_ERR_ARG, "af_get_state_dev: bad arguments");
    const InstDev &I = c->ih[inst];
    const size_t vb = vbytes(c);
    for (int z = 0; z < nkinds(c); z++)
        if (!dofs[z]) return fail(c, AF_ERR_ARG, "af_get_state_dev: null DoF array");
    const af_status os = after_caller(c, stream);
    if (os != AF_OK) return os;
    const char *base = (const char *)c->buf[0] + (size_t)I.off * vb;
    for (int z = 0; z < nkinds(c); z++)
        HIPOK(c, af4::convert_launch(c->prec, false, base + (size_t)z * I.kstride * vb, dofs[z], I.ncell, c->stream));
    InstState st;
    if (t) HIPOK(c, hipMemcpyAsync(&st, c->d_st + inst, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    if (t) *t = st.t;
    return AF_OK;
}

af_status af_step(af_ctx *c, int nsteps, double t_end, const double *dt_prescribed, double *dt_used)
{
    if (!c || nsteps < 0) return fail(c, AF_ERR_ARG, "af_step: bad arguments");
    af_status s = check_ready(c);
    if (s != AF_OK) return s;
    if (dt_prescribed)
        for (int i = 0; i < c->n_inst; i++)
            if (!(dt_prescribed[i] >= 0) || !std::isfinite(dt_prescribed[i]))
                return fail(c, AF_ERR_ARG, "af_step: prescribed dt must be finite and >= 0");
    if ((s = upload_ctl(c, t_end, dt_prescribed)) != AF_OK) return s;
    if (nsteps == 0) return finish_step(c, dt_used);
    const bool ws0 = !(c->keys_fresh && cfl_from_keys(c)), ws = !cfl_from_keys(c);
    c->keys_fresh = false;  // until the launch below has completed
    if (nsteps == 1) {
        HIPOK(c, enqueue_step(c, ws0, nullptr, nullptr));
    } else {
        if (!c->gexec || c->graph_steps != nsteps || c->graph_ws != ws0) {
            drop_graph(c);
            HIPOK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int k = 0; k < nsteps && e == hipSuccess; k++) e = enqueue_step(c, k == 0 ? ws0 : ws, nullptr, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(c, AF_ERR_DEVICE, std::string("graph capture: ") +
                                                  hipGetErrorString(e != hipSuccess ? e : e2));
            }
            c->graph = g;
            HIPOK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
            c->graph_steps = nsteps;
            c->graph_ws = ws0;
        }
        HIPOK(c, hipGraphLaunch(c->gexec, c->stream));
    }
    s = finish_step(c, dt_used);
    c->keys_fresh = s == AF_OK && cfl_from_keys(c);
    return s;
}

af_status af_step_timed(af_ctx *c, int nsteps, double t_end, const double *dt_prescribed, double *mean_stage_ms,
                        int *launches)
{
    if (!c || nsteps < 1) return fail(c, AF_ERR_ARG, "af_step_timed: bad arguments");
    af_status s = check_ready(c);
    if (s != AF_OK) return s;
    if ((s = upload_ctl(c, t_end, dt_prescribed)) != AF_OK) return s;
    const int per = num_stages(c->integ);
    std::vector<hipEvent_t> ev((size_t)2 * per * nsteps);
    for (auto &e : ev) HIPOK(c, hipEventCreate(&e));
    size_t next = 0;
    hipError_t err = hipSuccess;
    const bool ws0 = !(c->keys_fresh && cfl_from_keys(c)), ws = !cfl_from_keys(c);
    c->keys_fresh = false;
    for (int k = 0; k < nsteps && err == hipSuccess; k++) err = enqueue_step(c, k == 0 ? ws0 : ws, &ev, &next);
    hipError_t se = hipStreamSynchronize(c->stream);
    double total = 0;
    for (size_t k = 0; k + 1 < next; k += 2) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        total += ms;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess || se != hipSuccess)
        return fail(c, AF_ERR_DEVICE, std::string("af_step_timed: ") + hipGetErrorString(err != hipSuccess ? err : se));
    if (mean_stage_ms) *mean_stage_ms = next ? total / (next / 2) : 0.0;
    if (launches) *launches = (int)(next / 2);
    s = finish_step(c, nullptr);
    c->keys_fresh = s == AF_OK && cfl_from_keys(c);
    return s;
}

af_status af_autotune(af_ctx *c, int nsteps, int *chosen, double *ms_per_stage)
{
    if (!c || nsteps < 1) return fail(c, AF_ERR_ARG, "af_autotune: bad arguments");
    af_status s = check_ready(c);
    if (s != AF_OK) return s;
    const int nv = af4::stage_num_variants(c->dim);
    if (ms_per_stage)
        for (int v = 0; v < nv; v++) ms_per_stage[v] = -1.0;
    // the state (buffer A) and the per-instance scalars, restored after
    // every variant
    const size_t bytes = (size_t)c->total * vbytes(c);
    void *backup = nullptr;
    if (hipMalloc(&backup, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, AF_ERR_ALLOC, "af_autotune: no device memory for the state copy");
    }
    std::vector<InstState> st(c->n_inst);
    hipError_t e = hipMemcpyAsync(backup, c->buf[0], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.data(), c->d_st, sizeof(InstState) * c->n_inst, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    auto restore = [&]() -> hipError_t {
        hipError_t r = hipMemcpyAsync(c->buf[0], backup, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (r == hipSuccess)
            r = hipMemcpyAsync(c->d_st, st.data(), sizeof(InstState) * c->n_inst, hipMemcpyHostToDevice, c->stream);
        if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
        c->keys_fresh = false;  // the restored state's min / max are not reduced
        return r;
    };
    const int v0 = c->variant;
    if (e != hipSuccess) s = fail(c, AF_ERR_DEVICE, std::string("af_autotune: ") + hipGetErrorString(e));
    // one untimed pass first, so that the variant timed first does not pay
    // for clocks and caches still settling
    if (s == AF_OK) {
        double ms = 0.0;
        int launches = 0;
        s = af_step_timed(c, nsteps, 0.0, nullptr, &ms, &launches);
        if (s == AF_OK && (e = restore()) != hipSuccess)
            s = fail(c, AF_ERR_DEVICE, std::string("af_autotune: ") + hipGetErrorString(e));
    }
    // two timed passes, in index order and back, keeping each variant's
    // faster figure: neither a variant's position in the order nor one slow
    // measurement decides the choice
    std::vector<double> t(nv, -1.0);
    for (int pass = 0; pass < 2 && s == AF_OK; pass++)
        for (int k = 0; k < nv && s == AF_OK; k++) {
            const int v = pass == 0 ? k : nv - 1 - k;
            if (!af4::stage_supported(c->dim, c->prec, c->lim, c->si, c->caps, v)) continue;
            double ms = 0.0;
            int launches = 0;
            if ((s = af_set_variant(c, v)) != AF_OK) break;
            if ((s = af_step_timed(c, 1, 0.0, nullptr, &ms, &launches)) != AF_OK) break;
            if ((s = af_step_timed(c, nsteps, 0.0, nullptr, &ms, &launches)) != AF_OK) break;
            if ((e = restore()) != hipSuccess) {
                s = fail(c, AF_ERR_DEVICE, std::string("af_autotune: ") + hipGetErrorString(e));
                break;
            }
            t[v] = t[v] < 0 ? ms : std::min(t[v], ms);
        }
    int best = -1;
    for (int v = 0; v < nv && s == AF_OK; v++) {
        if (t[v] < 0) continue;
        if (ms_per_stage) ms_per_stage[v] = t[v];
        if (best < 0 || t[v] < 0.97 * t[best]) best = v;
    }
    if (s == AF_OK) {
        s = af_set_variant(c, best);
    } else {
        const std::string msg = c->err;
        (void)af_set_variant(c, v0);
        (void)restore();
        c->err = msg;
    }
    (void)hipFree(backup);
    if (s == AF_OK && chosen) *chosen = best;
    return s;
}

af_status af_limiter_activity(af_ctx *c, int inst, long long *counts)
{
    if (!c || inst < 0 || inst >= c->n_inst || !counts) return fail(c, AF_ERR_ARG, "af_limiter_activity: bad arguments");
    af_status s = check_ready(c);
    if (s != AF_OK) return s;
    if (!c->lim) return fail(c, AF_ERR_UNSUPPORTED, "af_limiter_activity: the limiter is off");
    // the generic kernel of one tile variant has the counting form; the
    // tile variant in use is restored after
    const int v0 = c->variant, vg = af4::count_variant(c->dim);
    if (!af4::stage_supported(c->dim, c->prec, c->lim, c->si, c->caps, vg))
        return fail(c, AF_ERR_UNSUPPORTED, "af_limiter_activity: the counting kernel does not fit this combination");
    if (!c->d_lact) {
        if (hipMalloc(&c->d_lact, sizeof(unsigned long long) * 2 * c->n_inst) != hipSuccess) {
            (void)hipGetLastError();
            c->d_lact = nullptr;
            return fail(c, AF_ERR_ALLOC, "af_limiter_activity: counters");
        }
    }
    std::vector<InstState> st(c->n_inst);
    HIPOK(c, hipMemcpyAsync(st.data(), c->d_st, sizeof(InstState) * c->n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    if (vg != v0 && (s = af_set_variant(c, vg)) != AF_OK) return s;
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipMemsetAsync(c->d_lact, 0, sizeof(unsigned long long) * 2 * c->n_inst, c->stream);
    if (e == hipSuccess && (s = upload_ctl(c, 0.0, nullptr)) != AF_OK) e = hipErrorUnknown;
    // the CFL step of the current state, then one forward-Euler stage into
    // the scratch buffer B with counting on
    if (e == hipSuccess && s == AF_OK)
        e = af4::wavespeed_launch(c->dim, c->prec, c->d_inst, c->d_chunks, c->nchunks, c->buf[0], c->d_st, c->d_wslot,
                                  c->stream);
    if (e == hipSuccess && s == AF_OK)
        e = af4::finalize_launch(c->n_inst, c->d_inst, c->d_ctl, c->d_dtp, c->d_st, c->dim, c->prec, nullptr,
                                 c->d_wslot, c->waves_per_block, c->max_chunks, c->stream);
    if (e == hipSuccess && s == AF_OK) {
        const StageSpec fe = {0, 1, -1, af4::kCombFE, 1.0, 0, 0, 0, 1.0, false};
        c->lact_on = true;
        e = launch_stage(c, fe, 1, c->lim, c->si, c->work_start[inst], c->work_count[inst]);
        c->lact_on = false;
    }
    if (e == hipSuccess && s == AF_OK)
        e = hipMemcpyAsync(h, c->d_lact + 2 * inst, sizeof h, hipMemcpyDeviceToHost, c->stream);
    // restore the per-instance scalars and the variant
    if (e == hipSuccess && s == AF_OK)
        e = hipMemcpyAsync(c->d_st, st.data(), sizeof(InstState) * c->n_inst, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && s == AF_OK) e = hipStreamSynchronize(c->stream);
    c->keys_fresh = false;
    const std::string msg = e != hipSuccess ? std::string("af_limiter_activity: ") + hipGetErrorString(e) : c->err;
    if (vg != v0) {
        const af_status s2 = af_set_variant(c, v0);
        if (s == AF_OK && e == hipSuccess) s = s2;
    }
    if (e != hipSuccess) return fail(c, AF_ERR_DEVICE, msg);
    if (s != AF_OK) return s;
    const long long ncell = c->ih[inst].ncell;
    counts[0] = c->dim * ncell;                                        // face fluxes
    counts[1] = (long long)h[0];                                       // of which limited
    counts[2] = c->ih[inst].nodc ? 0 : c->dim * ncell;                 // cell potentials
    counts[3] = (long long)h[1];                                       // of which limited
    return AF_OK;
}

af_status af_residual(af_ctx *c, int inst, double *const *rhs)
{
    if (!c || inst < 0 || inst >= c->n_inst || !rhs) return fail(c, AF_ERR_ARG, "af_residual: bad arguments");
    if (!c->have_state[inst]) return fail(c, AF_ERR_STATE, "af_residual before af_set_state");
    const StageSpec fe = {0, 1, -1, af4::kCombFE, 1.0, 0, 0, 0, 1.0, false};
    HIPOK(c, launch_stage(c, fe, af4::kStageRHS, false, false, c->work_start[inst], c->work_count[inst]));
    const InstDev &I = c->ih[inst];
    std::vector<char> stage((size_t)I.ncell * vbytes(c));
    const char *base = (const char *)c->buf[1] + (size_t)I.off * vbytes(c);
    for (int z = 0; z < nkinds(c); z++) {
        HIPOK(c, hipMemcpyAsync(stage.data(), base + (size_t)z * I.kstride * vbytes(c), stage.size(),
                                hipMemcpyDeviceToHost, c->stream));
        HIPOK(c, hipStreamSynchronize(c->stream));
        if (c->prec == 32) from_device_layout<float>(stage.data(), rhs[z], I.ncell);
        else from_device_layout<double>(stage.data(), rhs[z], I.ncell);
    }
    return AF_OK;
}

// af_norms_t from the nine FP64 reductions of norms_launch (sum u, sum |u|,
// sum u^2, max |u|, min / max average, min / max point value, non-finite
// count) and the cell volume; time, step and clamp fields zero.
static void norms_from_sums(const double *r, double vol, af_norms_t *out)
{
    std::memset(out, 0, sizeof *out);
    out->mass = r[0] * vol;
    out->l1_avg = r[1] * vol;
    out->l2_avg = std::sqrt(r[2] * vol);
    out->linf_avg = r[3];
    out->min_avg = r[4];
    out->max_avg = r[5];
    out->min_pv = r[6];
    out->max_pv = r[7];
    out->nonfinite = r[8] > 0 ? 1 : 0;
}

af_status af_norms(af_ctx *c, int inst, af_norms_t *out)
{
    if (!c || inst < 0 || inst >= c->n_inst || !out) return fail(c, AF_ERR_ARG, "af_norms: bad arguments");
    const InstDev &I = c->ih[inst];
    const char *base = (const char *)c->buf[0] + (size_t)I.off * vbytes(c);
    HIPOK(c, af4::norms_launch(c->prec, base, I.ncell, I.kstride, nkinds(c), c->d_npart, c->d_nout, c->stream));
    double r[9];
    InstState st;
    HIPOK(c, hipMemcpyAsync(r, c->d_nout, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipMemcpyAsync(&st, c->d_st + inst, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIPOK(c, hipStreamSynchronize(c->stream));
    norms_from_sums(r, I.vol, out);
    out->t = st.t;
    out->dt_last = st.dt;
    if (st.flags & 1u) out->nonfinite = 1;
    out->max_clamp = __builtin_bit_cast(double, st.clampmax);
    out->steps = st.steps;
    return AF_OK;
}

af_status af_norms_noalloc(int dim, int precision, const int *n, const double *lo, const double *hi, const void *dofs,
                           long long kind_stride, void *stream, af_norms_t *out)
{
    if (dim < 1 || dim > 3 || (precision != 32 && precision != 64) || !n || !lo || !hi || !dofs || !out)
        return fail(nullptr, AF_ERR_ARG, "af_norms_noalloc: bad arguments");
    long long ncell = 1;
    double vol = 1.0;
    for (int l = 0; l < dim; l++) {
        if (n[l] < 1 || !(hi[l] > lo[l])) return fail(nullptr, AF_ERR_ARG, "af_norms_noalloc: bad grid");
        ncell *= n[l];
        vol *= (hi[l] - lo[l]) / n[l];
    }
    // the kinds of the block must not overlap, and every index of the block
    // must fit the kernels' 64-bit element indexing
    const long long kinds = 1ll << dim;
    if (kind_stride < ncell || kind_stride > (1ll << 56) / kinds)
        return fail(nullptr, AF_ERR_ARG, "af_norms_noalloc: kind_stride must be at least the number of cells");
    double *scr = nullptr;
    hipError_t e = af4::noalloc_scratch(&scr);
    if (e != hipSuccess) return fail(nullptr, AF_ERR_DEVICE, std::string("af_norms_noalloc: scratch: ") + hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    double r[9];
    e = af4::norms_launch(precision, dofs, ncell, kind_stride, (int)kinds, scr, scr + 9 * af4::kNormBlocks, s);
    if (e == hipSuccess) e = hipMemcpyAsync(r, scr + 9 * af4::kNormBlocks, sizeof r, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(nullptr, AF_ERR_DEVICE, std::string("af_norms_noalloc: ") + hipGetErrorString(e));
    norms_from_sums(r, vol, out);
    return AF_OK;
}

af_status af_copy_rate(long long bytes, int reps, double *gb_per_s)
{
    if (bytes < 16 || reps < 1 || !gb_per_s) return fail(nullptr, AF_ERR_ARG, "af_copy_rate: bad arguments");
    const long long n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, n16 * 16);
    if (e == hipSuccess) e = hipMalloc(&b, n16 * 16);
    if (e != hipSuccess) {
        if (a) (void)hipFree(a);
        (void)hipGetLastError();
        return fail(nullptr, AF_ERR_ALLOC, "af_copy_rate: buffers");
    }
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, n16 * 16, s);
    if (e == hipSuccess) e = af4::copy16_launch(a, b, n16, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; r++) e = af4::copy16_launch(a, b, n16, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const std::string msg = e != hipSuccess ? std::string("af_copy_rate: ") + hipGetErrorString(e) : "";
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(nullptr, AF_ERR_DEVICE, msg);
    *gb_per_s = 2.0 * (double)n16 * 16.0 * reps / (ms * 1e-3) / 1e9;
    return AF_OK;
}

af_status af_work(const af_ctx *c, double *bytes_per_stage, double *cells, double *dofs)
{
    if (!c) return AF_ERR_ARG;
    double nc = 0;
    for (const InstDev &I : c->ih) nc += (double)I.ncell;
    // state arrays read or written per stage: input and output, plus X0 for
    // blended stages and X0, X1 for summed ones, averaged over the step
    double arrays = 0;
    for (int k = 0; k < num_stages(c->integ); k++) {
        const StageSpec &sp = stages_of(c->integ)[k];
        arrays += 2.0 + (sp.mode == af4::kCombBlend ? 1.0 : 0.0) + (sp.mode == af4::kCombSum ? 2.0 : 0.0);
    }
    const double per_cell_stage = arrays / num_stages(c->integ) * (1 << c->dim) * (double)vbytes(c);
    if (bytes_per_stage) *bytes_per_stage = per_cell_stage * nc;
    if (cells) *cells = nc;
    if (dofs) *dofs = nc * (1 << c->dim);
    return AF_OK;
}

}  // extern "C"
