/*
 * af.h -- C ABI of the MI355X (gfx950) implementation of the compact
 * fourth-order doubly conservative active flux (AF) method with monolithic
 * convex limiting for degenerate convection-diffusion equations
 *
 *     u_t + div f(u) = Lap a(u),   a(u) = int kappa,  kappa >= 0,
 *
 * on uniform Cartesian meshes in 1, 2 or 3 dimensions, periodic or (1D, 2D)
 * with Dirichlet or outflow ends (J. Duan, arXiv 2510.11527; the PDE is
 * Eq. (cde_conservative), the maximum principle [u_min, u_max] is stated in
 * Sec. 1 and its discrete form, for averages and point values, in Def. 5.1).
 *
 * Every call returns an af_status; no C++ exception crosses this boundary.
 * All host buffers are owned by the caller and copied by the library; the
 * context owns all device memory until af_destroy.  A context is not
 * thread-safe; distinct contexts are independent.
 *
 * DoF layout (Sec. 4 of the paper, "zeta order"): a state of a d-dimensional
 * instance is 2^d arrays of n0*n1*n2 values each, x fastest:
 *   1D: average, x-face point value
 *   2D: average, x-face, y-face, corner
 *   3D: average, x-face, y-face, z-face, (i+1/2,j+1/2,k), (i+1/2,j,k+1/2),
 *       (i,j+1/2,k+1/2), corner
 * The point value at a half index i+1/2 is stored at index i.
 */
#ifndef AF4_AF_H
#define AF4_AF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct af_ctx af_ctx;

typedef enum {
    AF_OK = 0,
    AF_ERR_ARG = -1,         /* invalid argument or problem description */
    AF_ERR_ALLOC = -2,       /* device or host allocation failed */
    AF_ERR_DEVICE = -3,      /* a HIP call failed; see af_last_error */
    AF_ERR_BOUNDS = -4,      /* state outside [umin, umax] with the limiter on */
    AF_ERR_NONFINITE = -5,   /* non-finite or divergent state */
    AF_ERR_CFL = -6,         /* CFL number outside the admissible range */
    AF_ERR_STATE = -7,       /* call out of order (e.g. step before set_state) */
    AF_ERR_UNSUPPORTED = -8  /* valid but not supported combination */
} af_status;

/* Convection flux f_l(u) per axis (Sec. 6 examples). */
typedef enum {
    AF_F_LINEAR = 0,  /* p0 * u                                  */
    AF_F_QUAD = 1,    /* p0 * u^2   (p0 = 1/2: Burgers)          */
    AF_F_BL = 2,      /* u^2 / (u^2 + (1-u)^2)  (Example 6.6)    */
    AF_F_BL_GRAV = 3  /* BL(u) * (1 - p1 (1-u)^2)  (Example 6.6) */
} af_flux_kind;

/* Diffusion potential a(u) = int kappa (Sec. 1). */
typedef enum {
    AF_A_LINEAR = 0,   /* p0 * u                                            */
    AF_A_POWER = 1,    /* p0 * u^p1  (porous medium, Eq. (pme))             */
    AF_A_DEADZONE = 2, /* p0 * sign(u) * max(0, |u| - p1)  (Examples 6.8/9) */
    AF_A_BL = 3,       /* p0 (2u^2 - 4u^3/3) on [0,1], constant outside     */
    AF_A_RAMP2 = 4     /* (p0/2) max(0, u - p1)^2, i.e. kappa = p0 max(0,u-p1) */
} af_diff_kind;

typedef enum {
    AF_RK_SSP3 = 0,   /* SSP-RK3, Shu-Osher form; R(z) of Sec. 3.2 */
    AF_RK_EULER = 1,  /* one forward-Euler stage per step (Sec. 5)  */
    AF_RK_SSP54 = 2   /* SSP-RK(5,4) of Spiteri and Ruuth, the paper's integrator
                         (Sec. 1; R(z) with eta = 0.004477718303076 in Sec. 3.2);
                         five stages, two more state buffers */
} af_integrator;

/* Ends of an axis (1D and 2D problems).  The paper runs its Examples
 * 6.5-6.9 with Dirichlet or outflow ends but states no ghost treatment; the
 * one used: a half-grid point on or beyond an open end -- ghost point values,
 * ghost cell averages (their centres) and the boundary points x_{-1/2},
 * x_{N-1/2} -- takes a boundary value: the Dirichlet value if one of the ends
 * it lies on or beyond is Dirichlet (lowest axis first), else (outflow) the
 * mean average of the domain cells whose closure contains the point moved
 * onto the boundary (one cell, two along an edge in 2D).  The stored point
 * values on the high ends (index N-1 of the faces normal to the axis, and of
 * the corners) are not unknowns: their input is ignored, a stage writes the
 * Dirichlet value (Dirichlet end) or passes the input through (outflow), and
 * the right-hand side there is 0.  The mass changes by the boundary fluxes. */
typedef enum {
    AF_BC_PERIODIC = 0,
    AF_BC_DIRICHLET = 1,  /* u = bc_value at the end */
    AF_BC_OUTFLOW = 2     /* zero-order extrapolation of the boundary cell's average */
} af_bc;

/* Form of the diffusion discretization. */
typedef enum {
    AF_DIFF_DC = 0,   /* doubly conservative (Secs. 2.2, 4): the paper's method */
    AF_DIFF_NODC = 1  /* App. A, 1D only: averages with the face fluxes
                         kappa(u_{i+1/2}) D_c(u)_{i+1/2}, point values with the
                         compact operator of Eq. (1d_diff_compact_kappa_u).  With
                         the limiter, the diffusion flux joins the convective
                         one in the face correction (one limited correction per
                         low-order state; the paper states no formula for it) */
} af_diffusion_form;

typedef struct {
    int dim;                 /* 1, 2 or 3 */
    int n[3];                /* cells per axis (>= 4 on used axes) */
    double lo[3], hi[3];     /* periodic box */
    int flux[3];             /* af_flux_kind per axis */
    double flux_par[3][2];   /* p0, p1 per axis */
    int diff;                /* af_diff_kind */
    double diff_par[2];      /* p0, p1 */
    double umin, umax;       /* bounds; NaN: min/max over the DoFs of the first af_set_state */
    double cfl;              /* C in dt = C / max_{l,faces}(alpha_l/dx_l + kappa_max/dx_l^2),
                                Eqs. (1d_av_pp_dt, multid_av_pp_dt); with the limiter every
                                forward-Euler stage needs C s <= 1/(2d), s its step in units of
                                dt: C <= 1/(2d) for SSP-RK3 and Euler, C <= 0.7541/d for SSP-RK(5,4) */
    int limiter;             /* 1: monolithic convex limiting of the averages (Sec. 5.1.1, 5.2.1)
                                and projection of the point values (Sec. 5.1.2) */
    int si_blend;            /* 1: smoothness-indicator blending (Sec. 5.1.3) */
    double si_gamma;         /* gamma of the blending */
    int precision;           /* 32 or 64: storage and stencil arithmetic */
    int integrator;          /* af_integrator */
    int diffusion_form;      /* af_diffusion_form; AF_DIFF_NODC needs dim = 1 and no
                                blending (else AF_ERR_UNSUPPORTED) */
    int bc[3][2];            /* af_bc of the low and high end of each axis: both periodic or
                                neither (AF_ERR_ARG); non-periodic ends need dim <= 2 and no
                                blending (AF_ERR_UNSUPPORTED) */
    double bc_value[3][2];   /* Dirichlet values; with the limiter inside [umin, umax]
                                (AF_ERR_BOUNDS, checked when the bounds are known) */
} af_problem;

typedef struct {
    double t;                /* time of the state */
    double dt_last;          /* last step size used */
    double mass;             /* FP64 sum of averages times the cell volume */
    double min_avg, max_avg; /* over the averages */
    double min_pv, max_pv;   /* over the point values */
    double l1_avg, l2_avg, linf_avg;  /* volume-weighted norms of the averages */
    double max_clamp;        /* largest safeguard clamp applied to an average so far */
    long long steps;         /* steps taken */
    int nonfinite;           /* 1 if a non-finite value was produced */
    int reserved;
} af_norms_t;

/* Creates a context holding n_inst independent instances (batched when
 * n_inst > 1: one launch per Runge-Kutta stage advances all of them, each
 * with its own time step).  All instances must share dim, precision,
 * limiter, si_blend and integrator (else AF_ERR_UNSUPPORTED); grids, fluxes,
 * potentials, bounds and CFL numbers may differ.  Validation: n >= 4 on used
 * axes, hi > lo, 0 < cfl, and with the limiter the stage bound on cfl above
 * (AF_ERR_CFL).  Allocates three state buffers per instance (five for
 * SSP-RK(5,4)) on the current HIP device. */
af_status af_create(int n_inst, const af_problem *probs, af_ctx **out);

/* Frees all device memory and graphs of the context.  NULL is accepted. */
af_status af_destroy(af_ctx *ctx);

/* Copies the state of instance inst from the host: dofs[0..2^d-1] point to
 * n0*n1*n2 doubles each, in zeta order (the DoFs of Sec. 2 and Sec. 4: cell
 * averages and the point values shared by neighbouring cells).  FP32
 * contexts round to nearest.  Validates before mutating: non-finite ->
 * AF_ERR_NONFINITE; with the limiter, a (rounded) value outside [umin, umax]
 * -> AF_ERR_BOUNDS, since the MPP property of Def. 5.1 starts from DoFs
 * inside the bounds.  If umin/umax were NaN at creation they are set here,
 * once, to the min/max of the (rounded) DoFs and Dirichlet values -- the
 * discrete form of the bounds of the initial data (Sec. 1).  In FP32 the
 * kernels clamp and limit against the nearest floats inside [umin, umax]. */
af_status af_set_state(af_ctx *ctx, int inst, const double *const *dofs, double t);

/* Copies the state of instance inst to the host (widened to double). */
af_status af_get_state(af_ctx *ctx, int inst, double *const *dofs, double *t);

/* af_set_state for DoFs in device memory: dofs (a host array of 2^d
 * pointers) points to 2^d device arrays of n0*n1*n2 doubles each, in zeta
 * order, readable by the context's device.  The arrays must be ready once
 * the work queued on `stream` (a hipStream_t of the HIP runtime this library
 * is linked against; NULL: the null stream) is done: the call waits for that
 * stream first.  Rounding (FP32 contexts: to nearest), the non-finite check
 * (after rounding) and the bounds of Def. 5.1 are those of af_set_state,
 * evaluated on the device; a rejected state leaves the context as it was.
 * Synchronizes the context stream before returning: the caller's arrays may
 * be reused or freed at once.  No host copy of the state is made. */
af_status af_set_state_dev(af_ctx *ctx, int inst, const double *const *dofs, double t, void *stream);

/* af_get_state to device memory: writes the state of instance inst, widened
 * to double, to the 2^d device arrays dofs[0..2^d-1] of n0*n1*n2 doubles
 * (zeta order), and the time to *t when t is not NULL.  Waits for `stream`
 * first (as af_set_state_dev) and synchronizes the context stream before
 * returning, so the arrays hold the state when the call returns. */
af_status af_get_state_dev(af_ctx *ctx, int inst, double *const *dofs, double *t, void *stream);

/* Advances every instance by nsteps steps.  Per step and instance, dt is
 * the CFL value computed on the device from the averages (FP64 reduction of
 * the interval maximum of |f_l'|, Eq. (1d_local_wave_speed)), or
 * dt_prescribed[inst] when dt_prescribed is not NULL; with t_end > 0 it is
 * clipped to t_end - t and an instance that has reached t_end stays put.
 * On return dt_used[inst] (if not NULL) holds the last step of each
 * instance.  Runs as one HIP graph launch when nsteps > 1.  Returns
 * AF_ERR_NONFINITE if any stage produced a non-finite value or the
 * averages diverged; the state is then readable but unspecified. */
af_status af_step(af_ctx *ctx, int nsteps, double t_end, const double *dt_prescribed, double *dt_used);

/* Semi-discrete right-hand side R(U) of instance inst, without limiting or
 * blending (Eq. (2d_af_dc); Eq. (1d_af_dc) in 1D), to rhs[0..2^d-1]. */
af_status af_residual(af_ctx *ctx, int inst, double *const *rhs);

/* Norms and diagnostics of instance inst, reduced on the device in FP64
 * over the stored DoFs: the mass (sum of averages times the cell volume,
 * conserved to round-off by the locally and doubly conservative updates of
 * Props 5.1/5.2 on periodic meshes), min/max of the averages and of the point
 * values (the bounds of Def. 5.1), the l1/l2/linf norms of the averages, the
 * time, last step and step count, the largest safeguard clamp and a
 * non-finite flag.  Sums are compensated (Neumaier) and reduced in a fixed
 * order (bitwise reproducible).  Synchronizes the context stream. */
af_status af_norms(af_ctx *ctx, int inst, af_norms_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture aside -- this call synchronizes -- tight serving loops, harnesses
 * that forbid hipMalloc): the norms of af_norms for a state held in the
 * caller's device memory, with no allocation at all.  dofs points to one
 * device block of (2^dim - 1) * kind_stride + n0*..*n_{dim-1} values of the
 * given precision (32: float, 64: double): DoF kind z (zeta order, average
 * first) at dofs + z * kind_stride, x fastest; kind_stride >= the number of
 * cells.  lo/hi give the cell volume.  The work is enqueued on stream
 * (hipStream_t, NULL: the null stream), which is then synchronized; out gets
 * mass, min/max of averages and point values, l1/l2/linf of the averages and
 * nonfinite, all reduced in FP64 exactly as af_norms does (same kernels, same
 * order: bit-identical results on the same data); t, dt_last, steps and
 * max_clamp are 0.  Scratch: the block partials live in a static device
 * array of the library (17,424 bytes, one per GPU, held until the process
 * ends; its size does not depend on the grid, so no grid is too large for
 * it).  Calls that overlap on one GPU (other host threads, other streams)
 * share that array and race; serialize them.  Errors: AF_ERR_ARG for a bad
 * dim, precision, grid, pointer or kind_stride; AF_ERR_DEVICE if a HIP call
 * fails (message in af_last_error(NULL)). */
af_status af_norms_noalloc(int dim, int precision, const int *n, const double *lo, const double *hi, const void *dofs,
                           long long kind_stride, void *stream, af_norms_t *out);

/* Message of the last error of the context (or of af_create if ctx is NULL). */
const char *af_last_error(const af_ctx *ctx);

/* Uses the given hipStream_t (passed as void*) for all further work of the
 * context; NULL restores the context's own stream.  Cached graphs are
 * dropped. */
af_status af_set_stream(af_ctx *ctx, void *stream);

/* Selects the stage-kernel tile variant (0 = default; see af_num_variants)
 * and returns AF_ERR_ARG for an out-of-range index.  Used by the tile
 * autotuner; cached graphs are dropped. */
af_status af_set_variant(af_ctx *ctx, int variant);
int af_num_variants(const af_ctx *ctx);
int af_get_variant(const af_ctx *ctx);
const char *af_variant_name(const af_ctx *ctx, int variant);

/* Times the stage kernels: runs nsteps steps like af_step, launching
 * eagerly with HIP events around every stage-kernel launch on the context
 * stream, and returns the mean stage-kernel duration in milliseconds and the
 * number of timed launches.  The state advances as with af_step. */
af_status af_step_timed(af_ctx *ctx, int nsteps, double t_end, const double *dt_prescribed, double *mean_stage_ms,
                        int *launches);

/* Tile autotuner: times every tile variant built for the context's
 * dimension, precision and flags on the current state of all instances and
 * selects the fastest by mean stage-kernel duration.  After one untimed pass
 * of nsteps steps, every variant runs one warm-up step and nsteps (>= 1) CFL
 * steps timed as af_step_timed, in two passes (index order, then reverse),
 * and keeps its faster figure; then, in index order, a variant replaces the
 * selection only when more than 3% faster, so that timing noise does not
 * move the choice.  The state, time, step count
 * and flags of every instance are restored after each variant, so the call
 * leaves the solution where it was; cached graphs are dropped.  Needs
 * af_set_state for every instance (AF_ERR_STATE); allocates one temporary
 * device copy of the state (AF_ERR_ALLOC if that fails), released before
 * returning.  On success *chosen (if not NULL) holds the selected variant
 * and ms_per_stage (if not NULL, af_num_variants entries) the measured mean
 * stage time of every variant, -1 for those not built.  On an error the
 * variant selected before the call is restored. */
af_status af_autotune(af_ctx *ctx, int nsteps, int *chosen, double *ms_per_stage);

/* Limiter activity of instance inst (Sec. 5.1.1, 5.2.1): one forward-Euler
 * stage of the current state with the current CFL step is evaluated, with
 * the generic stage kernel, into scratch memory, and the limiting parameters
 * below 1 are counted: counts[0] face fluxes evaluated (one per cell and
 * direction, the face c + 1/2), counts[1] of those with theta < 1,
 * counts[2] cell potentials evaluated (one per cell and direction; 0 in the
 * App. A form, which limits face fluxes only), counts[3] of those with
 * theta < 1.  The state, time, step count and flags are left as they were;
 * the tile variant in use is restored.  AF_ERR_UNSUPPORTED without the
 * limiter, AF_ERR_STATE before af_set_state; allocates 16 bytes per instance
 * of device memory on the first call (kept until af_destroy). */
af_status af_limiter_activity(af_ctx *ctx, int inst, long long *counts);

/* Algorithmic HBM bytes of one stage launch over all instances, averaged over
 * the stages of one step: (2 + 1 for stages that read U^n) * 2^d * cells *
 * value size.  Grid cells and DoFs of the context in *cells, *dofs. */
af_status af_work(const af_ctx *ctx, double *bytes_per_stage, double *cells, double *dofs);

/* Attainable-bandwidth reference for the roofline: times reps launches of a
 * streaming copy (16-byte elements) of `bytes` bytes between two buffers it
 * allocates on the current device and frees before returning, with HIP
 * events on a stream of its own, and returns the rate counting every byte
 * read and written, in GB/s (1e9 bytes per second).  AF_ERR_ARG for
 * bytes < 16, reps < 1 or a NULL result; AF_ERR_ALLOC if the buffers do not
 * fit; AF_ERR_DEVICE if a HIP call fails (message in af_last_error(NULL)). */
af_status af_copy_rate(long long bytes, int reps, double *gb_per_s);

#ifdef __cplusplus
}
#endif

#endif /* AF4_AF_H */
