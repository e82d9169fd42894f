"""Seeded synthetic workloads and initial data.

This module holds no arithmetic of the numerical method: it only builds
problem descriptions (plain dicts) and initial DoF arrays in FP64, with numpy
``default_rng`` (PCG64) streams, so that the GPU library and the CPU oracle
are fed the same inputs.  Exact solutions used by tests are also here; they
are closed forms of the PDE, not of the scheme.

Problem dict::

    {"name": str, "dim": d, "n": [n0, ..], "lo": [..], "hi": [..],
     "flux": [(kind, p0, p1), ...]   # per axis; kinds: linear c*u, quad c*u^2,
                                     # bl u^2/(u^2+(1-u)^2), bl_grav bl*(1-g(1-u)^2)
     "diff": (kind, p0, p1),         # linear k0*u, power c*u^m,
                                     # deadzone eps*sign(u)max(0,|u|-u0),
                                     # bl eps(2u^2-4u^3/3) on [0,1],
                                     # ramp2 (c/2) max(0,u-u0)^2
     "umin": .., "umax": .., "cfl": .., "limiter": bool, "si": bool,
     "si_gamma": .., "precision": 32|64, "t_end": .. or None, "steps": .. or None}

DoFs: list of 2^d float64 arrays in the zeta order of Sec. 4 of the paper
(average, then point values), each flat with x fastest; the point value at
i+1/2 is stored at index i.

Seeds: 251011527 + k for the k-th benchmark workload (k = 1..5).
"""
import math

import numpy as np

SEED_BASE = 251011527

# half-shift masks of the DoFs in zeta order (bit l set: half index in axis l)
ZETA_MASKS = {1: [0, 1], 2: [0, 1, 2, 3], 3: [0, 1, 2, 4, 3, 5, 6, 7]}


def dx_of(spec):
    return [(spec["hi"][l] - spec["lo"][l]) / spec["n"][l] for l in range(spec["dim"])]


def dof_coords(spec, mask):
    """Coordinates (one 1D array per axis) of the DoF points of one kind."""
    d = spec["dim"]
    dx = dx_of(spec)
    out = []
    for l in range(d):
        i = np.arange(spec["n"][l], dtype=np.float64)
        if mask >> l & 1:
            out.append(spec["lo"][l] + (i + 1.0) * dx[l])
        else:
            out.append(spec["lo"][l] + (i + 0.5) * dx[l])
    return out


def _outer_apply(fn_axes, spec):
    """Evaluate a separable product over the grid (x fastest): returns flat."""
    arr = fn_axes[0]
    for l in range(1, spec["dim"]):
        arr = np.multiply.outer(fn_axes[l], arr)
    return arr.reshape(-1)


def fourier_dofs(spec, modes):
    """DoFs of g(x) = sum_k A_k sin(2 pi k.x + phi_k) on a periodic box:
    averages exact (sinc products), point values sampled.  Returns the list
    of 2^d arrays (unscaled)."""
    d = spec["dim"]
    dx = dx_of(spec)
    L = [spec["hi"][l] - spec["lo"][l] for l in range(d)]
    dofs = []
    for mask in ZETA_MASKS[d]:
        xs = dof_coords(spec, mask)
        acc = np.zeros(int(np.prod(spec["n"][:d])))
        for (k, A, phi) in modes:
            # sin(sum theta_l + phi) = Im(e^{i phi} prod_l e^{i theta_l})
            axes = []
            for l in range(d):
                w = 2 * math.pi * k[l] / L[l]
                f = np.exp(1j * w * xs[l])
                if mask == 0 and k[l] != 0:
                    # cell average: sinc factor in every axis
                    z = w * dx[l] / 2
                    f = f * (math.sin(z) / z)
                axes.append(f)
            prod = _outer_apply(axes, spec)
            acc += A * np.imag(np.exp(1j * phi) * prod)
        dofs.append(acc)
    return dofs


def rescale01(dofs):
    g0 = min(float(x.min()) for x in dofs)
    g1 = max(float(x.max()) for x in dofs)
    return [(x - g0) / (g1 - g0) for x in dofs]


def bounds_of(dofs, precision=64):
    if precision == 32:
        dofs = [x.astype(np.float32).astype(np.float64) for x in dofs]
    return min(float(x.min()) for x in dofs), max(float(x.max()) for x in dofs)


def round_to(dofs, precision):
    if precision == 32:
        return [x.astype(np.float32).astype(np.float64) for x in dofs]
    return [np.array(x, dtype=np.float64) for x in dofs]


def _subsample_avg(spec, indicator, sub=16, chunk_rows=32):
    """Cell averages of a piecewise-constant 2D field by sub x sub midpoint
    sub-sampling; indicator(X, Y) returns values on coordinate grids."""
    nx, ny = spec["n"][0], spec["n"][1]
    dx, dy = dx_of(spec)
    xs = spec["lo"][0] + (np.arange(nx * sub) + 0.5) * dx / sub
    out = np.empty((ny, nx))
    for j0 in range(0, ny, chunk_rows):
        j1 = min(ny, j0 + chunk_rows)
        ys = spec["lo"][1] + (np.arange(j0 * sub, j1 * sub) + 0.5) * dy / sub
        vals = indicator(xs[None, :], ys[:, None])
        out[j0:j1] = vals.reshape(j1 - j0, sub, nx, sub).mean(axis=(1, 3))
    return out.reshape(-1)


def _point_dofs_2d(spec, field):
    d = 2
    dofs = []
    for mask in ZETA_MASKS[d][1:]:
        xs, ys = dof_coords(spec, mask)
        dofs.append(field(xs[None, :], ys[:, None]).reshape(-1))
    return dofs


# ---------------------------------------------------------------------------
# Benchmark workloads
# ---------------------------------------------------------------------------

def config1(seed=SEED_BASE + 1, n=80, cfl=0.3):
    """1D linear u_t + u_x = 0.01 u_xx on [0,1], u0 = sin(2 pi x + phi).
    The stated CFL 0.4 is unstable for SSP-RK3 with this scheme; 0.3 is the
    reading used (0.4 is kept for the divergence test)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0, 2 * math.pi)
    spec = dict(name="c1_linear_1d", dim=1, n=[n], lo=[0.0], hi=[1.0],
                flux=[("linear", 1.0, 0.0)], diff=("linear", 0.01, 0.0),
                cfl=cfl, limiter=False, si=False, si_gamma=1.0, precision=64,
                t_end=1.0, steps=None, phi=phi)
    dofs = rescale_free_fourier_1d(spec, phi, 0.0)
    spec["umin"], spec["umax"] = bounds_of(dofs)
    return spec, dofs


def rescale_free_fourier_1d(spec, phi, t, c=1.0, k0=0.01):
    """DoFs of exp(-4 pi^2 k0 t) sin(2 pi (x - c t) + phi) (exact solution)."""
    decay = math.exp(-4 * math.pi ** 2 * k0 * t)
    return [decay * x for x in fourier_dofs(spec, [((1,), 1.0, phi - 2 * math.pi * c * t)])]


def config2(seed=SEED_BASE + 2, n=512, cfl=0.05):
    """2D strongly degenerate Burgers, f = (u^2/2, u^2/2),
    a = 0.05 max(0, u - 0.25) (eps = 0.1 scale on kappa = 0.5 above 0.25),
    u0 = union of 12 axis-aligned periodic blocks painted in order."""
    rng = np.random.default_rng(seed)
    blocks = []
    for _ in range(12):
        x0 = rng.uniform(0, 1)
        y0 = rng.uniform(0, 1)
        w = rng.uniform(0.05, 0.3)
        h = rng.uniform(0.05, 0.3)
        v = rng.uniform(0, 1)
        blocks.append((x0, y0, w, h, v))
    spec = dict(name="c2_burgers_deadzone_2d", dim=2, n=[n, n], lo=[0.0, 0.0], hi=[1.0, 1.0],
                flux=[("quad", 0.5, 0.0), ("quad", 0.5, 0.0)], diff=("deadzone", 0.05, 0.25),
                cfl=cfl, limiter=True, si=False, si_gamma=1.0, precision=64, t_end=0.25, steps=None)

    def field(X, Y):
        out = np.zeros(np.broadcast(X, Y).shape)
        for (x0, y0, w, h, v) in blocks:
            inside = (np.mod(X - x0, 1.0) < w) & (np.mod(Y - y0, 1.0) < h)
            out = np.where(inside, v, out)
        return out

    dofs = [_subsample_avg(spec, field)] + _point_dofs_2d(spec, field)
    spec["umin"], spec["umax"] = bounds_of(dofs)
    return spec, dofs


def config3(seed=SEED_BASE + 3, n=1024, precision=64, cfl=0.05):
    """2D Buckley-Leverett with gravity on [-1.5,1.5]^2, kappa = 0.04 u(1-u),
    u0 = 1 inside a union of 5 disks (minimum-image distance), else 0."""
    rng = np.random.default_rng(seed)
    disks = []
    for _ in range(5):
        cx = rng.uniform(-1.5, 1.5)
        cy = rng.uniform(-1.5, 1.5)
        r = rng.uniform(0.2, 0.5)
        disks.append((cx, cy, r))
    spec = dict(name="c3_buckley_leverett_gravity_2d", dim=2, n=[n, n], lo=[-1.5, -1.5], hi=[1.5, 1.5],
                flux=[("bl", 0.0, 0.0), ("bl_grav", 0.0, 5.0)], diff=("bl", 0.01, 0.0),
                cfl=cfl, limiter=True, si=False, si_gamma=1.0, precision=precision, t_end=0.5, steps=None)

    def field(X, Y):
        out = np.zeros(np.broadcast(X, Y).shape)
        for (cx, cy, r) in disks:
            ddx = np.mod(X - cx + 1.5, 3.0) - 1.5
            ddy = np.mod(Y - cy + 1.5, 3.0) - 1.5
            out = np.where(ddx * ddx + ddy * ddy < r * r, 1.0, out)
        return out

    dofs = [_subsample_avg(spec, field)] + _point_dofs_2d(spec, field)
    dofs = round_to(dofs, precision)
    spec["umin"], spec["umax"] = bounds_of(dofs, precision)
    return spec, dofs


def _modes(rng, nmodes, d):
    ks = [k for k in np.ndindex(*([9] * d))]
    ks = [tuple(int(v) - 4 for v in k) for k in ks]
    ks = [k for k in ks if any(v != 0 for v in k)]
    out = []
    for _ in range(nmodes):
        k = ks[int(rng.integers(len(ks)))]
        A = rng.uniform(0, 1)
        phi = rng.uniform(0, 2 * math.pi)
        out.append((k, A, phi))
    return out


def config4(seed=SEED_BASE + 4, n_inst=256, sizes=(64, 128, 256, 512), cfl=0.05, steps=200,
            with_dofs=True, limiter=True):
    """Batch of independent 2D porous-medium/Burgers instances of uneven
    size: f = (u^2/2, u^2/2), a = c u^m, u0 = random 8-mode Fourier sum
    rescaled to [0,1].  Returns a list of (spec, dofs)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        N = int(sizes[int(rng.integers(len(sizes)))])
        c = rng.uniform(0.01, 0.1)
        m = int((2, 3)[int(rng.integers(2))])
        modes = _modes(rng, 8, 2)
        spec = dict(name="c4_batched_pme_burgers_2d[%d]" % i, dim=2, n=[N, N], lo=[0.0, 0.0], hi=[1.0, 1.0],
                    flux=[("quad", 0.5, 0.0), ("quad", 0.5, 0.0)], diff=("power", c, float(m)),
                    cfl=cfl, limiter=limiter, si=False, si_gamma=1.0, precision=32, t_end=None, steps=steps,
                    modes=modes)
        dofs = None
        if with_dofs:
            dofs = round_to(rescale01(fourier_dofs(spec, modes)), 32)
            spec["umin"], spec["umax"] = bounds_of(dofs, 32)
        else:
            spec["umin"], spec["umax"] = 0.0, 1.0
        out.append((spec, dofs))
    return out


def config4_dofs(spec):
    dofs = round_to(rescale01(fourier_dofs(spec, spec["modes"])), 32)
    return dofs


def config5(seed=SEED_BASE + 5, n=256, cfl=0.03, steps=100):
    """3D degenerate convection-diffusion, f = (u^2/2)x3,
    kappa = 0.1 max(0, u - 0.3), u0 = 6-mode Fourier sum rescaled to [0,1];
    FP32, limiter and smoothness-indicator blending (gamma = 1)."""
    rng = np.random.default_rng(seed)
    modes = _modes(rng, 6, 3)
    spec = dict(name="c5_degenerate_3d", dim=3, n=[n, n, n], lo=[0.0] * 3, hi=[1.0] * 3,
                flux=[("quad", 0.5, 0.0)] * 3, diff=("ramp2", 0.1, 0.3),
                cfl=cfl, limiter=True, si=True, si_gamma=1.0, precision=32, t_end=None, steps=steps,
                modes=modes)
    dofs = round_to(rescale01(fourier_dofs(spec, modes)), 32)
    spec["umin"], spec["umax"] = bounds_of(dofs, 32)
    return spec, dofs


def _ek_profile_antiderivative(x):
    """Antiderivative from -1 of the initial profile of the Evje-Karlsen
    example (1 on [-1, -0.4), -2.5 x on [-0.4, 0), 0 on [0, 1)), extended
    periodically with period 2 (the profile's integral over a period is 0.8)."""
    k = np.floor((x + 1.0) / 2.0)
    y = x - 2.0 * k
    g = np.where(y < -0.4, y + 1.0, np.where(y < 0.0, 0.8 - 1.25 * y * y, 0.8))
    return 0.8 * k + g


def config_nodc(seed=SEED_BASE + 6, n_inst=1024, n=8192, cfl=0.075, precision=64, diffusion_form="nodc",
                limiter=True):
    """Batch of 1D strongly degenerate problems for the diffusion form of
    App. A: a periodic stand-in of the Evje-Karlsen example (the paper's runs
    use Dirichlet data on [-1, 1]).  f = u^2/4, a = max(0, u - 1/2) (kappa
    jumps from 0 to 1 at u = 1/2: zero on a set of positive measure), initial
    profile of that example shifted by a uniform random offset in [-1, 1);
    averages exact, point values sampled; bounds [0, 1].  Returns a list of
    (spec, dofs)."""
    rng = np.random.default_rng(seed)
    out = []
    dx = 2.0 / n
    edges = -1.0 + dx * np.arange(n + 1)
    for i in range(n_inst):
        sh = rng.uniform(-1.0, 1.0)
        G = _ek_profile_antiderivative(edges - sh)
        avg = (G[1:] - G[:-1]) / dx
        xf = edges[1:] - sh
        yf = xf - 2.0 * np.floor((xf + 1.0) / 2.0)
        pv = np.where(yf < -0.4, 1.0, np.where(yf < 0.0, -2.5 * yf, 0.0))
        dofs = round_to([np.clip(avg, 0.0, 1.0), pv], precision)
        spec = dict(name="nodc_ek_1d[%d]" % i, dim=1, n=[n], lo=[-1.0], hi=[1.0], flux=[("quad", 0.25, 0.0)],
                    diff=("deadzone", 1.0, 0.5), umin=0.0, umax=1.0, cfl=cfl, limiter=limiter, si=False,
                    si_gamma=1.0, precision=precision, t_end=None, steps=None, diffusion_form=diffusion_form)
        out.append((spec, dofs))
    return out


def config_ek(seed=SEED_BASE + 7, n_inst=1024, n=8192, cfl=0.075, precision=64, diffusion_form="dc",
              limiter=True):
    """Batch of 1D problems of the Evje-Karlsen example as the paper runs it
    (Example 6.5): [-1, 1] with Dirichlet ends u(-1) = 1, u(1) = 0, f = u^2/4;
    the example's C^1 potential is replaced by a = max(0, u - 1/2) (kappa
    jumps from 0 to 1 at u = 1/2 instead of ramping over [0.5, 0.6]).  The
    initial profile (1, then -2.5 (x - s) on [s - 0.4, s), then 0) has its
    ramp shifted by s ~ U[-0.3, 0.3] per instance; averages exact, point
    values sampled, the boundary point x_{N-1/2} holding the Dirichlet value;
    bounds [0, 1].  Returns a list of (spec, dofs)."""
    rng = np.random.default_rng(seed)
    out = []
    dx = 2.0 / n
    edges = -1.0 + dx * np.arange(n + 1)
    for i in range(n_inst):
        sh = rng.uniform(-0.3, 0.3)
        y = edges - sh  # the unshifted profile's coordinate; y in [-1.3, 1.3]
        G = np.where(y < -0.4, y + 1.0, np.where(y < 0.0, 0.8 - 1.25 * y * y, 0.8))
        avg = (G[1:] - G[:-1]) / dx
        yf = y[1:]
        pv = np.where(yf < -0.4, 1.0, np.where(yf < 0.0, -2.5 * yf, 0.0))
        pv[-1] = 0.0
        dofs = round_to([np.clip(avg, 0.0, 1.0), pv], precision)
        spec = dict(name="ek_dirichlet_1d[%d]" % i, dim=1, n=[n], lo=[-1.0], hi=[1.0], flux=[("quad", 0.25, 0.0)],
                    diff=("deadzone", 1.0, 0.5), umin=0.0, umax=1.0, cfl=cfl, limiter=limiter, si=False,
                    si_gamma=1.0, precision=precision, t_end=None, steps=None, diffusion_form=diffusion_form,
                    bc=(("dirichlet", 1.0), ("dirichlet", 0.0)))
        out.append((spec, dofs))
    return out


# ---------------------------------------------------------------------------
# Small problems of the paper's examples, used by tests
# ---------------------------------------------------------------------------

def smooth_linear(d, n, c=1.0, k0=0.01, t=0.0, limiter=False):
    """Example 6.1: u = 1 + exp(-4 d pi^2 k0 t) sin(2 pi sum_l (x_l - c t))
    on [0,1]^d, f_l = c u, a = k0 u.  Returns (spec, DoFs at time t)."""
    spec = dict(name="ex61_smooth_linear_%dd" % d, dim=d, n=[n] * d, lo=[0.0] * d, hi=[1.0] * d,
                flux=[("linear", c, 0.0)] * d, diff=("linear", k0, 0.0), cfl=0.3 / d,
                limiter=limiter, si=False, si_gamma=1.0, precision=64, t_end=None, steps=None)
    dofs = smooth_linear_exact(spec, t, c, k0)
    spec["umin"], spec["umax"] = bounds_of(dofs)
    return spec, dofs


def smooth_linear_exact(spec, t, c=1.0, k0=0.01):
    d = spec["dim"]
    decay = math.exp(-4 * d * math.pi ** 2 * k0 * t)
    g = fourier_dofs(spec, [((1,) * d, 1.0, -2 * math.pi * c * t * d)])
    return [1.0 + decay * x for x in g]


def sin4_advection(n, t=0.0):
    """Example 6.2: u_t + u_x = 0, u = 1 + sin^4(2 pi (x - t)) on [0,1];
    bounds [1, 2].  sin^4 y = 3/8 - cos(2y)/2 + cos(4y)/8."""
    spec = dict(name="ex62_sin4_1d", dim=1, n=[n], lo=[0.0], hi=[1.0],
                flux=[("linear", 1.0, 0.0)], diff=("linear", 0.0, 0.0), cfl=0.3,
                limiter=True, si=False, si_gamma=1.0, precision=64, t_end=1.0, steps=None,
                umin=1.0, umax=2.0)
    s = -2 * math.pi * t
    # 3/8 - cos(2y)/2 + cos(4y)/8 with y = 2 pi x + s; cos(z) = sin(z + pi/2)
    g = fourier_dofs(spec, [((2,), -0.5, 2 * s + math.pi / 2), ((4,), 0.125, 4 * s + math.pi / 2)])
    return spec, [1.0 + 3.0 / 8.0 + x for x in g]


def barenblatt_value(m, d, x2, t):
    """Barenblatt solution B_m (Example 6.3) at squared radius x2, time t."""
    alpha = 1.0 / (m - 1 + 2.0 / d)
    core = 1 - alpha * (m - 1) / (2 * d * m) * x2 / t ** (2 * alpha / d)
    return t ** (-alpha) * np.maximum(0.0, core) ** (1.0 / (m - 1))


def barenblatt(d, m, n=80, t=1.0, sub=8, limiter=True):
    """Example 6.3 on [-L, L]^d (L = 6, 8, 10), initial data B_m(., t),
    averages by sub^d midpoint sub-sampling, point values sampled.  The
    support stays well inside the domain for t <= 2, so periodic wrap-around
    does not interact with it."""
    Lh = {1: 6.0, 2: 8.0, 3: 10.0}[d]
    spec = dict(name="ex63_barenblatt_%dd_m%d" % (d, m), dim=d, n=[n] * d, lo=[-Lh] * d, hi=[Lh] * d,
                flux=[("linear", 0.0, 0.0)] * d, diff=("power", 1.0, float(m)), cfl=0.1 / d,
                limiter=limiter, si=False, si_gamma=1.0, precision=64, t_end=None, steps=None)
    dx = dx_of(spec)
    dofs = []
    for mask in ZETA_MASKS[d]:
        coords = []
        for l in range(d):
            if mask >> l & 1:
                coords.append(dof_coords(spec, mask)[l][:, None])
            else:
                i = np.arange(n, dtype=np.float64)[:, None]
                s = (np.arange(sub, dtype=np.float64)[None, :] + 0.5) / sub - 0.5
                coords.append(spec["lo"][l] + (i + 0.5 + s) * dx[l])
        # squared radius on the product grid of (cell, subsample) per axis
        r2 = None
        for l in range(d):
            c2 = coords[l] ** 2
            r2 = c2 if r2 is None else np.add.outer(c2, r2)
        v = barenblatt_value(m, d, r2, t)
        # average over the subsample axes (odd axes of the outer product)
        sub_axes = tuple(2 * k + 1 for k in range(d))
        v = v.mean(axis=sub_axes)
        dofs.append(np.ascontiguousarray(v).reshape(-1))
    spec["umin"], spec["umax"] = 0.0, max(float(x.max()) for x in dofs)
    return spec, dofs
