"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU
oracle on identical seeded inputs.  Bar: relative l1 <= 1e-12 (FP64) and
<= 1e-5 (FP32, same FP32-rounded inputs), exact bounds with the limiter."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2510_11527_amd import af
from paper_2510_11527_amd import workloads as W
from gpu_common import TOL, check, check_residual, gpu_run, oracle_fe, prepare, random_state, rel_l1

pytestmark = pytest.mark.gpu

FLUXES = [("quad", 0.5, 0.0), ("bl", 0.0, 0.0), ("bl_grav", 0.0, 5.0), ("linear", -0.7, 0.0)]
DIFFS = [("power", 0.05, 2.0), ("deadzone", 0.05, 0.25), ("bl", 0.01, 0.0), ("ramp2", 0.1, 0.3), ("linear", 0.02, 0)]


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_spec(d, n, fl, df, limiter=False, si=False, precision=64, cfl=None):
    return dict(name="t", dim=d, n=[n + l for l in range(d)], lo=[0.0] * d, hi=[1.0 + 0.1 * l for l in range(d)],
                flux=[fl] * d, diff=df, umin=0.0, umax=1.0, limiter=limiter, si=si, si_gamma=1.0,
                precision=precision, cfl=cfl or 0.3 / (2 * d))


def state_for(spec, rng, smooth=False):
    d = spec["dim"]
    N = int(np.prod(spec["n"][:d]))
    if smooth:
        g = W.rescale01(W.fourier_dofs(spec, [((1,) * d, 1.0, 0.4), ((2,) + (0,) * (d - 1), 0.3, 1.1)]))
        return g
    U = [rng.uniform(0, 1, size=N) for _ in range(2 ** d)]
    U[0] = np.where(rng.uniform(size=N) < 0.6, U[0], rng.choice([0.0, 1.0], size=N))
    return U


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [64, 32])
def test_residual_matches_oracle(d, prec):
    rng = np.random.default_rng(10 * d + prec)
    n = {1: 37, 2: 21, 3: 9}[d]
    for k in range(4):
        spec = small_spec(d, n, FLUXES[k], DIFFS[(k + d) % 5], precision=prec)
        U = state_for(spec, rng, smooth=(k % 2 == 0))
        s, U = prepare(spec, U, prec)
        note("residual d=%d prec=%d flux=%s diff=%s n=%s" % (d, prec, FLUXES[k][0], DIFFS[(k + d) % 5][0], s["n"]))
        ctx = af.Context(s)
        ctx.set_state(0, U)
        R = ctx.residual(0)
        ctx.close()
        P = oracle.problem(s)
        Ro = oracle.rhs(P, U)
        check_residual(R, Ro, U, oracle.dt_cfl(P, U, s["cfl"]), prec, "d=%d k=%d" % (d, k))


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("lim,si", [(False, False), (True, False), (True, True), (False, True)])
def test_forward_euler_stage_matches_oracle(d, prec, lim, si):
    rng = np.random.default_rng(100 * d + prec + 7 * lim + 3 * si)
    n = {1: 41, 2: 19, 3: 9}[d]
    for k in range(2):
        fl, df = FLUXES[(k + d) % 4], DIFFS[(k + 2 * d) % 5]
        spec = small_spec(d, n, fl, df, limiter=lim, si=si, precision=prec)
        U = state_for(spec, rng, smooth=(k == 1))
        s, U = prepare(spec, U, prec)
        P = oracle.problem(s)
        dt = oracle.dt_cfl(P, U, s["cfl"])
        note("fe d=%d prec=%d lim=%d si=%d flux=%s diff=%s dt=%.3e" % (d, prec, lim, si, fl[0], df[0], dt))
        V, t, used, nrm = gpu_run(s, U, dts=[dt], integrator="euler")
        Vo, dg = oracle.fe(P, U, dt)
        check(V, Vo, prec, 1, "fe")
        if lim:
            assert min(v.min() for v in V) >= s["umin"] and max(v.max() for v in V) <= s["umax"]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("gamma", [0.25, 6.0])
def test_si_blending_strength_matches_oracle(d, prec, gamma):
    """Blending with gamma other than 1 (every other test uses 1, where a
    kernel that dropped gamma would still agree): one forward-Euler stage
    with the limiter, on rough random and smooth data, so that the weights
    exp(-gamma s) take intermediate values; in 3D on the marching and the
    generic kernel.  On the rough data the oracle's result at this gamma
    must differ from its result at gamma = 1 by far more than the tolerance
    (on smooth data s is small and the weights stay near 1 for any gamma)."""
    rng = np.random.default_rng(1000 * d + prec + int(4 * gamma))
    n = {1: 41, 2: 19, 3: 9}[d]
    tiles = ["3d-march-16x8x32", "generic-8x8x4"] if d == 3 else [None]
    for k in range(2):
        fl, df = FLUXES[(k + d) % 4] if d < 3 else FLUXES[3 * k % 4], DIFFS[(k + 2 * d) % 5]
        spec = small_spec(d, n, fl, df, limiter=True, si=True, precision=prec)
        spec["si_gamma"] = gamma
        U = state_for(spec, rng, smooth=(k == 1))
        s, U = prepare(spec, U, prec)
        P = oracle.problem(s)
        dt = oracle.dt_cfl(P, U, s["cfl"])
        Vo, _ = oracle.fe(P, U, dt)
        Vo1, _ = oracle.fe(oracle.problem(dict(s, si_gamma=1.0)), U, dt)
        sep = rel_l1(Vo, Vo1)
        if k == 0:
            assert sep > 100 * TOL[prec], ("gamma has no effect on this case", sep)
        for tile in tiles:
            variant = None
            if tile is not None:
                probe = af.Context(s)
                variant = [probe.variant_name(v) for v in range(probe.num_variants())].index(tile)
                probe.close()
            note("si gamma=%g d=%d prec=%d flux=%s diff=%s tile=%s: oracle gamma vs 1 rel_l1 %.2e"
                 % (gamma, d, prec, fl[0], df[0], tile, sep))
            V, _, _, _ = gpu_run(s, U, dts=[dt], integrator="euler", variant=variant)
            check(V, Vo, prec, 1, "si gamma %g" % gamma)
            assert min(v.min() for v in V) >= s["umin"] and max(v.max() for v in V) <= s["umax"]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("si", [False, True])
def test_limiter_with_bounds_around_zero(d, prec, si):
    """MPP bounds [-1, 1] (every other small case uses [0, 1], where a clamp
    or gap that took 0 for umin would agree): Burgers (f' changes sign
    inside the bounds) with linear diffusion and a linear flux against the
    grid with a dead-zone potential whose threshold is negative, on rough
    data with values at both bounds.  One forward-Euler stage; the unlimited
    oracle goes below -1, the limited GPU result matches
    the oracle and stays inside exactly; in 3D on the marching and the
    generic kernel."""
    n = {1: 41, 2: 19, 3: 9}[d]
    tiles = ["3d-march-16x8x32", "generic-8x8x4"] if d == 3 else [None]
    for k in range(2):
        fl = [("quad", 0.5, 0.0), ("linear", -0.7, 0.0)][k]
        df = [("linear", 0.02, 0), ("deadzone", 0.05, -0.25)][k]
        spec = dict(name="t", dim=d, n=[n + l for l in range(d)], lo=[0.0] * d, hi=[1.0 + 0.1 * l for l in range(d)],
                    flux=[fl] * d, diff=df, umin=-1.0, umax=1.0, limiter=True, si=si, si_gamma=1.0,
                    precision=prec, cfl=0.3 / (2 * d))
        rng = np.random.default_rng(50 * d + k + 5 * si + prec)
        N = int(np.prod(spec["n"]))
        U = [rng.uniform(-1, 1, size=N) for _ in range(2 ** d)]
        U[0] = np.where(rng.uniform(size=N) < 0.6, U[0], rng.choice([-1.0, 1.0], size=N))
        s, U = prepare(spec, U, prec)
        assert s["umin"] == -1.0 and s["umax"] == 1.0
        P = oracle.problem(s)
        dt = oracle.dt_cfl(P, U, s["cfl"])
        Vo, _ = oracle.fe(P, U, dt)
        Vu, _ = oracle.fe(oracle.problem(dict(s, limiter=False)), U, dt)
        assert min(v.min() for v in Vu) < -1.0 - 1e-3  # the limiter works at the negative bound
        for tile in tiles:
            variant = None
            if tile is not None:
                probe = af.Context(s)
                variant = [probe.variant_name(v) for v in range(probe.num_variants())].index(tile)
                probe.close()
            note("bounds [-1, 1] d=%d prec=%d si=%d flux=%s diff=%s tile=%s" % (d, prec, si, fl[0], df[0], tile))
            V, _, _, _ = gpu_run(s, U, dts=[dt], integrator="euler", variant=variant)
            check(V, Vo, prec, 1, "bounds [-1, 1]")
            assert min(v.min() for v in V) >= -1.0 and max(v.max() for v in V) <= 1.0


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("lim", [False, True])
def test_different_flux_per_axis_matches_oracle(d, prec, lim):
    """A different flux along each axis (the other small cases use one flux
    for all axes, where per-axis constants taken from the wrong axis would
    agree): Burgers, a linear flux against the grid and a linear flux along
    it, on a grid of unequal spacings; the CFL step and one forward-Euler
    stage, on every tile variant of the dimension."""
    n = {2: 19, 3: 9}[d]
    fl = [("quad", 0.5, 0.0), ("linear", -0.7, 0.0), ("linear", 0.3, 0.0)][:d]
    rng = np.random.default_rng(70 * d + prec + lim)
    spec = small_spec(d, n, fl[0], ("power", 0.05, 2.0), limiter=lim, precision=prec)
    spec["flux"] = fl
    U = state_for(spec, rng)
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    dto = oracle.dt_cfl(P, U, s["cfl"])
    Vo, _ = oracle.fe(P, U, dto)
    # the axes are not interchangeable here: the same data with the fluxes
    # of the first two axes swapped gives another result
    Vs, _ = oracle.fe(oracle.problem(dict(s, flux=[fl[1], fl[0]] + fl[2:])), U, dto)
    assert rel_l1(Vo, Vs) > 100 * TOL[prec]
    probe = af.Context(s)
    names = [probe.variant_name(v) for v in range(probe.num_variants())]
    probe.close()
    for v, name in enumerate(names):
        ctx = af.Context(s, integrator="euler")
        try:
            ctx.set_variant(v)
        except af.AFError as e:  # a variant whose kernel does not cover this case
            ctx.close()
            assert e.status == af.AF_ERR_UNSUPPORTED
            continue
        ctx.set_state(0, U)
        dtg = ctx.step(1)[0]
        V, _ = ctx.get_state(0)
        ctx.close()
        note("flux per axis d=%d prec=%d lim=%d tile=%s dt gpu %.17g oracle %.17g" % (d, prec, lim, name, dtg, dto))
        assert abs(dtg - dto) <= (1e-15 if prec == 64 else 1e-6) * dto
        Vo2, _ = oracle.fe(P, U, dtg)
        check(V, Vo2, prec, 1, "flux per axis " + name)
        if lim:
            assert min(v.min() for v in V) >= s["umin"] and max(v.max() for v in V) <= s["umax"]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [64, 32])
def test_instances_of_different_physics_in_one_context(d, prec):
    """One context holding instances with different flux and potential kinds
    (Burgers with a power law, Buckley-Leverett with its own potential, a
    linear flux with a dead zone, a linear flux along the grid with linear
    diffusion), of different sizes: three SSP-RK3 steps with the GPU's own
    CFL steps, each instance against the oracle replaying its steps.  Every
    tile variant that takes the mix."""
    n0 = {1: 41, 2: 17, 3: 9}[d]
    phys = [(("quad", 0.5, 0.0), ("power", 0.05, 2.0)), (("bl", 0.0, 0.0), ("bl", 0.01, 0.0)),
            (("linear", -0.7, 0.0), ("deadzone", 0.05, 0.25)), (("linear", 0.4, 0.0), ("linear", 0.02, 0))]
    rng = np.random.default_rng(90 * d + prec)
    items = []
    for i, (fl, df) in enumerate(phys):
        spec = small_spec(d, n0 + 3 * i, fl, df, limiter=True, si=(d != 2), precision=prec)
        U = state_for(spec, rng, smooth=(i % 2 == 1))
        items.append(prepare(spec, U, prec))
    specs = [s for s, _ in items]
    probe = af.Context(specs)
    names = [probe.variant_name(v) for v in range(probe.num_variants())]
    probe.close()
    ran = 0
    for v, name in enumerate(names):
        ctx = af.Context(specs)
        try:
            ctx.set_variant(v)
        except af.AFError as e:
            ctx.close()
            assert e.status == af.AF_ERR_UNSUPPORTED
            continue
        for i, (_, U) in enumerate(items):
            ctx.set_state(i, U)
        dts = [ctx.step(1) for _ in range(3)]
        note("mixed physics d=%d prec=%d tile=%s dt %s" % (d, prec, name, np.round(dts[0], 8).tolist()))
        for i, (s, U) in enumerate(items):
            V, _ = ctx.get_state(i)
            P = oracle.problem(s)
            assert abs(dts[0][i] - oracle.dt_cfl(P, U, s["cfl"])) <= (1e-15 if prec == 64 else 1e-6) * dts[0][i]
            Uo, _, _ = oracle.run(P, U, dts=[x[i] for x in dts])
            check(V, Uo, prec, 9, "mixed physics %s instance %d" % (name, i))
            assert min(x.min() for x in V) >= s["umin"] and max(x.max() for x in V) <= s["umax"]
        ctx.close()
        ran += 1
    assert ran >= 1


@pytest.mark.parametrize("d,n", [(1, 3001), (2, 2101)])
@pytest.mark.parametrize("prec", [64, 32])
def test_wave_speed_pass_on_rows_longer_than_a_chunk(d, n, prec):
    """Rows longer than a wave-speed chunk are split into segments, the last
    one ragged.  Buckley-Leverett fluxes (|f'| not convex: the pass runs
    every step) on averages in [0, 0.35], where |f'| increases, with the
    largest averages only in the last cells of a row: the CFL step depends on
    the ragged segment (without those cells the oracle's step is larger).
    The step of each of three SSP-RK3 steps against the oracle's for the
    GPU's state, and the state against the oracle replaying the steps."""
    fl = ("bl", 0.0, 0.0)
    spec = small_spec(d, 4, fl, ("bl", 0.01, 0.0), limiter=True, precision=prec)
    spec["n"] = [n, 4][:d]
    rng = np.random.default_rng(31 * d + prec)
    U = [0.3 * u for u in state_for(spec, rng, smooth=True)]
    U0 = U[0].reshape(spec["n"][::-1])
    U0[..., -3:] = 0.35  # the tail of every row
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    flat = [u.copy() for u in U]
    flat[0] = np.asarray(U[0]).reshape(spec["n"][::-1]).copy()
    flat[0][..., -3:] = 0.3
    flat[0] = flat[0].reshape(-1)
    assert oracle.dt_cfl(P, flat, s["cfl"]) > oracle.dt_cfl(P, U, s["cfl"]) * (1 + 1e-6)
    ctx = af.Context(s)
    ctx.set_state(0, U)
    dts = []
    for k in range(3):
        Vk, _ = ctx.get_state(0)
        dto = oracle.dt_cfl(P, Vk, s["cfl"])
        dtg = ctx.step(1)[0]
        note("long rows d=%d n=%d prec=%d step %d: dt gpu %.17g oracle %.17g" % (d, n, prec, k, dtg, dto))
        assert abs(dtg - dto) <= (1e-15 if prec == 64 else 1e-6) * dto
        dts.append(dtg)
    V, _ = ctx.get_state(0)
    ctx.close()
    Uo, _, _ = oracle.run(P, U, dts=dts)
    check(V, Uo, prec, 9, "long rows d=%d" % d)


def _steps_case(name):
    if name == "c2":
        spec, U = W.config2(n=48)
    elif name == "c3_64":
        spec, U = W.config3(n=48, precision=64)
    elif name == "c3_32":
        spec, U = W.config3(n=48, precision=32)
    elif name == "c4":
        spec, U = W.config4(n_inst=3, sizes=(32,))[2]
    elif name == "c5":
        spec, U = W.config5(n=12)
    elif name == "c1":
        spec, U = W.config1()
    return spec, U


@pytest.mark.parametrize("name", ["c1", "c2", "c3_64", "c3_32", "c4", "c5"])
def test_ssprk3_steps_match_oracle(name):
    """Ten SSP-RK3 steps with the oracle's own CFL time steps, prescribed to
    both sides (the config-like problems at reduced size)."""
    spec, U = _steps_case(name)
    prec = spec["precision"]
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    Uo, t, dts = oracle.run(P, U, nsteps=10, cfl=s["cfl"])
    note("steps %s prec=%d n=%s dt0=%.3e" % (name, prec, s["n"], dts[0]))
    V, tg, used, nrm = gpu_run(s, U, dts=dts)
    check(V, Uo, prec, 3 * len(dts), "ssprk3 " + name)
    assert abs(tg - t) <= 1e-15 * max(1.0, t) + 1e-300
    if s.get("limiter"):
        assert min(v.min() for v in V) >= s["umin"] and max(v.max() for v in V) <= s["umax"]
        ulp = np.spacing(np.float32(1.0)) if prec == 32 else np.spacing(1.0)
        assert nrm["max_clamp"] <= 4 * ulp * max(1.0, abs(s["umax"]), abs(s["umin"]))


@pytest.mark.parametrize("name", ["c1", "c2", "c3_64", "c3_32", "c4", "c5"])
def test_ssprk54_steps_match_oracle(name):
    """Ten SSP-RK(5,4) steps (the paper's integrator) with the oracle's CFL
    steps prescribed to both sides; exact bounds with the limiter."""
    spec, U = _steps_case(name)
    prec = spec["precision"]
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    Uo, t, dts = oracle.run(P, U, nsteps=10, cfl=s["cfl"], integrator="ssprk54")
    note("ssprk54 %s prec=%d n=%s dt0=%.3e" % (name, prec, s["n"], dts[0]))
    V, tg, used, nrm = gpu_run(s, U, dts=dts, integrator="ssprk54")
    check(V, Uo, prec, 5 * len(dts), "ssprk54 " + name)
    assert abs(tg - t) <= 1e-15 * max(1.0, t) + 1e-300
    if s.get("limiter"):
        assert min(v.min() for v in V) >= s["umin"] and max(v.max() for v in V) <= s["umax"]
        ulp = np.spacing(np.float32(1.0)) if prec == 32 else np.spacing(1.0)
        assert nrm["max_clamp"] <= 4 * ulp * max(1.0, abs(s["umax"]), abs(s["umin"]))


def test_ssprk54_cfl_bound():
    """With the limiter every forward-Euler stage must satisfy C s <= 1/(2d);
    the largest SSP-RK(5,4) stage step is s = b21/a21 = 0.66305 dt."""
    spec, U = W.config2(n=16)
    ok = dict(spec, cfl=0.25 / 0.6630508078509)
    af.Context(ok, integrator="ssprk54").close()
    with pytest.raises(af.AFError) as e:
        af.Context(dict(spec, cfl=0.25 / 0.66), integrator="ssprk54")
    assert e.value.status == af.AF_ERR_CFL


@pytest.mark.parametrize("name", ["c1", "c2", "c3_32", "c5"])
def test_cfl_time_step_matches_oracle(name):
    spec, U = _steps_case(name)
    prec = spec["precision"]
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    dto = oracle.dt_cfl(P, U, s["cfl"])
    ctx = af.Context(s)
    ctx.set_state(0, U)
    used = ctx.step(1)
    ctx.close()
    note("dt %s gpu=%.17g oracle=%.17g" % (name, used[0], dto))
    assert abs(used[0] - dto) <= (1e-15 if prec == 64 else 1e-6) * dto


def test_config1_full_run_matches_exact_and_oracle():
    spec, U = W.config1()
    P = oracle.problem(spec)
    Uo, t, dts = oracle.run(P, U, cfl=spec["cfl"], t_end=spec["t_end"])
    ctx = af.Context(spec)
    ctx.set_state(0, U)
    used = ctx.step(len(dts) + 3, t_end=spec["t_end"])  # extra steps are no-ops
    V, tg = ctx.get_state(0)
    nrm = ctx.norms(0)
    ctx.close()
    assert abs(tg - 1.0) < 1e-13 and nrm["steps"] == len(dts) == 480
    check(V, Uo, 64, 3 * len(dts), "1D linear to T = 1")
    ex = W.rescale_free_fourier_1d(spec, spec["phi"], 1.0)
    assert max(np.abs(a - b).mean() for a, b in zip(V, ex)) < 5e-6


def test_config1_stated_cfl_with_ssprk54_matches_oracle():
    """The 1D workload at its stated C = 0.4 with SSP-RK(5,4) to T = 1:
    GPU vs oracle and vs the exact solution."""
    spec, U = W.config1(cfl=0.4)
    P = oracle.problem(spec)
    Uo, t, dts = oracle.run(P, U, cfl=0.4, t_end=1.0, integrator="ssprk54")
    ctx = af.Context(spec, integrator="ssprk54")
    ctx.set_state(0, U)
    ctx.step(len(dts) + 2, t_end=1.0)
    V, tg = ctx.get_state(0)
    nrm = ctx.norms(0)
    ctx.close()
    assert abs(tg - 1.0) < 1e-13 and nrm["steps"] == len(dts)
    check(V, Uo, 64, 5 * len(dts), "1D linear SSP-RK(5,4) to T = 1")
    ex = W.rescale_free_fourier_1d(spec, spec["phi"], 1.0)
    assert max(np.abs(a - b).mean() for a, b in zip(V, ex)) < 2e-7


def test_divergence_is_reported():
    spec, U = W.config1(cfl=0.4)
    ctx = af.Context(spec)
    ctx.set_state(0, U)
    with pytest.raises(af.AFError) as e:
        ctx.step(400)
    assert e.value.status == af.AF_ERR_NONFINITE
    ctx.close()


def test_argument_validation():
    spec, U = W.config2(n=16)
    with pytest.raises(af.AFError) as e:
        af.Context(dict(spec, cfl=0.3))
    assert e.value.status == af.AF_ERR_CFL
    ctx = af.Context(spec)
    bad = [u.copy() for u in U]
    bad[1][3] = spec["umax"] + 0.5
    with pytest.raises(af.AFError) as e:
        ctx.set_state(0, bad)
    assert e.value.status == af.AF_ERR_BOUNDS
    bad[1][3] = math.nan
    with pytest.raises(af.AFError) as e:
        ctx.set_state(0, bad)
    assert e.value.status == af.AF_ERR_NONFINITE
    with pytest.raises(af.AFError) as e:
        ctx.step(1)
    assert e.value.status == af.AF_ERR_STATE
    ctx.close()


@pytest.mark.parametrize("d,fl,n", [(1, 2, 300), (2, 0, 70), (2, 2, 70), (3, 0, 20), (3, 0, 36)])
def test_tile_variants_agree(d, fl, n):
    """Tile shapes of one kernel family compute the same per-cell arithmetic
    (identical bits); different families agree to the parity tolerance.  In
    3D, 20 cells per axis fit one z walk of every marching tile; 36 give the
    32-plane walks a ragged last walk and every tile ragged x and y edges."""
    rng = np.random.default_rng(d + 10 * fl + n)
    spec = small_spec(d, n, FLUXES[fl], DIFFS[1], limiter=True, precision=32)
    U = state_for(spec, rng)
    s, U = prepare(spec, U, 32)
    ref = {}
    first = None
    ctx = af.Context(s)
    for v in range(ctx.num_variants()):
        name = ctx.variant_name(v)
        try:
            ctx.set_variant(v)
        except af.AFError as e:
            assert e.status == af.AF_ERR_UNSUPPORTED
            continue
        note("variant d=%d flux=%s %s" % (d, FLUXES[fl][0], name))
        ctx.set_state(0, U)
        ctx.step(2, dt=1e-4)
        V, _ = ctx.get_state(0)
        fam = name.rsplit("-", 1)[0]  # kernel family: the name without the tile
        if fam in ref:
            for a, b in zip(V, ref[fam]):
                assert np.array_equal(a, b), name
        else:
            ref[fam] = V
        if first is None:
            first = V
        check(V, first, 32, 6, "variant %s against the first variant" % name)
    ctx.close()


@pytest.mark.parametrize("d,prec", [(1, 64), (3, 32)])
def test_every_tile_variant_ssprk54_matches_oracle(d, prec):
    """Three SSP-RK(5,4) steps on every tile variant built for the problem --
    a forward-Euler stage, blending stages and the summing last stage, whose
    combinations read U^n prefetched by the kernels and X1 in their summing
    branch -- against the oracle with its CFL steps prescribed.  3D: 20 cells
    per axis give every marching tile ragged x and y edges and a walk shorter
    than the tile's; limiter and blending on."""
    if d == 1:
        spec = small_spec(1, 700, FLUXES[0], DIFFS[1], limiter=True, precision=prec)
        rng = np.random.default_rng(5401)
        U = state_for(spec, rng)
    else:
        spec, U = W.config5(n=20)
    s, U = prepare(spec, U, prec)
    P = oracle.problem(s)
    Uo, t, dts = oracle.run(P, U, nsteps=3, cfl=s["cfl"], integrator="ssprk54")
    ctx = af.Context(s, integrator="ssprk54")
    nv = ctx.num_variants()
    names = [ctx.variant_name(v) for v in range(nv)]
    ctx.close()
    ran = 0
    for v in range(nv):
        ctx = af.Context(s, integrator="ssprk54")
        try:
            ctx.set_variant(v)
        except af.AFError as e:
            assert e.status == af.AF_ERR_UNSUPPORTED
            ctx.close()
            continue
        ctx.close()
        note("ssprk54 every variant d=%d prec=%d %s n=%s" % (d, prec, names[v], s["n"]))
        V, tg, used, nrm = gpu_run(s, U, dts=dts, integrator="ssprk54", variant=v)
        check(V, Uo, prec, 5 * len(dts), "ssprk54 variant " + names[v])
        assert min(x.min() for x in V) >= s["umin"] and max(x.max() for x in V) <= s["umax"]
        ran += 1
    assert ran >= 3


@pytest.mark.parametrize("case", ["c4", "c5"])
def test_autotune_selects_a_built_variant_and_leaves_the_solution(case):
    """af_autotune times every built tile variant, keeps one within 3% of
    the fastest, and restores state, time and norms bit for bit; stepping on
    afterwards equals a fresh context on the chosen variant."""
    items = W.config4(n_inst=5, sizes=(40, 72)) if case == "c4" else [W.config5(n=14)]
    specs = [s for s, _ in items]
    ctx = af.Context(specs)
    with pytest.raises(af.AFError) as e:
        ctx.autotune(1)
    assert e.value.status == af.AF_ERR_STATE
    for i, (_, U) in enumerate(items):
        ctx.set_state(i, U)
    ctx.step(2)
    before = [ctx.get_state(i) for i in range(len(items))]
    nb = [ctx.norms(i) for i in range(len(items))]
    chosen, ms = ctx.autotune(2)
    built = [m for m in ms if m > 0]
    note("autotune %s: chosen %s, ms %s" % (case, ctx.variant_name(chosen), np.round(ms, 4)))
    assert ctx.variant() == chosen and ms[chosen] > 0 and len(built) >= 2
    assert min(built) >= 0.97 * ms[chosen] * (1 - 1e-12)
    for i in range(len(items)):
        V, t = ctx.get_state(i)
        assert t == before[i][1]
        for a, b in zip(V, before[i][0]):
            assert np.array_equal(a, b)
        assert ctx.norms(i) == nb[i]
    d1 = ctx.step(2)
    ref = af.Context(specs)
    ref.set_variant(chosen)
    for i, (V, t) in enumerate(before):
        ref.set_state(i, V, t)
    d2 = ref.step(2)
    assert np.array_equal(d1, d2)
    for i in range(len(items)):
        for a, b in zip(ctx.get_state(i)[0], ref.get_state(i)[0]):
            assert np.array_equal(a, b)
    ctx.close()
    ref.close()


@pytest.mark.parametrize("d,form,si", [(1, "dc", False), (2, "dc", False), (3, "dc", False), (1, "nodc", False),
                                       (2, "dc", True), (3, "dc", True)])
def test_limiter_activity_matches_oracle(d, form, si):
    """af_limiter_activity counts, in one FE stage with the CFL step, the face
    fluxes and cell potentials whose limiting parameter is below 1, once
    each.  The oracle evaluates every face from both its cells and every
    potential from three cells (periodic grid), so its count of theta < 1 is
    2 F + 3 P.  The call leaves state and variant as they were."""
    rng = np.random.default_rng(700 + 10 * d + (form == "nodc") + 3 * si)
    n = {1: 61, 2: 19, 3: 9}[d]
    spec = small_spec(d, n, ("quad", 0.5, 0.0), ("power", 0.05, 2.0), limiter=True, si=si, precision=64)
    spec["diffusion_form"] = form
    U = state_for(spec, rng)
    s, U = prepare(spec, U, 64)
    ctx = af.Context(s)
    v0 = ctx.variant()
    ctx.set_state(0, U)
    c = ctx.limiter_activity(0)
    note("limiter activity d=%d %s si=%d: %s" % (d, form, si, c))
    assert ctx.variant() == v0
    V, t = ctx.get_state(0)
    assert t == 0.0 and all(np.array_equal(a, b) for a, b in zip(V, U))
    P = oracle.problem(s)
    dt = oracle.dt_cfl(P, U, s["cfl"])
    _, dg = oracle.fe(P, U, dt)
    N = int(np.prod(s["n"][:d]))
    assert c["faces"] == d * N and c["potentials"] == (0 if form == "nodc" else d * N)
    assert dg["n_theta"] == 2 * c["faces"] + 3 * c["potentials"]
    lim = 2 * c["faces_limited"] + 3 * c["potentials_limited"]
    assert c["faces_limited"] > 0
    assert abs(lim - dg["n_theta_lt1"]) <= 2, (lim, dg["n_theta_lt1"])
    # stepping on is unaffected by the diagnostic
    d1 = ctx.step(2)
    ref = af.Context(s)
    ref.set_state(0, U)
    d2 = ref.step(2)
    assert np.array_equal(d1, d2)
    assert all(np.array_equal(a, b) for a, b in zip(ctx.get_state(0)[0], ref.get_state(0)[0]))
    ctx.close()
    ref.close()


def test_limiter_activity_fp32_and_validation():
    """FP32 contexts count too (within a few borderline decisions of the
    FP64 count on the same rounded data); without the limiter the call is
    unsupported, before af_set_state out of order."""
    rng = np.random.default_rng(77)
    spec = small_spec(2, 23, ("bl_grav", 0.0, 5.0), ("ramp2", 0.1, 0.3), limiter=True, precision=32)
    U = state_for(spec, rng)
    s32, U32 = prepare(spec, U, 32)
    ctx = af.Context(s32)
    with pytest.raises(af.AFError) as e:
        ctx.limiter_activity(0)
    assert e.value.status == af.AF_ERR_STATE
    ctx.set_state(0, U32)
    c32 = ctx.limiter_activity(0)
    ctx.close()
    s64 = dict(s32, precision=64)
    ctx = af.Context(s64)
    ctx.set_state(0, U32)
    c64 = ctx.limiter_activity(0)
    ctx.close()
    note("limiter activity fp32 %s fp64 %s" % (c32, c64))
    assert c32["faces"] == c64["faces"] and c32["potentials"] == c64["potentials"]
    assert 0 < c64["faces_limited"] < c64["faces"]
    tot = c64["faces"] + c64["potentials"]
    assert abs(c32["faces_limited"] - c64["faces_limited"]) + abs(c32["potentials_limited"] - c64["potentials_limited"]) <= 0.01 * tot
    ctx = af.Context(dict(s64, limiter=False))
    ctx.set_state(0, U32)
    with pytest.raises(af.AFError) as e:
        ctx.limiter_activity(0)
    assert e.value.status == af.AF_ERR_UNSUPPORTED
    ctx.close()


def test_table3_unlimited_extrema_on_the_gpu():
    """The HIP path itself reproduces Example 6.2's printed unlimited
    extrema (Table 3) to their four digits: FP64, SSP-RK(5,4) to T = 1 at
    CFL 0.05 from Simpson-rule initial averages, N = 20 ... 320."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mpp_tables.json")))["table3"]
    u0 = lambda s: 1.0 + np.sin(2 * np.pi * s) ** 4
    for i, N in enumerate(g["N"]):
        spec = dict(W.sin4_advection(N)[0], limiter=False, cfl=0.05)
        xc, xr = (np.arange(N) + 0.5) / N, (np.arange(N) + 1.0) / N
        U = [(u0(xr - 1.0 / N) + 4 * u0(xc) + u0(xr)) / 6, u0(xr)]
        ctx = af.Context(spec, integrator="ssprk54")
        ctx.set_state(0, U)
        ctx.step(20 * N + 20, t_end=1.0)
        V, t = ctx.get_state(0)
        ctx.close()
        got = (min(v.min() for v in V) - 1.0, max(v.max() for v in V) - 2.0)
        note("table 3 N=%d t=%.15f got %s printed %s" % (N, t, got, g["without"][i]))
        assert abs(t - 1.0) < 1e-12
        for a, b in zip(got, g["without"][i]):
            assert abs(a - b) <= 5e-4 * abs(b), (N, got, g["without"][i])


def test_table4_unlimited_minimum_on_the_gpu():
    """The 2D path reproduces Example 6.3's printed unlimited minimum at T
    (Table 4, m = 2, N = 80, t from 1 to 2, SSP-RK(5,4) at CFL 0.1, Simpson
    initial averages) to its four digits, in FP64."""
    import json
    import os
    t4 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mpp_tables.json")))["table4"]
    m, d, n, L = 2, 2, 80, 8.0
    spec, U = W.barenblatt(d, m, n=n, t=1.0, sub=2, limiter=False)
    dx = 2 * L / n
    xc = -L + (np.arange(n) + 0.5) * dx
    pts = lambda xo, yo: W.barenblatt_value(m, d, np.add.outer((xc + yo) ** 2, (xc + xo) ** 2), 1.0).reshape(-1)
    w = {-1: 1.0, 0: 4.0, 1: 1.0}
    U = [sum(w[a] * w[b] * pts(a * dx / 2, b * dx / 2) for a in (-1, 0, 1) for b in (-1, 0, 1)) / 36] + U[1:]
    ctx = af.Context(dict(spec, cfl=0.1), integrator="ssprk54")
    ctx.set_state(0, U, 1.0)
    ctx.step(2000, t_end=2.0)
    V, t = ctx.get_state(0)
    name = ctx.variant_name(ctx.variant())
    ctx.close()
    got = min(v.min() for v in V)
    ref = t4["2d"]["without"][t4["m"].index(m)]
    note("table 4 m=%d on %s: t=%.15f min %.6e printed %.4e" % (m, name, t, got, ref))
    assert abs(t - 2.0) < 1e-12
    assert abs(got - ref) <= 5e-4 * abs(ref), (got, ref)


def test_graph_equals_eager_and_checkpoint_resume():
    spec, U = W.config2(n=64)
    ctx = af.Context(spec)
    ctx.set_state(0, U)
    ctx.step(6)                     # one graph launch
    A, ta = ctx.get_state(0)
    ctx.set_state(0, U)
    for _ in range(3):
        ctx.step(1)                 # eager
    mid, tm = ctx.get_state(0)
    ctx.set_state(0, mid, tm)       # checkpoint / resume
    for _ in range(3):
        ctx.step(1)
    B, tb = ctx.get_state(0)
    ctx.close()
    assert ta == tb
    for a, b in zip(A, B):
        assert np.array_equal(a, b)


def test_batched_instances_match_oracle():
    """Uneven batched instances (config-4 construction, small sizes) in one
    context: each matches its own oracle run with its own CFL steps."""
    items = W.config4(n_inst=6, sizes=(16, 24, 40))
    specs = [s for s, _ in items]
    ctx = af.Context(specs)
    for i, (s, U) in enumerate(items):
        ctx.set_state(i, U)
    dts = []
    for _ in range(5):
        dts.append(ctx.step(1))
    for i, (s, U) in enumerate(items):
        V, _ = ctx.get_state(i)
        P = oracle.problem(s)
        Uo, _, odts = oracle.run(P, U, dts=[d[i] for d in dts])
        dto = oracle.dt_cfl(P, U, s["cfl"])
        assert abs(dts[0][i] - dto) <= 1e-6 * dto
        check(V, Uo, 32, 3 * len(dts), "batched instance %d" % i)
    ctx.close()


def _end_time_batch(kind):
    """Instances of different sizes (so different CFL steps) for one context."""
    if kind == "2d":  # batched porous-medium / Burgers instances, FP32
        return W.config4(n_inst=3, sizes=(16, 24, 40))
    if kind == "3d":  # degenerate 3D with blending, FP32
        return [W.config5(n=12), W.config5(n=20)]
    # App. A batch, FP64
    return W.config_nodc(n_inst=2, n=64) + W.config_nodc(seed=7, n_inst=1, n=160)


@pytest.mark.parametrize("kind,tile", [("2d", "2d-own-32x16"), ("2d", "generic-32x8"), ("3d", "3d-march-16x8x32"),
                                       ("3d", "generic-8x8x8"), ("1d", "generic-512")])
def test_instances_reaching_the_end_time_at_different_steps(kind, tile):
    """Stepping to a common end time, the instances of one context with
    larger CFL steps finish first; from then on the finalize gives them a
    zero step and every stage must leave them unchanged while the others go
    on.  Each instance against the oracle replaying its own nonzero steps,
    the time reached and the number of steps it took."""
    items = _end_time_batch(kind)
    specs = [s for s, _ in items]
    prec = specs[0]["precision"]
    dt0 = [oracle.dt_cfl(oracle.problem(s), U, s["cfl"]) for s, U in items]
    T = 3.5 * max(dt0)
    ctx = af.Context(specs)
    ctx.set_variant([ctx.variant_name(v) for v in range(ctx.num_variants())].index(tile))
    for i, (_, U) in enumerate(items):
        ctx.set_state(i, U)
    dts = []
    while len(dts) < 200:
        d = ctx.step(1, t_end=T)
        if not np.any(d > 0):
            break
        dts.append(d)
    dts = np.array(dts)
    taken = (dts > 0).sum(axis=0)
    note("end time %s %s: steps per instance %s" % (kind, tile, taken.tolist()))
    # some instance finished at least two steps before the last one
    assert taken.max() - taken.min() >= 2
    for i, (s, U) in enumerate(items):
        V, t = ctx.get_state(i)
        assert ctx.norms(i)["steps"] == taken[i]
        assert abs(t - T) <= 1e-12 * T
        # zero steps only after the instance's last step
        assert np.all(dts[: taken[i], i] > 0) and np.all(dts[taken[i]:, i] == 0)
        Uo, to, _ = oracle.run(oracle.problem(s), U, dts=list(dts[: taken[i], i]))
        assert abs(to - T) <= 1e-12 * T
        check(V, Uo, prec, 3 * int(taken[i]), "%s instance %d (%d steps)" % (kind, i, taken[i]))
    ctx.close()


def test_conservation_and_bounds_long_run():
    spec, U = W.config2(n=96)
    ctx = af.Context(spec)
    ctx.set_state(0, U)
    m0 = ctx.norms(0)["mass"]
    ctx.step(100)
    nrm = ctx.norms(0)
    ctx.close()
    assert abs(nrm["mass"] - m0) <= 1e-13 * abs(m0)
    assert nrm["min_avg"] >= spec["umin"] and nrm["max_avg"] <= spec["umax"]
    assert nrm["min_pv"] >= spec["umin"] and nrm["max_pv"] <= spec["umax"]
    assert nrm["max_clamp"] <= 4 * np.spacing(1.0)


@pytest.mark.parametrize("name,integ", [("c2", "ssprk3"), ("c4", "ssprk3"), ("c5", "ssprk3"), ("c1", "ssprk3"),
                                        ("c2", "euler"), ("c4", "ssprk54"), ("ek", "ssprk3"), ("ek", "ssprk54"),
                                        ("c2open", "ssprk3")])
def test_cfl_from_last_stage_minmax_equals_wave_speed_pass(name, integ):
    """For convex |f'| the last stage of a step reduces the min / max average
    and the next step's CFL step comes from them; it must equal, to the bit,
    the step the separate FP64 wave-speed pass computes on the same state."""
    if name == "c4":
        items = W.config4(n_inst=4, sizes=(32, 48))
    elif name == "ek":              # Dirichlet ends, 1D: ghost values in the min / max
        items = W.config_ek(n_inst=3, n=48)
    elif name == "c2open":          # Dirichlet and outflow ends, 2D (own-items kernel)
        spec, U = W.config2(n=40)
        g0, g1 = spec["umin"], 0.5 * (spec["umin"] + spec["umax"])
        items = [(dict(spec, bcs=[(("dirichlet", g1), ("dirichlet", g0)), ("outflow", "outflow")]), U)]
    else:
        items = [_steps_case(name)]
    specs = [s for s, _ in items]
    a = af.Context(specs, integrator=integ)
    for i, (_, U) in enumerate(items):
        a.set_state(i, U)
    a.step(1)                      # wave-speed pass
    a.step(3)                      # min / max of the last stage (graph)
    mids = [a.get_state(i) for i in range(len(items))]
    used_keys = a.step(1)
    b = af.Context(specs, integrator=integ)
    for i, (V, t) in enumerate(mids):
        b.set_state(i, V, t)
    used_ws = b.step(1)            # fresh state: wave-speed pass
    note("cfl %s %s keys=%s ws=%s" % (name, integ, used_keys[:2], used_ws[:2]))
    assert np.array_equal(np.asarray(used_keys), np.asarray(used_ws))
    for i in range(len(items)):
        A, ta = a.get_state(i)
        B, tb = b.get_state(i)
        assert ta == tb
        for x, y in zip(A, B):
            assert np.array_equal(x, y)
    a.close()
    b.close()


def test_fp32_bounds_without_an_exact_float_hold_exactly():
    """Bounds [0.7, 1.1] have no exact FP32 values and round outwards to
    nearest; the FP32 kernels clamp and limit against the nearest floats
    inside them, so every DoF stays inside the FP64 bounds the context was
    given, and the run still matches the oracle."""
    spec, U = W.config4(n_inst=1, sizes=(48,))[0]
    lo, hi = 0.7, 1.1
    flo = np.nextafter(np.float32(lo), np.float32(1)) if float(np.float32(lo)) < lo else np.float32(lo)
    fhi = np.nextafter(np.float32(hi), np.float32(-1)) if float(np.float32(hi)) > hi else np.float32(hi)
    assert float(np.float32(lo)) < lo and float(np.float32(hi)) > hi   # both round outwards
    U = [np.clip(np.float32(lo + (hi - lo) * u), flo, fhi).astype(np.float64) for u in U]
    s = dict(spec, umin=lo, umax=hi, precision=32)
    P = oracle.problem(s)
    Uo, t, dts = oracle.run(P, U, nsteps=20, cfl=s["cfl"])
    V, tg, used, nrm = gpu_run(s, U, dts=dts)
    note("fp32 bounds: min %.10g max %.10g" % (min(v.min() for v in V), max(v.max() for v in V)))
    assert min(v.min() for v in V) >= lo and max(v.max() for v in V) <= hi
    assert nrm["min_avg"] >= lo and nrm["max_avg"] <= hi and nrm["min_pv"] >= lo and nrm["max_pv"] <= hi
    check(V, Uo, 32, 3 * len(dts), "fp32 bounds")


def test_copy_rate_reference():
    """af_copy_rate, the attainable-bandwidth reference of the roofline: a
    plausible HBM rate (above 1 TB/s, not above the 8 TB/s peak by more than
    timing noise) for a 1 GiB streaming copy."""
    r = af.copy_rate(1 << 30, 10)
    note("copy rate %.1f GB/s" % r)
    assert 1000.0 < r < 8400.0
