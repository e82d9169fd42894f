"""GPU parity at the full sizes of the benchmarked workloads, in the launch
configuration the benchmark times: one context per workload with all its
instances batched, built by the benchmark's own workload and context code,
default tile variant.

* One forward-Euler stage with the CFL step is compared, element by element,
  with the FP64 oracle on sampled cells that the oracle computes one by one:
  every combination of the first and last cells of the first two tiles and of
  the last cells of each axis (tile edges, corners, ragged tails), plus random
  cells and random cells whose average lies strictly inside the bounds.
  Bar: relative l1 over the sample per DoF kind within the FP64 / FP32
  tolerance, every sampled value within the element-wise bound of one stage,
  every value inside [umin, umax].
* One SSP-RK3 step is checked for what holds at any size: total mass to
  round-off (FP64 reduction; periodic instances, where no flux crosses an
  end), averages and point values inside [umin, umax] exactly, nothing
  clamped by the safeguard beyond rounding.
"""
import itertools
import re
import sys

import numpy as np
import pytest

import bench
import oracle
from paper_2510_11527_amd import af
from gpu_common import TOL, abs_bound, check

pytestmark = pytest.mark.gpu

WORKLOADS = ["c2", "c3", "c3f32", "c4", "c5", "nodc", "ek"]


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tile_of(name, d):
    """Tile extents from a variant name such as generic-512, 2d-own-32x16 or
    generic-8x8x4."""
    t = [int(v) for v in re.findall(r"\d+", name.split("-")[-1])]
    return (t + [1, 1])[:d]


def has_open_end(spec):
    return any((e if isinstance(e, str) else e[0]) != "periodic" for ax in oracle.boundary_ends(spec) for e in ax)


def sample_cells(spec, U, tile, rng, nrand):
    d = spec["dim"]
    n = spec["n"][:d]
    axes = []
    for l in range(d):
        t, nl = tile[l], n[l]
        axes.append(sorted({0, min(t - 1, nl - 1), min(t, nl - 1), min(2 * t - 1, nl - 1), nl - 2, nl - 1}))
    cells = set()
    for c in itertools.product(*axes):
        idx, stride = 0, 1
        for l in range(d):
            idx += c[l] * stride
            stride *= n[l]
        cells.add(idx)
    total = int(np.prod(n))
    cells.update(int(v) for v in rng.integers(0, total, size=nrand))
    # cells where the state varies (fronts of piecewise-constant data)
    active = np.flatnonzero((U[0] > spec["umin"]) & (U[0] < spec["umax"]))
    if active.size:
        cells.update(int(v) for v in rng.choice(active, size=min(nrand, active.size), replace=False))
    return np.array(sorted(cells), dtype=np.int64)


@pytest.mark.parametrize("wl", WORKLOADS)
def test_full_size_forward_euler_stage_matches_oracle_on_sampled_cells(wl):
    fe_sampled(wl)


@pytest.mark.parametrize("tile", ["3d-march-8x8x32", "3d-march-16x8x256"])
def test_full_size_3d_stage_on_the_autotuned_tiles(tile):
    """The 3D workload at full size on the marching tiles the autotuner
    chooses between (bench.py times whichever it picks), sampled cells
    against the oracle."""
    fe_sampled("c5", tile)


def fe_sampled(wl, tile_name=None):
    name, items = bench.workload(wl)
    prec = items[0][0]["precision"]
    d = items[0][0]["dim"]
    variant = None
    if tile_name is not None:
        probe = af.Context(items[0][0])
        variant = [probe.variant_name(v) for v in range(probe.num_variants())].index(tile_name)
        probe.close()
    ctx = bench.make_ctx(items, integrator="euler", variant=variant)
    vname = ctx.variant_name(ctx.variant())
    tile = tile_of(vname, d)
    note("full-size fe %s (%d instances, variant %s)" % (name, len(items), vname))
    dts = ctx.step(1)
    rng = np.random.default_rng(2510 + len(wl))
    nrand = 48 if len(items) == 1 else 6
    num = np.zeros(2 ** d)
    den = np.zeros(2 ** d)
    ncmp = 0
    worst = 0.0   # largest |gpu - oracle| / abs_bound over the sample
    for i, (s, U) in enumerate(items):
        V, _ = ctx.get_state(i)
        cells = sample_cells(s, U, tile, rng, nrand)
        Vo, _ = oracle.fe_cells(oracle.problem(s), U, dts[i], cells)
        G = np.stack([np.asarray(V[z])[cells] for z in range(2 ** d)], axis=1)
        assert np.all(np.isfinite(G))
        assert G.min() >= s["umin"] and G.max() <= s["umax"], (i, G.min(), G.max())
        num += np.abs(G - Vo).sum(axis=0)
        den += np.abs(Vo).sum(axis=0)
        ncmp += cells.size
        worst = max(worst, float(np.abs(G - Vo).max()) / abs_bound(prec, float(np.abs(Vo).max()), 1))
    ctx.close()
    err = float(np.max(num / den))
    note("  %d sampled cells, relative l1 %.3e, max |gpu - oracle| at %.3f of the element-wise bound" % (ncmp, err, worst))
    assert err <= TOL[prec], err
    assert worst <= 1.0, worst


@pytest.mark.parametrize("wl", WORKLOADS)
def test_full_size_step_conserves_mass_and_bounds(wl):
    name, items = bench.workload(wl)
    prec = items[0][0]["precision"]
    ctx = bench.make_ctx(items)
    note("full-size step %s (%d instances, variant %s)" % (name, len(items), ctx.variant_name(ctx.variant())))
    m0 = [ctx.norms(i)["mass"] for i in range(len(items))]
    ctx.step(1)
    # the face fluxes telescope, so the mass moves only by the rounding of
    # the stored averages (a few units in the last place of the storage
    # precision per cell, in random sign: sqrt(N) growth) and by the rounding
    # of the FP64 reduction itself (about eps |mass| per level of its tree)
    eps = float(np.finfo(np.float32 if prec == 32 else np.float64).eps)
    for i, (s, _) in enumerate(items):
        nrm = ctx.norms(i)
        d = s["dim"]
        ncell = int(np.prod(s["n"][:d]))
        vol = float(np.prod([(s["hi"][l] - s["lo"][l]) / s["n"][l] for l in range(d)]))
        umag = max(abs(s["umin"]), abs(s["umax"]))
        tol = 16 * eps * np.sqrt(ncell) * umag * vol + 64 * np.finfo(np.float64).eps * abs(m0[i])
        if not has_open_end(s):
            assert abs(nrm["mass"] - m0[i]) <= tol, (i, nrm["mass"], m0[i], tol)
        assert nrm["min_avg"] >= s["umin"] and nrm["max_avg"] <= s["umax"], i
        assert nrm["min_pv"] >= s["umin"] and nrm["max_pv"] <= s["umax"], i
        assert nrm["max_clamp"] <= 4 * eps * max(abs(s["umin"]), abs(s["umax"]), 1.0), (i, nrm["max_clamp"])
    ctx.close()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_minimum_grid_matches_oracle(d):
    """Four cells per axis, the smallest grid accepted: every halo (three cells
    with the smoothness indicators) wraps around the periodic instance, in a
    batch next to a larger instance.  One limited, blended FE stage in FP64
    and FP32 against the oracle over all DoFs."""
    rng = np.random.default_rng(400 + d)
    for prec in (64, 32):
        items = []
        for n in (4, 11):
            spec = dict(name="min", dim=d, n=[n] * d, lo=[0.0] * d, hi=[1.0] * d, flux=[("quad", 0.5, 0.0)] * d,
                        diff=("power", 0.05, 2.0), umin=0.0, umax=1.0, limiter=True, si=True, si_gamma=1.0,
                        precision=prec, cfl=0.05)
            U = [rng.uniform(0, 1, size=n ** d) for _ in range(2 ** d)]
            if prec == 32:
                U = [u.astype(np.float32).astype(np.float64) for u in U]
            items.append((spec, U))
        ctx = bench.make_ctx(items, integrator="euler")
        note("minimum grid d=%d prec=%d variant %s" % (d, prec, ctx.variant_name(ctx.variant())))
        dts = ctx.step(1)
        for i, (s, U) in enumerate(items):
            V, _ = ctx.get_state(i)
            Vo, _ = oracle.fe(oracle.problem(s), U, dts[i])
            check(V, Vo, prec, 1, "minimum grid d=%d instance %d" % (d, i))
            assert min(v.min() for v in V) >= 0.0 and max(v.max() for v in V) <= 1.0
        ctx.close()


def test_instance_beyond_2_pow_31_dofs_matches_oracle():
    """One 2D FP64 instance of 23200^2 cells: its DoF block holds more than
    2^31 values (17 GB), past every 32-bit offset.  The own-items kernel,
    which addresses a block with 32-bit byte offsets, is not selected; the
    default (table) kernel and the generic kernel, both with 64-bit offsets,
    each run one limited FE stage that matches the oracle on sampled cells,
    among them the last cells, whose offsets exceed 2^31."""
    n = 23200
    ncell = n * n
    assert 4 * ncell > 2 ** 31
    rng = np.random.default_rng(2311)
    spec = dict(name="big", dim=2, n=[n, n], lo=[0.0, 0.0], hi=[1.0, 1.0], flux=[("quad", 0.5, 0.0)] * 2,
                diff=("power", 0.05, 2.0), umin=0.0, umax=1.0, limiter=True, si=False, si_gamma=1.0,
                precision=64, cfl=0.075)
    U = [rng.random(ncell) for _ in range(4)]
    ctx = bench.make_ctx([(spec, U)], integrator="euler")
    names = [ctx.variant_name(v) for v in range(ctx.num_variants())]
    generic = next(v for v, nm in enumerate(names) if nm.startswith("generic"))
    dt = None
    for v in (ctx.variant(), generic):
        ctx.set_variant(v)
        ctx.set_state(0, U)
        note("instance of %d cells, variant %s" % (ncell, names[v]))
        assert "own" not in names[v]
        if dt is None:
            dt = ctx.step(1)[0]
        else:
            ctx.step(1, dt=dt)
        V, _ = ctx.get_state(0)
        cells = sample_cells(spec, U, tile_of(names[v], 2), rng, 64)
        cells = np.unique(np.concatenate([cells, np.arange(ncell - 40, ncell), ncell - n + np.arange(40)]))
        Vo, _ = oracle.fe_cells(oracle.problem(spec), U, dt, cells)
        G = np.stack([V[z][cells] for z in range(4)], axis=1)
        del V
        err = float(np.max(np.abs(G - Vo).sum(axis=0) / np.abs(Vo).sum(axis=0)))
        ma = float(np.abs(G - Vo).max())
        note("  %d sampled cells, relative l1 %.3e, max_abs %.3e" % (cells.size, err, ma))
        assert err <= TOL[64], err
        assert ma <= abs_bound(64, float(np.abs(Vo).max()), 1), ma
        assert G.min() >= 0.0 and G.max() <= 1.0
    ctx.close()
