"""GPU parity at the full sizes of the benchmarked workloads, in the launch
configuration the benchmark times: one context per workload with all its
instances batched, built by the benchmark's own workload and context code,
default tile variant.

* One forward-Euler stage with the CFL step is compared, element by element,
  with the FP64 oracle on sampled cells that the oracle computes one by one:
  every combination of the first and last cells of the first two tiles and of
  the last cells of each axis (tile edges, corners, ragged tails), plus random
  cells and random cells whose average lies strictly inside the bounds.  Bar: relative l1 over the sample per DoF kind within the FP64 /
  FP32 tolerance, every value inside [umin, umax].
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
from gpu_common import TOL

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
    name, items = bench.workload(wl)
    prec = items[0][0]["precision"]
    d = items[0][0]["dim"]
    ctx = bench.make_ctx(items, integrator="euler")
    vname = ctx.variant_name(ctx.variant())
    tile = tile_of(vname, d)
    note("full-size fe %s (%d instances, variant %s)" % (name, len(items), vname))
    dts = ctx.step(1)
    rng = np.random.default_rng(2510 + len(wl))
    nrand = 48 if len(items) == 1 else 6
    num = np.zeros(2 ** d)
    den = np.zeros(2 ** d)
    ncmp = 0
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
    ctx.close()
    err = float(np.max(num / den))
    note("  %d sampled cells, relative l1 %.3e" % (ncmp, err))
    assert err <= TOL[prec], err


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
