"""Full-grid parity and the FP64 reductions at the benchmark sizes.

* Ten SSP-RK3 steps of the 2D degenerate Burgers workload (512^2, FP64) and
  of the 2D Buckley-Leverett workload (1024^2, FP64), in the benchmark's
  launch configuration, against the oracle on every DoF, the oracle's CFL
  steps prescribed to both sides.
* af_norms after those steps against independent sums of the state read
  back (math.fsum, numpy min/max) and the mass against the oracle's state:
  the FP64 reductions of the paper's conservation and bounds (mass conserved
  to round-off, Props 5.1/5.2; bounds of Def. 5.1).
* The same norms checks on sampled instances of the batched FP32 workload
  after ten CFL steps, each instance against its own oracle run.
"""
import math
import sys

import numpy as np
import pytest

import bench
import oracle
from gpu_common import check

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def independent_norms(spec, V):
    d = spec["dim"]
    vol = float(np.prod([(spec["hi"][l] - spec["lo"][l]) / spec["n"][l] for l in range(d)]))
    a = np.asarray(V[0], dtype=np.float64)
    pv = np.concatenate([np.asarray(v, dtype=np.float64) for v in V[1:]])
    return {"mass": math.fsum(a) * vol, "l1_avg": math.fsum(np.abs(a)) * vol,
            "l2_avg": math.sqrt(math.fsum(a * a) * vol), "linf_avg": float(np.abs(a).max()),
            "min_avg": float(a.min()), "max_avg": float(a.max()), "min_pv": float(pv.min()),
            "max_pv": float(pv.max()), "abs_mass": math.fsum(np.abs(a)) * vol}


def check_norms(nrm, ref, what):
    """Sums within 4e-16 of the sum of magnitudes (compensated reduction;
    about one unit in the last place of the result), extrema exact."""
    note("  norms %s: mass %.17g vs %.17g" % (what, nrm["mass"], ref["mass"]))
    assert abs(nrm["mass"] - ref["mass"]) <= 4e-16 * ref["abs_mass"], (what, nrm["mass"], ref["mass"])
    assert abs(nrm["l1_avg"] - ref["l1_avg"]) <= 4e-16 * ref["l1_avg"], what
    assert abs(nrm["l2_avg"] - ref["l2_avg"]) <= 4e-16 * ref["l2_avg"], what
    for k in ("linf_avg", "min_avg", "max_avg", "min_pv", "max_pv"):
        assert nrm[k] == ref[k], (what, k, nrm[k], ref[k])
    assert nrm["nonfinite"] == 0


@pytest.mark.parametrize("wl", ["c2", "c3"])
def test_full_grid_ten_steps_match_oracle_and_norms(wl):
    name, items = bench.workload(wl)
    (spec, U), = items
    P = oracle.problem(spec)
    note("full grid %s: oracle, 10 steps" % name)
    Uo, t, dts = oracle.run(P, U, nsteps=10, cfl=spec["cfl"])
    ctx = bench.make_ctx(items)
    note("full grid %s: GPU, variant %s" % (name, ctx.variant_name(ctx.variant())))
    for dt in dts:
        ctx.step(1, dt=dt)
    V, tg = ctx.get_state(0)
    nrm = ctx.norms(0)
    ctx.close()
    check(V, Uo, 64, 30, "full grid " + name)
    assert abs(tg - t) <= 1e-15 * t
    ref = independent_norms(spec, V)
    check_norms(nrm, ref, name)
    # the mass of the oracle's state: both conserve it to round-off
    ro = independent_norms(spec, Uo)
    assert abs(nrm["mass"] - ro["mass"]) <= 1e-15 * ro["abs_mass"], (nrm["mass"], ro["mass"])
    m0 = independent_norms(spec, U)["mass"]
    note("  mass drift over 10 steps: gpu %.3e, oracle %.3e (relative)" % (
        (nrm["mass"] - m0) / abs(m0), (ro["mass"] - m0) / abs(m0)))
    assert abs(nrm["mass"] - m0) <= 1e-14 * ro["abs_mass"]


def test_batched_fp32_norms_and_sampled_instances_match_oracle():
    """The batched FP32 workload (256 instances) after ten CFL steps: for
    four sampled instances, one of every grid size, af_norms against
    independent sums of the FP32 state read back (FP64 reductions), and the
    state against the oracle run with the same steps."""
    name, items = bench.workload("c4")
    ctx = bench.make_ctx(items)
    note("batched %s: variant %s" % (name, ctx.variant_name(ctx.variant())))
    dts = [ctx.step(1) for _ in range(10)]
    picks = []
    for size in (64, 128, 256, 512):
        picks.append(next(i for i, (s, _) in enumerate(items) if s["n"][0] == size))
    for i in picks:
        s, U = items[i]
        V, _ = ctx.get_state(i)
        nrm = ctx.norms(i)
        check_norms(nrm, independent_norms(s, V), "instance %d (%d^2)" % (i, s["n"][0]))
        Uo, _, _ = oracle.run(oracle.problem(s), U, dts=[d[i] for d in dts])
        check(V, Uo, 32, 30, "instance %d" % i)
        ro = independent_norms(s, Uo)
        # FP32 storage: each stored average rounds by half an ulp
        assert abs(nrm["mass"] - ro["mass"]) <= 30 * 2.0 ** -24 * ro["abs_mass"], (nrm["mass"], ro["mass"])
    ctx.close()
