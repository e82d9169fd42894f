"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on identical inputs and compare."""
import numpy as np

import oracle
from paper_2510_11527_amd import af
from paper_2510_11527_amd import workloads as W

TOL = {64: 1e-12, 32: 1e-5}   # relative l1 over all DoFs, vs the FP64 oracle


def rel_l1(a, b):
    """max over DoF kinds of ||a - b||_1 / ||b||_1."""
    out = 0.0
    for x, y in zip(a, b):
        den = np.abs(y).sum()
        num = np.abs(np.asarray(x) - np.asarray(y)).sum()
        out = max(out, num / den if den > 0 else num)
    return out


def prepare(spec, dofs, precision):
    """Inputs both sides see: rounded to the GPU storage precision, with the
    bounds of the rounded data."""
    s = dict(spec)
    s["precision"] = precision
    U = W.round_to(dofs, precision)
    if "umin" not in spec or precision == 32:
        s["umin"], s["umax"] = W.bounds_of(U, precision)
    return s, U


def gpu_run(spec, U, dts=None, nsteps=None, integrator="ssprk3", variant=None, t_end=0.0):
    ctx = af.Context(spec, integrator=integrator)
    if variant is not None:
        ctx.set_variant(variant)
    ctx.set_state(0, U)
    used = []
    if dts is not None:
        for dt in dts:
            used.append(ctx.step(1, dt=dt)[0])
    else:
        for _ in range(nsteps):
            used.append(ctx.step(1, t_end=t_end)[0])
    V, t = ctx.get_state(0)
    nrm = ctx.norms(0)
    ctx.close()
    return V, t, used, nrm


def oracle_fe(spec, U, dt):
    P = oracle.problem(spec)
    V, dg = oracle.fe(P, U, dt)
    return V, dg


def random_state(d, n, rng, lo=0.0, hi=1.0, smooth=False):
    N = n ** d
    if smooth:
        spec = dict(dim=d, n=[n] * d, lo=[0.0] * d, hi=[1.0] * d)
        modes = [(tuple(int(v) for v in rng.integers(-2, 3, size=d)), rng.uniform(0.2, 1), rng.uniform(0, 6.28))
                 for _ in range(3)]
        modes = [m for m in modes if any(m[0])] or [((1,) * d, 1.0, 0.3)]
        g = W.rescale01(W.fourier_dofs(spec, modes))
        return [lo + (hi - lo) * x for x in g]
    U = [rng.uniform(lo, hi, size=N) for _ in range(2 ** d)]
    U[0] = np.where(rng.uniform(size=N) < 0.6, U[0], rng.choice([lo, hi], size=N))
    return U
