"""af_norms_noalloc, the entry point for callers that cannot allocate: the
norms of a state held in the caller's device memory, reduced with the
library's static scratch array, against af_norms of a context holding the
same state (same kernels and order: identical results) and against
independent sums on the host.  Two calls in a row, the second on a smaller
grid, so that the shared scratch holds the first call's partials when the
second starts.

The caller's device memory and stream come from the HIP runtime the library
itself is linked against (through ctypes), as a caller of the C ABI would
hold them."""
import ctypes
import math
import sys

import numpy as np
import pytest

from paper_2510_11527_amd import af
from paper_2510_11527_amd import workloads as W
from hip_mem import DeviceBlock, hip

pytestmark = pytest.mark.gpu

FIELDS = ["mass", "min_avg", "max_avg", "min_pv", "max_pv", "l1_avg", "l2_avg", "linf_avg", "nonfinite"]


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cases():
    # FP32 2D batched-workload instances (256^2 then 40^2) and FP64 3D
    # (24^3 then 6^3)
    big = W.config4(n_inst=1, sizes=(256,))[0]
    small = W.config4(n_inst=1, sizes=(40,), seed=77)[0]
    yield "fp32 2d", [(dict(s, precision=32), W.round_to(U, 32)) for s, U in (big, small)]
    s3, U3 = W.config5(n=24)
    t3, V3 = W.config5(n=6, seed=78)
    yield "fp64 3d", [(dict(s3, precision=64, si=False), U3), (dict(t3, precision=64, si=False), V3)]


@pytest.mark.parametrize("case", ["fp32 2d", "fp64 3d"])
def test_norms_noalloc_matches_af_norms_on_two_calls(case):
    pairs = dict(cases())[case]
    stream = ctypes.c_void_p()
    assert hip().hipStreamCreate(ctypes.byref(stream)) == 0
    for k, (spec, U) in enumerate(pairs):
        d, prec = spec["dim"], spec["precision"]
        note("norms_noalloc %s call %d: n=%s" % (case, k, spec["n"][:d]))
        ctx = af.Context(spec)
        ctx.set_state(0, U)
        ref = ctx.norms(0)
        ctx.close()
        B = DeviceBlock(U, prec, pad=37 + 64 * k)
        got = af.norms_noalloc(d, prec, spec["n"][:d], spec["lo"][:d], spec["hi"][:d], B.ptr.value, B.kstride,
                               stream.value)
        B.free()
        for f in FIELDS:
            assert got[f] == ref[f], (case, k, f, got[f], ref[f])
        assert got["t"] == 0.0 and got["steps"] == 0 and got["max_clamp"] == 0.0
        # independent sums of the same (stored) values
        vol = float(np.prod([(spec["hi"][l] - spec["lo"][l]) / spec["n"][l] for l in range(d)]))
        avg = np.asarray(U[0], dtype=np.float64)
        assert abs(got["mass"] - math.fsum(avg) * vol) <= 1e-15 * math.fsum(np.abs(avg)) * vol
        assert abs(got["l1_avg"] - math.fsum(np.abs(avg)) * vol) <= 1e-15 * got["l1_avg"]
        assert abs(got["l2_avg"] - math.sqrt(math.fsum(avg * avg) * vol)) <= 1e-15 * got["l2_avg"]
        assert got["min_avg"] == avg.min() and got["max_avg"] == avg.max() and got["linf_avg"] == np.abs(avg).max()
        pv = np.concatenate([np.asarray(u, dtype=np.float64) for u in U[1:]])
        assert got["min_pv"] == pv.min() and got["max_pv"] == pv.max() and got["nonfinite"] == 0
    assert hip().hipStreamDestroy(stream) == 0


def test_norms_noalloc_rejects_bad_arguments():
    """Rejected on the host before any device work (the pointer is never
    dereferenced)."""
    B = DeviceBlock([np.zeros(64)] * 4, 64, pad=0)
    for args in [(2, 64, [8, 8], B.kstride - 1),    # kinds would overlap
                 (2, 16, [8, 8], B.kstride),        # no such precision
                 (2, 64, [8, 0], B.kstride),        # empty axis
                 (4, 64, [8, 8], B.kstride)]:       # no such dimension
        with pytest.raises(af.AFError) as e:
            af.norms_noalloc(args[0], args[1], args[2], [0, 0], [1, 1], B.ptr.value, args[3])
        assert e.value.status == af.AF_ERR_ARG
    B.free()
