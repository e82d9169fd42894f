"""ctypes binding of the AF library (include/af.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libaf4.so; this module
never computes any part of it.  Importing it loads the library and fails
loudly if it has not been built (``python -m paper_2510_11527_amd.build``).
"""
import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaf4.so")

AF_OK, AF_ERR_ARG, AF_ERR_ALLOC, AF_ERR_DEVICE, AF_ERR_BOUNDS = 0, -1, -2, -3, -4
AF_ERR_NONFINITE, AF_ERR_CFL, AF_ERR_STATE, AF_ERR_UNSUPPORTED = -5, -6, -7, -8
STATUS_NAMES = {0: "AF_OK", -1: "AF_ERR_ARG", -2: "AF_ERR_ALLOC", -3: "AF_ERR_DEVICE", -4: "AF_ERR_BOUNDS",
                -5: "AF_ERR_NONFINITE", -6: "AF_ERR_CFL", -7: "AF_ERR_STATE", -8: "AF_ERR_UNSUPPORTED"}
FLUX = {"linear": 0, "quad": 1, "bl": 2, "bl_grav": 3}
DIFF = {"linear": 0, "power": 1, "deadzone": 2, "bl": 3, "ramp2": 4}
DIFFUSION_FORMS = {"dc": 0, "nodc": 1}
BC_KINDS = {"periodic": 0, "dirichlet": 1, "outflow": 2}
INTEGRATORS = {"ssprk3": 0, "euler": 1, "ssprk54": 2}

EXPORTS = ["af_create", "af_destroy", "af_set_state", "af_get_state", "af_step", "af_residual", "af_norms",
           "af_last_error", "af_set_stream", "af_set_variant", "af_num_variants", "af_variant_name",
           "af_step_timed", "af_work", "af_get_variant", "af_autotune", "af_limiter_activity", "af_norms_noalloc", "af_copy_rate",
           "af_set_state_dev", "af_get_state_dev"]


class AfProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("flux", ctypes.c_int * 3),
        ("flux_par", (ctypes.c_double * 2) * 3),
        ("diff", ctypes.c_int),
        ("diff_par", ctypes.c_double * 2),
        ("umin", ctypes.c_double),
        ("umax", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int),
        ("si_blend", ctypes.c_int),
        ("si_gamma", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("integrator", ctypes.c_int),
        ("diffusion_form", ctypes.c_int),
        ("bc", (ctypes.c_int * 2) * 3),
        ("bc_value", (ctypes.c_double * 2) * 3),
    ]


class AfNorms(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("mass", ctypes.c_double),
                ("min_avg", ctypes.c_double), ("max_avg", ctypes.c_double), ("min_pv", ctypes.c_double),
                ("max_pv", ctypes.c_double), ("l1_avg", ctypes.c_double), ("l2_avg", ctypes.c_double),
                ("linf_avg", ctypes.c_double), ("max_clamp", ctypes.c_double), ("steps", ctypes.c_longlong),
                ("nonfinite", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def lib():
    """Load libaf4.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libaf4.so is not built; run python -m paper_2510_11527_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(dp)
        vp = ctypes.c_void_p
        L.af_create.argtypes = [ctypes.c_int, ctypes.POINTER(AfProblem), ctypes.POINTER(vp)]
        L.af_destroy.argtypes = [vp]
        L.af_set_state.argtypes = [vp, ctypes.c_int, pp, ctypes.c_double]
        L.af_get_state.argtypes = [vp, ctypes.c_int, pp, dp]
        L.af_step.argtypes = [vp, ctypes.c_int, ctypes.c_double, dp, dp]
        L.af_step_timed.argtypes = [vp, ctypes.c_int, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.af_residual.argtypes = [vp, ctypes.c_int, pp]
        L.af_norms.argtypes = [vp, ctypes.c_int, ctypes.POINTER(AfNorms)]
        L.af_last_error.argtypes = [vp]
        L.af_last_error.restype = ctypes.c_char_p
        L.af_set_stream.argtypes = [vp, vp]
        L.af_set_variant.argtypes = [vp, ctypes.c_int]
        L.af_num_variants.argtypes = [vp]
        L.af_get_variant.argtypes = [vp]
        L.af_variant_name.argtypes = [vp, ctypes.c_int]
        L.af_variant_name.restype = ctypes.c_char_p
        L.af_work.argtypes = [vp, dp, dp, dp]
        L.af_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        L.af_limiter_activity.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
        ip = ctypes.POINTER(ctypes.c_int)
        L.af_norms_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, dp, vp, ctypes.c_longlong, vp,
                                       ctypes.POINTER(AfNorms)]
        L.af_copy_rate.argtypes = [ctypes.c_longlong, ctypes.c_int, dp]
        L.af_set_state_dev.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.c_double, vp]
        L.af_get_state_dev.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), dp, vp]
        for name in EXPORTS:
            if name not in ("af_last_error", "af_num_variants", "af_variant_name", "af_get_variant"):
                getattr(L, name).restype = ctypes.c_int
        L.af_num_variants.restype = ctypes.c_int
        L.af_get_variant.restype = ctypes.c_int
        _lib = L
    return _lib


class AFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def make_problem(spec, precision=None, integrator="ssprk3"):
    """af_problem from a problem dict (see workloads.py)."""
    P = AfProblem()
    d = int(spec["dim"])
    P.dim = d
    for l in range(3):
        P.n[l] = int(spec["n"][l]) if l < d else 1
        P.lo[l] = float(spec["lo"][l]) if l < d else 0.0
        P.hi[l] = float(spec["hi"][l]) if l < d else 1.0
    for l in range(d):
        kind, *par = spec["flux"][l]
        P.flux[l] = FLUX[kind]
        for k, v in enumerate(par[:2]):
            P.flux_par[l][k] = float(v)
    kind, *par = spec["diff"]
    P.diff = DIFF[kind]
    for k, v in enumerate(par[:2]):
        P.diff_par[k] = float(v)
    P.umin = float(spec.get("umin", math.nan))
    P.umax = float(spec.get("umax", math.nan))
    P.cfl = float(spec.get("cfl", 0.1))
    P.limiter = int(bool(spec.get("limiter", False)))
    P.si_blend = int(bool(spec.get("si", False)))
    P.si_gamma = float(spec.get("si_gamma", 1.0))
    P.precision = int(precision or spec.get("precision", 64))
    P.integrator = INTEGRATORS[integrator]
    P.diffusion_form = DIFFUSION_FORMS[spec.get("diffusion_form", "dc")]
    # ends per axis ("bcs": [(low, high), ...]; "bc": those of axis 0); each
    # end "periodic", "outflow" or ("dirichlet", value)
    ends = list(spec.get("bcs", [])) or ([spec["bc"]] if "bc" in spec else [])
    for l, pair in enumerate(ends):
        for e in range(2):
            kind = pair[e] if isinstance(pair[e], str) else pair[e][0]
            P.bc[l][e] = BC_KINDS[kind]
            P.bc_value[l][e] = 0.0 if isinstance(pair[e], str) else float(pair[e][1])
    return P


def _pp(arrs):
    dp = ctypes.POINTER(ctypes.c_double)
    a = (dp * len(arrs))()
    for i, x in enumerate(arrs):
        a[i] = x.ctypes.data_as(dp)
    return a


class Context:
    """Owns one af_ctx.  Methods mirror the C entry points."""

    def __init__(self, specs, precision=None, integrator="ssprk3"):
        if isinstance(specs, dict):
            specs = [specs]
        self.specs = list(specs)
        self.dim = int(self.specs[0]["dim"])
        arr = (AfProblem * len(self.specs))(*[make_problem(s, precision, integrator) for s in self.specs])
        self.precision = arr[0].precision
        h = ctypes.c_void_p()
        st = lib().af_create(len(self.specs), arr, ctypes.byref(h))
        if st != AF_OK:
            raise AFError(st, lib().af_last_error(None).decode())
        self.h = h
        self.ncells = [int(np.prod([s["n"][l] for l in range(self.dim)])) for s in self.specs]

    def _check(self, st):
        if st != AF_OK:
            raise AFError(st, lib().af_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().af_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, inst, dofs, t=0.0):
        a = [np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1)) for x in dofs]
        self._check(lib().af_set_state(self.h, int(inst), _pp(a), float(t)))

    def get_state(self, inst):
        out = [np.empty(self.ncells[inst]) for _ in range(1 << self.dim)]
        t = ctypes.c_double()
        self._check(lib().af_get_state(self.h, int(inst), _pp(out), ctypes.byref(t)))
        return out, t.value

    def set_state_dev(self, inst, ptrs, t=0.0, stream_ptr=None):
        """af_set_state_dev: ptrs holds 2^d device addresses (integers) of
        FP64 arrays of ncells[inst] values, in zeta order."""
        a = (ctypes.c_void_p * len(ptrs))(*[int(p) for p in ptrs])
        self._check(lib().af_set_state_dev(self.h, int(inst), a, float(t), stream_ptr))

    def get_state_dev(self, inst, ptrs, stream_ptr=None):
        """af_get_state_dev: the state, widened to FP64, to the device arrays
        at ptrs; returns the time."""
        a = (ctypes.c_void_p * len(ptrs))(*[int(p) for p in ptrs])
        t = ctypes.c_double()
        self._check(lib().af_get_state_dev(self.h, int(inst), a, ctypes.byref(t), stream_ptr))
        return t.value

    def step(self, nsteps=1, t_end=0.0, dt=None):
        n = len(self.specs)
        dp = ctypes.POINTER(ctypes.c_double)
        used = np.empty(n)
        presc = None
        if dt is not None:
            presc = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).copy())
        st = lib().af_step(self.h, int(nsteps), float(t_end or 0.0),
                           presc.ctypes.data_as(dp) if presc is not None else None, used.ctypes.data_as(dp))
        self._check(st)
        return used

    def step_timed(self, nsteps=1, t_end=0.0, dt=None):
        n = len(self.specs)
        dp = ctypes.POINTER(ctypes.c_double)
        presc = None
        if dt is not None:
            presc = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).copy())
        ms = ctypes.c_double()
        cnt = ctypes.c_int()
        self._check(lib().af_step_timed(self.h, int(nsteps), float(t_end or 0.0),
                                        presc.ctypes.data_as(dp) if presc is not None else None,
                                        ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def residual(self, inst):
        out = [np.empty(self.ncells[inst]) for _ in range(1 << self.dim)]
        self._check(lib().af_residual(self.h, int(inst), _pp(out)))
        return out

    def norms(self, inst):
        n = AfNorms()
        self._check(lib().af_norms(self.h, int(inst), ctypes.byref(n)))
        return n.as_dict()

    def set_stream(self, stream_ptr):
        self._check(lib().af_set_stream(self.h, ctypes.c_void_p(stream_ptr)))

    def num_variants(self):
        return lib().af_num_variants(self.h)

    def variant_name(self, v):
        return lib().af_variant_name(self.h, int(v)).decode()

    def set_variant(self, v):
        self._check(lib().af_set_variant(self.h, int(v)))

    def variant(self):
        return lib().af_get_variant(self.h)

    def limiter_activity(self, inst):
        """Counts of af_limiter_activity: face fluxes, of which limited, cell
        potentials, of which limited (one forward-Euler stage of the current
        state; the state is left unchanged)."""
        c = (ctypes.c_longlong * 4)()
        self._check(lib().af_limiter_activity(self.h, int(inst), c))
        return {"faces": c[0], "faces_limited": c[1], "potentials": c[2], "potentials_limited": c[3]}

    def autotune(self, nsteps=5):
        """Select the fastest tile variant on the current state (af_autotune);
        returns the chosen index and the mean stage time per variant (ms, -1
        for variants not built)."""
        ms = np.empty(self.num_variants())
        chosen = ctypes.c_int()
        self._check(lib().af_autotune(self.h, int(nsteps), ctypes.byref(chosen),
                                      ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return chosen.value, ms

    def work(self):
        b, c, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().af_work(self.h, ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return {"bytes_per_stage": b.value, "cells": c.value, "dofs": d.value}


def norms_noalloc(dim, precision, n, lo, hi, dofs_ptr, kind_stride, stream_ptr=None):
    """af_norms_noalloc: norms of a state in caller device memory (one block,
    DoF kind z at dofs_ptr + z * kind_stride values), computed without any
    allocation.  dofs_ptr and stream_ptr are device addresses / a stream
    handle as integers (e.g. a torch tensor's data_ptr() and a torch
    stream's cuda_stream)."""
    nn = (ctypes.c_int * 3)(*[int(v) for v in (list(n) + [1, 1, 1])[:3]])
    ll = (ctypes.c_double * 3)(*[float(v) for v in (list(lo) + [0.0, 0.0, 0.0])[:3]])
    hh = (ctypes.c_double * 3)(*[float(v) for v in (list(hi) + [1.0, 1.0, 1.0])[:3]])
    out = AfNorms()
    st = lib().af_norms_noalloc(int(dim), int(precision), nn, ll, hh, ctypes.c_void_p(int(dofs_ptr)),
                                int(kind_stride), ctypes.c_void_p(stream_ptr or None), ctypes.byref(out))
    if st != AF_OK:
        raise AFError(st, lib().af_last_error(None).decode())
    return out.as_dict()


def copy_rate(nbytes=1 << 30, reps=20):
    """af_copy_rate: GB/s of a streaming device copy (read + write bytes)."""
    r = ctypes.c_double()
    st = lib().af_copy_rate(int(nbytes), int(reps), ctypes.byref(r))
    if st != AF_OK:
        raise AFError(st, lib().af_last_error(None).decode())
    return r.value

