"""Readings of the limiter tested against the limited columns of Table 3.

TEST INFRASTRUCTURE ONLY (a record of hypotheses, used by the tests): the
GPU library never imports it.

Example 6.2 runs u_t + u_x = 0 with u = 1 + sin^4(2 pi (x - t)) on the
periodic [0, 1] to T = 1 with SSP-RK(5,4) and prints the discrete
(min - u_min, max - u_max) over all DoFs with and without the limiter of
Sec. 5.1.  The unlimited columns are reproduced by the C oracle to their
four digits; the limited ones are not.  This module re-implements the 1D
scheme for this one problem (f = u, a = 0, so alpha = 1, the LLF flux is the
upwind average and u^{L,+}_i is the average itself) in vectorised numpy,
with switches for the details the paper leaves open or that an
implementation might read differently:

* ``factor``: the multiple of mu in theta^c.  Eq.
  (1d_convection_limiting_parameter) prints 6 mu (one third of each limited
  state is the convection part); with a = 0 the two diffusion thirds equal
  u^{L,+-}, so the bound on the whole state needs only 2 mu.
* ``step``: the step size the limited forward-Euler operator is built with in
  each Runge-Kutta term a U + b dt L(U): ``"ratio"`` (b/a) dt, which makes the
  term a times a limited forward-Euler stage (the form the oracle uses);
  ``"dt"`` the step dt^n of the formulas of Sec. 5.1; ``"b"`` b dt.
* ``projection``: point values clamped inside every forward-Euler stage
  (``"stage_fe"``, Sec. 5.1.2 applied per stage), after every Runge-Kutta
  combination (``"combination"``) or once per step (``"step"``).
* ``low``: low-order states from the stage input (``"stage"``) or from U^n
  (``"un"``).
* ``where``: limiting in every stage (``"all"``), only in the last stage
  (``"last"``), or once per step on the step's time-averaged face flux
  against the low-order step of dt from U^n (``"step_fct"``).
* ``init``: initial averages by Simpson's rule on the initial point values
  or exact.
"""
import numpy as np

# SSP-RK(5,4), Shu-Osher coefficients (Spiteri and Ruuth 2002; the same
# published values the C oracle uses)
_B10 = 0.391752226571890
_A20, _A21, _B21 = 0.444370493651235, 0.555629506348765, 0.368410593050371
_A30, _A32, _B32 = 0.620101851488403, 0.379898148511597, 0.251891774271694
_A40, _A43, _B43 = 0.178079954393132, 0.821920045606868, 0.544974750228521
_A52, _A53, _B53 = 0.517231671970585, 0.096059710526147, 0.063692468666290
_A54, _B54 = 0.386708617503269, 0.226007483236906

UMIN, UMAX = 1.0, 2.0


def _theta(zl, zh):
    """Theta(z^L, z^H) of Sec. 5.1.1: the largest blend keeping the state in
    [u_min, u_max]."""
    out = np.ones_like(zl)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(zh < UMIN, (zl - UMIN) / (zl - zh), out)
        out = np.where(zh > UMAX, (zl - UMAX) / (zl - zh), out)
    return np.clip(out, 0.0, 1.0)


def _rhs(ub, up, dx):
    """Unlimited semi-discrete right-hand side for f = u (Eqs. 1d_conv_av,
    1d_conv_pnt with alpha = 1: f^+ = u, f^- = 0; centre by Simpson)."""
    um = np.roll(up, 1)
    uc = (6 * ub - um - up) / 4
    Rp = -(um - 6 * uc + 3 * up + 2 * np.roll(uc, -1)) / (3 * dx)
    return -(up - um) / dx, Rp


def _fe(ub, up, h, dx, o, src=None, limit=True):
    """One forward-Euler stage of step h, limited per Sec. 5.1.1/5.1.2."""
    Ra, Rp = _rhs(ub, up, dx)
    upn = up + h * Rp
    if o["projection"] == "stage_fe":
        upn = np.clip(upn, UMIN, UMAX)
    if not limit:
        return ub + h * Ra, upn
    mu = h / dx
    s = ub if src is None else src
    Lp = s                                   # u^{L,+}_i (LLF with alpha = 1)
    Lm = s - 2 * mu * (s - np.roll(s, 1))    # u^{L,-}_i
    df = up - s                              # f^H - f^L at i+1/2
    k = o["factor"] * mu
    th = np.minimum(_theta(Lp, Lp - k * df), _theta(np.roll(Lm, -1), np.roll(Lm, -1) + k * df))
    flim = s + th * df
    return ub - mu * (flim - np.roll(flim, 1)), upn


def _step(ub, up, dt, dx, o):
    U0 = (ub, up)
    src = ub if o["low"] == "un" else None

    def term(U, a, b, limit=True):
        h = {"ratio": b / a * dt, "dt": dt, "b": b * dt}[o["step"]]
        V = _fe(U[0], U[1], h, dx, o, src=src, limit=limit)
        return tuple(a * u + b * dt * (v - u) / h for u, v in zip(U, V))

    def P(U):
        return (U[0], np.clip(U[1], UMIN, UMAX)) if o["projection"] == "combination" else U

    if o["where"] == "step_fct":
        return _step_fct(ub, up, dt, dx, o)
    early = o["where"] == "all"
    last = o["where"] in ("all", "last")
    U1 = P(term(U0, 1.0, _B10, early))
    t = term(U1, _A21, _B21, early); U2 = P(tuple(_A20 * x + y for x, y in zip(U0, t)))
    t = term(U2, _A32, _B32, early); U3 = P(tuple(_A30 * x + y for x, y in zip(U0, t)))
    t = term(U3, _A43, _B43, early); U4 = P(tuple(_A40 * x + y for x, y in zip(U0, t)))
    t1, t2 = term(U3, _A53, _B53, last), term(U4, _A54, _B54, last)
    U5 = tuple(_A52 * a + b + c for a, b, c in zip(U2, t1, t2))
    if o["projection"] in ("combination", "step"):
        U5 = (U5[0], np.clip(U5[1], UMIN, UMAX))
    return U5


def _step_fct(ub, up, dt, dx, o):
    """Unlimited SSP-RK(5,4) step; its time-averaged face flux limited once
    against the low-order forward-Euler step of dt from U^n."""
    U0 = (ub, up)
    L = lambda U: _rhs(U[0], U[1], dx)
    l0 = L(U0); U1 = tuple(u + _B10 * dt * r for u, r in zip(U0, l0))
    l1 = L(U1); U2 = tuple(_A20 * x + _A21 * y + _B21 * dt * r for x, y, r in zip(U0, U1, l1))
    l2 = L(U2); U3 = tuple(_A30 * x + _A32 * y + _B32 * dt * r for x, y, r in zip(U0, U2, l2))
    l3 = L(U3); U4 = tuple(_A40 * x + _A43 * y + _B43 * dt * r for x, y, r in zip(U0, U3, l3))
    l4 = L(U4)
    U5 = tuple(_A52 * a + _A53 * b + _B53 * dt * c + _A54 * d + _B54 * dt * e
               for a, b, c, d, e in zip(U2, U3, l3, U4, l4))
    # the face flux f(u_{i+1/2}) of each stage, combined like the stages
    f = [U[1] for U in (U0, U1, U2, U3, U4)]
    g1 = _B10 * f[0]
    g2 = _A21 * g1 + _B21 * f[1]
    g3 = _A32 * g2 + _B32 * f[2]
    g4 = _A43 * g3 + _B43 * f[3]
    fbar = _A52 * g2 + _A53 * g3 + _B53 * f[3] + _A54 * g4 + _B54 * f[4]
    mu = dt / dx
    Lm = ub - 2 * mu * (ub - np.roll(ub, 1))
    df = fbar - ub
    k = o["factor"] * mu
    th = np.minimum(_theta(ub, ub - k * df), _theta(np.roll(Lm, -1), np.roll(Lm, -1) + k * df))
    flim = ub + th * df
    return ub - mu * (flim - np.roll(flim, 1)), np.clip(U5[1], UMIN, UMAX)


DEFAULTS = dict(limiter=True, factor=6.0, step="ratio", projection="stage_fe", low="stage",
                where="all", init="simpson", cfl=0.05)


def run(N, **kw):
    """(min - u_min, max - u_max) over all DoFs at T = 1 on N cells."""
    o = dict(DEFAULTS, **kw)
    dx = 1.0 / N
    u0 = lambda s: 1.0 + np.sin(2 * np.pi * s) ** 4
    xc, xr = (np.arange(N) + 0.5) / N, (np.arange(N) + 1.0) / N
    if o["init"] == "simpson":
        ub = (u0(xr - dx) + 4 * u0(xc) + u0(xr)) / 6
    else:
        # antiderivative of sin^4(2 pi x) = 3/8 - cos(4 pi x)/2 + cos(8 pi x)/8
        F = lambda x: 3 / 8 * x - np.sin(4 * np.pi * x) / (8 * np.pi) + np.sin(8 * np.pi * x) / (64 * np.pi)
        ub = 1.0 + (F(xr) - F(xr - dx)) / dx
    up = u0(xr)
    nst = int(np.ceil(1.0 / (o["cfl"] * dx) - 1e-9))
    dt = 1.0 / nst
    for _ in range(nst):
        if o["limiter"]:
            ub, up = _step(ub, up, dt, dx, o)
        else:
            ub, up = _step(ub, up, dt, dx, dict(o, where="none", projection="none"))
    return (min(ub.min(), up.min()) - UMIN, max(ub.max(), up.max()) - UMAX)


if __name__ == "__main__":
    import sys
    Ns = [int(x) for x in (sys.argv[1] if len(sys.argv) > 1 else "20,40,80").split(",")]
    for kw in [{}, dict(factor=2.0), dict(factor=2.0, step="dt", cfl=0.07)]:
        print(kw, ["%+.3e/%+.3e" % run(N, **kw) for N in Ns], flush=True)
