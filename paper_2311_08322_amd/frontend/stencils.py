"""The benchmark stencils of the GT4Py paper (Sec. 3.1) written in the
frontend's language: the horizontal diffusion, the implicit vertical
advection and their time step, plus the damping-form diffusion written with
if/else and an external constant to exercise those parts of the language.
The arithmetic follows the stated definitions operation for operation."""
from __future__ import annotations

from . import BACKWARD, FORWARD, PARALLEL, Field, computation, function, interval, stencil  # noqa: F401


@function
def lap_of(f):
    return 4.0 * f - ((f[-1, 0, 0] + f[1, 0, 0]) + (f[0, -1, 0] + f[0, 1, 0]))


@stencil
def hdiff(u: Field, out: Field, *, coeff: float):
    with computation(PARALLEL), interval(...):
        lap = lap_of(u)
        flx = lap[1, 0, 0] - lap
        flx = 0.0 if flx * (u[1, 0, 0] - u) > 0.0 else flx
        fly = lap[0, 1, 0] - lap
        fly = 0.0 if fly * (u[0, 1, 0] - u) > 0.0 else fly
        out = u - coeff * ((flx - flx[-1, 0, 0]) + (fly - fly[0, -1, 0]))


@stencil(externals={"SIGN": -1.0})
def hdiff_damping(u: Field, out: Field, *, coeff: float):
    with computation(PARALLEL), interval(...):
        lap = SIGN * lap_of(u)  # noqa: F821 (external)
        flx = lap[1, 0, 0] - lap
        if flx * (u[1, 0, 0] - u) > 0.0:
            flx = 0.0
        fly = lap[0, 1, 0] - lap
        if fly * (u[0, 1, 0] - u) > 0.0:
            fly = 0.0
        out = u - coeff * ((flx - flx[-1, 0, 0]) + (fly - fly[0, -1, 0]))


@stencil
def vadv(u: Field, data: Field, w: Field, out: Field, *, dt_dz: float):
    # coefficients: a_0 = 0 and c_{nk-1} = 0, the interval boundaries
    with computation(PARALLEL):
        with interval(0, 1):
            a = 0.0
        with interval(1, None):
            a = -0.25 * dt_dz * w
    with computation(PARALLEL):
        with interval(0, -1):
            c = 0.25 * dt_dz * w[0, 0, 1]
        with interval(-1, None):
            c = 0.0
    with computation(FORWARD):
        with interval(0, 1):
            m = 1.0 + abs(a) + abs(c)
            cp = c / m
            dp = (u + data) / m
        with interval(1, None):
            m = (1.0 + abs(a) + abs(c)) - a * cp[0, 0, -1]
            cp = c / m
            dp = ((u + data) - a * dp[0, 0, -1]) / m
    with computation(BACKWARD):
        with interval(-1, None):
            out = dp
        with interval(0, -1):
            out = dp - cp * out[0, 0, 1]


@stencil
def step(u: Field, data: Field, w: Field, out: Field, *, coeff: float, dt_dz: float):
    with computation(PARALLEL), interval(...):
        lap = lap_of(u)
        flx = lap[1, 0, 0] - lap
        flx = 0.0 if flx * (u[1, 0, 0] - u) > 0.0 else flx
        fly = lap[0, 1, 0] - lap
        fly = 0.0 if fly * (u[0, 1, 0] - u) > 0.0 else fly
        h = u - coeff * ((flx - flx[-1, 0, 0]) + (fly - fly[0, -1, 0]))
    with computation(PARALLEL):
        with interval(0, 1):
            a = 0.0
        with interval(1, None):
            a = -0.25 * dt_dz * w
    with computation(PARALLEL):
        with interval(0, -1):
            c = 0.25 * dt_dz * w[0, 0, 1]
        with interval(-1, None):
            c = 0.0
    with computation(FORWARD):
        with interval(0, 1):
            m = 1.0 + abs(a) + abs(c)
            cp = c / m
            dp = (h + data) / m
        with interval(1, None):
            m = (1.0 + abs(a) + abs(c)) - a * cp[0, 0, -1]
            cp = c / m
            dp = ((h + data) - a * dp[0, 0, -1]) / m
    with computation(BACKWARD):
        with interval(-1, None):
            out = dp
        with interval(0, -1):
            out = dp - cp * out[0, 0, 1]


ALL = {"hdiff": hdiff, "hdiff_damping": hdiff_damping, "vadv": vadv, "step": step}
