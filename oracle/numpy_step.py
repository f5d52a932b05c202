"""The time step written as whole-array NumPy operations: the CPU analogue of
the paper's ``numpy`` backend (Sec. 2.3 lists it beside the generated C++
backends; Sec. 3.1 compares the two), kept as context for the benchmark.

TEST INFRASTRUCTURE ONLY: used by the CPU-baseline leg of the benchmark and
by the test-suite, never by the product path.  It shares no code with the
HIP library or with ``oracle.c``.

Each stage is one array expression over a whole level range, with the same
association as the oracle's loops, and NumPy contracts nothing into fused
multiply-adds, so the result equals the oracle's bit for bit (a CPU test
checks exactly that; the oracle's own pins then carry over).  The Thomas
sweep is vectorised over the columns and runs its levels in order
(FORWARD elimination, BACKWARD substitution, Sec. 2.2).

Layout as the oracle: padded ``u`` (nk, nj+4, ni+4), interior ``data``
(nk, nj, ni), staggered ``w`` (nk+1, nj, ni).
"""
from __future__ import annotations

import numpy as np


def hdiff_interior(u: np.ndarray, coeff: float) -> np.ndarray:
    """Flux-limited fourth-order diffusion of the interior (stated form,
    scalar coefficient, limiter decided in FP64)."""
    nk, pj, pi = u.shape
    nj, ni = pj - 4, pi - 4
    # lap on the box i in [-1, ni], j in [-1, nj] (padded index = i + 2)
    cen = u[:, 1:nj + 3, 1:ni + 3]
    s = (u[:, 1:nj + 3, 0:ni + 2] + u[:, 1:nj + 3, 2:ni + 4]) + (u[:, 0:nj + 2, 1:ni + 3] + u[:, 2:nj + 4, 1:ni + 3])
    lap = 4.0 * cen - s  # lap[k, j + 1, i + 1]
    # x-fluxes between (i, j) and (i+1, j), i in [-1, ni), j in [0, nj)
    fx = lap[:, 1:nj + 1, 1:ni + 2] - lap[:, 1:nj + 1, 0:ni + 1]
    gx = u[:, 2:nj + 2, 2:ni + 3] - u[:, 2:nj + 2, 1:ni + 2]
    fx = np.where(fx * gx > 0.0, 0.0, fx)  # fx[k, j, i + 1]
    # y-fluxes between (i, j) and (i, j+1), i in [0, ni), j in [-1, nj)
    fy = lap[:, 1:nj + 2, 1:ni + 1] - lap[:, 0:nj + 1, 1:ni + 1]
    gy = u[:, 2:nj + 3, 2:ni + 2] - u[:, 1:nj + 2, 2:ni + 2]
    fy = np.where(fy * gy > 0.0, 0.0, fy)  # fy[k, j + 1, i]
    div = (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])
    return u[:, 2:nj + 2, 2:ni + 2] - coeff * div


def thomas(d: np.ndarray, w: np.ndarray, dt_dz: float) -> np.ndarray:
    """x = T^{-1} d for every column at once: a_k = -r/4 w_k (k >= 1),
    c_k = r/4 w_{k+1} (k <= nk-2), b_k = 1 + |a_k| + |c_k|."""
    nk = d.shape[0]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    zero = np.zeros(d.shape[1:])
    for k in range(nk):
        a = (-0.25 * dt_dz) * w[k] if k >= 1 else zero
        c = (0.25 * dt_dz) * w[k + 1] if k <= nk - 2 else zero
        b = 1.0 + np.abs(a) + np.abs(c)
        if k == 0:
            cp[0] = c / b
            dp[0] = d[0] / b
        else:
            m = b - a * cp[k - 1]
            cp[k] = c / m
            dp[k] = (d[k] - a * dp[k - 1]) / m
    x = np.empty_like(d)
    x[nk - 1] = dp[nk - 1]
    for k in range(nk - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def step(u: np.ndarray, data: np.ndarray, w: np.ndarray, coeff: float, dt_dz: float) -> np.ndarray:
    """One time step: the diffused interior plus the forcing is the right-hand
    side of the column solve; returns the padded next state (halo carried)."""
    nxt = u.copy()
    nk, nj, ni = data.shape
    if nk * nj * ni == 0:
        return nxt
    nxt[:, 2:nj + 2, 2:ni + 2] = thomas(hdiff_interior(u, coeff) + data, w, dt_dz)
    return nxt
