"""Pure-Python loop version of the forward stencils, for tiny domains only.

TEST INFRASTRUCTURE ONLY.  A second, independently written CPU reference of
the horizontal diffusion and the vertical Thomas solve (the benchmark
stencils named in Sec. 3.1, with the workload's definition of their
formulas, which the paper does not print), used to cross-check ``oracle.c`` on domains of a few hundred
points.  Same array conventions as ``oracle.py``.
"""
from __future__ import annotations


def _lap(u, i, j, k):
    # u is indexed with the padded offset (+2, +2)
    c = u[k][j + 2][i + 2]
    s = (u[k][j + 2][i + 1] + u[k][j + 2][i + 3]) + (u[k][j + 1][i + 2] + u[k][j + 3][i + 2])
    return 4.0 * c - s


def hdiff(u, coeff):
    """u: nested lists or array (nk, nj+4, ni+4). Returns interior out, mx, my as lists."""
    nk = len(u)
    nj = len(u[0]) - 4
    ni = len(u[0][0]) - 4
    out = [[[0.0] * ni for _ in range(nj)] for _ in range(nk)]
    mx = [[[0] * (ni + 1) for _ in range(nj)] for _ in range(nk)]
    my = [[[0] * ni for _ in range(nj + 1)] for _ in range(nk)]
    for k in range(nk):
        lap = {}
        for j in range(-1, nj + 1):
            for i in range(-1, ni + 1):
                lap[(i, j)] = _lap(u, i, j, k)
        fx = {}
        for j in range(nj):
            for i in range(-1, ni):
                f = lap[(i + 1, j)] - lap[(i, j)]
                g = u[k][j + 2][i + 3] - u[k][j + 2][i + 2]
                kept = not (f * g > 0.0)
                mx[k][j][i + 1] = int(kept)
                fx[(i, j)] = f if kept else 0.0
        fy = {}
        for j in range(-1, nj):
            for i in range(ni):
                f = lap[(i, j + 1)] - lap[(i, j)]
                g = u[k][j + 3][i + 2] - u[k][j + 2][i + 2]
                kept = not (f * g > 0.0)
                my[k][j + 1][i] = int(kept)
                fy[(i, j)] = f if kept else 0.0
        for j in range(nj):
            for i in range(ni):
                div = (fx[(i, j)] - fx[(i - 1, j)]) + (fy[(i, j)] - fy[(i, j - 1)])
                out[k][j][i] = u[k][j + 2][i + 2] - coeff * div
    return out, mx, my


def thomas_column(dcol, wcol, dt_dz):
    """One column: dcol has nk entries, wcol nk+1. Returns x (list)."""
    nk = len(dcol)
    a = [0.0] * nk
    c = [0.0] * nk
    for k in range(1, nk):
        a[k] = -0.25 * dt_dz * wcol[k]
    for k in range(nk - 1):
        c[k] = 0.25 * dt_dz * wcol[k + 1]
    b = [1.0 + abs(a[k]) + abs(c[k]) for k in range(nk)]
    cp = [0.0] * nk
    dp = [0.0] * nk
    for k in range(nk):
        m = b[k] - (a[k] * cp[k - 1] if k > 0 else 0.0)
        cp[k] = c[k] / m
        dp[k] = (dcol[k] - (a[k] * dp[k - 1] if k > 0 else 0.0)) / m
    x = [0.0] * nk
    for k in range(nk - 1, -1, -1):
        x[k] = dp[k] - (cp[k] * x[k + 1] if k < nk - 1 else 0.0)
    return x
