"""Independent per-cell fifth-order Lax-Friedrichs Euler code (pure Python).

Written from the textbook definitions (ideal-gas Euler flux, five-cell
upwind-biased interpolant, Rusanov flux, Shu-Osher SSP-RK3) on a periodic
1D line, with Python floats and explicit loops.  It shares nothing with the
oracle and serves to pin it at alpha = 0, where the entropic pressure
vanishes and IGR reduces to the plain scheme.
"""

import math


def _prim(q, gamma):
    rho, mx, my, mz, E = q
    u = mx / rho
    p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho)
    return rho, u, p


def _flux_x(q, gamma):
    rho, mx, my, mz, E = q
    _, u, p = _prim(q, gamma)
    return [mx, mx * u + p, my * u, mz * u, (E + p) * u], abs(u) + math.sqrt(gamma * p / rho)


def rhs_1d(cells, dx, gamma):
    """cells: list of n 5-lists (periodic).  Returns dU/dt per cell."""
    n = len(cells)
    at = lambda i: cells[i % n]
    face_flux = []
    for f in range(n + 1):           # face between cells f-1 and f
        i = f - 1
        qL, qR = [], []
        for c in range(5):
            a, b, m, d, e = (at(i + o)[c] for o in (-2, -1, 0, 1, 2))
            qL.append((2 * a - 13 * b + 47 * m + 27 * d - 3 * e) / 60.0)
            b2, m2, d2, e2, g2 = (at(i + o)[c] for o in (-1, 0, 1, 2, 3))
            qR.append((-3 * b2 + 27 * m2 + 47 * d2 - 13 * e2 + 2 * g2) / 60.0)
        FL, sL = _flux_x(qL, gamma)
        FR, sR = _flux_x(qR, gamma)
        lam = max(sL, sR)
        face_flux.append([0.5 * (FL[c] + FR[c]) - 0.5 * lam * (qR[c] - qL[c]) for c in range(5)])
    return [[-(face_flux[i + 1][c] - face_flux[i][c]) / dx for c in range(5)] for i in range(n)]


def rk3_1d(cells, dx, dt, gamma):
    L0 = rhs_1d(cells, dx, gamma)
    u1 = [[cells[i][c] + dt * L0[i][c] for c in range(5)] for i in range(len(cells))]
    L1 = rhs_1d(u1, dx, gamma)
    u2 = [[0.75 * cells[i][c] + 0.25 * (u1[i][c] + dt * L1[i][c]) for c in range(5)] for i in range(len(cells))]
    L2 = rhs_1d(u2, dx, gamma)
    return [[cells[i][c] / 3.0 + 2.0 / 3.0 * (u2[i][c] + dt * L2[i][c]) for c in range(5)] for i in range(len(cells))]
