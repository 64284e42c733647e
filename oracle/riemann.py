"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

TEST INFRASTRUCTURE ONLY.  Used to pin the whole IGR scheme on the planar
Sod problem: IGR smooths shocks over a width set by alpha ~ dx^2 ("Shock
treatment with information geometric regularization"), so the discrete
solution must approach the vanishing-viscosity (exact entropy) solution as
the grid is refined.

Written from the textbook construction (pressure functions for a shock or a
rarefaction on each side, Newton iteration for the star pressure, sampling
of the self-similar solution); nothing here comes from the paper, which
prints no worked example.  Pinned by the classical Sod star state stored in
tests/golden/sod_star_state.json and by the Rankine-Hugoniot relations
checked in tests.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Side:
    rho: float
    u: float
    p: float


@dataclass
class StarState:
    p: float
    u: float
    rho_l: float
    rho_r: float


def _sound(s: Side, gamma: float) -> float:
    return math.sqrt(gamma * s.p / s.rho)


def _pressure_function(p: float, s: Side, gamma: float):
    """f_K(p) and its derivative: velocity jump across the K-wave."""
    c = _sound(s, gamma)
    if p > s.p:  # shock
        a = 2.0 / ((gamma + 1.0) * s.rho)
        b = (gamma - 1.0) / (gamma + 1.0) * s.p
        q = math.sqrt(a / (p + b))
        return (p - s.p) * q, q * (1.0 - 0.5 * (p - s.p) / (p + b))
    ratio = p / s.p  # rarefaction
    ex = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * c / (gamma - 1.0) * (ratio ** ex - 1.0)
    df = ratio ** (-(gamma + 1.0) / (2.0 * gamma)) / (s.rho * c)
    return f, df


def star_state(left: Side, right: Side, gamma: float = 1.4, tol: float = 1e-15) -> StarState:
    """Star-region pressure, velocity and the two star densities."""
    du = right.u - left.u
    p = max(1e-12, 0.5 * (left.p + right.p))
    for _ in range(200):
        fl, dfl = _pressure_function(p, left, gamma)
        fr, dfr = _pressure_function(p, right, gamma)
        step = (fl + fr + du) / (dfl + dfr)
        p_new = max(1e-14, p - step)
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _pressure_function(p, left, gamma)
    fr, _ = _pressure_function(p, right, gamma)
    u = 0.5 * (left.u + right.u) + 0.5 * (fr - fl)
    g1 = (gamma - 1.0) / (gamma + 1.0)

    def star_rho(s: Side):
        r = p / s.p
        if p > s.p:
            return s.rho * (r + g1) / (g1 * r + 1.0)
        return s.rho * r ** (1.0 / gamma)

    return StarState(p=p, u=u, rho_l=star_rho(left), rho_r=star_rho(right))


def wave_speeds(left: Side, right: Side, gamma: float = 1.4) -> dict:
    """Speeds of the wave fronts (head/tail for a rarefaction, the shock
    speed for a shock) and of the contact."""
    st = star_state(left, right, gamma)
    out = {"contact": st.u}
    for name, s, sign, rho_star in (("left", left, -1.0, st.rho_l), ("right", right, 1.0, st.rho_r)):
        c = _sound(s, gamma)
        if st.p > s.p:
            out[name + "_shock"] = s.u + sign * c * math.sqrt(
                (gamma + 1.0) / (2.0 * gamma) * st.p / s.p + (gamma - 1.0) / (2.0 * gamma))
        else:
            c_star = math.sqrt(gamma * st.p / rho_star)
            out[name + "_head"] = s.u + sign * c
            out[name + "_tail"] = st.u + sign * c_star
    return out


def sample(left: Side, right: Side, xi: np.ndarray, gamma: float = 1.4):
    """(rho, u, p) of the self-similar solution at xi = (x - x0) / t."""
    st = star_state(left, right, gamma)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    g = gamma
    for idx, x in np.ndenumerate(xi):
        if x <= st.u:
            s, sign, rho_star = left, 1.0, st.rho_l
        else:
            s, sign, rho_star = right, -1.0, st.rho_r
        c = _sound(s, g)
        # mirror the right side onto the left-side formulas via sign
        xs = sign * x
        us = sign * s.u
        ustar = sign * st.u
        if st.p > s.p:  # shock on this side
            S = us - c * math.sqrt((g + 1) / (2 * g) * st.p / s.p + (g - 1) / (2 * g))
            if xs <= S:
                r, v, q = s.rho, us, s.p
            else:
                r, v, q = rho_star, ustar, st.p
        else:  # rarefaction on this side
            head = us - c
            c_star = math.sqrt(g * st.p / rho_star)
            tail = ustar - c_star
            if xs <= head:
                r, v, q = s.rho, us, s.p
            elif xs >= tail:
                r, v, q = rho_star, ustar, st.p
            else:
                v = 2.0 / (g + 1) * (c + 0.5 * (g - 1) * us + xs)
                cf = 2.0 / (g + 1) * (c + 0.5 * (g - 1) * (us - xs))
                r = s.rho * (cf / c) ** (2.0 / (g - 1))
                q = s.p * (cf / c) ** (2.0 * g / (g - 1))
        rho[idx], u[idx], p[idx] = r, sign * v, q
    return rho, u, p


def cell_averages(left: Side, right: Side, x0: float, t: float, edges: np.ndarray,
                  gamma: float = 1.4, sub: int = 64):
    """Cell averages of the conserved variables (rho, rho u, E) of the exact
    solution at time t over the cells [edges[i], edges[i+1]] (midpoint rule
    with ``sub`` points per cell)."""
    edges = np.asarray(edges, dtype=np.float64)
    h = np.diff(edges)
    frac = (np.arange(sub) + 0.5) / sub
    xs = edges[:-1, None] + h[:, None] * frac[None, :]
    rho, u, p = sample(left, right, (xs - x0) / t, gamma)
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return rho.mean(1), (rho * u).mean(1), E.mean(1)
