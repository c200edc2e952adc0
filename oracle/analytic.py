"""Analytic solutions of the paper's shock problems (Sec. 4.2-4.4).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

* Sod: the exact solution of the Riemann problem for an ideal gas, by the
  textbook method (pressure function with shock / rarefaction branches,
  root for the star pressure, sampling on x/t), as in Toro, "Riemann Solvers
  and Numerical Methods for Fluid Dynamics", ch. 4.
* Noh: the closed form quoted in Sec. 4.3 (shock radius, pre-shock density
  growth, post-shock density jump).  Post-shock temperature: all inflow
  kinetic energy becomes heat, T = m v0^2 / f.
* Sedov-Taylor: the self-similar ODEs of the Euler equations behind a strong
  shock, integrated from the Rankine-Hugoniot state at the shock inwards;
  the constant of the shock-radius law in Sec. 4.4 follows from the energy
  integral.

Ideal gas with f = 3 velocity components, gamma = 1 + 2/f = 5/3 (the
printed "1 + 1/f" in Sec. 4 contradicts the values 2 and 5/3 it quotes).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq


# --------------------------------------------------------------------------
# Sod / exact Riemann solver
# --------------------------------------------------------------------------
def _pressure_fn(p, rho, pk, ak, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * ak / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def riemann_star(left, right, gamma):
    """Star-region pressure and velocity for states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")

    def f(p):
        return _pressure_fn(p, rl, pl, al, gamma) + _pressure_fn(p, rr, pr, ar, gamma) + (ur - ul)

    lo, hi = 1e-14 * min(pl, pr), 10.0 * max(pl, pr)
    while f(hi) < 0.0:
        hi *= 10.0
    ps = brentq(f, lo, hi, xtol=1e-15 * hi, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_pressure_fn(ps, rr, pr, ar, gamma) - _pressure_fn(ps, rl, pl, al, gamma))
    return ps, us


def riemann_sample(s, left, right, gamma, star=None):
    """(rho, u, p) at similarity coordinate s = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    ps, us = riemann_star(left, right, gamma) if star is None else star
    if s <= us:
        a = math.sqrt(g * pl / rl)
        if ps > pl:
            sl = ul - a * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if s <= sl:
                return rl, ul, pl
            r = rl * (ps / pl + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * ps / pl + 1.0)
            return r, us, ps
        head = ul - a
        a_star = a * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        tail = us - a_star
        if s <= head:
            return rl, ul, pl
        if s > tail:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (a + 0.5 * (g - 1.0) * ul + s)
        c = 2.0 / (g + 1.0) * (a + 0.5 * (g - 1.0) * (ul - s))
        return rl * (c / a) ** (2.0 / (g - 1.0)), u, pl * (c / a) ** (2.0 * g / (g - 1.0))
    a = math.sqrt(g * pr / rr)
    if ps > pr:
        sr = ur + a * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if s >= sr:
            return rr, ur, pr
        r = rr * (ps / pr + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * ps / pr + 1.0)
        return r, us, ps
    head = ur + a
    a_star = a * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    tail = us + a_star
    if s >= head:
        return rr, ur, pr
    if s < tail:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1.0) * (-a + 0.5 * (g - 1.0) * ur + s)
    c = 2.0 / (g + 1.0) * (a - 0.5 * (g - 1.0) * (ur - s))
    return rr * (c / a) ** (2.0 / (g - 1.0)), u, pr * (c / a) ** (2.0 * g / (g - 1.0))


def sod_profile(x, t, left, right, gamma=5.0 / 3.0, x0=0.5):
    """Arrays (rho, u, p) at positions x and time t > 0."""
    star = riemann_star(left, right, gamma)
    out = np.array([riemann_sample((xi - x0) / t, left, right, gamma, star) for xi in np.atleast_1d(x)])
    return out[:, 0], out[:, 1], out[:, 2]


# --------------------------------------------------------------------------
# Noh (Sec. 4.3)
# --------------------------------------------------------------------------
def noh_profile(r, t, n0=1.0, v0=1.0, gamma=5.0 / 3.0, d=2, mass=1.0, f=3):
    """Number density, radial velocity and pressure at radius r, time t."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    rs = 0.5 * (gamma - 1.0) * v0 * t
    inside = r < rs
    n = np.where(inside, n0 * ((gamma + 1.0) / (gamma - 1.0)) ** d,
                 n0 * (1.0 + v0 * t / np.maximum(r, 1e-300)) ** (d - 1))
    vr = np.where(inside, 0.0, -v0)
    temp = mass * v0 * v0 / f
    p = np.where(inside, n * temp, 0.0)
    return n, vr, p, rs


# --------------------------------------------------------------------------
# Sedov-Taylor blast wave (Sec. 4.4)
# --------------------------------------------------------------------------
def sedov_similarity(gamma=5.0 / 3.0, j=3, lam_min=1e-4, npts=4000):
    """Self-similar profiles behind a strong shock into a cold uniform gas.

    With R(t) the shock radius, delta = 2 / (j + 2), R' = delta R / t and
    lam = r / R:  u = R' f(lam), rho = rho0 g(lam), p = rho0 R'^2 h(lam).
    Mass, momentum and entropy conservation give
        (f - lam) g' + g (f' + (j - 1) f / lam) = 0
        (delta - 1)/delta f + (f - lam) f' + h' / g = 0
        2 (delta - 1)/delta + (f - lam) (h'/h - gamma g'/g) = 0,
    started from the strong-shock jump f = h = 2/(gamma+1),
    g = (gamma+1)/(gamma-1) at lam = 1.  The energy integral
        E = sigma_j rho0 R'^2 R^j  int_0^1 (g f^2 / 2 + h/(gamma-1)) lam^(j-1) dlam
    fixes xi0 in R = xi0 (E t^2 / rho0)^(1/(j+2)).
    Returns (lam, f, g, h, xi0) with lam increasing."""
    g_ = gamma
    dl = 2.0 / (j + 2.0)
    k = (dl - 1.0) / dl

    def rhs(lam, y):
        f, g, h = y
        D = f - lam
        num = -k * f + (h / (g * D)) * (g_ * (j - 1.0) * f / lam + 2.0 * k)
        den = D - g_ * h / (g * D)
        fp = num / den
        gp = -g * (fp + (j - 1.0) * f / lam) / D
        hp = h * (g_ * gp / g - 2.0 * k / D)
        return [fp, gp, hp]

    y0 = [2.0 / (g_ + 1.0), (g_ + 1.0) / (g_ - 1.0), 2.0 / (g_ + 1.0)]
    lam_eval = np.geomspace(1.0, lam_min, npts)
    sol = solve_ivp(rhs, (1.0, lam_min), y0, t_eval=lam_eval, rtol=1e-11, atol=1e-14, method="DOP853")
    if not sol.success:
        raise RuntimeError(sol.message)
    lam = sol.t[::-1]
    f, g, h = sol.y[0][::-1], sol.y[1][::-1], sol.y[2][::-1]
    integrand = (0.5 * g * f * f + h / (g_ - 1.0)) * lam ** (j - 1)
    # Close the gap [0, lam_min] with the leading power of the integrand.
    integral = np.trapezoid(integrand, lam) + integrand[0] * lam[0] / j
    sigma_j = {1: 2.0, 2: 2.0 * math.pi, 3: 4.0 * math.pi}[j]
    xi0 = (1.0 / (sigma_j * dl * dl * integral)) ** (1.0 / (j + 2.0))
    return lam, f, g, h, xi0


def sedov_profile(r, t, energy=1.0, rho0=1.0, gamma=5.0 / 3.0, j=3, sim=None):
    """(rho, u, p, R) at radius r and time t for a point blast of energy E."""
    lam, f, g, h, xi0 = sedov_similarity(gamma, j) if sim is None else sim
    R = xi0 * (energy * t * t / rho0) ** (1.0 / (j + 2.0))
    Rdot = 2.0 / (j + 2.0) * R / t
    x = np.atleast_1d(np.asarray(r, dtype=np.float64)) / R
    inside = x < 1.0
    rho = np.where(inside, rho0 * np.interp(x, lam, g), rho0)
    u = np.where(inside, Rdot * np.interp(x, lam, f), 0.0)
    p = np.where(inside, rho0 * Rdot * Rdot * np.interp(x, lam, h), 0.0)
    return rho, u, p, R
