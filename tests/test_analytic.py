"""Pins of the analytic solutions (Sec. 4.2-4.4) and of the unit
conventions, against numbers the paper prints (tests/golden) and textbook
invariants."""
import json
import math
import os

import numpy as np
import pytest

from oracle import analytic as A

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_sod_star_state_textbook():
    """Toro's test 1 (gamma = 1.4): p* = 0.30313, u* = 0.92745."""
    ps, us = A.riemann_star((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert ps == pytest.approx(0.30313, abs=2e-5)
    assert us == pytest.approx(0.92745, abs=2e-5)


def _state(s, L, R, g, star):
    return A.riemann_sample(s, L, R, g, star)


def test_sod_jump_conditions():
    """Rankine-Hugoniot across the shock, continuity of u and p across the
    contact, constant entropy and Riemann invariant through the fan."""
    g = 5.0 / 3.0
    L, R = (8.0, 0.0, 10.0), (1.0, 0.0, 1.0)
    ps, us = A.riemann_star(L, R, g)
    star = (ps, us)
    rr, ur, pr = R
    rs = _state(us + 1e-9, L, R, g, star)[0]
    S = (rs * us - rr * ur) / (rs - rr)               # mass flux fixes the speed
    e = lambda r, u, p: p / ((g - 1) * r) + 0.5 * u * u
    assert rs * us * (us - S) + ps == pytest.approx(rr * ur * (ur - S) + pr, rel=1e-10)
    assert rs * e(rs, us, ps) * (us - S) + ps * us == pytest.approx(
        rr * e(rr, ur, pr) * (ur - S) + pr * ur, rel=1e-9)
    assert _state(S - 1e-7, L, R, g, star)[0] == pytest.approx(rs, rel=1e-9)
    assert _state(S + 1e-7, L, R, g, star) == pytest.approx(R)
    lft = _state(us - 1e-9, L, R, g, star)
    rgt = _state(us + 1e-9, L, R, g, star)
    assert lft[1] == pytest.approx(rgt[1], rel=1e-12) and lft[2] == pytest.approx(rgt[2], rel=1e-12)
    assert lft[0] > rgt[0]
    aL = math.sqrt(g * L[2] / L[0])
    for s in np.linspace(-aL + 1e-6, us - 1e-3, 7):
        r, u, p = _state(s, L, R, g, star)
        if r == L[0]:
            continue
        assert p / r ** g == pytest.approx(L[2] / L[0] ** g, rel=1e-10)
        assert u + 2 * math.sqrt(g * p / r) / (g - 1) == pytest.approx(2 * aL / (g - 1), rel=1e-10)


def test_sod_equal_states_do_nothing():
    rho, u, p = A.sod_profile(np.linspace(0, 1, 11), 0.1, (2.0, 0.0, 3.0), (2.0, 0.0, 3.0))
    assert np.allclose(rho, 2.0) and np.allclose(u, 0.0, atol=1e-12) and np.allclose(p, 3.0)


def test_sod_normalisation_of_the_2d_run():
    """n_l = (8/9) N / (V/2) and p_l = n_l T_l reproduce the printed numbers,
    which fixes p = n T and the 8:1 split with n_r = 0.125 n_l."""
    s = GOLD["sod_2d"]
    half_area = 0.5 * s["box"][0] * s["box"][1]
    n_l = (1.0 / (1.0 + s["n_r_over_n_l"])) * s["N"] / half_area
    assert n_l == pytest.approx(s["n_l"], rel=2e-3)
    assert n_l * s["T_l"] == pytest.approx(s["p_l"], rel=2e-3)


@pytest.mark.parametrize("key", ["noh_2d", "noh_3d"])
def test_noh_printed_shock_state(key):
    """Shock density, temperature and pressure of the paper's Noh runs,
    from the closed form with T = m v0^2 / f and p = n T."""
    s = GOLD[key]
    n, vr, p, rs = A.noh_profile([1e-6], t=1.0, n0=s["n0"], v0=s["v_r0"], gamma=s["gamma"], d=s["d"], f=s["f"])
    if "n_shock_over_n0" in s:
        assert n[0] / s["n0"] == pytest.approx(s["n_shock_over_n0"], rel=1e-12)
    assert s["v_r0"] ** 2 / s["f"] == pytest.approx(s["T_shock"], rel=1e-12)
    assert p[0] == pytest.approx(s["p_shock"], rel=5e-3)


def test_noh_cylinder_gamma_5_3():
    n, vr, p, rs = A.noh_profile(np.array([0.1, 0.3, 0.5]), t=0.6, n0=1.0, v0=1.0, gamma=5 / 3, d=2)
    assert rs == pytest.approx(0.2)
    assert n[0] == pytest.approx(16.0)
    assert n[1] == pytest.approx(1 + 0.6 / 0.3) and n[2] == pytest.approx(1 + 0.6 / 0.5)
    assert p[0] == pytest.approx(16.0 / 3.0)


def test_sedov_constants():
    """Taylor's xi0 = 1.033 for gamma = 1.4 (spherical); xi0 near 1.15 for
    gamma = 5/3; the shock density n0 (gamma+1)/(gamma-1) of Sec. 4.4."""
    lam, f, g, h, xi0 = A.sedov_similarity(1.4, 3)
    assert xi0 == pytest.approx(1.033, abs=1e-3)
    lam, f, g, h, xi0 = A.sedov_similarity(5 / 3, 3)
    assert 1.14 < xi0 < 1.16
    assert g[-1] == pytest.approx(GOLD["sedov"]["n_shock_over_n0_gamma_5_3"], rel=1e-12)
    assert g[0] < 1e-6


def test_sedov_profile_holds_the_blast_energy():
    sim = A.sedov_similarity(5 / 3, 3)
    E, t = 2.5, 0.3
    rho, u, p, R = A.sedov_profile(np.array([0.0]), t, energy=E, sim=sim)
    r = np.linspace(1e-6, R * (1 - 1e-9), 200001)
    rho, u, p, _ = A.sedov_profile(r, t, energy=E, sim=sim)
    e = 0.5 * rho * u * u + p / (2.0 / 3.0)
    assert np.trapezoid(e * 4 * np.pi * r * r, r) == pytest.approx(E, rel=2e-3)
    mass = np.trapezoid(rho * 4 * np.pi * r * r, r)
    assert mass == pytest.approx(4 / 3 * np.pi * R ** 3, rel=2e-3)
