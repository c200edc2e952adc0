"""Pins of the oracle's random-partner mode (REF_PAIR_RANDOM: the usual DSMC
rule of Sec. 2.3, partners drawn at random inside a scattering cell, in
place of the point-of-closest-approach criteria).

- The pairs form a matching inside each c-bin: every particle in at most one
  pair, both partners in the same c-bin, floor(n_c / 2) pairs per c-bin.
- The matching is uniform: the three matchings of four particles come up
  equally often over many steps (chi-square).
- The collision rate is the kinetic-theory one: summed over steps, the
  colliding pairs equal the sum over c-bins of
  floor(n_c / 2) (n_c - 1) sigma <g> dt / V_c, with <g> the mean relative
  speed of the velocity sample itself (in space and in the plane).  With
  about six particles per c-bin this fixes the acceptance rule (the factor
  n_c - 1 rather than n_c, sigma, dt, the c-bin volume and the direction of
  the comparison) independently of its arithmetic.
- Collisions keep momentum and energy, and a mono-speed gas relaxes to the
  Maxwell-Boltzmann speed distribution.
- The mode cannot be combined with ranking by contact time, and the
  search-only entry points reject it."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1210_8084_amd import workloads as W

P, R = W.PERIODIC, W.REFLECT


def _ncells(g):
    return int(np.prod(g["ncell"]))


def _cells(st, g):
    idx = []
    for a, k in enumerate(("x", "y", "z")):
        t = (st[k] - g["lo"][a]) * (g["ncell"][a] / (g["hi"][a] - g["lo"][a]))
        idx.append(np.clip(np.floor(t), 0, g["ncell"][a] - 1).astype(np.int64))
    return idx[0] + g["ncell"][0] * (idx[1] + g["ncell"][1] * idx[2])


def test_pairs_form_a_matching_inside_each_bin(oracle):
    w = W.random_box(n=3001, seed=31, ncell=(6, 5, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.6)
    st0 = W.copy_state(w.state)
    cell = _cells(st0, w.grid)
    # A huge cross section: every formed pair collides and is listed.
    out = oracle.step(W.copy_state(w.state), w.grid, dict(w.params, sigma=1e6, pair_random=True))
    c = out["counters"]
    counts = np.bincount(cell, minlength=_ncells(w.grid))
    formed = int(np.sum(counts // 2))
    assert c[oracle.CNT["tests"]] == formed
    assert c[oracle.CNT["pairs"]] == formed
    assert c[oracle.CNT["cand"]] == c[oracle.CNT["have_best"]] == 2 * formed
    pairs = np.asarray(out["pairs"])
    ids = pairs.ravel()
    assert len(np.unique(ids)) == len(ids)            # everyone at most once
    assert np.all(pairs[:, 0] < pairs[:, 1])
    pos = {int(i): k for k, i in enumerate(st0["id"])}
    for a, b in pairs:
        assert cell[pos[int(a)]] == cell[pos[int(b)]]


def test_matching_is_uniform(oracle):
    """Four particles in one c-bin: the matchings {01|23}, {02|13},
    {03|12} are equally likely."""
    st = W.make_state([0.1, 0.2, 0.3, 0.4], [0.5] * 4, [0.5] * 4, [1.0, -1.0, 0.5, -0.5], [0.0] * 4, [0.0] * 4)
    g = W.grid((0, 0, 0), (1, 1, 1), (1, 1, 1), (P, P, P))
    p = dict(W.params(sigma=1e6, dt=1e-3, seed=5), pair_random=True)
    seen = {}
    for s in range(3000):
        out = oracle.step(W.copy_state(st), g, dict(p, step=s), moments=False)
        key = tuple(sorted(tuple(map(int, q)) for q in out["pairs"]))
        seen[key] = seen.get(key, 0) + 1
    assert len(seen) == 3
    obs = np.array(list(seen.values()))
    assert stats.chisquare(obs).pvalue > 1e-3


def _mean_pair_speed(V, rng, m):
    i = rng.integers(0, V.shape[1], m)
    j = rng.integers(0, V.shape[1], m)
    keep = i != j
    return float(np.mean(np.sqrt(((V[:, i[keep]] - V[:, j[keep]]) ** 2).sum(axis=0))))


@pytest.mark.parametrize("planar", [False, True])
def test_collision_rate_is_the_kinetic_rate(oracle, planar):
    n, steps = 6000, 30
    rng = np.random.default_rng(17 + planar)
    if planar:
        x, y = rng.uniform(0, 1, size=(2, n))
        v = rng.normal(0.0, 1.0, size=(2, n))
        st = W.make_state(x, y, np.zeros(n), v[0], v[1], np.zeros(n))
        g = W.grid((0, 0, -0.5), (1, 1, 0.5), (30, 30, 1), (P, P, P))
        vol = 1.0 / 900
        sigma = 0.008
    else:
        pos = rng.uniform(0, 1, size=(3, n))
        v = rng.normal(0.0, 1.0, size=(3, n))
        st = W.make_state(*pos, *v)
        g = W.grid((0, 0, 0), (1, 1, 1), (10, 10, 10), (P, P, P))
        vol = 1e-3
        sigma = 0.006
    dt = 2e-3
    p = dict(W.params(sigma=sigma, dt=dt, seed=9), planar=planar, pair_random=True)
    got = want = 0.0
    for s in range(steps):
        V = np.stack([st["vx"], st["vy"]] + ([] if planar else [st["vz"]]))
        gbar = _mean_pair_speed(V, rng, 200_000)
        counts = np.bincount(_cells(st, g), minlength=_ncells(g))
        prob = (counts - 1).clip(min=0) * sigma * gbar * dt / vol
        assert prob.max() < 1.0
        want += float(np.sum((counts // 2) * prob))
        out = oracle.step(st, g, dict(p, step=s), moments=False)
        got += float(out["counters"][oracle.CNT["pairs"]])
    assert want > 1500
    assert abs(got - want) <= 5.0 * math.sqrt(want), (got, want)


def test_random_partners_conserve_and_relax_to_maxwell(oracle):
    n = 20000
    rng = np.random.default_rng(23)
    d = rng.normal(size=(3, n))
    d /= np.sqrt((d * d).sum(axis=0))
    st = W.make_state(*rng.uniform(0, 1, size=(3, n)), *d)
    g = W.grid((0, 0, 0), (1, 1, 1), (4, 4, 4), (P, P, P))
    vol = 1.0 / 64
    # about a quarter of the particles collide per step
    sigma = 0.5 / ((n / 64 - 1) * (4 / math.sqrt(math.pi) / math.sqrt(3.0)) * 0.01 / vol)
    p = dict(W.params(sigma=sigma, dt=0.01, seed=4), pair_random=True)
    e0 = float(np.sum(d * d))
    p0 = d.sum(axis=1)
    for s in range(30):
        out = oracle.step(st, g, dict(p, step=s), moments=False)
    V = np.stack([st["vx"], st["vy"], st["vz"]])
    assert float(np.sum(V * V)) == pytest.approx(e0, rel=1e-12)
    assert np.allclose(V.sum(axis=1), p0, atol=1e-9)
    # Maxwell-Boltzmann with <v^2> = 1: each component normal with variance 1/3
    assert stats.kstest(V[0] * math.sqrt(3.0), "norm").pvalue > 1e-3
    assert out["counters"][oracle.CNT["pairs"]] > 0.1 * n / 2


def test_random_partners_reject_other_uses(oracle):
    w = W.random_box(n=200, seed=41)
    p = dict(w.params, pair_random=True)
    with pytest.raises(ValueError):
        oracle.step(W.copy_state(w.state), w.grid, dict(p, rank_time=True))
    with pytest.raises(ValueError):
        oracle.best(w.state, w.grid, p)
    with pytest.raises(ValueError):
        oracle.step_sample(w.state, w.grid, p, np.arange(5))
