"""Pins of the oracle's alternative criterion 3 (Sec. 2.4: the final partner
can be chosen by the shortest collision time instead of the smallest
distance).  The collision time is the earlier overlap time t_o1, the first
contact of the effective radii.

- A hand-built case where the two rules must disagree.
- Brute force against numpy's own polynomial roots of the overlap quadratic,
  |u|^2 t^2 + 2 (u.r) t + |r|^2 - D^2 = 0, on random systems.
- The candidate set does not depend on the ranking."""
import math

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

P, R = W.PERIODIC, W.REFLECT


def test_time_and_distance_rankings_disagree_where_they_must(oracle):
    """A moves along +x at speed 1.  B sits 0.3 ahead, 0.05 off axis, and is
    touched first, at t_o1 = 0.3 - sqrt(0.1^2 - 0.05^2).  C sits 0.5 ahead on
    the axis: d_min = 0, touched at t = 0.4."""
    st = W.make_state([0.0, 0.3, 0.5], [0.0, 0.05, 0.0], [0.0, 0.0, 0.0],
                      [1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    g = W.grid((-1, -1, -1), (2, 2, 2), (1, 1, 1), (R, R, R))
    D = 0.1
    p = W.params(sigma=math.pi * D * D, dt=1.0)
    b_dist, d2_dist = oracle.best(st, g, p, oracle.MODE_ALL)
    b_time, d2_time = oracle.best(st, g, dict(p, rank_time=True), oracle.MODE_ALL)
    assert b_dist[0] == 2 and d2_dist[0] == 0.0
    assert b_time[0] == 1 and d2_time[0] == pytest.approx(0.05 ** 2, rel=1e-12)
    # B and C each see only A as a candidate
    assert b_dist[1] == b_time[1] == 0 and b_dist[2] == b_time[2] == 0


@pytest.mark.parametrize("seed,bc", [(1, (P, P, P)), (2, (R, P, R))])
def test_earliest_contact_by_brute_force(oracle, seed, bc):
    """For every particle, the partner chosen by time is the candidate whose
    smaller root of the overlap quadratic (numpy.roots) is the smallest."""
    w = W.random_box(n=400, seed=seed, ncell=(3, 3, 3), bc=bc, d_over_w=0.8, dt_over=0.8)
    st, g, p = w.state, w.grid, dict(w.params, rank_time=True)
    b, _ = oracle.best(st, g, p, oracle.MODE_ALL)
    D2 = p["sigma"] / math.pi
    L = np.array([h - l for l, h in zip(g["lo"], g["hi"])])
    per = np.array([c == P for c in g["bc"]])
    n = w.n
    checked = 0
    for i in range(n):
        ri = np.array([st[k][i] for k in ("x", "y", "z")])
        vi = np.array([st[k][i] for k in ("vx", "vy", "vz")])
        best_t, best_j = math.inf, -1
        for j in range(n):
            if j == i:
                continue
            rj = np.array([st[k][j] for k in ("x", "y", "z")])
            vj = np.array([st[k][j] for k in ("vx", "vy", "vz")])
            ok, _, _ = oracle.pair_test(g, w.params, ri, vi, rj, vj)
            if not ok:
                continue
            r = ri - rj
            r = np.where(per & (r > L / 2), r - L, np.where(per & (r < -L / 2), r + L, r))
            u = vi - vj
            roots = np.roots([u @ u, 2.0 * (u @ r), r @ r - D2])
            t1 = float(np.min(roots.real))
            if t1 < best_t:
                best_t, best_j = t1, j
        assert b[i] == best_j, i
        checked += best_j >= 0
    assert checked > 100


def test_ranking_leaves_the_candidates_alone(oracle):
    w = W.random_box(n=3000, seed=3, ncell=(6, 5, 4), d_over_w=0.7, dt_over=0.6)
    o_d = oracle.step(W.copy_state(w.state), w.grid, w.params)
    o_t = oracle.step(W.copy_state(w.state), w.grid, dict(w.params, rank_time=True))
    c = oracle.CNT
    for k in ("tests", "cand", "have_best", "alive"):
        assert o_d["counters"][c[k]] == o_t["counters"][c[k]]
    assert o_t["counters"][c["pairs"]] > 200 and o_d["counters"][c["pairs"]] > 200
    # with many candidates per particle the two rules pick different matchings
    assert set(map(tuple, o_d["pairs"].tolist())) != set(map(tuple, o_t["pairs"].tolist()))
