"""Pins of the oracle's collider update (Sec. 3, position-update equation)
and of its collisional virial (Sec. 4, stress-tensor equation) against the
geometry of a pair built by hand.

The pair: A at (1.75, 2, 2) moving +x at unit speed, B at
(2.25, 2 + by, 2 + bz) moving -x.  Relative position r = (-0.5, -by, -bz),
relative velocity u = (2, 0, 0), so the point of closest approach is at
t_poca = 0.25 exactly, where A sits at (2, 2, 2) and B at (2, 2 + by, 2 + bz):
their separation, oriented from B to A, is s = (0, -by, -bz).  The step is
dt = 0.75, so the two legs of the split move (t_poca and dt - t_poca = 0.5)
differ and a swap of the old and new velocities shows.  Everything here is a
dyadic rational, exact in binary.  The box [0, 4]^3 is large enough that no
wall is reached."""
import math

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

R = W.REFLECT
TP, DT = 0.25, 0.75
EPS = float(np.finfo(np.float64).eps)
S = np.array([0.0, -0.125, -0.0625])   # separation at closest approach, B -> A
POCA_A = np.array([2.0, 2.0, 2.0])
POCA_B = POCA_A - S


def pair_state(masses=None):
    st = W.make_state(x=[1.75, 2.25], y=[2.0, 2.125], z=[2.0, 2.0625],
                      vx=[1.0, -1.0], vy=[0.0, 0.0], vz=[0.0, 0.0], ids=[0, 1])
    if masses is not None:
        st["mass"] = np.array(masses, dtype=np.float64)
    return st


def run(oracle, seed, masses=None, nobin=(1, 1, 1)):
    st = pair_state(masses)
    v0 = np.array([[st["vx"][k], st["vy"][k], st["vz"][k]] for k in range(2)])
    g = W.grid((0, 0, 0), (4, 4, 4), (1, 1, 1), (R, R, R), nobin)
    # D = 0.25 > |s| = 0.1398: the pair is a candidate.
    p = W.params(sigma=math.pi * 0.0625, dt=DT, seed=seed)
    out = oracle.step(st, g, p)
    assert out["pairs"].tolist() == [[0, 1]]
    r1 = np.array([[st["x"][k], st["y"][k], st["z"][k]] for k in range(2)])
    v1 = np.array([[st["vx"][k], st["vy"][k], st["vz"][k]] for k in range(2)])
    return r1, v0, v1, out, g


def test_pair_geometry_is_as_built(oracle):
    st = pair_state()
    g = W.grid((0, 0, 0), (4, 4, 4), (1, 1, 1), (R, R, R))
    ok, d2, tp = oracle.pair_test(g, W.params(sigma=math.pi * 0.0625, dt=DT),
                                  [st["x"][0], st["y"][0], st["z"][0]], [1.0, 0.0, 0.0],
                                  [st["x"][1], st["y"][1], st["z"][1]], [-1.0, 0.0, 0.0])
    assert ok
    assert tp == TP
    assert d2 == float(S @ S)


@pytest.mark.parametrize("masses", [None, [1.0, 3.0]])
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_colliders_leave_from_their_point_of_closest_approach(oracle, seed, masses):
    """Sec. 3: a collider moves with its old velocity up to t_poca and with
    its new one for the rest of the step.  Running each particle back along
    its new velocity for dt - t_poca must land on the point of closest
    approach that the geometry fixes, the two points the impact parameter
    apart."""
    r1, v0, v1, _, _ = run(oracle, seed, masses)
    assert not np.allclose(v1, v0)
    back = r1 - v1 * (DT - TP)
    tol = 4 * EPS * 4.0
    assert np.all(np.abs(back[0] - POCA_A) <= tol), back[0]
    assert np.all(np.abs(back[1] - POCA_B) <= tol), back[1]
    assert np.all(np.abs((back[0] - back[1]) - S) <= 2 * tol)


@pytest.mark.parametrize("masses", [None, [1.0, 3.0]])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_virial_is_half_separation_times_momentum_change(oracle, seed, masses):
    """Sec. 4, stress tensor: the collisional part adds s_a dp_a / (2 dt) for
    each collider, s the separation at closest approach (from the partner)
    and dp the particle's momentum change; summed over the pair, s dp_A / dt
    since dp_B = -dp_A.  Built from the geometric s, not from the oracle's
    own r + t_poca u."""
    r1, v0, v1, out, _ = run(oracle, seed, masses)
    m = np.array(masses if masses is not None else [1.0, 1.0])
    dpA = m[0] * (v1[0] - v0[0])
    dpB = m[1] * (v1[1] - v0[1])
    assert np.all(np.abs(dpA + dpB) <= 8 * EPS * (np.abs(dpA) + 1.0))
    want = S * dpA / DT
    got = out["moments"][0, 7:10]
    scale = np.abs(S).max() * np.abs(dpA).max() / DT
    assert np.all(np.abs(got - want) <= 8 * EPS * scale), (got, want)
    assert got[0] == 0.0  # no separation along x at closest approach
    assert out["globals"][5] == pytest.approx(float(want.sum()), abs=8 * EPS * scale)
    assert out["moments"][0, 10] == 2.0


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_each_collider_carries_half_the_virial_to_its_own_bin(oracle, seed):
    """With two o-bins along x the colliders end on opposite sides of x = 2
    (they leave along +-n from the same x); each bin then holds one
    collider's term, s dp_A / (2 dt) either way (-s dp_B = s dp_A)."""
    r1, v0, v1, out, g = run(oracle, seed, nobin=(2, 1, 1))
    if r1[0, 0] == r1[1, 0]:
        pytest.skip("direction without an x component")
    dpA = v1[0] - v0[0]
    want = 0.5 * S * dpA / DT
    scale = np.abs(S).max() * np.abs(dpA).max() / DT
    M = out["moments"]
    assert M[0, 0] == 1.0 and M[1, 0] == 1.0
    for b in (0, 1):
        assert np.all(np.abs(M[b, 7:10] - want) <= 8 * EPS * scale), (b, M[b, 7:10], want)
        assert M[b, 10] == 1.0
