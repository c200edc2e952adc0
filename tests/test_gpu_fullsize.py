"""GPU checks of the FP32 path and of the full-size workloads.

FP32 handle: not bit-comparable with the FP64 oracle, so it is checked by
properties (per-collision conservation to FP32 rounding, pair validity under
the FP64 criteria, free streaming) and statistics (collision fraction).

Full sizes (16M-particle Sedov, 4M Sod, 8M Noh, the 4M 2D blast, the 8M
spherical Noh, the 16M Sedov with the adaptive time step): one step in the launch
configuration of the benchmark; sampled particles are recomputed one by one
by the oracle (their closest candidates, their partners' closest candidates,
their post-step state)."""
import math
import sys

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R, P, A = W.REFLECT, W.PERIODIC, W.ABSORB
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def T():
    from paper_1210_8084_amd import tpkmc
    assert torch.cuda.is_available(), "GPU test without a visible GPU"
    tpkmc.lib()
    return tpkmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rounded32(state):
    """The FP32 input as the FP32 handle sees it, widened back to float64."""
    out = W.copy_state(state)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        out[k] = state[k].astype(np.float32).astype(np.float64)
    return out


def one_step(T, w, precision, flags, state=None, pair_cap=None):
    g = w.grid
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=precision)
    dst = T.to_device(w.state if state is None else state, precision)
    cap = (w.n // 2 + 1) if pair_cap is None else pair_cap
    out = T.make_outputs(1, T.nobins(g), pair_cap=cap)
    eng.step(dst, g, w.params, out, flags=flags)
    torch.cuda.synchronize()
    host, o = T.to_host(dst), out.host()
    eng.close()
    del dst
    torch.cuda.empty_cache()
    return host, o


# ---------------------------------------------------------------- FP32
def test_fp32_per_collision_conservation(T):
    w = W.random_box(n=20000, seed=3, ncell=(10, 10, 10), bc=(P, P, P), d_over_w=0.8, dt_over=0.5)
    st0 = rounded32(w.state)
    got, o = one_step(T, w, T.FP32, T.EMIT_PAIRS)
    pairs = o["pairs"]
    assert len(pairs) > 2000
    idx0 = np.argsort(st0["id"])
    idx1 = np.argsort(got["id"])
    v0 = np.stack([st0[k][idx0] for k in ("vx", "vy", "vz")], axis=1)
    v1 = np.stack([got[k][idx1] for k in ("vx", "vy", "vz")], axis=1)
    a, b = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    scale = np.linalg.norm(v0[a], axis=1) + np.linalg.norm(v0[b], axis=1)
    dp = np.abs((v1[a] + v1[b]) - (v0[a] + v0[b])).max(axis=1)
    assert np.all(dp <= 8 * EPS32 * scale)
    e0 = (v0[a] ** 2).sum(1) + (v0[b] ** 2).sum(1)
    e1 = (v1[a] ** 2).sum(1) + (v1[b] ** 2).sum(1)
    assert np.all(np.abs(e1 - e0) <= 16 * EPS32 * e0)
    # Global FP64 sums of the FP32 state: energy kept to FP32 rounding.
    ek0 = 0.5 * float((v0 ** 2).sum())
    assert o["globals"][0][3] == pytest.approx(ek0, rel=1e-6)


def test_fp32_pairs_satisfy_the_criteria(T, oracle):
    """Every FP32 pair passes the FP64 three-criterion test on the same
    (FP32-rounded) input, up to FP32 rounding at the boundaries."""
    w = W.random_box(n=20000, seed=4, ncell=(10, 8, 6), bc=(R, P, P), d_over_w=0.7, dt_over=0.5)
    st0 = rounded32(w.state)
    got, o = one_step(T, w, T.FP32, T.EMIT_PAIRS, state=st0)
    idx = np.argsort(st0["id"])
    D2 = w.params["sigma"] / math.pi
    strict = 0
    for a, b in o["pairs"][:3000]:
        ia, ib = idx[a], idx[b]
        ri = [st0[k][ia] for k in ("x", "y", "z")]
        vi = [st0[k][ia] for k in ("vx", "vy", "vz")]
        rj = [st0[k][ib] for k in ("x", "y", "z")]
        vj = [st0[k][ib] for k in ("vx", "vy", "vz")]
        ok, d2, tp = oracle.pair_test(w.grid, w.params, ri, vi, rj, vj)
        if ok:
            strict += 1
            continue
        loose = dict(w.params, sigma=w.params["sigma"] * (1 + 1e-4), dt=w.params["dt"] * (1 + 1e-4))
        assert oracle.pair_test(w.grid, loose, ri, vi, rj, vj)[0]
    assert strict >= 0.995 * min(3000, len(o["pairs"]))


def test_fp32_collision_fraction_matches_oracle(T, oracle):
    """Same initial state, FP32 GPU vs FP64 oracle: the fraction of
    colliding particles per step agrees to statistical noise."""
    w = W.equilibration(n=40000, seed=5, lam_over_dx=1e-3, ncell=(16, 16, 16))
    g = w.grid
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP32)
    dst = T.to_device(w.state, T.FP32)
    out = T.make_outputs(1, T.nobins(g))
    st = W.copy_state(w.state)
    fg, fo = [], []
    for s in range(8):
        p = dict(w.params, step=s)
        eng.step(dst, g, p, out)
        torch.cuda.synchronize()
        fg.append(2 * out.host()["counters"][0][1] / w.n)
        fo.append(2 * oracle.step(st, g, p)["counters"][1] / w.n)
    eng.close()
    assert abs(np.mean(fg) - np.mean(fo)) < 0.01
    assert 0.4 < np.mean(fg) < 0.7


def test_fp32_free_streaming(T, oracle):
    w = W.random_box(n=5000, seed=6, ncell=(4, 4, 4), bc=(R, P, R), dt_over=1.0)
    w.params["sigma"] = 0.0
    st0 = rounded32(w.state)
    got, o = one_step(T, w, T.FP32, 0, state=st0)
    want = W.copy_state(st0)
    oracle.step(want, w.grid, w.params)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(got[k], want[k], rtol=0, atol=4 * EPS32)
    for k in ("vx", "vy", "vz"):
        assert np.array_equal(np.abs(got[k]), np.abs(st0[k]))
    assert o["counters"][0][1] == 0


# ---------------------------------------------------------------- full sizes
def _sampled_parity(T, oracle, w, precision, flags, nsample, seed):
    st_in = w.state if precision == T.FP64 else rounded32(w.state)
    _say(f"{w.name} n={w.n} precision={precision}: GPU step")
    got, o = one_step(T, w, precision, flags, state=st_in, pair_cap=0)
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(w.n, size=nsample, replace=False))
    _say("oracle sample")
    ref, partner, alive = oracle.step_sample(st_in, w.grid, w.params, sample)
    inv = np.empty(w.n, dtype=np.int64)
    inv[got["id"].astype(np.int64)] = np.arange(w.n)
    rows = inv[st_in["id"][sample].astype(np.int64)]
    g = np.stack([got[k][rows] for k in ("x", "y", "z", "vx", "vy", "vz")], axis=1)
    return got, o, sample, ref, partner, alive, g


def _sedov_adaptive():
    w = W.sedov()
    w.params = dict(w.params, dt=1.0, adaptive_dt=True)
    return w


@pytest.mark.parametrize("make", [
    lambda: W.sedov(),
    lambda: W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4),
    lambda: W.noh(),
    lambda: W.sedov2d(),
    lambda: W.noh3d(),
    _sedov_adaptive,
], ids=["sedov16M", "sod4M", "noh8M", "sedov2d4M", "noh3d8M", "sedov16M-adaptive"])
def test_fp64_fullsize_sampled_bit_exact(T, oracle, make):
    w = make()
    got, o, sample, ref, partner, alive, g = _sampled_parity(T, oracle, w, T.FP64, T.ALLOW_REORDER, 3000, 1)
    assert np.array_equal(g, ref), f"{np.sum(np.any(g != ref, axis=1))} sampled particles differ"
    c = o["counters"][0]
    assert c[0] == w.n
    assert c[2] == oracle.count_tests(w.state, w.grid)
    assert o["globals"][0][7] == oracle.step_dt(w.state, w.grid, w.params)
    frac = (partner >= 0).mean()
    assert abs(2 * c[1] / w.n - frac) < 5 * math.sqrt(frac * (1 - frac) / len(sample)) + 1e-3
    del got


def test_fp32_sedov_16M_sampled(T, oracle):
    """The benchmark's configuration (FP32, records kept in c-bin order,
    moments on): sampled particles against the FP64 oracle on the same
    FP32-rounded input."""
    w = W.sedov()
    got, o, sample, ref, partner, alive, g = _sampled_parity(
        T, oracle, w, T.FP32, T.ALLOW_REORDER, 4000, 2)
    st_in = rounded32(w.state)
    rows = np.arange(len(sample))
    pos_tol = 8 * EPS32 * (1.0 + np.abs(ref[:, 3:]).max() * w.params["dt"])
    same = np.all(np.abs(g[:, :3] - ref[:, :3]) <= pos_tol, axis=1)
    collided_ref = partner >= 0
    # Free-streaming samples agree to FP32 rounding; colliders move to the
    # same place up to the (rare) FP32 tie or boundary decisions.
    assert same[~collided_ref].mean() > 0.999
    assert same.mean() > 0.99
    c = o["counters"][0]
    assert c[0] == w.n
    assert abs(int(c[2]) - oracle.count_tests(st_in, w.grid)) <= 1e-5 * c[2]
    frac = collided_ref.mean()
    assert abs(2 * c[1] / w.n - frac) < 5 * math.sqrt(max(frac * (1 - frac), 1e-4) / len(rows)) + 2e-3
    m = o["moments"]
    assert m[:, 0].sum() == w.n
    assert o["globals"][0][3] == pytest.approx(1.0 + 0.5 * (w.n - w.info["n_blast"]) / w.n *
                                               (1e-3 * w.info["v_blast"]) ** 2, rel=1e-4)


@pytest.mark.parametrize("make", [
    lambda: W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4),
    lambda: W.noh(),
], ids=["sod4M", "noh8M"])
def test_fp64_fullsize_trajectory_sampled_bit_exact(T, oracle, make):
    """Five FP64 steps of the dense full-size runs: every transition is
    checked on the GPU's own state before the step, so the GPU FP64 path
    follows the oracle's trajectory bit for bit on these configurations
    (sampled particles and their partners, the test count, the time step).
    This is what lets whole runs at these sizes use the GPU FP64 path in
    place of the oracle, which is too slow for them."""
    w = make()
    g = w.grid
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP64)
    dst = T.to_device(w.state, T.FP64)
    out = T.make_outputs(1, T.nobins(g), pair_cap=w.n // 2 + 1)
    rng = np.random.default_rng(5)
    for s in range(5):
        p = dict(w.params, step=s)
        before = T.to_host(dst)
        _say(f"{w.name} n={w.n} FP64 step {s}")
        eng.step(dst, g, p, out, flags=T.ALLOW_REORDER | T.EMIT_PAIRS)
        torch.cuda.synchronize()
        after = T.to_host(dst)
        o = out.host()
        # 1000 particles at random and 1000 of the GPU's colliders (the
        # cold inflow of the implosion's first steps collides rarely).
        inv0 = np.empty(w.n, dtype=np.int64)
        inv0[before["id"].astype(np.int64)] = np.arange(w.n)
        coll = inv0[o["pairs"].ravel().astype(np.int64)]
        pick = rng.choice(coll, size=min(1000, len(coll)), replace=False) if len(coll) else coll
        sample = np.unique(np.concatenate([rng.choice(w.n, size=1000, replace=False), pick]))
        ref, partner, alive = oracle.step_sample(before, g, p, sample)
        inv = np.empty(w.n, dtype=np.int64)
        inv[after["id"].astype(np.int64)] = np.arange(w.n)
        rows = inv[before["id"][sample].astype(np.int64)]
        got = np.stack([after[k][rows] for k in ("x", "y", "z", "vx", "vy", "vz")], axis=1)
        assert np.array_equal(got, ref), f"step {s}: {np.sum(np.any(got != ref, axis=1))} sampled particles differ"
        c = o["counters"][0]
        assert c[2] == oracle.count_tests(before, g)
        assert c[0] == w.n
        assert c[1] > 0
        # every sampled GPU collider has the oracle's partner
        assert (partner[np.isin(sample, pick)] >= 0).all()
        _say(f"  {len(sample)} sampled, {int((partner >= 0).sum())} colliders, {int(c[1])} pairs")
    eng.close()
    del dst
    torch.cuda.empty_cache()
