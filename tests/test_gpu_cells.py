"""c-bins split by speed, chosen by the autotuner (S10 of the partner
search).  Two particles of speed at most v_c that meet the criteria of
Sec. 2.4 within a step start at most D + 2 v_c dt apart, so the slow
particles are searched on c-bins refined down to that width and the fast
ones on the configured c-bins against every particle of their configured
neighbourhood; nothing but the search's work changes, at any speeds.

 - FP64: steps on split c-bins equal the oracle's on the configured ones bit
   for bit (state, pairs, counters other than the search's work counters,
   moments): a shock tube; boxes holding a fast population (walls, periodic
   axes including one of three configured c-bins, absorbing walls, the
   plane, contact-time ranking); a tube whose speeds are raised after tuning.
 - Random partners (their draw depends on the c-bin) keep the configured
   c-bins; a planar grid keeps one c-bin on z; the speed bound is 2 v_rms
   for a thermal gas and 6 v_rms for a point blast (bit-exact too).
 - FP32: the tuned handle's pairs equal an untuned handle's, also through a
   captured graph, with fast particles, and inside a batch."""
import math

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R, P, A = W.REFLECT, W.PERIODIC, W.ABSORB
WORK = ("tests", "cand")


@pytest.fixture(scope="module")
def T():
    from paper_1210_8084_amd import tpkmc
    assert torch.cuda.is_available(), "GPU test without a visible GPU"
    tpkmc.lib()
    return tpkmc


def tube(n=20_000, seed=5, planar=False):
    """A shock tube whose cross-section is one periodic c-bin, with a time
    step small enough that the pair reach is a few percent of it."""
    w = (W.sod2d if planar else W.sod)(n=n, seed=seed, ncell=10, nobin=10, dt=1e-4)
    return w


def engine(T, w, precision):
    g = w.grid
    return T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=precision)


def test_fp64_refined_tube_equals_oracle(T, oracle):
    w = tube()
    g, p = w.grid, w.params
    eng = engine(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, g, p)])
    cells = eng.tuned_cells(0)
    print("configured", g["ncell"], "tuned", cells, "speed bound", eng.tuned_speed(0), flush=True)
    assert cells[1] >= 3 and cells[2] >= 3 and np.prod(cells) >= 4 * np.prod(g["ncell"])
    out = T.make_outputs(1, T.nobins(g), pair_cap=w.n)
    st = W.copy_state(w.state)
    for s in range(3):
        eng.step(dst, g, dict(p, step=s), out, flags=T.EMIT_PAIRS)
        torch.cuda.synchronize()
        go = out.host()
        ro = oracle.step(st, g, dict(p, step=s))
        got = T.to_host(dst)
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(got[k], st[k]), (s, k)
        assert sorted(map(tuple, go["pairs"].tolist())) == sorted(map(tuple, np.asarray(ro["pairs"]).tolist()))
        gc, rc = go["counters"][0], ro["counters"]
        for name, k in T.CNT.items():
            if name not in WORK:
                assert gc[k] == rc[k], (s, name)
        assert gc[T.CNT["tests"]] * 4 < rc[T.CNT["tests"]], (gc[T.CNT["tests"]], rc[T.CNT["tests"]])
        assert np.array_equal(go["moments"][:, 0], ro["moments"][:, 0])
        assert rc[T.CNT["pairs"]] > 100
    eng.close()


def test_random_partners_and_plane_keep_their_cells(T):
    w = tube()
    g, p = w.grid, dict(w.params, pair_random=True)
    eng = engine(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, g, p)])
    assert eng.tuned_cells(0) == tuple(g["ncell"]) and eng.tuned_speed(0) == 0.0
    eng.close()
    w2 = tube(planar=True)
    eng = engine(T, w2, T.FP64)
    dst = T.to_device(w2.state, T.FP64)
    eng.autotune(dst, [(0, w2.n, w2.grid, w2.params)])
    c = eng.tuned_cells(0)
    assert c[2] == 1 and c[1] >= 3
    eng.close()


def fast_box(n, seed, ncell, bc, planar=False, rank_time=False, fast_frac=0.001, fast_speed=10.0):
    """A Gaussian gas (unit speed per component) with a fraction of fast
    particles at fast_speed, isotropic; D is a quarter of the smallest
    configured c-bin and the gas moves 2% of it per step, so the slow
    particles' reach lets the autotuner refine their c-bins about 1.5 times
    per axis while the fast ones stay above the speed bound."""
    w = W.random_box(n=n, seed=seed, ncell=ncell, bc=bc, d_over_w=0.25, dt_over=0.02)
    rng = np.random.default_rng(seed + 100)
    fast = rng.random(n) < fast_frac
    d = rng.normal(size=(3, n))
    d /= np.sqrt((d * d).sum(axis=0))
    for k, a in enumerate(("vx", "vy", "vz")):
        w.state[a] = np.where(fast, fast_speed * d[k], w.state[a])
    p = dict(w.params, rank_time=rank_time)
    if planar:
        # In the plane sigma = 2 D.
        wmin = min((h - l) / c for l, h, c in zip(w.grid["lo"], w.grid["hi"], w.grid["ncell"]) if c > 1)
        p = dict(p, planar=True, sigma=2.0 * 0.25 * wmin)
        w.state["z"] = np.full(n, 0.5 * (w.grid["lo"][2] + w.grid["hi"][2]))
        w.state["vz"] = np.zeros(n)
    w.params = p
    return w


def fp64_steps_equal_oracle(T, oracle, w, steps=3, after_tune=None):
    """FP64 steps on the autotuned (split) c-bins against the oracle on the
    configured ones; returns the tuned c-bins and the speed bound."""
    g, p = w.grid, w.params
    eng = engine(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, g, p)])
    cells, vc = eng.tuned_cells(0), eng.tuned_speed(0)
    st = W.copy_state(w.state)
    if after_tune:
        after_tune(st)
        dst = T.to_device(st, T.FP64)
    out = T.make_outputs(1, T.nobins(g), pair_cap=w.n)
    n_fast = 0
    for s in range(steps):
        v = np.sqrt(st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)
        n_fast += int(((v > vc) & (st["alive"] != 0)).sum())
        eng.step(dst, g, dict(p, step=s), out, flags=T.EMIT_PAIRS)
        torch.cuda.synchronize()
        go = out.host()
        ro = oracle.step(st, g, dict(p, step=s))
        got = T.to_host(dst)
        for k in ("x", "y", "z", "vx", "vy", "vz", "alive"):
            assert np.array_equal(got[k], st[k]), (s, k)
        assert sorted(map(tuple, go["pairs"].tolist())) == sorted(map(tuple, np.asarray(ro["pairs"]).tolist()))
        gc, rc = go["counters"][0], ro["counters"]
        for name, k in T.CNT.items():
            if name not in WORK:
                assert gc[k] == rc[k], (s, name)
        assert np.array_equal(go["moments"][:, 0], ro["moments"][:, 0])
        assert rc[T.CNT["pairs"]] > 50
    eng.close()
    return cells, vc, n_fast


CASES = {
    "walls": dict(ncell=(6, 5, 4), bc=(R, R, R)),
    "periodic": dict(ncell=(3, 6, 5), bc=(P, P, P)),
    "absorb": dict(ncell=(6, 5, 4), bc=(A, P, R)),
    "plane": dict(ncell=(8, 6, 1), bc=(R, P, P), planar=True),
    "contact time": dict(ncell=(6, 5, 4), bc=(P, R, P), rank_time=True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_split_with_fast_particles_equals_oracle(T, oracle, case):
    kw = dict(CASES[case])
    w = fast_box(n=24_000, seed=41, **kw)
    cells, vc, n_fast = fp64_steps_equal_oracle(T, oracle, w)
    print(case, "configured", w.grid["ncell"], "tuned", cells, "speed bound", vc, "fast", n_fast, flush=True)
    refined = [a for a in range(3) if cells[a] > w.grid["ncell"][a]]
    assert len(refined) >= 2 and vc > 0.0
    assert n_fast > 60


def small_blast():
    return W.sedov(n=30_000, seed=3, kn=1e-2, ncell=8, nobin=4)


def test_speed_bound_follows_the_energy(T):
    """A thermal gas takes the bound 2 v_rms; a point blast, whose few fast
    particles hold nearly all the kinetic energy (more than half of it above
    2 v_rms), takes 6 v_rms, above which at most 1/36 of the particles can
    ever be while the energy is conserved."""
    for w, factor in ((fast_box(n=30_000, seed=4, ncell=(8, 8, 8), bc=(R, R, R), fast_frac=0.0), 2.0),
                      (small_blast(), 6.0)):
        eng = engine(T, w, T.FP32)
        dst = T.to_device(w.state, T.FP32)
        eng.autotune(dst, [(0, w.n, w.grid, w.params)])
        st = W.copy_state(w.state, dtype=np.float32)
        v_rms = math.sqrt(float(np.mean(st["vx"].astype(np.float64) ** 2 + st["vy"].astype(np.float64) ** 2
                                        + st["vz"].astype(np.float64) ** 2)))
        assert np.prod(eng.tuned_cells(0)) > np.prod(w.grid["ncell"])
        assert abs(eng.tuned_speed(0) - factor * v_rms) <= 1e-9 * factor * v_rms, (eng.tuned_speed(0), v_rms)
        eng.close()


def test_fp64_blast_split_equals_oracle(T, oracle):
    """The blast on its split c-bins: its blast particles are the fast ones
    at first, then the particles they heat."""
    w = small_blast()
    cells, vc, n_fast = fp64_steps_equal_oracle(T, oracle, w, steps=3)
    assert np.prod(cells) > np.prod(w.grid["ncell"]) and n_fast >= 30


def test_fp64_speeds_raised_after_tuning_equal_oracle(T, oracle):
    """Tuned on a cold tube; then a tenth of the particles move 30 times
    faster, far above the speed bound: they are searched on the configured
    c-bins and the steps still equal the oracle's."""
    w = tube()

    def raise_speeds(st):
        sel = np.arange(w.n) % 10 == 3
        for k in ("vx", "vy", "vz"):
            st[k] = np.where(sel, 30.0 * st[k], st[k])

    cells, vc, n_fast = fp64_steps_equal_oracle(T, oracle, w, after_tune=raise_speeds)
    assert np.prod(cells) > np.prod(w.grid["ncell"]) and n_fast > 1000

def _fp32_pairs(T, w, tune, steps=2, graph=False):
    g, p = w.grid, w.params
    eng = engine(T, w, T.FP32)
    dst = T.to_device(w.state, T.FP32)
    if tune:
        eng.autotune(dst, [(0, w.n, g, p)])
    else:
        eng.set_search(2, 64)
    out = T.make_outputs(1, T.nobins(g), pair_cap=w.n)
    pairs = []
    for s in range(steps):
        if graph:
            eng.run(dst, [(0, w.n, g, dict(p, step=s))], 1, out, flags=T.EMIT_PAIRS)
        else:
            eng.step(dst, g, dict(p, step=s), out, flags=T.EMIT_PAIRS)
        torch.cuda.synchronize()
        pairs.append(set(map(tuple, out.host()["pairs"].tolist())))
    cells = eng.tuned_cells(0) if tune else None
    eng.close()
    return pairs, cells


@pytest.mark.parametrize("graph", [False, True], ids=["step", "graph"])
@pytest.mark.parametrize("kind", ["tube", "fast particles"])
def test_fp32_tuned_cells_keep_the_pairs(T, graph, kind):
    w = tube(n=60_000, seed=7) if kind == "tube" else fast_box(n=60_000, seed=8, ncell=(6, 5, 4), bc=(R, P, P))
    ref, _ = _fp32_pairs(T, w, tune=False)
    got, cells = _fp32_pairs(T, w, tune=True, graph=graph)
    assert np.prod(cells) > np.prod(w.grid["ncell"])
    for a, b in zip(ref, got):
        # Equal up to exact ties of d_min^2, broken by record order.
        assert len(a ^ b) <= 1e-3 * len(a), (len(a), len(a ^ b))
        assert len(a) > 1000


def test_batch_refines_each_position_by_its_own_instance(T):
    """A refinable tube and a random-partner box in one batch: the tube's
    position is refined, the box's keeps its c-bins, and the tube's FP64
    steps still equal its steps alone on the configured c-bins."""
    t = tube(n=12_000, seed=9)
    b = W.random_box(n=3000, seed=10, ncell=(3, 3, 3), bc=(P, P, P), d_over_w=0.6, dt_over=0.5)
    b.state["id"] = b.state["id"] + np.uint32(1_000_000)
    bp = dict(b.params, pair_random=True, instance=1)
    st = {k: np.concatenate([t.state[k], b.state[k]]) for k in ("x", "y", "z", "vx", "vy", "vz", "id", "alive")}
    specs = [(0, t.n, t.grid, t.params), (t.n, b.n, b.grid, bp)]
    eng = T.Engine(max_particles=t.n + b.n, max_cells=T.ncells(t.grid) + T.ncells(b.grid) + 2,
                   max_obins=T.nobins(t.grid) + T.nobins(b.grid), precision=T.FP64, max_instances=2)
    dst = T.to_device(st, T.FP64)
    eng.autotune(dst, specs)
    assert np.prod(eng.tuned_cells(0)) > np.prod(t.grid["ncell"])
    assert eng.tuned_cells(1) == tuple(b.grid["ncell"])
    out = T.make_outputs(2, T.nobins(t.grid) + T.nobins(b.grid))
    eng.step_batched(dst, specs, out)
    torch.cuda.synchronize()
    got = T.to_host(dst)
    eng.close()
    alone = T.Engine(max_particles=t.n, max_cells=T.ncells(t.grid) + 1, max_obins=T.nobins(t.grid),
                     precision=T.FP64)
    d1 = T.to_device(t.state, T.FP64)
    alone.step(d1, t.grid, t.params, T.make_outputs(1, T.nobins(t.grid)))
    torch.cuda.synchronize()
    ref = T.to_host(d1)
    alone.close()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k][:t.n], ref[k]), k


def test_search_order_is_results_neutral(T):
    """The search's work-group order (contiguous per XCD, or chunks dealt
    round-robin) changes no result: FP64 states and pairs of a two-instance
    batch are bit-identical under every order, over full rounds and the
    partial last one."""
    t = tube(n=100_000, seed=11)
    b = W.random_box(n=40_000, seed=12, ncell=(8, 8, 8), bc=(P, R, P), d_over_w=0.6, dt_over=0.5)
    b.state["id"] = b.state["id"] + np.uint32(1_000_000)
    st = {k: np.concatenate([t.state[k], b.state[k]]) for k in ("x", "y", "z", "vx", "vy", "vz", "id", "alive")}
    specs = [(0, t.n, t.grid, t.params), (t.n, b.n, b.grid, dict(b.params, instance=1))]
    ref = None
    for order in (0, 1, 16, 128):
        eng = T.Engine(max_particles=t.n + b.n, max_cells=T.ncells(t.grid) + T.ncells(b.grid) + 2,
                       max_obins=T.nobins(t.grid) + T.nobins(b.grid), precision=T.FP64, max_instances=2)
        eng.set_search(2, 64)
        eng.set_search_order(order)
        assert eng.search_order() == order
        dst = T.to_device(st, T.FP64)
        out = T.make_outputs(2, T.nobins(t.grid) + T.nobins(b.grid), pair_cap=t.n + b.n)
        pairs = []
        for s in range(2):
            eng.step_batched(dst, [(o, c, g, dict(p, step=s)) for o, c, g, p in specs], out, flags=T.EMIT_PAIRS)
            torch.cuda.synchronize()
            pairs.append(sorted(map(tuple, out.host()["pairs"].tolist())))
        got = T.to_host(dst)
        eng.set_search(2, 64)
        assert eng.search_order() == 16  # fixing the shape resets the order to the default
        eng.close()
        if ref is None:
            ref = (got, pairs)
            assert len(pairs[0]) > 1000
            continue
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(got[k], ref[0][k]), (order, k)
        assert pairs == ref[1], order
