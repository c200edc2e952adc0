"""Results-neutral c-bins chosen by the autotuner (S10 of the partner
search): where a c-bin is at least D + 2 v_max dt wide on an axis, every pair
that can meet the criteria of Sec. 2.4 in a step lies inside the stencil, so
c-bins refined down to that width (with a margin) change nothing but the
search's work.

 - FP64: after autotune refines a tube's c-bins, steps equal the oracle's on
   the configured c-bins bit for bit (state, pairs, counters other than the
   search's work counters), with far fewer pair tests.
 - Random partners (their draw depends on the c-bin) keep the configured
   c-bins; a planar grid keeps one c-bin on z.
 - Each step checks the reach with its own v_max: speeds raised after
   tuning set TPKMC_STATUS_CELLS.
 - FP32: the tuned handle's pairs equal an untuned handle's, also through a
   captured graph and inside a batch."""
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
    print("configured", g["ncell"], "tuned", cells, flush=True)
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
    assert eng.status() & T.STATUS_CELLS == 0
    eng.close()


def test_random_partners_and_plane_keep_their_cells(T):
    w = tube()
    g, p = w.grid, dict(w.params, pair_random=True)
    eng = engine(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, g, p)])
    assert eng.tuned_cells(0) == tuple(g["ncell"])
    eng.close()
    w2 = tube(planar=True)
    eng = engine(T, w2, T.FP64)
    dst = T.to_device(w2.state, T.FP64)
    eng.autotune(dst, [(0, w2.n, w2.grid, w2.params)])
    c = eng.tuned_cells(0)
    assert c[2] == 1 and c[1] >= 3
    eng.close()


def test_speeds_beyond_the_tuned_reach_are_flagged(T):
    w = tube()
    g, p = w.grid, w.params
    eng = engine(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, g, p)])
    out = T.make_outputs(1, T.nobins(g))
    eng.step(dst, g, p, out)
    assert eng.status() & T.STATUS_CELLS == 0
    for k in ("vx", "vy", "vz"):
        dst[k].mul_(8.0)
    eng.step(dst, g, dict(p, step=1), out)
    assert eng.status() & T.STATUS_CELLS
    eng.close()


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
def test_fp32_tuned_cells_keep_the_pairs(T, graph):
    w = tube(n=60_000, seed=7)
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
        assert eng.search_order() == 0  # fixing the shape resets the order
        eng.close()
        if ref is None:
            ref = (got, pairs)
            assert len(pairs[0]) > 1000
            continue
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(got[k], ref[0][k]), (order, k)
        assert pairs == ref[1], order
