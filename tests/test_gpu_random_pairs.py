"""GPU parity of the random-partner mode (TPKMC_PAIR_RANDOM, the usual DSMC
rule of Sec. 2.3) against the oracle.

- FP64: bit-identical state, counters, pair lists and moments over two
  steps, on boxes with walls, periodic and absorbing axes, dense and sparse
  c-bins, a plane, per-particle masses and particles outside the box.
- FP32: the first step from an FP32-exact state forms and accepts exactly
  the oracle's pairs (keys are integers and the acceptance is decided in
  double on both sides); energy and the momentum along the periodic axis
  are kept.
- A batch mixing a closest-approach instance and a random-partner instance
  equals the two separate oracle runs.
- Bad combinations are refused before any launch."""
import sys

import numpy as np
import pytest
import torch

from paper_1210_8084_amd import workloads as W
from test_gpu_parity import assert_outputs_match, assert_state_equal

pytestmark = pytest.mark.gpu

P, R, A = W.PERIODIC, W.REFLECT, W.ABSORB


@pytest.fixture(scope="module")
def T():
    from paper_1210_8084_amd import tpkmc
    assert torch.cuda.is_available(), "GPU test without a visible GPU"
    tpkmc.lib()
    return tpkmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pairset(pairs):
    return sorted(map(tuple, np.asarray(pairs).tolist()))


def _gpu(T, w, precision, steps, flags=None):
    flags = T.EMIT_PAIRS if flags is None else flags
    g = w.grid
    eng = T.Engine(max_particles=max(w.n, 1), max_cells=T.ncells(g) + 1, max_obins=T.nobins(g),
                   precision=precision)
    dst = T.to_device(w.state, precision)
    out = T.make_outputs(1, T.nobins(g), pair_cap=w.n)
    outs = []
    for s in range(steps):
        eng.step(dst, g, dict(w.params, step=s), out, flags=flags)
        torch.cuda.synchronize()
        outs.append(out.host())
    eng.close()
    return T.to_host(dst), outs


def _oracle(oracle, w, steps):
    st = W.copy_state(w.state)
    outs = [oracle.step(st, w.grid, dict(w.params, step=s)) for s in range(steps)]
    return st, outs


def _match(got, gouts, want, routs, mass):
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, mass)


CASES = [
    dict(seed=101, n=3000, ncell=(6, 5, 4), bc=(R, P, P)),
    dict(seed=102, n=2999, ncell=(3, 3, 3), bc=(P, P, P)),
    dict(seed=103, n=4000, ncell=(20, 10, 8), bc=(R, R, R)),
    dict(seed=104, n=3000, ncell=(1, 1, 1), bc=(P, P, P)),
    dict(seed=105, n=3000, ncell=(5, 5, 5), bc=(A, R, A)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp64_random_partners_bit_exact(T, oracle, case):
    w = W.random_box(n=case["n"], seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.1,
                     dt_over=0.1, nobin=(3, 2, 1))
    w.params = dict(w.params, pair_random=True)
    w.state = W.shuffle_state(w.state, seed=case["seed"])
    _say(f"random partners fp64 {case}")
    got, gouts = _gpu(T, w, T.FP64, 2)
    want, routs = _oracle(oracle, w, 2)
    _match(got, gouts, want, routs, w.params["mass"])
    c = routs[0]["counters"]
    assert c[oracle.CNT["tests"]] > 100          # pairs formed
    assert 0 < c[oracle.CNT["pairs"]] <= c[oracle.CNT["tests"]]


def test_fp64_random_partners_plane_masses_outside(T, oracle):
    w = W.random_plane(n=5000, seed=106, ncell=(12, 9), bc=(R, P), d_over_w=0.1, dt_over=0.1)
    w.params = dict(w.params, pair_random=True)
    rng = np.random.default_rng(7)
    w.state["mass"] = rng.uniform(0.5, 2.0, w.n)
    sel = rng.random(w.n) < 0.03
    w.state["x"][sel] = -0.01 * rng.random(int(sel.sum()))   # just outside the wall
    _say("random partners fp64 plane + masses")
    got, gouts = _gpu(T, w, T.FP64, 2)
    want, routs = _oracle(oracle, w, 2)
    _match(got, gouts, want, routs, 2.0)
    assert np.all(got["vz"] == 0.0)


def test_fp32_random_partners_first_step_pairs(T, oracle):
    w = W.random_box(n=20000, seed=107, ncell=(10, 8, 6), bc=(R, R, P), d_over_w=0.15, dt_over=0.1)
    w.params = dict(w.params, pair_random=True)
    # An FP32-exact state: the oracle then sees exactly the GPU's inputs.
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        w.state[k] = w.state[k].astype(np.float32).astype(np.float64)
    _say("random partners fp32 first step")
    got, gouts = _gpu(T, w, T.FP32, 1)
    want, routs = _oracle(oracle, w, 1)
    assert gouts[0]["counters"][0].tolist()[1:4] == routs[0]["counters"].tolist()[1:4]
    assert _pairset(gouts[0]["pairs"]) == _pairset(routs[0]["pairs"])
    m = w.params["mass"]
    # walls along x and y reverse momentum; z is periodic
    assert abs(float(np.sum(got["vz"], dtype=np.float64)) - float(np.sum(w.state["vz"]))) < 1e-3
    e0 = 0.5 * m * sum(float(np.sum(w.state[k] ** 2)) for k in ("vx", "vy", "vz"))
    e1 = 0.5 * m * sum(float(np.sum(got[k].astype(np.float64) ** 2)) for k in ("vx", "vy", "vz"))
    assert e1 == pytest.approx(e0, rel=1e-5)


def test_batch_mixes_the_two_rules(T, oracle):
    ws = [W.random_box(n=3000, seed=108, ncell=(6, 5, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.6),
          W.random_box(n=2500, seed=109, ncell=(5, 4, 3), bc=(R, R, R), d_over_w=0.1, dt_over=0.1)]
    ws[1].params = dict(ws[1].params, pair_random=True)
    for k, w in enumerate(ws):
        w.params = dict(w.params, instance=k, seed=500 + k)
    st = {k: np.concatenate([w.state[k] for w in ws]) for k in ("x", "y", "z", "vx", "vy", "vz", "alive")}
    st["id"] = np.concatenate([ws[0].state["id"], ws[1].state["id"] + np.uint32(ws[0].n)]).astype(np.uint32)
    specs = [(0, ws[0].n, ws[0].grid, ws[0].params), (ws[0].n, ws[1].n, ws[1].grid, ws[1].params)]
    n = ws[0].n + ws[1].n
    eng = T.Engine(max_particles=n, max_cells=sum(T.ncells(w.grid) + 1 for w in ws),
                   max_obins=sum(T.nobins(w.grid) for w in ws), precision=T.FP64, max_instances=2)
    dst = T.to_device(st, T.FP64)
    out = T.make_outputs(2, sum(T.nobins(w.grid) for w in ws), pair_cap=n)
    eng.step_batched(dst, specs, out, flags=T.EMIT_PAIRS)
    torch.cuda.synchronize()
    got, go = T.to_host(dst), out.host()
    eng.close()
    want_pairs = []
    for k, w in enumerate(ws):
        ref = W.copy_state(w.state)
        ref["id"] = st["id"][specs[k][0]:specs[k][0] + w.n].copy()
        ro = oracle.step(ref, w.grid, w.params)
        sl = slice(specs[k][0], specs[k][0] + w.n)
        for key in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(got[key][sl], ref[key]), (k, key)
        assert go["counters"][k].tolist() == ro["counters"].tolist(), k
        want_pairs += _pairset(ro["pairs"])
    assert _pairset(go["pairs"]) == sorted(want_pairs)


def test_random_partners_refuse_contact_ranking(T):
    w = W.random_box(n=100, seed=110)
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(w.grid) + 1, max_obins=T.nobins(w.grid),
                   precision=T.FP64)
    dst = T.to_device(w.state, T.FP64)
    out = T.make_outputs(1, T.nobins(w.grid))
    with pytest.raises(T.TpkmcError):
        eng.step(dst, w.grid, dict(w.params, pair_random=True, rank_time=True), out)
    eng.close()


def test_fp64_random_partners_dense_bins_and_tube(T, oracle):
    """The Sod tube with a few hundred particles per c-bin (the in-bin rank
    loop at its longest): two steps bit-identical to the oracle."""
    w = W.sod(n=200_000, seed=111, ncell=50, nobin=10, dt=1e-4)
    w.params = dict(w.params, pair_random=True)
    _say("random partners fp64 sod 200k, 50 c-bins")
    got, gouts = _gpu(T, w, T.FP64, 2, flags=T.EMIT_PAIRS | T.ALLOW_REORDER)
    want, routs = _oracle(oracle, w, 2)
    # reordered arrays: compare particle by particle
    a, b = np.argsort(got["id"]), np.argsort(want["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k][a], want[k][b]), k
    for go, ro in zip(gouts, routs):
        assert go["counters"][0].tolist() == ro["counters"].tolist()
        assert _pairset(go["pairs"]) == _pairset(ro["pairs"])
    assert routs[0]["counters"][oracle.CNT["pairs"]] > 1000


def test_graph_run_random_partners(T, oracle):
    """tpkmc_run replays the step with the step counter advanced on the
    device: the random keys follow it, as in plain steps and the oracle."""
    w = W.random_box(n=4000, seed=112, ncell=(8, 6, 5), bc=(R, R, P), d_over_w=0.15, dt_over=0.1)
    w.params = dict(w.params, pair_random=True, step=3)
    g = w.grid
    kw = dict(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP64)
    K = 4
    e1 = T.Engine(**kw)
    d1 = T.to_device(w.state, T.FP64)
    o1 = T.make_outputs(1, T.nobins(g))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        e1.run(d1, [(0, w.n, g, w.params)], K, o1, stream=stream)
    stream.synchronize()
    got = T.to_host(d1)
    e1.close()
    ref = W.copy_state(w.state)
    for s in range(K):
        ro = oracle.step(ref, g, dict(w.params, step=3 + s))
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(got[k], ref[k]), k
    assert o1.host()["counters"][0].tolist() == ro["counters"].tolist()
