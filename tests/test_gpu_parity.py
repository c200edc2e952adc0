"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP64 handle: accepted pairs, post-step state (bit for bit), alive flags and
counters must equal the oracle's; global sums and moments agree to rounding
(they are summed in a different order).  Inputs span several work-groups,
ragged tails, every boundary type, degenerate grids (1 or 2 periodic bins),
empty and dead inputs."""
import math
import sys

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R, P, A = W.REFLECT, W.PERIODIC, W.ABSORB


@pytest.fixture(scope="module")
def T():
    from paper_1210_8084_amd import tpkmc
    assert torch.cuda.is_available(), "GPU test without a visible GPU"
    tpkmc.lib()
    return tpkmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def engine_for(T, w, precision, n_inst=1):
    g = w.grid
    return T.Engine(max_particles=max(w.n, 1), max_cells=T.ncells(g) + 1, max_obins=T.nobins(g),
                    precision=precision, max_instances=n_inst)


def gpu_steps(T, w, precision, steps=1, flags=None, pair_cap=None, state=None, shape=None):
    flags = T.EMIT_PAIRS if flags is None else flags
    eng = engine_for(T, w, precision)
    if shape is not None:
        eng.set_search(*shape)
    dst = T.to_device(w.state if state is None else state, precision)
    cap = w.n // 2 + 1 if pair_cap is None else pair_cap
    out = T.make_outputs(1, T.nobins(w.grid), pair_cap=cap)
    outs = []
    for s in range(steps):
        p = dict(w.params, step=w.params.get("step", 0) + s)
        eng.step(dst, w.grid, p, out, flags=flags)
        torch.cuda.synchronize()
        outs.append(out.host())
    status = eng.status()
    eng.close()
    return T.to_host(dst), outs, status


def oracle_steps(oracle, w, steps=1):
    st = W.copy_state(w.state)
    outs = []
    for s in range(steps):
        p = dict(w.params, step=w.params.get("step", 0) + s)
        outs.append(oracle.step(st, w.grid, p))
    return st, outs


def pairset(pairs):
    return sorted(map(tuple, np.asarray(pairs).tolist()))


def assert_state_equal(got, want, exact=True):
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        if exact:
            bad = np.flatnonzero(~((got[k] == want[k]) | (np.isnan(got[k]) & np.isnan(want[k]))))
            assert bad.size == 0, f"{k}: {bad.size} differ, first {bad[:5]} got {got[k][bad[:3]]} want {want[k][bad[:3]]}"
    assert np.array_equal(got["id"], want["id"])
    assert np.array_equal(got["alive"], want["alive"])


def assert_outputs_match(go, ro, mass):
    gc, rc = go["counters"][0], ro["counters"]
    assert gc.tolist() == rc.tolist(), f"counters {gc} vs {rc}"
    assert pairset(go["pairs"]) == pairset(ro["pairs"])
    gg, rg = go["globals"][0], ro["globals"]
    scale = abs(rg[3]) + 1e-300
    for k in (0, 1, 2):
        assert abs(gg[k] - rg[k]) <= 1e-12 * math.sqrt(scale * rg[6] * 2) + 1e-300
    for k in (3, 6):
        assert gg[k] == pytest.approx(rg[k], rel=1e-13)
    assert gg[4] == rg[4]
    assert gg[7] == rg[7]  # the time step used
    assert gg[5] == pytest.approx(rg[5], rel=1e-9, abs=1e-12 * scale)
    gm, rm = go["moments"], ro["moments"]
    assert np.array_equal(gm[:, 0], rm[:, 0])
    assert np.array_equal(gm[:, 10], rm[:, 10])
    np.testing.assert_allclose(gm[:, 11], rm[:, 11], rtol=1e-12, atol=0)
    # Sums over up to a few thousand particles in another order: relative
    # error ~ count * eps of the largest magnitude involved.
    vmax = math.sqrt(rg[4])
    for a in range(3):
        tol_p = 1e-12 * mass * rm[:, 0].max() * vmax
        np.testing.assert_allclose(gm[:, 1 + a], rm[:, 1 + a], rtol=0, atol=tol_p)
        np.testing.assert_allclose(gm[:, 4 + a], rm[:, 4 + a], rtol=1e-9, atol=tol_p * vmax)
        np.testing.assert_allclose(gm[:, 7 + a], rm[:, 7 + a], rtol=1e-9,
                                   atol=1e-12 * (abs(rm[:, 7 + a]).max() + 1e-300))


CASES = [
    dict(seed=1, ncell=(6, 5, 4), bc=(R, P, P)),
    dict(seed=2, ncell=(3, 3, 3), bc=(P, P, P)),
    dict(seed=3, ncell=(2, 1, 5), bc=(P, P, R)),
    dict(seed=4, ncell=(1, 1, 1), bc=(P, P, P)),
    dict(seed=5, ncell=(7, 2, 3), bc=(R, R, R)),
    dict(seed=6, ncell=(9, 4, 1), bc=(P, R, P)),
    dict(seed=7, ncell=(5, 5, 5), bc=(A, R, A)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
@pytest.mark.parametrize("n", [1000, 2999])
def test_fp64_one_step_bit_exact(T, oracle, case, n):
    w = W.random_box(n=n, seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.7, dt_over=0.6,
                     nobin=(3, 2, 1))
    w.state = W.shuffle_state(w.state, seed=case["seed"] + 100)
    _say(f"case {case} n={n}")
    got, gouts, status = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    assert_state_equal(got, want)
    assert_outputs_match(gouts[0], routs[0], w.params["mass"])
    assert routs[0]["counters"][1] > 50
    assert status & T.STATUS_PAIR_OVERFLOW == 0


@pytest.mark.parametrize("case", [CASES[0], CASES[3], CASES[4], CASES[6]],
                         ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
@pytest.mark.parametrize("shape", [(1, 64), (1, 256)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_fp64_one_record_per_lane_bit_exact(T, oracle, case, shape):
    """One record per lane: on dense bins the wave-uniform walk takes two
    neighbours per iteration, on sparse ones each lane walks its own rows;
    two steps stay bit-identical to the oracle."""
    w = W.random_box(n=2999, seed=case["seed"] + 30, ncell=case["ncell"], bc=case["bc"], d_over_w=0.7,
                     dt_over=0.6, nobin=(3, 2, 1))
    _say(f"one-record case {case} shape {shape}")
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=2, shape=shape)
    want, routs = oracle_steps(oracle, w, steps=2)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, w.params["mass"])
    assert routs[0]["counters"][1] > 50


def test_fp64_trajectory_bit_exact(T, oracle):
    """Ten steps: the state stays bit-identical to the oracle's."""
    w = W.random_box(n=4000, seed=11, ncell=(8, 4, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.4)
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=10)
    want, routs = oracle_steps(oracle, w, steps=10)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert go["counters"][0].tolist() == ro["counters"].tolist()


def test_fp64_sod_100k_bit_exact(T, oracle):
    """The 100k-particle FP64 Sod tube (200 c-bins): three steps, pair lists
    and states bit-exact."""
    w = W.sod()
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=3)
    want, routs = oracle_steps(oracle, w, steps=3)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, w.params["mass"])
    assert routs[0]["counters"][1] > 10000


def test_reorder_keeps_the_same_particles(T, oracle):
    w = W.random_box(n=3000, seed=12, ncell=(6, 5, 4), d_over_w=0.7, dt_over=0.5)
    got, gouts, _ = gpu_steps(T, w, T.FP64, flags=T.EMIT_PAIRS | T.ALLOW_REORDER)
    want, routs = oracle_steps(oracle, w)
    og, ow = np.argsort(got["id"]), np.argsort(want["id"])
    for k in ("x", "y", "z", "vx", "vy", "vz", "id", "alive"):
        assert np.array_equal(got[k][og], want[k][ow])
    assert pairset(gouts[0]["pairs"]) == pairset(routs[0]["pairs"])


def test_empty_single_and_dead(T, oracle):
    w = W.random_box(n=1, seed=3)
    got, gouts, _ = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    assert_state_equal(got, want)
    assert gouts[0]["counters"][0].tolist() == routs[0]["counters"].tolist()
    w = W.random_box(n=500, seed=4)
    w.state["alive"][:] = 0
    got, gouts, _ = gpu_steps(T, w, T.FP64)
    assert_state_equal(got, w.state)
    assert gouts[0]["counters"][0].tolist() == [0] * 8
    w = W.random_box(n=0, seed=4)
    eng = engine_for(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    out = T.make_outputs(1, T.nobins(w.grid), pair_cap=4)
    eng.step(dst, w.grid, w.params, out, flags=T.EMIT_PAIRS)
    torch.cuda.synchronize()
    assert out.host()["counters"][0].tolist() == [0] * 8


def test_nonfinite_and_fast_particles(T, oracle):
    w = W.random_box(n=2000, seed=5)
    w.state["y"][10] = np.nan
    w.state["vz"][11] = np.inf
    w.state["vx"][:5] = 4.0 * 0.15 / w.params["dt"]
    got, gouts, status = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    assert_state_equal(got, want)
    assert gouts[0]["counters"][0].tolist() == routs[0]["counters"].tolist()
    assert status & T.STATUS_NONFINITE and status & T.STATUS_FAST


def test_pair_list_overflow(T, oracle):
    w = W.random_box(n=3000, seed=6, d_over_w=0.8, dt_over=0.6)
    got, gouts, status = gpu_steps(T, w, T.FP64, pair_cap=10)
    want, routs = oracle_steps(oracle, w)
    assert status & T.STATUS_PAIR_OVERFLOW
    assert gouts[0]["counters"][0][1] == routs[0]["counters"][1] > 10
    assert len(gouts[0]["pairs"]) == 10
    assert set(pairset(gouts[0]["pairs"])) <= set(pairset(routs[0]["pairs"]))
    assert_state_equal(got, want)


def _batch():
    ws = [W.sod(n=6000, seed=21, ncell=40, nobin=8, dt=1e-3),
          W.noh(n=5000, seed=22, ncell=16, dt=5e-3),
          W.sedov(n=7000, seed=23, ncell=9, nobin=3, blast_fraction=0.01),
          W.random_box(n=3000, seed=24, ncell=(3, 3, 3), bc=(A, A, A), d_over_w=0.7, dt_over=0.6)]
    for k, w in enumerate(ws):
        w.params["instance"] = k
        w.params["seed"] = 1000 + k
    return ws


def _concat(ws):
    st = {k: np.concatenate([w.state[k] for w in ws]) for k in ("x", "y", "z", "vx", "vy", "vz", "alive")}
    ids, off = [], 0
    for w in ws:
        ids.append(w.state["id"] + np.uint32(off))
        off += w.n
    st["id"] = np.concatenate(ids).astype(np.uint32)
    specs, off = [], 0
    for w in ws:
        specs.append((off, w.n, w.grid, w.params))
        off += w.n
    return st, specs


def test_batched_equals_separate_oracle_runs(T, oracle):
    ws = _batch()
    st, specs = _concat(ws)
    n = len(st["x"])
    eng = T.Engine(max_particles=n, max_cells=sum(T.ncells(w.grid) + 1 for w in ws),
                   max_obins=sum(T.nobins(w.grid) for w in ws), precision=T.FP64, max_instances=len(ws))
    dst = T.to_device(st, T.FP64)
    out = T.make_outputs(len(ws), sum(T.nobins(w.grid) for w in ws), pair_cap=n)
    eng.step_batched(dst, specs, out, flags=T.EMIT_PAIRS)
    torch.cuda.synchronize()
    got = T.to_host(dst)
    go = out.host()
    eng.close()
    mo = 0
    for k, w in enumerate(ws):
        ref_state = W.copy_state(w.state)
        ref_state["id"] = st["id"][specs[k][0]:specs[k][0] + w.n].copy()
        ro = oracle.step(ref_state, w.grid, w.params)
        sl = slice(specs[k][0], specs[k][0] + w.n)
        assert_state_equal({kk: v[sl] for kk, v in got.items()}, ref_state)
        assert go["counters"][k].tolist() == ro["counters"].tolist()
        nb = T.nobins(w.grid)
        assert np.array_equal(go["moments"][mo:mo + nb, 0], ro["moments"][:, 0])
        mo += nb
    assert pairset(go["pairs"]) == sorted(
        sum([pairset(oracle.step(dict(W.copy_state(w.state), id=st["id"][s[0]:s[0] + w.n].copy()),
                                 w.grid, w.params)["pairs"]) for w, s in zip(ws, specs)], []))


def test_graph_run_equals_plain_steps(T, oracle):
    """tpkmc_run (one captured step replayed K times, step counter on the
    device) equals K plain steps and the oracle."""
    ws = _batch()[:3]
    st, specs = _concat(ws)
    n = len(st["x"])
    kw = dict(max_particles=n, max_cells=sum(T.ncells(w.grid) + 1 for w in ws),
              max_obins=sum(T.nobins(w.grid) for w in ws), precision=T.FP64, max_instances=len(ws))
    K = 4
    e1 = T.Engine(**kw)
    d1 = T.to_device(st, T.FP64)
    o1 = T.make_outputs(len(ws), kw["max_obins"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        e1.run(d1, specs, K, o1, stream=stream)
    stream.synchronize()
    e2 = T.Engine(**kw)
    d2 = T.to_device(st, T.FP64)
    o2 = T.make_outputs(len(ws), kw["max_obins"])
    for s in range(K):
        sp = [(off, cnt, g, dict(p, step=p["step"] + s)) for off, cnt, g, p in specs]
        e2.step_batched(d2, sp, o2)
    torch.cuda.synchronize()
    h1, h2 = T.to_host(d1), T.to_host(d2)
    assert_state_equal(h1, h2)
    # The first run tunes the handle, whose c-bins may be split by speed:
    # every counter but the search's work counters is the plain steps'.
    c1, c2 = o1.host()["counters"], o2.host()["counters"]
    keep = [k for name, k in T.CNT.items() if name not in ("tests", "cand")]
    assert c1[:, keep].tolist() == c2[:, keep].tolist()
    for k, w in enumerate(ws):
        ref_state = W.copy_state(w.state)
        ref_state["id"] = st["id"][specs[k][0]:specs[k][0] + w.n].copy()
        for s in range(K):
            oracle.step(ref_state, w.grid, dict(w.params, step=w.params["step"] + s))
        sl = slice(specs[k][0], specs[k][0] + w.n)
        assert_state_equal({kk: v[sl] for kk, v in h1.items()}, ref_state)
    # A second run on the same handle continues from the new state.
    with torch.cuda.stream(stream):
        e1.run(d1, [(o, c, g, dict(p, step=p["step"] + K)) for o, c, g, p in specs], 1, o1, stream=stream)
    stream.synchronize()
    e1.close(); e2.close()


def test_autotune_is_results_neutral(T, oracle):
    w = W.random_box(n=5000, seed=31, ncell=(8, 6, 5), d_over_w=0.7, dt_over=0.5)
    eng = engine_for(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    eng.autotune(dst, [(0, w.n, w.grid, w.params)])
    assert np.array_equal(T.to_host(dst)["x"], w.state["x"])
    out = T.make_outputs(1, T.nobins(w.grid), pair_cap=w.n)
    eng.step(dst, w.grid, w.params, out, flags=T.EMIT_PAIRS)
    torch.cuda.synchronize()
    want, routs = oracle_steps(oracle, w)
    assert_state_equal(T.to_host(dst), want)
    eng.close()


def test_invalid_arguments_are_rejected_before_launch(T):
    w = W.random_box(n=100, seed=1)
    eng = engine_for(T, w, T.FP64)
    dst = T.to_device(w.state, T.FP64)
    bad_grids = [dict(w.grid, ncell=(0, 1, 1)), dict(w.grid, hi=(0.0, 0.8, 0.6)),
                 dict(w.grid, bc=(3, 0, 0)), dict(w.grid, ncell=(1000, 1000, 1000))]
    for g in bad_grids:
        assert eng.step(dst, g, w.params, rc_only=True) in (T.EINVAL, T.ECAPACITY)
    for p in (dict(w.params, dt=0.0), dict(w.params, sigma=-1.0), dict(w.params, mass=0.0),
              dict(w.params, instance=1 << 24), dict(w.params, dt=float("nan"))):
        assert eng.step(dst, w.grid, p, rc_only=True) == T.EINVAL
    big = T.to_device(W.random_box(n=200, seed=1).state, T.FP64)
    assert eng.step(big, w.grid, w.params, rc_only=True) == T.ECAPACITY
    noalive = dict(dst)
    noalive["alive"] = None
    G, Pp = T.make_grid(dict(w.grid, bc=(A, A, A))), T.make_params(w.params)
    S = T.particles(noalive, with_alive=False)
    import ctypes
    rc = T.lib().tpkmc_step(eng.h, ctypes.byref(G), ctypes.byref(Pp), ctypes.byref(S), None, None)
    assert rc == T.EINVAL
    assert T.lib().tpkmc_step(None, ctypes.byref(G), ctypes.byref(Pp), ctypes.byref(S), None, None) == T.EINVAL
    eng.close()


def test_fp64_sqrt_and_division_are_correctly_rounded(T, oracle):
    """The pair path's divisions and square roots round like the host's
    (checked through the state: colliders' velocities use sqrt, t_poca a
    division), over many collisions with wide value ranges."""
    w = W.random_box(n=6000, seed=77, ncell=(6, 6, 6), bc=(P, P, P), d_over_w=0.9, dt_over=0.8, speed=37.0)
    got, _, _ = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    assert routs[0]["counters"][1] > 1000
    assert_state_equal(got, want)


# ------------------------------------------------------------ adaptive dt
def _adaptive(w, cap=1.0):
    w.params = dict(w.params, dt=float(cap), adaptive_dt=True)
    return w


@pytest.mark.parametrize("case", CASES[:5], ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp64_adaptive_step_bit_exact(T, oracle, case):
    """The adaptive time step of Sec. 3 is taken on the device: the same
    dt, pairs and state as the oracle, bit for bit."""
    w = _adaptive(W.random_box(n=2500, seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.7,
                               dt_over=0.6, nobin=(3, 2, 1)))
    w.state["vx"][7] *= 3.0  # a clear fastest particle
    _say(f"adaptive case {case}")
    got, gouts, status = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    dt = oracle.step_dt(w.state, w.grid, w.params)
    assert routs[0]["globals"][7] == dt
    assert (dt < 1.0) if max(case["ncell"]) > 1 else (dt == 1.0)  # one c-bin per axis: the cap
    assert_state_equal(got, want)
    assert_outputs_match(gouts[0], routs[0], w.params["mass"])
    if min(case["ncell"]) > 1:  # every axis bounds the step
        assert routs[0]["counters"][oracle.CNT["fast"]] <= 1


def test_fp64_adaptive_trajectory_and_cap(T, oracle):
    """Eight adaptive steps: dt changes from step to step with v_max and
    the state stays bit-identical; a small cap wins over the rule."""
    w = _adaptive(W.random_box(n=4000, seed=12, ncell=(8, 4, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.4))
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=8)
    want, routs = oracle_steps(oracle, w, steps=8)
    assert_state_equal(got, want)
    dts = [o["globals"][0][7] for o in gouts]
    assert dts == [o["globals"][7] for o in routs]
    assert len(set(dts)) > 1
    cap = 0.5 * min(dts)
    w2 = _adaptive(W.random_box(n=4000, seed=12, ncell=(8, 4, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.4), cap)
    _, gouts2, _ = gpu_steps(T, w2, T.FP64, steps=2)
    assert [o["globals"][0][7] for o in gouts2] == [cap, cap]


def test_graph_run_adapts_dt_on_the_device(T, oracle):
    """tpkmc_run with adaptive instances: each replay takes its own dt from
    the current state; instance 1 keeps its fixed dt."""
    ws = _batch()[:3]
    _adaptive(ws[0], cap=1.0)
    _adaptive(ws[2], cap=1.0)
    st, specs = _concat(ws)
    n = len(st["x"])
    kw = dict(max_particles=n, max_cells=sum(T.ncells(w.grid) + 1 for w in ws),
              max_obins=sum(T.nobins(w.grid) for w in ws), precision=T.FP64, max_instances=len(ws))
    K = 5
    eng = T.Engine(**kw)
    d1 = T.to_device(st, T.FP64)
    out = T.make_outputs(len(ws), kw["max_obins"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eng.run(d1, specs, K, out, stream=stream)
    stream.synchronize()
    h1 = T.to_host(d1)
    go = out.host()
    eng.close()
    for k, w in enumerate(ws):
        ref_state = W.copy_state(w.state)
        ref_state["id"] = st["id"][specs[k][0]:specs[k][0] + w.n].copy()
        dts = []
        for s in range(K):
            ro = oracle.step(ref_state, w.grid, dict(w.params, step=w.params["step"] + s))
            dts.append(ro["globals"][7])
        sl = slice(specs[k][0], specs[k][0] + w.n)
        assert_state_equal({kk: v[sl] for kk, v in h1.items()}, ref_state)
        assert go["globals"][k][7] == dts[-1]
        if k == 1:
            assert dts == [w.params["dt"]] * K
        else:
            assert len(set(dts)) > 1


def test_fp32_adaptive_dt_matches_the_rule(T, oracle):
    """FP32 state: v_max and dt are evaluated in double from the float
    components, so the dt equals the oracle's rule on the float state."""
    w = _adaptive(W.random_box(n=30000, seed=13, ncell=(12, 10, 8), bc=(P, P, P), d_over_w=0.5, dt_over=0.4))
    f32 = W.copy_state(w.state, dtype=np.float32)
    as64 = W.copy_state(f32)
    dt = oracle.step_dt(as64, w.grid, w.params)
    got, gouts, status = gpu_steps(T, w, T.FP32, state=f32)
    assert gouts[0]["globals"][0][7] == dt
    assert gouts[0]["counters"][0][T.CNT["fast"]] <= 1


# ------------------------------------------------------------ planar (2D) gas
PLANE_CASES = [
    dict(seed=31, ncell=(6, 5), bc=(R, P)),
    dict(seed=32, ncell=(3, 3), bc=(P, P)),
    dict(seed=33, ncell=(1, 7), bc=(P, R)),
    dict(seed=34, ncell=(2, 1), bc=(P, P)),
    dict(seed=35, ncell=(9, 4), bc=(A, R)),
]


@pytest.mark.parametrize("case", PLANE_CASES, ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp64_planar_step_bit_exact(T, oracle, case):
    """Two-dimensional gas: in-plane scattering directions and D = sigma/2,
    bit for bit against the oracle over three steps."""
    w = W.random_plane(n=2999, seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.7,
                       dt_over=0.5)
    w.state = W.shuffle_state(w.state, seed=case["seed"])
    _say(f"planar case {case}")
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=3)
    want, routs = oracle_steps(oracle, w, steps=3)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, w.params["mass"])
    assert routs[0]["counters"][1] > 100
    assert np.all(got["vz"] == 0.0) and np.all(got["z"] == 0.0)


def test_fp64_planar_adaptive_batched_with_spatial(T, oracle):
    """One batch holding a 2D Sod strip with the adaptive step and a 3D box:
    each instance equals its own oracle run."""
    ws = [_adaptive(W.sod2d(n=8000, seed=41, ncell=40, nobin=8), cap=1.0),
          W.random_box(n=3000, seed=42, ncell=(4, 3, 3), bc=(R, P, P), d_over_w=0.7, dt_over=0.5)]
    for k, w in enumerate(ws):
        w.params["instance"] = k
    st, specs = _concat(ws)
    n = len(st["x"])
    eng = T.Engine(max_particles=n, max_cells=sum(T.ncells(w.grid) + 1 for w in ws),
                   max_obins=sum(T.nobins(w.grid) for w in ws), precision=T.FP64, max_instances=len(ws))
    dst = T.to_device(st, T.FP64)
    out = T.make_outputs(len(ws), sum(T.nobins(w.grid) for w in ws), pair_cap=n)
    for s in range(2):
        eng.step_batched(dst, [(o, c, g, dict(p, step=s)) for o, c, g, p in specs], out, flags=T.EMIT_PAIRS)
    torch.cuda.synchronize()
    got, go = T.to_host(dst), out.host()
    eng.close()
    for k, w in enumerate(ws):
        ref_state = W.copy_state(w.state)
        ref_state["id"] = st["id"][specs[k][0]:specs[k][0] + w.n].copy()
        for s in range(2):
            ro = oracle.step(ref_state, w.grid, dict(w.params, step=s))
        sl = slice(specs[k][0], specs[k][0] + w.n)
        assert_state_equal({kk: v[sl] for kk, v in got.items()}, ref_state)
        assert go["counters"][k].tolist() == ro["counters"].tolist()
        assert go["globals"][k][7] == ro["globals"][7]


def test_fp32_planar_keeps_the_plane_and_conserves(T, oracle):
    """FP32 2D blast: z and vz stay exactly as given, energy and the pair
    count track the FP64 oracle."""
    w = W.sedov2d(n=60000, seed=43, ncell=60, nobin=10, blast_fraction=0.02)
    f32 = W.copy_state(w.state, dtype=np.float32)
    got, gouts, _ = gpu_steps(T, w, T.FP32, steps=4, state=f32)
    assert np.all(got["vz"] == 0.0) and np.all(got["z"] == 0.0)
    e0 = 0.5 * w.params["mass"] * float(sum((f32[k].astype(np.float64) ** 2).sum() for k in ("vx", "vy")))
    assert gouts[-1]["globals"][0][3] == pytest.approx(e0, rel=2e-5)
    want, routs = oracle_steps(oracle, w, steps=1)
    assert gouts[0]["counters"][0][1] == pytest.approx(routs[0]["counters"][1], rel=0.05)


def test_planar_needs_one_bin_along_z(T):
    w = W.random_plane(n=500, seed=44)
    g = dict(w.grid, ncell=(6, 5, 2), nobin=(6, 5, 2))
    eng = T.Engine(max_particles=500, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP64)
    dst = T.to_device(w.state, T.FP64)
    assert eng.step(dst, g, w.params, None, rc_only=True) == T.EINVAL
    eng.close()


# ------------------------------------------------------------ search shapes
SHAPES = [(1, 256), (2, 128), (2, 64), (4, 64)]


def _fp32_run(T, w, shape, steps=2):
    eng = engine_for(T, w, T.FP32)
    eng.set_search(*shape)
    assert eng.get_search() == shape
    dst = T.to_device(W.copy_state(w.state, dtype=np.float32), T.FP32)
    out = T.make_outputs(1, T.nobins(w.grid), pair_cap=w.n)
    hs = []
    for s in range(steps):
        eng.step(dst, w.grid, dict(w.params, step=s), out, flags=T.EMIT_PAIRS)
        torch.cuda.synchronize()
        hs.append(out.host())
    eng.close()
    return T.to_host(dst), hs


SHAPE_CASES = [
    dict(seed=51, ncell=(7, 5, 4), bc=(R, P, P)),
    dict(seed=52, ncell=(3, 3, 3), bc=(P, P, P)),
    dict(seed=53, ncell=(2, 1, 6), bc=(P, P, R)),
    dict(seed=54, ncell=(1, 1, 1), bc=(P, P, P)),
    dict(seed=55, ncell=(4, 2, 9), bc=(P, R, P)),
    dict(seed=56, ncell=(6, 6, 6), bc=(A, R, A)),
]


@pytest.mark.parametrize("case", SHAPE_CASES, ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp32_search_shapes_are_identical(T, case):
    """Every launch shape of the FP32 partner search (records per lane,
    work-group size) gives the same pairs, state and counters."""
    w = W.random_box(n=3001, seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.7, dt_over=0.5)
    _say(f"shapes case {case}")
    ref_state, ref_out = _fp32_run(T, w, SHAPES[0])
    assert ref_out[0]["counters"][0][1] > 50
    for v in SHAPES[1:]:
        st, outs = _fp32_run(T, w, v)
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.array_equal(st[k], ref_state[k]), (v, k)
        for o, r in zip(outs, ref_out):
            assert o["counters"][0].tolist() == r["counters"][0].tolist(), v
            assert pairset(o["pairs"]) == pairset(r["pairs"]), v


def test_search_shape_arguments(T):
    w = W.random_box(n=100, seed=65)
    eng = engine_for(T, w, T.FP32)
    for bad in ((3, 64), (4, 256), (2, 32), (0, 64)):
        with pytest.raises(T.TpkmcError):
            eng.set_search(*bad)
    eng.set_search(1, 64)
    assert eng.get_search() == (1, 64)
    eng.close()


# ------------------------------------------------------------ criterion 3 by time
@pytest.mark.parametrize("case", CASES[:4] + [CASES[6]], ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp64_rank_by_contact_time_bit_exact(T, oracle, case):
    """Criterion 3 by earliest contact (TPKMC_RANK_TIME): the same pairs and
    state as the oracle, bit for bit, over two steps."""
    w = W.random_box(n=2500, seed=case["seed"] + 70, ncell=case["ncell"], bc=case["bc"], d_over_w=0.8,
                     dt_over=0.6, nobin=(3, 2, 1))
    w.params = dict(w.params, rank_time=True)
    _say(f"rank-time case {case}")
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=2)
    want, routs = oracle_steps(oracle, w, steps=2)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, w.params["mass"])
    assert routs[0]["counters"][1] > 50


def test_fp32_rank_by_contact_time(T, oracle):
    """FP32 with the time ranking: every launch shape agrees, and the pair
    count tracks the FP64 oracle's."""
    w = W.random_box(n=20000, seed=77, ncell=(10, 8, 6), bc=(P, P, R), d_over_w=0.8, dt_over=0.6)
    w.params = dict(w.params, rank_time=True)
    s0, o0 = _fp32_run(T, w, (2, 128), steps=1)
    s1, o1 = _fp32_run(T, w, (1, 64), steps=1)
    assert pairset(o0[0]["pairs"]) == pairset(o1[0]["pairs"])
    ro = oracle.step(W.copy_state(W.copy_state(w.state, dtype=np.float32)), w.grid, w.params)
    assert o0[0]["counters"][0][1] == pytest.approx(ro["counters"][1], rel=0.02)
    common = set(pairset(o0[0]["pairs"])) & set(pairset(ro["pairs"]))
    assert len(common) > 0.97 * len(ro["pairs"])


# ------------------------------------------------------------ mixtures
@pytest.mark.parametrize("case", CASES[:3] + [CASES[6]], ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_fp64_mixture_bit_exact(T, oracle, case):
    """Per-particle masses: mass-weighted scattering, moments and sums; the
    state and pairs equal the oracle's bit for bit over two steps."""
    w = W.random_box(n=2999, seed=case["seed"] + 90, ncell=case["ncell"], bc=case["bc"], d_over_w=0.7,
                     dt_over=0.6, nobin=(3, 2, 1))
    w.state["mass"] = np.random.default_rng(case["seed"]).uniform(0.3, 3.0, w.n)
    w.state = W.shuffle_state(w.state, seed=case["seed"] + 9)
    _say(f"mixture case {case}")
    got, gouts, _ = gpu_steps(T, w, T.FP64, steps=2)
    want, routs = oracle_steps(oracle, w, steps=2)
    assert_state_equal(got, want)
    for go, ro in zip(gouts, routs):
        assert_outputs_match(go, ro, 3.0)
    assert routs[0]["counters"][1] > 50


def test_mixture_reorder_keeps_masses_with_their_particles(T, oracle):
    """With ALLOW_REORDER the mass array is permuted with the ids; an invalid
    mass makes its particle non-finite on both sides."""
    w = W.random_box(n=4000, seed=95, ncell=(6, 5, 4), d_over_w=0.6, dt_over=0.5)
    m = np.random.default_rng(3).uniform(0.5, 2.0, w.n)
    m[17] = 0.0
    m[18] = np.nan
    w.state["mass"] = m
    got, gouts, status = gpu_steps(T, w, T.FP64, flags=T.ALLOW_REORDER | T.EMIT_PAIRS)
    want, routs = oracle_steps(oracle, w)
    by_id = {int(i): k for k, i in enumerate(got["id"])}
    for k in range(w.n):
        gk = by_id[int(w.state["id"][k])]
        assert (got["mass"][gk] == m[k]) or (np.isnan(m[k]) and np.isnan(got["mass"][gk]))
        assert got["x"][gk] == want["x"][k] or (np.isnan(want["x"][k]) and np.isnan(got["x"][gk]))
    assert gouts[0]["counters"][0].tolist() == routs[0]["counters"].tolist()
    assert routs[0]["counters"][oracle.CNT["nonfinite"]] == 2
    assert status & T.STATUS_NONFINITE


def test_fp32_mixture_conserves(T, oracle):
    """FP32 mixture: momentum and energy kept to FP32 rounding, the pair count
    tracks the oracle's."""
    w = W.random_box(n=20000, seed=96, ncell=(10, 8, 6), bc=(P, P, P), d_over_w=0.6, dt_over=0.5)
    w.state["mass"] = np.where(np.arange(w.n) % 3 == 0, 4.0, 1.0)
    f32 = W.copy_state(w.state, dtype=np.float32)
    got, gouts, _ = gpu_steps(T, w, T.FP32, steps=3, state=f32)
    m = f32["mass"].astype(np.float64)
    p0 = [float(np.sum(m * f32[k].astype(np.float64))) for k in ("vx", "vy", "vz")]
    p1 = [float(np.sum(m * got[k])) for k in ("vx", "vy", "vz")]
    e0 = 0.5 * float(np.sum(m * sum(f32[k].astype(np.float64) ** 2 for k in ("vx", "vy", "vz"))))
    e1 = 0.5 * float(np.sum(m * sum(got[k] ** 2 for k in ("vx", "vy", "vz"))))
    assert e1 == pytest.approx(e0, rel=2e-6)
    assert np.allclose(p1, p0, atol=2e-6 * math.sqrt(2 * e0 * m.sum()))
    assert gouts[-1]["globals"][0][6] == pytest.approx(m.sum(), rel=1e-12)
    ro = oracle.step(W.copy_state(f32), w.grid, w.params)
    assert gouts[0]["counters"][0][1] == pytest.approx(ro["counters"][1], rel=0.02)


def _boundary_pairs(n_pairs, seed, D, dt):
    """Pairs placed on the edges of criteria 1 and 2 (closest approach just
    before or after the end of the step, closest distance just below or above
    D), one pair per c-bin of a lattice of bins much wider than their reach,
    so their separations lie at |r|^2 = D^2 + |u|^2 dt^2."""
    rng = np.random.default_rng(seed)
    nb = int(np.ceil(n_pairs ** (1.0 / 3.0)))
    wb = 0.01
    k = np.arange(n_pairs)
    c = np.stack([(k % nb + 0.5) * wb, (k // nb % nb + 0.5) * wb, (k // (nb * nb) + 0.5) * wb])
    u = rng.normal(size=(3, n_pairs))
    u *= rng.uniform(0.3, 2.0, n_pairs) / np.sqrt((u * u).sum(axis=0))
    q = rng.normal(size=(3, n_pairs))
    q -= u * (q * u).sum(axis=0) / (u * u).sum(axis=0)
    q /= np.sqrt((q * q).sum(axis=0))
    e1 = rng.choice([-1.0, 1.0], n_pairs) * 10 ** rng.uniform(-13, -6, n_pairs)
    e2 = rng.choice([-1.0, 1.0], n_pairs) * 10 ** rng.uniform(-13, -6, n_pairs)
    r = -u * dt * (1.0 - e1) + q * D * (1.0 - e2)
    va = 0.05 * rng.normal(size=(3, n_pairs))
    pa, pb = c + 0.5 * r, c - 0.5 * r
    vb = va - u
    st = W.make_state(*np.concatenate([pa, pb], axis=1), *np.concatenate([va, vb], axis=1))
    g = W.grid((0, 0, 0), (nb * wb,) * 3, (nb,) * 3, (P, P, P))
    p = W.params(sigma=math.pi * D * D, dt=dt, seed=seed)

    class Wl:
        pass
    w = Wl()
    w.state, w.grid, w.params, w.n = st, g, p, 2 * n_pairs
    return w


def test_fp64_pairs_on_the_edges_of_both_criteria(T, oracle):
    """Pairs on the edges of both criteria: the accepted pairs and the state
    stay bit-identical to the oracle's, and both outcomes occur."""
    w = _boundary_pairs(4000, seed=61, D=1e-3, dt=1e-3)
    got, gouts, _ = gpu_steps(T, w, T.FP64)
    want, routs = oracle_steps(oracle, w)
    assert_state_equal(got, want)
    assert pairset(gouts[0]["pairs"]) == pairset(routs[0]["pairs"])
    assert gouts[0]["counters"][0].tolist() == routs[0]["counters"].tolist()
    accepted = routs[0]["counters"][oracle.CNT["pairs"]]
    assert 0.1 * 4000 < accepted < 0.9 * 4000


def _mix_by_enumeration(oracle, st, grid, params):
    """(tests, s0 < 0, s0 < 0 < s1) over the unordered pairs of every c-bin's
    neighbourhood, s0 and s1 in the order of the pair test (no FMA)."""
    n = len(st["x"])
    cells = np.array([oracle.cell_of(grid, st["x"][i], st["y"][i], st["z"][i])[0] for i in range(n)])
    L = [grid["hi"][a] - grid["lo"][a] for a in range(3)]
    tests = s0n = c1n = 0
    for i in range(n):
        nb = set(oracle.stencil(grid, int(cells[i])))
        J = np.array([j for j in range(i + 1, n) if int(cells[j]) in nb], dtype=np.int64)
        if len(J) == 0:
            continue
        r = [st[k][i] - st[k][J] for k in ("x", "y", "z")]
        for a in range(3):
            if grid["bc"][a] == P:
                r[a] = np.where(r[a] > 0.5 * L[a], r[a] - L[a], np.where(r[a] < -(0.5 * L[a]), r[a] + L[a], r[a]))
        u = [st[k][i] - st[k][J] for k in ("vx", "vy", "vz")]
        s0 = (r[0] * u[0] + r[1] * u[1]) + r[2] * u[2]
        vv = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
        s1 = s0 + vv * params["dt"]
        tests += len(J)
        s0n += int((s0 < 0).sum())
        c1n += int(((s0 < 0) & (s1 > 0)).sum())
    return tests, s0n, c1n


@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"s{c['seed']}-{c['ncell']}-{c['bc']}")
def test_search_mix_counts(T, oracle, case):
    """tpkmc_search_mix counts the pair tests, the approaching pairs and those
    meeting criterion 1: in FP64 exactly an enumeration of the neighbourhood
    pairs; in FP32 the same up to rounding of s0 and s1.  The state is left
    untouched."""
    w = W.random_box(n=1500, seed=case["seed"], ncell=case["ncell"], bc=case["bc"], d_over_w=0.7, dt_over=0.6)
    want = _mix_by_enumeration(oracle, w.state, w.grid, w.params)
    assert want[0] == oracle.count_tests(w.state, w.grid)
    st32 = W.copy_state(w.state)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        st32[k] = w.state[k].astype(np.float32).astype(np.float64)
    want32 = _mix_by_enumeration(oracle, st32, w.grid, w.params)
    for prec in (T.FP64, T.FP32):
        eng = engine_for(T, w, prec)
        dst = T.to_device(w.state, prec)
        before = T.to_host(dst)
        got = eng.search_mix(dst, [(0, w.n, w.grid, w.params)])
        after = T.to_host(dst)
        eng.close()
        for k in ("x", "y", "z", "vx", "vy", "vz", "id"):
            assert np.array_equal(before[k], after[k])
        _say(f"mix {case} prec={prec}: gpu {got} enumeration {want}")
        if prec == T.FP64:
            assert got == want
        else:
            assert got[0] == want32[0]
            assert abs(got[1] - want32[1]) <= 3 and abs(got[2] - want32[2]) <= 3
