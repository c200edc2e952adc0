"""Exact o-bin moments on the GPU (Sec. 4: count, bulk momentum, velocity
spread and virial per o-bin).  The library forms each sum in integers, so
the sums cannot depend on the order in which particles are met:

 - bit-identical moments for equal inputs: repeated runs, caller order
   against ALLOW_REORDER, every search launch shape, and an instance alone
   against the same instance placed second in a batch (FP64 and FP32, over
   several steps, so the o-bin shifts evolve too);
 - FP64: counts, momenta, spreads and masses within a few ulp of the exact
   sums (math.fsum) over the oracle's post-step state, which the GPU state
   equals bit for bit; plain summation of a few hundred terms typically
   misses these bounds by an order of magnitude.  O-bins of more than 4096
   particles round their terms to a quantum 2^h times coarser (h = 1 per
   doubling), so that their sums fit one int64: within 2^h times the bound."""
import math

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R, P, A = W.REFLECT, W.PERIODIC, W.ABSORB
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def T():
    from paper_1210_8084_amd import tpkmc
    assert torch.cuda.is_available(), "GPU test without a visible GPU"
    tpkmc.lib()
    return tpkmc


def run(T, w, precision, steps, flags=0, shape=None, batched_behind=None):
    """Moments of each step; with batched_behind, w is the second instance
    of a batch whose first instance is that workload."""
    g = w.grid
    specs = [w] if batched_behind is None else [batched_behind, w]
    n = sum(s.n for s in specs)
    eng = T.Engine(max_particles=n, max_cells=sum(T.ncells(s.grid) + 1 for s in specs),
                   max_obins=sum(T.nobins(s.grid) for s in specs), precision=precision, max_instances=len(specs))
    if shape:
        eng.set_search(*shape)
    dtype = np.float64 if precision == T.FP64 else np.float32
    states = [W.copy_state(s.state, dtype=dtype) for s in specs]
    cat = {k: np.concatenate([st[k] for st in states]) for k in states[0]}
    dst = T.to_device(cat, precision)
    nob = sum(T.nobins(s.grid) for s in specs)
    out = T.make_outputs(len(specs), nob)
    mo = T.nobins(specs[0].grid) if batched_behind is not None else 0
    res = []
    for s in range(steps):
        if batched_behind is None:
            eng.step(dst, g, dict(w.params, step=s), out, flags=flags)
        else:
            # The instance under test keeps its instance number (0), so its
            # random draws are those of the run alone.
            inst = [(0, specs[0].n, specs[0].grid, dict(specs[0].params, step=s, instance=1)),
                    (specs[0].n, w.n, g, dict(w.params, step=s, instance=0))]
            eng.step_batched(dst, inst, out, flags=flags)
        torch.cuda.synchronize()
        res.append(out.host()["moments"][mo:mo + T.nobins(g)].copy())
    eng.close()
    return res


def workload(seed, mass=False):
    w = W.random_box(n=6000, seed=seed, ncell=(6, 5, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.6,
                     nobin=(3, 2, 2))
    if mass:
        w.state["mass"] = np.random.default_rng(seed).uniform(0.3, 3.0, w.n)
    w.state = W.shuffle_state(w.state, seed=seed + 5)
    return w


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mass", [False, True], ids=["scalar-mass", "mixture"])
def test_moments_do_not_depend_on_order_shape_or_batch(T, prec, mass):
    precision = T.FP64 if prec == "fp64" else T.FP32
    w = workload(21, mass)
    other = W.random_box(n=2500, seed=22, ncell=(3, 3, 3), bc=(P, P, P), d_over_w=0.7, dt_over=0.6, nobin=(2, 1, 1))
    other.state["id"] = other.state["id"] + np.uint32(1_000_000)
    if mass:
        other.state["mass"] = np.full(other.n, 1.5)
    base = run(T, w, precision, 3)
    variants = {
        "repeat": run(T, w, precision, 3),
        "reorder": run(T, w, precision, 3, flags=T.ALLOW_REORDER),
        "shape 1x256": run(T, w, precision, 3, shape=(1, 256)),
        "shape 4x64 reorder": run(T, w, precision, 3, flags=T.ALLOW_REORDER, shape=(4, 64)),
        "second in a batch": run(T, w, precision, 3, batched_behind=other),
    }
    assert base[0][:, 0].sum() == w.n and base[-1][:, 10].sum() > 100
    for name, v in variants.items():
        for s in range(3):
            assert np.array_equal(v[s].view(np.uint64), base[s].view(np.uint64)), (name, s)


def obin_index(st, g):
    idx = np.zeros(len(st["x"]), dtype=np.int64)
    mul = 1
    for a, k in enumerate(("x", "y", "z")):
        lo, hi, nb = g["lo"][a], g["hi"][a], g["nobin"][a]
        t = (st[k] - lo) * (nb / (hi - lo))
        b = np.where(t >= 0.0, np.minimum(np.floor(np.where(t >= 0.0, t, 0.0)), nb - 1), 0).astype(np.int64)
        idx += b * mul
        mul *= nb
    return idx


def headroom(n):
    c = 0 if n <= 1 else int(n - 1).bit_length()  # ceil(log2 n)
    return max(0, c - 12)


@pytest.mark.parametrize("mass", [False, True], ids=["scalar-mass", "mixture"])
@pytest.mark.parametrize("steps", [1, 4])
def test_fp64_moments_are_exact_sums(T, oracle, mass, steps):
    check_exact_sums(T, oracle, workload(31, mass), mass, steps)


@pytest.mark.parametrize("n", [9000, 20000])
def test_fp64_large_obin_sums(T, oracle, n):
    """One o-bin of 9000 or 20000 particles: headroom 2 or 3."""
    w = W.random_box(n=n, seed=41, ncell=(6, 5, 4), bc=(R, P, P), d_over_w=0.7, dt_over=0.6, nobin=(1, 1, 1))
    assert headroom(n) in (2, 3)
    check_exact_sums(T, oracle, w, False, 2)
    # The same state twice: bit-identical.
    a, b = run(T, w, T.FP64, 2), run(T, w, T.FP64, 2, flags=T.ALLOW_REORDER)
    for s in range(2):
        assert np.array_equal(a[s].view(np.uint64), b[s].view(np.uint64))


def check_exact_sums(T, oracle, w, mass, steps):
    got = run(T, w, T.FP64, steps)[-1]
    st = W.copy_state(w.state)
    speed = lambda q: math.sqrt(float(np.max(q["vx"] ** 2 + q["vy"] ** 2 + q["vz"] ** 2)))
    vmax = speed(st)  # bounds the o-bin shifts, which are clamped to the pre-step largest speed
    for s in range(steps):
        ro = oracle.step(st, w.grid, dict(w.params, step=s))
        vmax = max(vmax, speed(st))
    nob = T.nobins(w.grid)
    alive = (st["alive"] != 0) & np.isfinite(st["x"])
    ob = obin_index(st, w.grid)
    m_all = st["mass"] if mass else np.full(w.n, w.params["mass"])
    assert np.array_equal(got[:, 0], ro["moments"][:, 0])
    assert np.array_equal(got[:, 10], ro["moments"][:, 10])
    checked = 0
    for b in range(nob):
        sel = alive & (ob == b)
        assert int(sel.sum()) == int(ro["moments"][b, 0])  # the same o-bin rule as the oracle's
        if not sel.any():
            assert np.all(got[b] == 0.0)
            continue
        m = m_all[sel]
        hq = 2.0 ** headroom(int(sel.sum()))  # the quantum's headroom
        mass_b = math.fsum(m) if mass else sel.sum() * w.params["mass"]
        assert abs(got[b, 11] - mass_b) <= 2 * EPS * mass_b * hq
        for a, k in enumerate(("vx", "vy", "vz")):
            v = st[k][sel]
            p = math.fsum(m * v)
            tol = 4 * hq * EPS * (math.fsum(np.abs(m * v)) + 2 * mass_b * vmax)
            assert abs(got[b, 1 + a] - p) <= tol, (b, a, got[b, 1 + a], p, tol)
            vb = p / mass_b
            spread = math.fsum(m * (v - vb) ** 2)
            tol2 = 8 * hq * EPS * math.fsum(m * (np.abs(v) + vmax) ** 2)
            assert abs(got[b, 4 + a] - spread) <= tol2, (b, a, got[b, 4 + a], spread, tol2)
        checked += 1
    assert checked >= nob - 1
