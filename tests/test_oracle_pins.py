"""Pins of the FP64 oracle's building blocks against what the paper and the
mathematics fix: the three-criterion pair test (Sec. 2.4, Sec. 3), the
neighbourhood of a c-bin (Sec. 3), the random directions of the scattering
(Sec. 3) and the Philox generator behind them."""
import itertools
import math

import numpy as np
import pytest

from paper_1210_8084_amd import workloads as W

GRID = W.grid((0, 0, 0), (1, 1, 1), (4, 4, 4), (W.REFLECT,) * 3)


def params(D, dt):
    return W.params(sigma=math.pi * D * D, dt=dt)


# ---------------------------------------------------------------- pair test
def test_head_on_impact_parameter(oracle):
    """i moves along +x at speed s towards j at rest, offset by b: the point
    of closest approach is at t = dist / s with separation exactly b."""
    s, dist, b, D, dt = 2.0, 0.01, 0.003, 0.004, 0.01
    ok, d2, tp = oracle.pair_test(GRID, params(D, dt), [0.5, 0.5, 0.5], [s, 0, 0],
                                  [0.5 + dist, 0.5 + b, 0.5], [0, 0, 0])
    assert ok
    assert d2 == pytest.approx(b * b, rel=1e-12)
    assert tp == pytest.approx(dist / s, rel=1e-12)


def test_receding_pair_is_rejected(oracle):
    ok, _, _ = oracle.pair_test(GRID, params(0.004, 0.01), [0.5, 0.5, 0.5], [-2.0, 0, 0],
                                [0.51, 0.501, 0.5], [0, 0, 0])
    assert not ok


def test_closest_approach_after_the_step_is_rejected(oracle):
    """Criterion 1: chi < 0 needs the closest approach inside [t, t + dt]."""
    s, dist, D = 1.0, 0.02, 0.004
    P = params(D, dt=0.9 * dist / s)
    ok, _, _ = oracle.pair_test(GRID, P, [0.5, 0.5, 0.5], [s, 0, 0], [0.5 + dist, 0.501, 0.5], [0, 0, 0])
    assert not ok
    P = params(D, dt=1.1 * dist / s)
    ok, _, _ = oracle.pair_test(GRID, P, [0.5, 0.5, 0.5], [s, 0, 0], [0.5 + dist, 0.501, 0.5], [0, 0, 0])
    assert ok


@pytest.mark.parametrize("factor,expect", [(1 - 1e-9, True), (1 + 1e-9, False)])
def test_radius_boundary(oracle, factor, expect):
    """Criterion 2 at d_min = D (1 -/+ 1e-9)."""
    D = 0.004
    b = D * factor
    ok, _, _ = oracle.pair_test(GRID, params(D, 0.01), [0.5, 0.5, 0.5], [1.0, 0, 0],
                                [0.505, 0.5 + b, 0.5], [0, 0, 0])
    assert ok is expect


def test_matches_the_papers_overlap_quadratic(oracle):
    """Criterion 2 as printed: the overlap times t_o solve
    |v|^2 t^2 + 2 (v.r) t + |r|^2 - D^2 = 0 and must be real; together with
    criterion 1 (closest approach inside the step).  Checked with numpy's
    polynomial roots on random pairs."""
    rng = np.random.default_rng(7)
    D, dt = 0.05, 0.05
    P = params(D, dt)
    G = W.grid((0, 0, 0), (1, 1, 1), (1, 1, 1), (W.REFLECT,) * 3)
    agree = 0
    for _ in range(3000):
        ri = rng.uniform(0.4, 0.6, 3)
        rj = ri + rng.normal(0, 0.03, 3)
        vi, vj = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
        ok, d2, tp = oracle.pair_test(G, P, ri, vi, rj, vj)
        r, v = ri - rj, vi - vj
        roots = np.roots([v @ v, 2 * (v @ r), r @ r - D * D])
        real = bool(np.all(np.abs(np.imag(roots)) < 1e-12 * max(1.0, np.max(np.abs(roots)))))
        tpoca = -(r @ v) / (v @ v)
        expect = real and 0.0 < tpoca < dt
        dmin2 = np.sum((r + tpoca * v) ** 2)
        if abs(dmin2 - D * D) < 1e-9 * D * D or min(abs(tpoca), abs(tpoca - dt)) < 1e-12:
            continue  # too close to a boundary for the root test's tolerance
        assert ok == expect
        if ok:
            assert d2 == pytest.approx(dmin2, rel=1e-9, abs=1e-18)
            assert tp == pytest.approx(tpoca, rel=1e-12)
        agree += 1
    assert agree > 2900


def test_closest_approach_by_dense_sampling(oracle):
    """d_min^2 and t_poca equal the minimum of |r + u t|^2 over a fine grid
    of t in [0, dt] (brute force on the trajectory)."""
    rng = np.random.default_rng(11)
    G = W.grid((0, 0, 0), (1, 1, 1), (1, 1, 1), (W.REFLECT,) * 3)
    P = params(0.2, 0.1)
    checked = 0
    ts = np.linspace(0.0, 0.1, 200001)
    for _ in range(200):
        ri, vi = rng.uniform(0.45, 0.55, 3), rng.normal(0, 1, 3)
        rj, vj = rng.uniform(0.45, 0.55, 3), rng.normal(0, 1, 3)
        ok, d2, tp = oracle.pair_test(G, P, ri, vi, rj, vj)
        if not ok:
            continue
        path = (ri - rj)[None, :] + ts[:, None] * (vi - vj)[None, :]
        dist2 = np.sum(path * path, axis=1)
        k = int(np.argmin(dist2))
        assert d2 == pytest.approx(dist2[k], rel=1e-6, abs=1e-12)
        assert abs(tp - ts[k]) <= 2 * (ts[1] - ts[0]) + 1e-6
        checked += 1
    assert checked > 20


def test_bitwise_symmetric(oracle):
    """Swapping i and j negates r, u and the PoCA separation exactly, so
    d_min^2 and t_poca are bit-identical both ways."""
    rng = np.random.default_rng(5)
    G = W.grid((0, 0, 0), (1, 1, 1), (1, 1, 1), (W.REFLECT, W.PERIODIC, W.PERIODIC))
    P = params(0.3, 0.2)
    hits = 0
    for _ in range(2000):
        ri, rj = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
        vi, vj = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
        a = oracle.pair_test(G, P, ri, vi, rj, vj)
        b = oracle.pair_test(G, P, rj, vj, ri, vi)
        assert a[0] == b[0]
        if a[0]:
            hits += 1
            assert a[1] == b[1] and a[2] == b[2]
    assert hits > 50


def test_periodic_minimum_image(oracle):
    """Across a periodic face the pair is tested at its nearest image."""
    G = W.grid((0, 0, 0), (1, 1, 1), (4, 4, 4), (W.PERIODIC,) * 3)
    P = params(0.004, 0.01)
    ok, d2, tp = oracle.pair_test(G, P, [0.995, 0.5, 0.5], [1.0, 0, 0], [0.002, 0.502, 0.5], [0, 0, 0])
    assert ok
    assert d2 == pytest.approx(0.002 ** 2, rel=1e-9)
    assert tp == pytest.approx(0.007, rel=1e-9)
    Gr = W.grid((0, 0, 0), (1, 1, 1), (4, 4, 4), (W.REFLECT,) * 3)
    ok, _, _ = oracle.pair_test(Gr, P, [0.995, 0.5, 0.5], [1.0, 0, 0], [0.002, 0.502, 0.5], [0, 0, 0])
    assert not ok


# ---------------------------------------------------------------- c-bins
@pytest.mark.parametrize("ncell,bc", [
    ((5, 4, 3), (0, 0, 0)), ((5, 4, 3), (1, 1, 1)), ((1, 1, 1), (1, 1, 1)),
    ((2, 2, 2), (1, 1, 1)), ((3, 1, 2), (1, 0, 1)), ((7, 2, 1), (0, 1, 1)), ((1, 3, 4), (2, 1, 0))])
def test_stencil_is_the_3x3x3_neighbourhood(oracle, ncell, bc):
    """Every cell within one index per axis (wrapped on periodic axes),
    listed once, by a set-based enumeration written independently."""
    g = W.grid((0, 0, 0), (1, 1, 1), ncell, bc)
    nx, ny, nz = ncell
    for cz, cy, cx in itertools.product(range(nz), range(ny), range(nx)):
        want = set()
        for d in itertools.product((-1, 0, 1), repeat=3):
            c = [cx + d[0], cy + d[1], cz + d[2]]
            okc = True
            for a, n in enumerate(ncell):
                if bc[a] == W.PERIODIC:
                    c[a] %= n
                elif not 0 <= c[a] < n:
                    okc = False
            if okc:
                want.add(c[0] + nx * (c[1] + ny * c[2]))
        assert oracle.stencil(g, cx + nx * (cy + ny * cz)) == sorted(want)


def test_cell_of_floor_and_clamp(oracle):
    g = W.grid((-1, 0, 2), (1, 1, 3), (8, 3, 2), (0, 0, 0))
    assert oracle.cell_of(g, -1.0, 0.0, 2.0)[1] == (0, 0, 0)
    assert oracle.cell_of(g, 0.999999, 0.5, 2.75)[1] == (7, 1, 1)
    assert oracle.cell_of(g, 1.0, 1.0, 3.0)[1] == (7, 2, 1)        # hi edge clamps
    assert oracle.cell_of(g, -1.5, -0.1, 1.0)[1] == (0, 0, 0)      # below lo clamps
    assert oracle.cell_of(g, -0.75, 0.34, 2.49)[1] == (1, 1, 0)
    flat, c = oracle.cell_of(g, 0.3, 0.9, 2.6)
    assert flat == c[0] + 8 * (c[1] + 3 * c[2])


# ---------------------------------------------------------------- RNG
def test_philox_avalanche_and_key_dependence(oracle):
    """A counter-based bijection: flipping any single counter or key bit
    flips about half of the 128 output bits."""
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        base = oracle.philox(ctr, key)
        bit = int(rng.integers(0, 192))
        c2, k2 = ctr.copy(), key.copy()
        if bit < 128:
            c2[bit // 32] ^= np.uint32(1 << (bit % 32))
        else:
            k2[(bit - 128) // 32] ^= np.uint32(1 << ((bit - 128) % 32))
        out = oracle.philox(c2, k2)
        flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out)))
    assert 60 < np.mean(flips) < 68
    assert min(flips) > 30


def test_philox_uniform_bytes(oracle):
    """Chi-square of the output bytes over consecutive counters."""
    words = np.array([oracle.philox([i, 7, 0, 0], [123, 456]) for i in range(4000)], dtype=np.uint32)
    b = words.view(np.uint8).ravel()
    hist = np.bincount(b, minlength=256)
    exp = len(b) / 256.0
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert 180 < chi2 < 340  # 255 dof, ~4 sigma either side


def test_directions_are_unit_and_isotropic(oracle):
    """Marsaglia's construction gives unit vectors uniform on the sphere:
    mean 0, <n_a^2> = 1/3, and (Archimedes) n_z uniform on [-1, 1]."""
    from scipy.stats import kstest
    ns = []
    for k in range(20000):
        n, used = oracle.direction(99, 3, 1, k, k + 1)
        assert 1 <= used <= 255
        assert abs(float(n @ n) - 1.0) <= 8e-16
        ns.append(n)
    ns = np.array(ns)
    assert np.all(np.abs(ns.mean(axis=0)) < 0.02)
    assert np.all(np.abs((ns ** 2).mean(axis=0) - 1 / 3) < 0.01)
    assert kstest(ns[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(ns[:, 1], ns[:, 0])
    assert kstest(phi, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-3


def test_direction_depends_on_every_key_field(oracle):
    base, _ = oracle.direction(1, 2, 3, 4, 5)
    for args in [(2, 2, 3, 4, 5), (1, 3, 3, 4, 5), (1, 2, 4, 4, 5), (1, 2, 3, 5, 5), (1, 2, 3, 4, 6)]:
        assert not np.array_equal(oracle.direction(*args)[0], base)
    assert np.array_equal(oracle.direction(1, 2, 3, 4, 5)[0], base)


# The oracle's Philox4x32-10 against an independent implementation: rocRAND's
# (its header ships with ROCm), compiled here for the host at test time, so
# that no third-party answer is stored in this repository.
_ROCRAND_PROBE = r"""
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
struct open_engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};
int main() {
    open_engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


def test_philox_matches_rocrand(oracle, tmp_path):
    import os
    import shutil
    import subprocess
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    header = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(header)):
        pytest.skip("hipcc or the rocRAND header is not installed")
    src, exe = tmp_path / "philox.cpp", tmp_path / "philox"
    src.write_text(_ROCRAND_PROBE)
    subprocess.run([hipcc, "--cuda-host-only", "-O1", "-o", str(exe), str(src)], check=True, timeout=120,
                   capture_output=True)
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 2 ** 32, size=(3000, 6), dtype=np.uint64)
    rows[:6] = [[0] * 6, [2 ** 32 - 1] * 6, [0, 0, 0, 0, 2 ** 32 - 1, 2 ** 32 - 1],
                [2 ** 32 - 1] * 4 + [0, 0], [1, 2, 3, 4, 5, 6], [7, 0, 0, 255, 1, 0]]
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True, timeout=60)
    theirs = np.array([[int(v) for v in line.split()] for line in res.stdout.splitlines()], dtype=np.uint64)
    assert theirs.shape == (len(rows), 4)
    ours = np.array([oracle.philox(r[:4].astype(np.uint32), r[4:].astype(np.uint32)) for r in rows],
                    dtype=np.uint64)
    assert np.array_equal(ours, theirs)
