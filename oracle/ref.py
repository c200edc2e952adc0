"""ctypes binding of the plain FP64 CPU oracle (``tpkmc_ref.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark use this module; the GPU library never does.  It
imports nothing from the GPU package.

A particle state is a mapping with float64 arrays ``x y z vx vy vz``, a
uint32 array ``id`` and an optional uint8 array ``alive``.  A grid is a
mapping with ``lo hi`` (3 floats), ``ncell bc nobin`` (3 ints); params hold
``sigma mass dt seed step instance``.  Arrays are updated in place by
:func:`step`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpkmc_ref.c")
LIB = os.path.join(HERE, "libtpkmc_ref.so")

MODE_BINNED, MODE_BRUTE, MODE_ALL = 0, 1, 2
CNT = dict(alive=0, pairs=1, tests=2, cand=3, fast=4, nonfinite=5, absorbed=6, have_best=7)
GLB = dict(px=0, py=1, pz=2, ekin=3, vmax2=4, virial=5, mass=6, dt=7)
M_STRIDE = 12
M_MASS = 11      # moments slot: sum m
ADAPTIVE_DT = 1  # ref_params.flags: step length from the rule of Sec. 3
PLANAR = 2       # ref_params.flags: two-dimensional gas (x-y plane)
RANK_TIME = 4    # ref_params.flags: criterion 3 by earliest contact time
PAIR_RANDOM = 8  # ref_params.flags: random partners inside each c-bin (DSMC rule)


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Grid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("ncell", ctypes.c_int32 * 3), ("bc", ctypes.c_int32 * 3),
                ("nobin", ctypes.c_int32 * 3), ("pad", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("step", ctypes.c_uint64),
                ("instance", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


_lib = None
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.ref_philox4x32_10.argtypes = [_P, _P, _P]
        L.ref_philox4x32_10.restype = None
        L.ref_direction.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint32, _P]
        L.ref_direction.restype = ctypes.c_int
        L.ref_direction_planar.argtypes = L.ref_direction.argtypes
        L.ref_direction_planar.restype = ctypes.c_int
        L.ref_cell_of.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P]
        L.ref_cell_of.restype = ctypes.c_int32
        L.ref_stencil.argtypes = [_P, ctypes.c_int32, _P]
        L.ref_stencil.restype = ctypes.c_int
        L.ref_pair_test.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P]
        L.ref_pair_test.restype = ctypes.c_int
        L.ref_best.argtypes = [_P, _P, ctypes.c_int64] + [_P] * 8 + [ctypes.c_int, ctypes.c_int, _P, _P]
        L.ref_best.restype = ctypes.c_int
        L.ref_best_sample.argtypes = ([_P, _P, ctypes.c_int64] + [_P] * 8 +
                                      [ctypes.c_int64, _P, ctypes.c_int, _P, _P])
        L.ref_best_sample.restype = ctypes.c_int
        L.ref_step_sample.argtypes = ([_P, _P, ctypes.c_int64] + [_P] * 9 +
                                      [ctypes.c_int64, _P, ctypes.c_int, _P, _P, _P])
        L.ref_step_sample.restype = ctypes.c_int
        L.ref_step_dt.argtypes = [_P, _P, ctypes.c_int64] + [_P] * 7
        L.ref_step_dt.restype = ctypes.c_double
        L.ref_count_tests.argtypes = [_P, ctypes.c_int64] + [_P] * 7
        L.ref_count_tests.restype = ctypes.c_uint64
        L.ref_step.argtypes = ([_P, _P, ctypes.c_int64] + [_P] * 9 +
                               [ctypes.c_int, ctypes.c_int, _P, ctypes.c_int64, _P, _P, _P])
        L.ref_step.restype = ctypes.c_int
        L.ref_last_phase_ms.argtypes = [_P]
        L.ref_last_phase_ms.restype = None
        _lib = L
    return _lib


def make_grid(g) -> Grid:
    G = Grid()
    for a in range(3):
        G.lo[a] = float(g["lo"][a])
        G.hi[a] = float(g["hi"][a])
        G.ncell[a] = int(g["ncell"][a])
        G.bc[a] = int(g["bc"][a])
        G.nobin[a] = int(g.get("nobin", g["ncell"])[a])
    return G


def make_params(p) -> Params:
    P = Params()
    P.sigma = float(p["sigma"])
    P.mass = float(p.get("mass", 1.0))
    P.dt = float(p["dt"])
    P.seed = int(p.get("seed", 0))
    P.step = int(p.get("step", 0))
    P.instance = int(p.get("instance", 0))
    P.flags = ((ADAPTIVE_DT if p.get("adaptive_dt") else 0) | (PLANAR if p.get("planar") else 0) |
               (RANK_TIME if p.get("rank_time") else 0) |
               (PAIR_RANDOM if p.get("pair_random") else 0))
    return P


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check_state(s):
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        a = s[k]
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError(f"state[{k}] must be contiguous float64")
    if s["id"].dtype != np.uint32 or not s["id"].flags.c_contiguous:
        raise TypeError("state[id] must be contiguous uint32")
    al = s.get("alive")
    if al is not None and (al.dtype != np.uint8 or not al.flags.c_contiguous):
        raise TypeError("state[alive] must be contiguous uint8")
    return len(s["x"])


def _state_ptrs(s):
    return [_ptr(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "id")] + [_ptr(s.get("alive"))]


def _mass_ptr(s, n):
    """Per-particle masses (float64, one per particle) or None."""
    m = s.get("mass")
    if m is None:
        return None
    if m.dtype != np.float64 or len(m) != n or not m.flags["C_CONTIGUOUS"]:
        raise ValueError("state['mass'] must be contiguous float64 of length n")
    return _ptr(m)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def direction(seed, step, instance, idA, idB, planar=False):
    n = np.zeros(3)
    f = lib().ref_direction_planar if planar else lib().ref_direction
    used = f(seed, step, instance, idA, idB, _ptr(n))
    return n, used


def cell_of(grid, x, y, z):
    G = make_grid(grid)
    c = np.zeros(3, dtype=np.int32)
    flat = lib().ref_cell_of(ctypes.byref(G), x, y, z, _ptr(c))
    return int(flat), tuple(int(v) for v in c)


def stencil(grid, cell):
    G = make_grid(grid)
    out = np.zeros(27, dtype=np.int32)
    k = lib().ref_stencil(ctypes.byref(G), int(cell), _ptr(out))
    if k < 0:
        raise ValueError("bad grid or cell")
    return sorted(int(v) for v in out[:k])


def pair_test(grid, params, ri, vi, rj, vj):
    """(is_candidate, d2, t_poca) of the ordered pair (i, j)."""
    G, P = make_grid(grid), make_params(params)
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (ri, vi, rj, vj)]
    d2 = ctypes.c_double(0.0)
    tp = ctypes.c_double(0.0)
    ok = lib().ref_pair_test(ctypes.byref(G), ctypes.byref(P), *[_ptr(a) for a in arr],
                             ctypes.byref(d2), ctypes.byref(tp))
    if ok < 0:
        raise ValueError("bad grid or params")
    return bool(ok), d2.value, tp.value


def best(state, grid, params, mode=MODE_BINNED, nthreads=0):
    n = _check_state(state)
    G, P = make_grid(grid), make_params(params)
    b = np.full(n, -1, dtype=np.int64)
    d2 = np.zeros(n)
    rc = lib().ref_best(ctypes.byref(G), ctypes.byref(P), n, *_state_ptrs(state),
                        mode, nthreads, _ptr(b), _ptr(d2))
    if rc:
        raise ValueError(f"ref_best failed ({rc})")
    return b, d2


def best_sample(state, grid, params, sample, nthreads=0):
    n = _check_state(state)
    G, P = make_grid(grid), make_params(params)
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    b = np.full(len(smp), -1, dtype=np.int64)
    d2 = np.zeros(len(smp))
    rc = lib().ref_best_sample(ctypes.byref(G), ctypes.byref(P), n, *_state_ptrs(state),
                               len(smp), _ptr(smp), nthreads, _ptr(b), _ptr(d2))
    if rc:
        raise ValueError(f"ref_best_sample failed ({rc})")
    return b, d2


def step_sample(state, grid, params, sample, nthreads=0):
    """Post-step state of the listed particles as :func:`step` would leave
    it (binned mode), without touching ``state``.  Returns (state (k, 6) as
    x y z vx vy vz, partner index or -1, alive after the step)."""
    n = _check_state(state)
    G, P = make_grid(grid), make_params(params)
    smp = np.ascontiguousarray(sample, dtype=np.int64)
    out = np.zeros((len(smp), 6))
    partner = np.full(len(smp), -1, dtype=np.int64)
    alive = np.zeros(len(smp), dtype=np.uint8)
    rc = lib().ref_step_sample(ctypes.byref(G), ctypes.byref(P), n, *_state_ptrs(state), _mass_ptr(state, n),
                               len(smp), _ptr(smp), nthreads, _ptr(out), _ptr(partner), _ptr(alive))
    if rc:
        raise ValueError(f"ref_step_sample failed ({rc})")
    return out, partner, alive


def step_dt(state, grid, params):
    """Time step a step of this state would use (the adaptive rule of Sec. 3
    when ``params["adaptive_dt"]``, else ``params["dt"]``)."""
    n = _check_state(state)
    G, P = make_grid(grid), make_params(params)
    ptrs = _state_ptrs(state)
    dt = lib().ref_step_dt(ctypes.byref(G), ctypes.byref(P), n, *ptrs[:6], ptrs[7])
    if dt < 0:
        raise ValueError("ref_step_dt failed")
    return float(dt)


def count_tests(state, grid):
    n = _check_state(state)
    G = make_grid(grid)
    ptrs = _state_ptrs(state)
    return int(lib().ref_count_tests(ctypes.byref(G), n, *ptrs[:6], ptrs[7]))


def nobins(grid):
    nb = grid.get("nobin", grid["ncell"])
    return int(nb[0]) * int(nb[1]) * int(nb[2])


def step(state, grid, params, mode=MODE_BINNED, nthreads=0, pair_cap=None, moments=True):
    """One collision step in place.  Returns a dict with ``pairs`` ((k, 2)
    uint32, rows (idA, idB), idA < idB), ``counters`` (uint64[8]),
    ``globals`` (float64[8]) and ``moments`` ((nobin, 11) float64)."""
    n = _check_state(state)
    G, P = make_grid(grid), make_params(params)
    cap = n // 2 + 1 if pair_cap is None else int(pair_cap)
    pairs = np.zeros((max(cap, 1), 2), dtype=np.uint32)
    counters = np.zeros(8, dtype=np.uint64)
    glob = np.zeros(8)
    mom = np.zeros((nobins(grid), M_STRIDE)) if moments else None
    rc = lib().ref_step(ctypes.byref(G), ctypes.byref(P), n, *_state_ptrs(state), _mass_ptr(state, n), mode,
                        nthreads, _ptr(pairs), cap, _ptr(counters), _ptr(mom), _ptr(glob))
    if rc:
        raise ValueError(f"ref_step failed ({rc})")
    k = min(int(counters[CNT["pairs"]]), cap)
    return dict(pairs=pairs[:k].copy(), counters=counters, globals=glob, moments=mom)


PHASES = ("bin", "search", "pair", "scatter", "move", "moments")


def last_phase_ms():
    """Wall time (ms) of each phase of the last :func:`step` in this process."""
    out = np.zeros(len(PHASES))
    lib().ref_last_phase_ms(_ptr(out))
    return dict(zip(PHASES, out.tolist()))
