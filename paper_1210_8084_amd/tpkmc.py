"""Thin ctypes binding of libtpkmc (``include/tpkmc.h``).

Argument marshalling only: every step of the collision step runs in the HIP
kernels of ``libtpkmc.so``.  PyTorch provides device memory (tensors) and
streams.  There is no fallback: if the library is not built or no GPU is
visible, :func:`lib` raises.

Particle state on the device is a dict of tensors ``x y z vx vy vz``
(float64 for an FP64 engine, float32 for FP32), ``id`` (int32 storage read
as uint32) and ``alive`` (uint8).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpkmc.so")

FP64, FP32 = 0, 1
REFLECT, PERIODIC, ABSORB = 0, 1, 2
EMIT_PAIRS, ALLOW_REORDER, ADAPTIVE_DT, PLANAR, RANK_TIME, PAIR_RANDOM = 1, 2, 4, 8, 16, 32
STATUS_PAIR_OVERFLOW, STATUS_NONFINITE, STATUS_FAST = 1, 2, 4
CNT = dict(alive=0, pairs=1, tests=2, cand=3, fast=4, nonfinite=5, absorbed=6, have_best=7)
GLB = dict(px=0, py=1, pz=2, ekin=3, vmax2=4, virial=5, mass=6, dt=7)
PHASES = ("clear", "key", "scan", "scatter", "search", "move", "finalize")
MOMENT_STRIDE = 12

OK, EINVAL, ENOMEM, EHIP, ECAPACITY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class TpkmcError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("max_particles", ctypes.c_int64), ("max_cells", ctypes.c_int64),
                ("max_obins", ctypes.c_int64), ("max_instances", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Grid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("ncell", ctypes.c_int32 * 3), ("bc", ctypes.c_int32 * 3),
                ("nobin", ctypes.c_int32 * 3), ("pad", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("step", ctypes.c_uint64),
                ("instance", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz")] + \
               [("id", ctypes.c_void_p), ("alive", ctypes.c_void_p), ("mass", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_void_p), ("pair_cap", ctypes.c_int64), ("counters", ctypes.c_void_p),
                ("moments", ctypes.c_void_p), ("globals", ctypes.c_void_p)]


class Instance(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("count", ctypes.c_int64), ("grid", Grid), ("params", Params)]


_lib = None
_P = ctypes.c_void_p


def lib():
    """Load libtpkmc.so (built in-tree by ``build.build()``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtpkmc.so is not built ({LIB_PATH}); run paper_1210_8084_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.tpkmc_version.restype = ctypes.c_int
        L.tpkmc_strerror.restype = ctypes.c_char_p
        L.tpkmc_strerror.argtypes = [ctypes.c_int]
        L.tpkmc_create.argtypes = [_P, _P]
        L.tpkmc_destroy.argtypes = [_P]
        L.tpkmc_step.argtypes = [_P, _P, _P, _P, _P, _P]
        L.tpkmc_step_batched.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P]
        L.tpkmc_run.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]
        L.tpkmc_autotune.argtypes = [_P, _P, _P, ctypes.c_int32, _P]
        L.tpkmc_status.argtypes = [_P, _P]
        L.tpkmc_profile_enable.argtypes = [_P, ctypes.c_int32]
        L.tpkmc_profile_read.argtypes = [_P, _P, _P, ctypes.c_int32]
        L.tpkmc_set_search.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
        L.tpkmc_get_search.argtypes = [_P, _P, _P]
        L.tpkmc_step_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]
        L.tpkmc_search_mix.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P]
        L.tpkmc_tuned_cells.argtypes = [_P, ctypes.c_int32, _P]
        L.tpkmc_tuned_speed.argtypes = [_P, ctypes.c_int32, _P]
        L.tpkmc_search_order.argtypes = [_P, _P]
        L.tpkmc_set_search_order.argtypes = [_P, ctypes.c_int32]
        for f in ("tpkmc_create", "tpkmc_destroy", "tpkmc_step", "tpkmc_step_batched", "tpkmc_run",
                  "tpkmc_autotune", "tpkmc_status", "tpkmc_profile_enable", "tpkmc_profile_read",
                  "tpkmc_set_search", "tpkmc_get_search", "tpkmc_step_noalloc", "tpkmc_search_mix",
                  "tpkmc_tuned_cells", "tpkmc_tuned_speed", "tpkmc_search_order", "tpkmc_set_search_order"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().tpkmc_strerror(int(code)).decode()
    except RuntimeError:
        return "unknown"


def _check(code, what):
    if code != OK:
        raise TpkmcError(code, what)


def make_grid(g) -> Grid:
    G = Grid()
    for a in range(3):
        G.lo[a], G.hi[a] = float(g["lo"][a]), float(g["hi"][a])
        G.ncell[a], G.bc[a] = int(g["ncell"][a]), int(g["bc"][a])
        G.nobin[a] = int(g.get("nobin", g["ncell"])[a])
    return G


def make_params(p, flags=0) -> Params:
    P = Params()
    P.sigma, P.mass, P.dt = float(p["sigma"]), float(p.get("mass", 1.0)), float(p["dt"])
    P.seed, P.step = int(p.get("seed", 0)), int(p.get("step", 0))
    P.instance, P.flags = int(p.get("instance", 0)), int(flags)
    if p.get("adaptive_dt"):
        P.flags |= ADAPTIVE_DT
    if p.get("planar"):
        P.flags |= PLANAR
    if p.get("rank_time"):
        P.flags |= RANK_TIME
    if p.get("pair_random"):
        P.flags |= PAIR_RANDOM
    return P


def nobins(g) -> int:
    nb = g.get("nobin", g["ncell"])
    return int(nb[0]) * int(nb[1]) * int(nb[2])


def ncells(g) -> int:
    return int(g["ncell"][0]) * int(g["ncell"][1]) * int(g["ncell"][2])


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def to_device(state, precision=FP64, device="cuda"):
    """Copy a host state (numpy, float64) to device tensors."""
    torch = _torch()
    dt = torch.float64 if precision == FP64 else torch.float32
    out = {k: torch.as_tensor(np.ascontiguousarray(state[k]), device=device).to(dt).contiguous()
           for k in ("x", "y", "z", "vx", "vy", "vz")}
    out["id"] = torch.as_tensor(np.ascontiguousarray(state["id"]).view(np.int32), device=device).contiguous()
    alive = state.get("alive")
    if alive is None:
        alive = np.ones(len(state["x"]), np.uint8)
    out["alive"] = torch.as_tensor(np.ascontiguousarray(alive, dtype=np.uint8), device=device).contiguous()
    if state.get("mass") is not None:
        out["mass"] = torch.as_tensor(np.ascontiguousarray(state["mass"]), device=device).to(dt).contiguous()
    return out


def to_host(dstate):
    """Device state -> numpy (float64 for either precision; ids as uint32)."""
    out = {k: dstate[k].detach().cpu().numpy().astype(np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
    out["id"] = dstate["id"].detach().cpu().numpy().view(np.uint32).copy()
    out["alive"] = dstate["alive"].detach().cpu().numpy().copy()
    if dstate.get("mass") is not None:
        out["mass"] = dstate["mass"].detach().cpu().numpy().astype(np.float64)
    return out


def particles(dstate, with_alive=True) -> Particles:
    S = Particles()
    S.n = int(dstate["x"].numel())
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        setattr(S, k, dstate[k].data_ptr())
    S.id = dstate["id"].data_ptr()
    S.alive = dstate["alive"].data_ptr() if with_alive and dstate.get("alive") is not None else None
    S.mass = dstate["mass"].data_ptr() if dstate.get("mass") is not None else None
    return S


@dataclass
class DeviceOutputs:
    counters: object
    globals: object
    moments: object
    pairs: object
    pair_cap: int

    def struct(self) -> Outputs:
        O = Outputs()
        O.pairs = self.pairs.data_ptr() if self.pairs is not None else None
        O.pair_cap = int(self.pair_cap)
        O.counters = self.counters.data_ptr() if self.counters is not None else None
        O.moments = self.moments.data_ptr() if self.moments is not None else None
        O.globals = self.globals.data_ptr() if self.globals is not None else None
        return O

    def host(self, n_pairs=None):
        c = self.counters.cpu().numpy().view(np.uint64) if self.counters is not None else None
        out = dict(counters=c,
                   globals=self.globals.cpu().numpy() if self.globals is not None else None,
                   moments=self.moments.cpu().numpy() if self.moments is not None else None)
        if self.pairs is not None:
            k = int(c[:, CNT["pairs"]].sum()) if (n_pairs is None and c is not None) else int(n_pairs or 0)
            k = min(k, self.pair_cap)
            out["pairs"] = self.pairs[:k].cpu().numpy().view(np.uint32).copy()
        return out


def make_outputs(n_inst=1, n_obins=0, pair_cap=0, device="cuda", moments=True, globals_=True, counters=True):
    torch = _torch()
    return DeviceOutputs(
        counters=torch.zeros((n_inst, 8), dtype=torch.int64, device=device) if counters else None,
        globals=torch.zeros((n_inst, 8), dtype=torch.float64, device=device) if globals_ else None,
        moments=torch.zeros((max(n_obins, 1), MOMENT_STRIDE), dtype=torch.float64, device=device)
        if (moments and n_obins > 0) else None,
        pairs=torch.zeros((max(pair_cap, 1), 2), dtype=torch.int32, device=device) if pair_cap > 0 else None,
        pair_cap=int(pair_cap))


def _stream_ptr(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def step_noalloc(dstate, grid, params, out=None, flags=0, precision=FP64, device=0, stream=None, rc_only=False):
    """One step through ``tpkmc_step_noalloc``: no handle, scratch in the
    library's static device array (no device allocation)."""
    G, P, S = make_grid(grid), make_params(params, flags), particles(dstate)
    O = out.struct() if out is not None else Outputs()
    rc = lib().tpkmc_step_noalloc(int(precision), int(device), ctypes.byref(G), ctypes.byref(P), ctypes.byref(S),
                                  ctypes.byref(O), _P(_stream_ptr(stream)))
    if rc_only:
        return rc
    _check(rc, "tpkmc_step_noalloc")


class Engine:
    """Owns one tpkmc handle (device scratch sized by the capacities)."""

    def __init__(self, max_particles, max_cells, max_obins=1, precision=FP64, max_instances=1, device=0):
        self.precision = precision
        cfg = Config(max_particles=int(max_particles), max_cells=int(max_cells), max_obins=int(max_obins),
                     max_instances=int(max_instances), precision=int(precision), device=int(device), flags=0)
        h = ctypes.c_void_p()
        _check(lib().tpkmc_create(ctypes.byref(cfg), ctypes.byref(h)), "tpkmc_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().tpkmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dstate, grid, params, out=None, flags=0, stream=None, rc_only=False):
        G, P, S = make_grid(grid), make_params(params, flags), particles(dstate)
        O = out.struct() if out is not None else Outputs()
        rc = lib().tpkmc_step(self.h, ctypes.byref(G), ctypes.byref(P), ctypes.byref(S), ctypes.byref(O),
                              _P(_stream_ptr(stream)))
        if rc_only:
            return rc
        _check(rc, "tpkmc_step")

    @staticmethod
    def instances(specs, flags=0):
        """specs: list of (offset, count, grid, params)."""
        arr = (Instance * len(specs))()
        for k, (off, cnt, g, p) in enumerate(specs):
            arr[k].offset, arr[k].count = int(off), int(cnt)
            arr[k].grid = make_grid(g)
            arr[k].params = make_params(p, flags)
        return arr

    def step_batched(self, dstate, specs, out=None, flags=0, stream=None):
        arr = self.instances(specs, flags)
        S = particles(dstate)
        O = out.struct() if out is not None else Outputs()
        _check(lib().tpkmc_step_batched(self.h, ctypes.byref(S), arr, len(specs), ctypes.byref(O),
                                        _P(_stream_ptr(stream))), "tpkmc_step_batched")

    def run(self, dstate, specs, nsteps, out=None, flags=0, stream=None):
        arr = self.instances(specs, flags)
        S = particles(dstate)
        O = out.struct() if out is not None else Outputs()
        _check(lib().tpkmc_run(self.h, ctypes.byref(S), arr, len(specs), int(nsteps), ctypes.byref(O),
                               _P(_stream_ptr(stream))), "tpkmc_run")

    def autotune(self, dstate, specs, stream=None):
        arr = self.instances(specs)
        S = particles(dstate)
        _check(lib().tpkmc_autotune(self.h, ctypes.byref(S), arr, len(specs), _P(_stream_ptr(stream))),
               "tpkmc_autotune")

    def search_mix(self, dstate, specs, stream=None):
        """(tests, approaching, meeting criterion 1) of the search on this
        state; the state is not modified."""
        arr = self.instances(specs)
        S = particles(dstate)
        counts = np.zeros(3, dtype=np.uint64)
        _check(lib().tpkmc_search_mix(self.h, ctypes.byref(S), arr, len(specs), counts.ctypes.data_as(_P),
                                      _P(_stream_ptr(stream))), "tpkmc_search_mix")
        return tuple(int(v) for v in counts)

    def search_order(self):
        """Work-group order of the search: 0 contiguous per XCD, S chunks of S."""
        v = ctypes.c_int32(0)
        _check(lib().tpkmc_search_order(self.h, ctypes.byref(v)), "tpkmc_search_order")
        return int(v.value)

    def set_search_order(self, order):
        _check(lib().tpkmc_set_search_order(self.h, int(order)), "tpkmc_set_search_order")

    def tuned_cells(self, k=0):
        """The slow particles' c-bins per axis that autotune chose for batch
        position k."""
        n = (ctypes.c_int32 * 3)()
        _check(lib().tpkmc_tuned_cells(self.h, int(k), n), "tpkmc_tuned_cells")
        return tuple(int(v) for v in n)

    def tuned_speed(self, k=0):
        """Speed bound of the slow particles at batch position k (0: no split)."""
        v = ctypes.c_double()
        _check(lib().tpkmc_tuned_speed(self.h, int(k), ctypes.byref(v)), "tpkmc_tuned_speed")
        return float(v.value)

    def set_search(self, group, block):
        """Fix the partner-search launch shape: `group` records per lane (1, 2
        or 4) and `block` lanes per work-group (64, 128 or 256)."""
        _check(lib().tpkmc_set_search(self.h, int(group), int(block)), "tpkmc_set_search")

    def get_search(self):
        g, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().tpkmc_get_search(self.h, ctypes.byref(g), ctypes.byref(b)), "tpkmc_get_search")
        return int(g.value), int(b.value)

    def status(self) -> int:
        v = ctypes.c_int32(0)
        _check(lib().tpkmc_status(self.h, ctypes.byref(v)), "tpkmc_status")
        return int(v.value)

    def profile(self, on=True):
        _check(lib().tpkmc_profile_enable(self.h, 1 if on else 0), "tpkmc_profile_enable")

    def profile_read(self):
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int64)
        _check(lib().tpkmc_profile_read(self.h, ms.ctypes.data_as(_P), n.ctypes.data_as(_P), len(PHASES)),
               "tpkmc_profile_read")
        return {ph: (float(ms[k]), int(n[k])) for k, ph in enumerate(PHASES)}
