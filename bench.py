#!/usr/bin/env python3
"""Benchmark of the collision step on one MI355X.

A step is one pass of the whole path (bin key, prefix sum, scatter into
c-bin order, closest-partner search, pairing + scattering + move + moments,
per-instance reduction) over one batch of particles already resident in
HBM.  Default workload: the 16M-particle Sedov blast (128^3 c-bins, 64^3
o-bins, Kn = 1e-3, a 600-step run) with FP32 state and FP64 moments,
particle arrays kept in c-bin order between steps.

The K timed steps are spread over the run, because its c-bins fill up as
the blast front sweeps the box: a third at its start, a third at its middle
and a third at its end, the steps between them advanced untimed by graph
replay.  The whole run is also timed end to end.

Prints ONE JSON line: particle-steps/s as `value`, PCA pair tests/s, the
roofline of the dominant kernel (the partner search, timed with HIP events
recorded by the library on the stream it launches on; its FLOPs from the
measured arithmetic mix of the pair tests), per-phase times, the batched
ensemble against plain per-instance FP64 steps, and the CPU oracle timed
on bounded samples of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one unordered pair test (criteria 1-2 of Sec. 2.4, in
# the order of the step): 11 FLOP decide s0 = r.u (three differences of
# positions and of velocities, three products, two sums); the pairs that
# approach (s0 < 0) take 7 more for |u|^2 and s1 = s0 + |u|^2 dt; the pairs
# that meet criterion 1 (s0 < 0 < s1) take 12 more for t_poca = -s0 / |u|^2,
# the separation r + t_poca u there and its square d_min^2.
FLOP_S0, FLOP_S1, FLOP_DMIN = 11, 7, 12
PEAK_FLOPS = {"fp32": 157.3e12, "fp64": 78.6e12}
HBM_PEAK = 8.0e12


WORKLOAD_NAMES = {"sedov16M": "16M-particle Sedov", "sod4M": "4M-particle Sod", "sod4M_kn0.1": "4M-particle Sod at Kn 0.1",
                  "noh8M": "8M-particle Noh", "sod100k": "100k-particle Sod"}


def note(msg):
    """Progress on stderr (stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1210_8084_amd import workloads as W
    if name == "sedov16M":
        return W.sedov()
    if name == "sod4M":
        return W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4, steps=500)
    if name == "sod4M_kn0.1":
        return W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4, kn=1e-1, steps=500)
    if name == "noh8M":
        return W.noh()
    if name == "sod100k":
        return W.sod()
    raise SystemExit(f"unknown workload {name}")


def phase_bytes(rs, n, ncell_tot, nobin, reorder, colliders=0):
    """Algorithmic HBM bytes per launch of each phase (rs = bytes per real):
    what each kernel must read and write once, as listed per kernel in the
    design notes.  The move phase runs two kernels, the move and the moment
    pass (listed also on their own)."""
    rec = 8 * rs
    pkey = 8 if rs == 4 else 4   # FP32: 64-bit (d_min^2, partner) key; FP64: partner index
    acc = 128                    # exact sums of one o-bin
    src = 0 if reorder else 4
    # record, own and partner's partner key in; state, id, alive, collided flag
    # out; colliders' virial terms out
    move = n * (rec + 2 * pkey + 6 * rs + 4 + 1 + 1 + src) + colliders * 3 * rs
    # state, alive and collided flag in (colliders' virial terms too); per
    # o-bin shift and exponents in, exact sums out
    moments = n * (6 * rs + 1 + 1 + src) + colliders * 3 * rs + nobin * (24 + acc)
    return {
        "clear": 4 * ncell_tot + acc * nobin,
        # state and alive in, rank out
        "key": n * (6 * rs + 1 + 4),
        "scan": 12 * ncell_tot,
        # state, id, alive, rank, start[key] in; record (and FP32 key init, permutation) out
        "scatter": n * (6 * rs + 4 + 1 + 4 + 4 + rec + (8 if rs == 4 else 0) + src),
        # records and the c-bin starts in (each once), partner key or index out
        "search": n * (rec + pkey) + 4 * ncell_tot,
        "move": move + moments,
        "k_move": move,
        "k_moments": moments,
        "finalize": 0,
    }


def kernel_code_sha256(path):
    """SHA-256 of a kernel source with its comments and blank lines removed:
    the counter summaries stay valid across comment edits, not code edits."""
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
    return hashlib.sha256("\n".join(line for line in lines if line.strip()).encode()).hexdigest()


def read_traffic(workload, precision, shape, cbins):
    """HBM bytes per search launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source, in the launch
    shape (records per lane, lanes per work-group) and on the c-bins this run
    uses."""
    path = os.path.join(ROOT, "profiles", f"search_{workload}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_1210_8084_amd", "csrc", "tpkmc_kernels.h")
    if vals.get("kernel_code_sha256") != kernel_code_sha256(src):
        return None
    if vals.get("search_shape") != f"{shape[0]},{shape[1]}":
        return None
    if vals.get("search_cbins") != ",".join(str(int(c)) for c in cbins):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def _slab(w, frac):
    """The x < (lo + L / frac) slab of the state: the same density and c-bin
    size on 1/frac of the c-bins along x."""
    g = w.grid
    nx = max(1, g["ncell"][0] // frac)
    hi_x = g["lo"][0] + (g["hi"][0] - g["lo"][0]) * nx / g["ncell"][0]
    sel = w.state["x"] < hi_x
    st = {k: np.ascontiguousarray(v[sel]) for k, v in w.state.items()}
    sg = dict(g, hi=(hi_x, g["hi"][1], g["hi"][2]), ncell=(nx, g["ncell"][1], g["ncell"][2]),
              nobin=(max(1, g["nobin"][0] // frac), g["nobin"][1], g["nobin"][2]))
    return st, sg, hi_x


def cpu_baseline(w, nthreads):
    """The oracle as it stands, on bounded samples of the same workload, on
    `nthreads` host threads and on one: one full step of an x-slab with the
    same density and c-bin size (the lower half with every thread, 1/32 of
    the box on one thread) for uniform workloads, else the closest-partner
    search of a random particle subset scaled to all particles."""
    from oracle import ref
    if w.name in ("sedov", "equilibration"):
        res = {}
        for label, frac, nt in (("all", 2, nthreads), ("one_thread", 32, 1)):
            note(f"CPU oracle: {label} ({nt} threads)")
            st, sg, hi_x = _slab(w, frac)
            n = len(st["x"])
            t0 = time.perf_counter()
            ref.step(st, sg, w.params, nthreads=nt)
            t = time.perf_counter() - t0
            res[label] = dict(value=n / t, threads=nt, seconds=round(t, 3),
                              phases_ms={k: round(v, 1) for k, v in ref.last_phase_ms().items()},
                              sample=(f"one oracle step of the x < {hi_x:g} slab of the same state: {n} particles, "
                                      f"{sg['ncell'][0]}x{sg['ncell'][1]}x{sg['ncell'][2]} c-bins"))
        return res
    res = {}
    rng = np.random.default_rng(0)
    for label, frac, nt in (("all", 64, nthreads), ("one_thread", 1024, 1)):
        sub = np.sort(rng.choice(w.n, size=max(1, w.n // frac), replace=False))
        t0 = time.perf_counter()
        ref.best_sample(w.state, w.grid, w.params, sub, nthreads=nt)
        t = (time.perf_counter() - t0) * (w.n / len(sub))
        res[label] = dict(value=w.n / t, threads=nt, seconds=round(t * len(sub) / w.n, 3),
                          sample=(f"oracle closest-partner search of {len(sub)} random particles (1/{frac}), "
                                  f"time scaled to all {w.n}"))
    return res


def batched_ensemble(args, K, Wm):
    """64 independent Sod/Noh/Sedov instances (log-uniform sizes and Knudsen
    numbers) stepped together: FP32 state, one captured HIP graph per run,
    launch shape from the autotuner; against the same instances run one
    after another as plain FP64 steps (default launch shape) over the same
    steps from the same state.  The L1 distance between the two runs' o-bin
    density profiles after those steps bounds the difference of their L1
    errors against any reference profile (triangle inequality)."""
    import torch
    from paper_1210_8084_amd import tpkmc as T
    from paper_1210_8084_amd import workloads as W
    note("batched ensemble: drawing 64 instances")
    ws = W.batched(n_inst=64, seed=1, scale=args.batch_scale)
    st = {k: np.concatenate([w.state[k] for w in ws]) for k in ("x", "y", "z", "vx", "vy", "vz", "alive")}
    ids, specs, off = [], [], 0
    for w in ws:
        ids.append(w.state["id"].astype(np.int64) + off)
        specs.append((off, w.n, w.grid, w.params))
        off += w.n
    st["id"] = np.concatenate(ids).astype(np.uint32)
    ntot = off
    nobs = [T.nobins(w.grid) for w in ws]
    ncell = sum(T.ncells(w.grid) + 1 for w in ws)
    nob = sum(nobs)
    stream = torch.cuda.Stream()
    eng = T.Engine(max_particles=ntot, max_cells=ncell, max_obins=nob, precision=T.FP32, max_instances=len(ws))
    with torch.cuda.stream(stream):
        dst = T.to_device(st, T.FP32)
        out = T.make_outputs(len(ws), nob)
    torch.cuda.synchronize()
    eng.autotune(dst, specs, stream=stream)
    flags = T.ALLOW_REORDER
    eng.run(dst, specs, Wm, out, flags=flags, stream=stream)
    torch.cuda.synchronize()
    # Per-kernel times from one plain batched step with event profiling.
    eng.profile(True)
    eng.profile_read()
    eng.step_batched(dst, [(o, c, g, dict(p, step=p["step"] + Wm)) for o, c, g, p in specs], out, flags=flags,
                     stream=stream)
    torch.cuda.synchronize()
    prof = eng.profile_read()
    eng.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.run(dst, [(o, c, g, dict(p, step=p["step"] + Wm + 1)) for o, c, g, p in specs], K, out, flags=flags,
            stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c = out.host()["counters"]
    alive_last = float(c[:, T.CNT["alive"]].sum())
    value = alive_last * K / elapsed
    counts32 = out.moments[:, 0].cpu().numpy()
    note(f"batched ensemble: FP32 graph {1e3 * elapsed / K:.2f} ms per step; plain FP64 comparator")
    eng.close()
    del dst
    torch.cuda.empty_cache()
    # The same instances one after another, plain FP64 steps over the same
    # Wm + 1 + K steps; the first step of each instance is not timed.
    nsteps = Wm + 1 + K
    t64, ps64 = 0.0, 0.0
    l1 = []
    kinds = []
    ob0 = 0
    for k, w in enumerate(ws):
        if k % 16 == 0:
            note(f"batched ensemble: plain FP64 instance {k}/{len(ws)}")
        g, p = w.grid, w.params
        e = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP64)
        d = T.to_device(w.state, T.FP64)
        o = T.make_outputs(1, T.nobins(g))
        e.step(d, g, dict(p, step=p["step"]), o, flags=flags, stream=stream)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s in range(1, nsteps):
            e.step(d, g, dict(p, step=p["step"] + s), o, flags=flags, stream=stream)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - ts
        ps64 += w.n * (nsteps - 1)
        c64 = o.moments[:, 0].cpu().numpy()
        c32 = counts32[ob0:ob0 + nobs[k]]
        ob0 += nobs[k]
        l1.append(float(np.abs(c32 - c64).sum() / max(c64.sum(), 1.0)))
        kinds.append(w.info["kind"])
        e.close()
        del d
    torch.cuda.empty_cache()
    v64 = ps64 / t64
    l1 = np.array(l1)
    return {
        "value": value, "unit": "particle-steps/s", "instances": len(ws), "particles": ntot,
        "ms_per_step": 1e3 * elapsed / K, "steps": K,
        "plain_fp64_sequential": {"value": v64, "unit": "particle-steps/s", "steps_per_instance": nsteps - 1},
        "batched_fp32_over_plain_fp64": value / v64,
        "l1_density_fp32_vs_fp64": {
            "after_steps": nsteps, "mean": float(l1.mean()), "max": float(l1.max()),
            **{kind: float(l1[[x == kind for x in kinds]].mean()) for kind in ("sod", "noh", "sedov")}},
        "search_ms": round(prof["search"][0], 3),
        "phases_ms": {ph: round(ms / n, 4) for ph, (ms, n) in prof.items() if n},
    }


def run_batched(args):
    """The batched ensemble as the workload of its own JSON line."""
    K, Wm = args.steps, args.warmup
    b = batched_ensemble(args, K, Wm)
    line = {
        "metric": "particle-steps/s (batched ensemble: 64 Sod/Noh/Sedov instances, FP32 state, one HIP graph)",
        "value": b["value"], "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": b["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded initial states of the paper's test problems)",
        "config": {"workload": "batched64", "instances": b["instances"], "particles": b["particles"],
                   "sizes": "log-uniform 5e4-2e6" if args.batch_scale == 1.0 else f"scaled x{args.batch_scale}",
                   "kn": "log-uniform 1e-3-1e-1", "state_precision": "fp32", "moments": "fp64"},
        "plain_fp64_sequential": b["plain_fp64_sequential"],
        "batched_fp32_over_plain_fp64": b["batched_fp32_over_plain_fp64"],
        "l1_density_fp32_vs_fp64": b["l1_density_fp32_vs_fp64"],
        "phases": b["phases_ms"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def windows_of(total, K, Wm):
    """Timed windows (first step, steps) over a run of `total` steps: a third
    of K at its start (after Wm warm-up steps), a third at its middle and a
    third at its end; a single window when the run is too short."""
    if total < Wm + 3 * K or K < 3:
        return [(Wm, K)]
    k2 = K // 3
    k1 = K - 2 * k2
    return [(Wm, k1), (total // 2, k2), (total - k2, k2)]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sedov16M")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-whole-run", action="store_true", help="skip the end-to-end timing of the whole run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-ensemble keys")
    ap.add_argument("--start-only", action="store_true",
                    help="time all K steps from the start of the run (no windows at its middle and end)")
    ap.add_argument("--search", default="auto",
                    help="'auto': the autotuner's results-neutral choice of c-bins and search launch shape; or a "
                         "fixed shape 'G,B' (records per lane, lanes per work-group) on the configured c-bins")
    ap.add_argument("--search-order", type=int, default=None,
                    help="search work-group order in place of the tuned one: 0 contiguous per XCD, S > 0 chunks "
                         "of S work-groups dealt round-robin")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="batched ensemble: scale every instance size")
    ap.add_argument("--batch-steps", type=int, default=10, help="batched ensemble: timed steps")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the run, copy a 1 GiB device buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the collision step on a single GPU and "
              "does not shard it across GPUs; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched64":
        run_batched(args)
        return

    import ctypes
    import torch
    from paper_1210_8084_amd import tpkmc as T

    note(f"workload {args.workload}")
    w = make_workload(args.workload)
    prec = T.FP32 if args.precision == "fp32" else T.FP64
    rs = 4 if prec == T.FP32 else 8
    g, p = w.grid, w.params
    ncell_tot, nob = T.ncells(g) + 1, T.nobins(g)
    eng = T.Engine(max_particles=w.n, max_cells=ncell_tot, max_obins=nob, precision=prec)
    stream = torch.cuda.Stream()
    flags = T.ALLOW_REORDER
    K, Wm = args.steps, args.warmup
    with torch.cuda.stream(stream):
        dst = T.to_device(w.state, prec)
        moments = torch.zeros((nob, T.MOMENT_STRIDE), dtype=torch.float64, device="cuda")
        counters = torch.zeros((max(K, 1), 8), dtype=torch.int64, device="cuda")
        glob = torch.zeros((max(K, 1), 8), dtype=torch.float64, device="cuda")
        gcount = torch.zeros((1, 8), dtype=torch.int64, device="cuda")
        gglob = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    gout = T.DeviceOutputs(counters=gcount, globals=gglob, moments=moments, pairs=None, pair_cap=0)

    def step(k_step, k_out):
        G, P, S = T.make_grid(g), T.make_params(dict(p, step=k_step), flags), T.particles(dst)
        O = T.Outputs()
        O.pairs, O.pair_cap = None, 0
        O.counters = counters[k_out].data_ptr()
        O.globals = glob[k_out].data_ptr()
        O.moments = moments.data_ptr()
        rc = T.lib().tpkmc_step(eng.h, ctypes.byref(G), ctypes.byref(P), ctypes.byref(S), ctypes.byref(O),
                                ctypes.c_void_p(stream.cuda_stream))
        if rc:
            raise T.TpkmcError(rc, "tpkmc_step")

    def advance(first, nsteps):
        if nsteps > 0:
            eng.run(dst, [(0, w.n, g, dict(p, step=first))], nsteps, gout, flags=flags, stream=stream)

    torch.cuda.synchronize()
    if args.search == "auto":
        eng.autotune(dst, [(0, w.n, g, p)], stream=stream)
    else:
        eng.set_search(*[int(v) for v in args.search.split(",")])
    if args.search_order is not None:
        eng.set_search_order(args.search_order)
    for k in range(Wm):
        step(k, 0)
    torch.cuda.synchronize()

    wins = [(Wm, K)] if args.start_only else windows_of(w.steps, K, Wm)
    at = Wm
    elapsed, k_out = 0.0, 0
    prof_tot = {}
    win_rows = []
    flops = 0.0
    search_s = 0.0
    for first, kw in wins:
        note(f"timed window at step {first} ({kw} steps)")
        advance(at, first - at)
        torch.cuda.synchronize()
        tests_w, s0_w, c1_w = eng.search_mix(dst, [(0, w.n, g, dict(p, step=first))], stream=stream)
        eng.profile(True)
        eng.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(kw):
            step(first + k, k_out + k)
        torch.cuda.synchronize()
        dt_w = time.perf_counter() - t0
        prof = eng.profile_read()
        eng.profile(False)
        elapsed += dt_w
        c = counters[k_out:k_out + kw].cpu().numpy()
        k_out += kw
        at = first + kw
        for ph, (ms, n) in prof.items():
            a = prof_tot.setdefault(ph, [0.0, 0])
            a[0] += ms
            a[1] += n
        f_test = FLOP_S0 + (FLOP_S1 * s0_w + FLOP_DMIN * c1_w) / max(tests_w, 1)
        tests_steps = float(c[:, T.CNT["tests"]].sum())
        flops += tests_steps * f_test
        search_s += prof["search"][0] / 1e3
        win_rows.append({"first_step": first, "steps": kw, "ms_per_step": round(1e3 * dt_w / kw, 4),
                         "search_ms": round(prof["search"][0] / max(prof["search"][1], 1), 4),
                         "pairs_per_step": float(c[:, T.CNT["pairs"]].mean()),
                         "pair_tests_per_step": tests_steps / kw,
                         "approaching_fraction": round(s0_w / max(tests_w, 1), 4),
                         "criterion1_fraction": round(c1_w / max(tests_w, 1), 5),
                         "flop_per_pair_test": round(f_test, 3)})
    c = counters[:K].cpu().numpy()
    alive = float(c[:, T.CNT["alive"]].sum())
    tests = float(c[:, T.CNT["tests"]].sum())
    pairs = float(c[:, T.CNT["pairs"]].sum())
    value = alive / elapsed
    ms_per_step = 1e3 * elapsed / K

    whole = None
    if not args.no_whole_run and w.steps > 0:
        note(f"whole run: {w.steps} steps")
        with torch.cuda.stream(stream):
            fresh = T.to_device(w.state, prec)
            for k in dst:
                dst[k].copy_(fresh[k])
            del fresh
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        advance(0, w.steps)
        torch.cuda.synchronize()
        tw = time.perf_counter() - tw0
        alive_end = float(gcount[0, T.CNT["alive"]].cpu())
        whole = {"steps": w.steps, "ms_per_step": round(1e3 * tw / w.steps, 4),
                 "value": alive_end * w.steps / tw, "unit": "particle-steps/s",
                 "timing": "one HIP graph of the step replayed for every step of the run, from the initial state"}

    search_ms, search_n = prof_tot["search"]
    achieved = flops / search_s if search_s > 0 else 0.0
    peak = PEAK_FLOPS[args.precision]
    shape = eng.get_search()
    shape = (shape[0], min(shape[1], 256 // shape[0]))
    order = eng.search_order()
    cbins = list(eng.tuned_cells(0)) if args.search == "auto" else list(g["ncell"])
    traffic = read_traffic(args.workload, args.precision, shape, cbins)
    bytes_per = phase_bytes(rs, w.n, int(np.prod(cbins)) + 1, nob, True, colliders=2 * pairs / max(K, 1))
    phases = {}
    for ph, (ms, n) in prof_tot.items():
        if n:
            avg = ms / n
            b = bytes_per.get(ph, 0)
            phases[ph] = {"ms": round(avg, 5), "alg_GBps": round(b / (avg / 1e3) / 1e9, 1) if b else None,
                          "hbm_frac": round(b / (avg / 1e3) / HBM_PEAK, 3) if b else None}
    eng.close()
    del dst
    torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        batched = batched_ensemble(args, args.batch_steps, 2)

    cpu = None
    if not args.no_cpu:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res = cpu_baseline(w, nthreads)
        cpu = {"value": res["all"]["value"], "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
               "sample": res["all"]["sample"], "seconds": res["all"]["seconds"],
               "phases_ms": res["all"].get("phases_ms"),
               "one_thread": res["one_thread"], "host": host_info()}

    line = {
        "metric": f"particle-steps/s (collision step, {WORKLOAD_NAMES[args.workload]}, "
                  f"{args.precision.upper()} state)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == T.FP32 else "f64",
        "data": "synthetic (seeded initial state of the paper's test problem)",
        "config": {"workload": args.workload, "particles": w.n, "ncell": list(g["ncell"]),
                   "search_cbins": cbins,
                   "nobin": list(g["nobin"]), "kn": w.info.get("kn"), "run_steps": w.steps,
                   "state_precision": args.precision, "moments": "fp64",
                   "particle_order": "c-bin order kept between steps",
                   "timed_steps": "start, middle and end of the run" if len(wins) == 3 else "start of the run"},
        "pair_tests_per_s": tests / elapsed,
        "pairs_per_step": pairs / K,
        "windows": win_rows,
        "whole_run": whole,
        "roofline": {"kernel": "k_search (closest-partner search)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "algorithmic_bytes": bytes_per["search"],
                     "search_shape": list(shape),
                     "search_order": order,
                     "avg_launch_ms": search_ms / max(search_n, 1),
                     "flop_per_pair_test": flops / max(tests, 1.0),
                     "flop_model": f"{FLOP_S0} per test + {FLOP_S1} per approaching pair + {FLOP_DMIN} per pair "
                                   "meeting criterion 1, counts from tpkmc_search_mix"},
        "phases": phases,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dstb = torch.empty_like(src)
        for _ in range(3):
            dstb.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": src.numel() * 4, "copies": 3}), flush=True)


if __name__ == "__main__":
    main()
