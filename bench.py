#!/usr/bin/env python3
"""Benchmark of the collision step on one MI355X.

A step is one pass of the whole path (bin key, prefix sum, scatter into
c-bin order, closest-partner search, pairing + scattering + move + moments,
per-instance reduction) over one batch of particles already resident in
HBM.  Default workload: the 16M-particle Sedov blast (128^3 c-bins, 64^3
o-bins, Kn = 1e-3) with FP32 state and FP64 moments, particle arrays kept in
c-bin order between steps.

Prints ONE JSON line: particle-steps/s as `value`, PCA pair tests/s, the
roofline of the dominant kernel (the partner search, timed with HIP events
recorded by the library on the stream it launches on), per-phase times and
the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one unordered pair test: criterion 1 (closest approach
# reached within the step) must be decided for every pair of the
# neighbourhood -- six coordinate differences, the dot products r.u and |u|^2
# (3 products + 2 sums each) and s1 = r.u + |u|^2 dt (2 FLOP).
FLOP_PER_TEST = 18
PEAK_FLOPS = {"fp32": 157.3e12, "fp64": 78.6e12}
HBM_PEAK = 8.0e12
MOMENT_VALUES = 12  # doubles per o-bin


WORKLOAD_NAMES = {"sedov16M": "16M-particle Sedov", "sod4M": "4M-particle Sod", "sod4M_kn0.1": "4M-particle Sod at Kn 0.1",
                  "noh8M": "8M-particle Noh", "sod100k": "100k-particle Sod"}


def make_workload(name):
    from paper_1210_8084_amd import workloads as W
    if name == "sedov16M":
        return W.sedov()
    if name == "sod4M":
        return W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4)
    if name == "sod4M_kn0.1":
        return W.sod(n=4_000_000, ncell=1000, nobin=200, dt=1.134e-4, kn=1e-1)
    if name == "noh8M":
        return W.noh()
    if name == "sod100k":
        return W.sod()
    raise SystemExit(f"unknown workload {name}")


def phase_bytes(rs, n, ncell_tot, nobin, reorder):
    """Algorithmic HBM bytes per launch of each phase (rs = bytes per real)."""
    rec = 8 * rs
    return {
        "clear": 4 * ncell_tot + 8 * MOMENT_VALUES * nobin,
        "key": n * (6 * rs + 1 + 4),
        "scan": 12 * ncell_tot,
        "scatter": n * (6 * rs + 4 + 1 + 4 + 4 + rec + (0 if reorder else 4)),
        "search": n * (rec + 4) + 4 * ncell_tot,
        "move": n * (rec + 4 + 6 * rs + 1 + (4 if reorder else 4)) + 2 * 8 * MOMENT_VALUES * nobin,
        "finalize": 0,
    }


def kernel_code_sha256(path):
    """SHA-256 of a kernel source with its comments and blank lines removed:
    the counter summaries stay valid across comment edits, not code edits."""
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
    return hashlib.sha256("\n".join(line for line in lines if line.strip()).encode()).hexdigest()


def read_traffic(workload, precision, shape):
    """HBM bytes per search launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and in the launch
    shape (records per lane, lanes per work-group) this run uses."""
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
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, nthreads):
    """The oracle as it stands, on a bounded sample of the same workload:
    one full step of the lower half (an x-slab with the same density and
    c-bin size) for uniform workloads, about ten seconds on 16 host threads,
    else the closest-partner search of a random particle subset scaled to
    all particles."""
    from oracle import ref
    from paper_1210_8084_amd import workloads as W
    g = w.grid
    if w.name in ("sedov", "equilibration"):
        frac = 2
        nx = g["ncell"][0] // frac
        hi_x = g["lo"][0] + (g["hi"][0] - g["lo"][0]) * nx / g["ncell"][0]
        sel = w.state["x"] < hi_x
        st = {k: np.ascontiguousarray(v[sel]) for k, v in w.state.items()}
        sg = dict(g, hi=(hi_x, g["hi"][1], g["hi"][2]), ncell=(nx, g["ncell"][1], g["ncell"][2]),
                  nobin=(max(1, g["nobin"][0] // frac), g["nobin"][1], g["nobin"][2]))
        n = len(st["x"])
        t0 = time.perf_counter()
        ref.step(st, sg, w.params, nthreads=nthreads)
        t = time.perf_counter() - t0
        sample = (f"one oracle step of the x < {hi_x:g} slab of the same state: {n} particles, "
                  f"{sg['ncell'][0]}x{sg['ncell'][1]}x{sg['ncell'][2]} c-bins")
        return n / t, sample
    frac = 64
    rng = np.random.default_rng(0)
    sub = np.sort(rng.choice(w.n, size=max(1, w.n // frac), replace=False))
    t0 = time.perf_counter()
    ref.best_sample(w.state, g, w.params, sub, nthreads=nthreads)
    t = (time.perf_counter() - t0) * (w.n / len(sub))
    sample = (f"oracle closest-partner search of {len(sub)} random particles (1/{frac}), "
              f"time scaled to all {w.n}")
    return w.n / t, sample


def run_batched(args):
    """64 independent Sod/Noh/Sedov instances (log-uniform sizes and Knudsen
    numbers) stepped together: FP32 state, one captured HIP graph per run,
    launch shape from the autotuner; compared with the same instances run one
    after another as plain FP64 steps with the default launch shape."""
    import ctypes
    import torch
    from paper_1210_8084_amd import tpkmc as T
    from paper_1210_8084_amd import workloads as W
    ws = W.batched(n_inst=64, seed=1, scale=args.batch_scale)
    st = {k: np.concatenate([w.state[k] for w in ws]) for k in ("x", "y", "z", "vx", "vy", "vz", "alive")}
    ids, specs, off = [], [], 0
    for w in ws:
        ids.append(w.state["id"].astype(np.int64) + off)
        specs.append((off, w.n, w.grid, w.params))
        off += w.n
    st["id"] = np.concatenate(ids).astype(np.uint32)
    ntot = off
    ncell = sum(T.ncells(w.grid) + 1 for w in ws)
    nob = sum(T.nobins(w.grid) for w in ws)
    K, Wm = args.steps, args.warmup
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
    tests_one = float(out.host()["counters"][:, T.CNT["tests"]].sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.run(dst, [(o, c, g, dict(p, step=p["step"] + Wm + 1)) for o, c, g, p in specs], K, out, flags=flags,
            stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c = out.host()["counters"]
    alive_last = float(c[:, T.CNT["alive"]].sum())
    value = alive_last * K / elapsed
    eng.close()
    del dst
    torch.cuda.empty_cache()
    # The same instances one after another, plain FP64 steps.
    Kp = max(1, args.fp64_steps)
    t64 = 0.0
    ps64 = 0.0
    for w in ws:
        g, p = w.grid, w.params
        e = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=T.FP64)
        d = T.to_device(w.state, T.FP64)
        o = T.make_outputs(1, T.nobins(g))
        e.step(d, g, p, o, stream=stream)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(Kp):
            e.step(d, g, dict(p, step=1 + k), o, stream=stream)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - ts
        ps64 += w.n * Kp
        e.close()
        del d
    torch.cuda.empty_cache()
    v64 = ps64 / t64
    search_ms, search_n = prof["search"]
    achieved = tests_one * FLOP_PER_TEST / (search_ms / 1e3) if search_ms > 0 else 0.0
    line = {
        "metric": "particle-steps/s (batched ensemble: 64 Sod/Noh/Sedov instances, FP32 state, one HIP graph)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded initial states of the paper's test problems)",
        "config": {"workload": "batched64", "instances": len(ws), "particles": ntot,
                   "sizes": "log-uniform 5e4-2e6" if args.batch_scale == 1.0 else f"scaled x{args.batch_scale}",
                   "kn": "log-uniform 1e-3-1e-1", "state_precision": "fp32", "moments": "fp64"},
        "plain_fp64_sequential": {"value": v64, "unit": "particle-steps/s", "steps_per_instance": Kp},
        "batched_fp32_over_plain_fp64": value / v64,
        "roofline": {"kernel": "k_search (closest-partner search)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FLOPS["fp32"] / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FLOPS["fp32"], "traffic": None,
                     "avg_launch_ms": search_ms / max(search_n, 1), "flop_per_pair_test": FLOP_PER_TEST},
        "phases": {ph: {"ms": round(ms / n, 5)} for ph, (ms, n) in prof.items() if n},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sedov16M")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--search", default="2,64",
                    help="search launch shape 'G,B' (records per lane, lanes per work-group), or 'auto' for the "
                         "autotuner's choice.  The default is the library's default shape, the one the "
                         "profiles in profiles/ were taken with; the autotuner's timings of the near-equal "
                         "(2, 64) and (2, 128) shapes differ by a few per cent from run to run")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="batched64: scale every instance size")
    ap.add_argument("--fp64-steps", type=int, default=5, help="batched64: plain FP64 steps per instance")
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

    import torch
    from paper_1210_8084_amd import tpkmc as T

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

    def outputs(k):
        O = T.Outputs()
        O.pairs, O.pair_cap = None, 0
        O.counters = counters[k].data_ptr()
        O.globals = glob[k].data_ptr()
        O.moments = moments.data_ptr()
        return O

    def step(k_step, k_out):
        import ctypes
        G, P, S = T.make_grid(g), T.make_params(dict(p, step=k_step), flags), T.particles(dst)
        O = outputs(k_out)
        rc = T.lib().tpkmc_step(eng.h, ctypes.byref(G), ctypes.byref(P), ctypes.byref(S), ctypes.byref(O),
                                ctypes.c_void_p(stream.cuda_stream))
        if rc:
            raise T.TpkmcError(rc, "tpkmc_step")

    torch.cuda.synchronize()
    if args.search == "auto":
        eng.autotune(dst, [(0, w.n, g, p)], stream=stream)
    else:
        eng.set_search(*[int(v) for v in args.search.split(",")])
    for k in range(Wm):
        step(k, 0)
    torch.cuda.synchronize()
    eng.profile(True)
    eng.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(Wm + k, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = eng.profile_read()
    eng.profile(False)
    elapsed = t1 - t0
    c = counters[:K].cpu().numpy()
    alive = float(c[:, T.CNT["alive"]].sum())
    tests = float(c[:, T.CNT["tests"]].sum())
    pairs = float(c[:, T.CNT["pairs"]].sum())
    value = alive / elapsed
    ms_per_step = 1e3 * elapsed / K

    graph_ms = None
    if not args.no_graph:
        spec = [(0, w.n, g, dict(p, step=Wm + K))]
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        gout = T.DeviceOutputs(counters=counters[:1], globals=glob[:1], moments=moments, pairs=None, pair_cap=0)
        eng.run(dst, spec, K, gout, flags=flags, stream=stream)
        torch.cuda.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - tg0) / K

    search_ms, search_n = prof["search"]
    search_s = search_ms / 1e3
    achieved = tests * FLOP_PER_TEST / search_s if search_s > 0 else 0.0
    peak = PEAK_FLOPS[args.precision]
    shape = eng.get_search()
    shape = (shape[0], min(shape[1], 256 // shape[0]))
    traffic = read_traffic(args.workload, args.precision, shape)
    bytes_per = phase_bytes(rs, w.n, ncell_tot, nob, True)
    phases = {}
    for ph, (ms, n) in prof.items():
        if n:
            avg = ms / n
            b = bytes_per.get(ph, 0)
            phases[ph] = {"ms": round(avg, 5), "alg_GBps": round(b / (avg / 1e3) / 1e9, 1) if b else None}

    cpu = None
    if not args.no_cpu:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        v_cpu, sample = cpu_baseline(w, nthreads)
        cpu = {"value": v_cpu, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
               "sample": sample}

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
                   "nobin": list(g["nobin"]), "kn": w.info.get("kn"), "state_precision": args.precision,
                   "moments": "fp64", "particle_order": "c-bin order kept between steps"},
        "pair_tests_per_s": tests / elapsed,
        "pairs_per_step": pairs / K,
        "graph_ms_per_step": graph_ms,
        "roofline": {"kernel": "k_search (closest-partner search)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "algorithmic_bytes": bytes_per["search"],
                     "search_shape": list(shape),
                     "avg_launch_ms": search_ms / max(search_n, 1),
                     "flop_per_pair_test": FLOP_PER_TEST},
        "phases": phases,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    eng.close()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dstb = torch.empty_like(src)
        for _ in range(3):
            dstb.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": src.numel() * 4, "copies": 3}), flush=True)


if __name__ == "__main__":
    main()
