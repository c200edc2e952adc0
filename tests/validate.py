"""Physics validation of the GPU collision step on the paper's shock problems.

Runs the Sod tube (Sec. 4.2), the cylindrical Noh implosion (Sec. 4.3) and
the Sedov blast (Sec. 4.4) on the GPU library, in FP32 and FP64, as
three-dimensional gases (f = 3, gamma = 5/3) and as two-dimensional ones
(f = 2, gamma = 2, the paper's 2D runs), and reports L1 errors of the number
density and pressure profiles against the analytic solutions, the FP32-FP64
difference of those errors, and the conservation of particles, momentum and
energy over the run.

Test infrastructure, like ``oracle/``: it scores the GPU runs against the
analytic solutions in ``oracle/analytic.py``; nothing in the library imports
it.

Usage:  python tests/validate.py [--out file.json] [--quick] [--only ...] [--seeds ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _run(w, precision, steps, progress=None, rank_time=False, pair_random=False):
    """Advance workload w by `steps` steps on the GPU; returns host state,
    the last step's moments and per-step globals/counters.  rank_time:
    criterion 3 by earliest contact instead of closest approach; pair_random:
    random partners inside each c-bin (the DSMC rule) instead of criteria 1-3."""
    import torch
    from paper_1210_8084_amd import tpkmc as T
    g, p = w.grid, dict(w.params, rank_time=rank_time, pair_random=pair_random)
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=precision)
    dst = T.to_device(w.state, precision)
    out = T.make_outputs(1, T.nobins(g))
    glob = torch.zeros((steps, 8), dtype=torch.float64, device="cuda")
    cnt = torch.zeros((steps, 8), dtype=torch.int64, device="cuda")
    eng.autotune(dst, [(0, w.n, g, p)])
    cells, speed_bound = list(eng.tuned_cells(0)), eng.tuned_speed(0)
    t0 = time.perf_counter()
    for s in range(steps):
        o = T.DeviceOutputs(counters=cnt[s:s + 1], globals=glob[s:s + 1], moments=out.moments, pairs=None,
                            pair_cap=0)
        eng.step(dst, g, dict(p, step=s), o, flags=T.ALLOW_REORDER)
        if progress and (s + 1) % progress == 0:
            torch.cuda.synchronize()
            print(f"  {w.name} step {s + 1}/{steps}", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = eng.status()
    host = T.to_host(dst)
    res = dict(state=host, moments=out.moments.cpu().numpy(), globals=glob.cpu().numpy(),
               counters=cnt.cpu().numpy().view(np.uint64), wall=wall, status=status, cells=cells,
               speed_bound=speed_bound)
    eng.close()
    del dst
    torch.cuda.empty_cache()
    return res


def _conservation(w, r):
    g0 = r["globals"][0]
    gl = r["globals"][-1]
    m = w.params["mass"]
    e0 = 0.5 * m * sum(float(np.sum(w.state[k] ** 2)) for k in ("vx", "vy", "vz"))
    if w.params.get("planar"):
        assert np.all(r["state"]["vz"] == 0.0), "a 2D run left the plane"
    alive = r["counters"][:, 0]
    return dict(energy_rel_drift=float(abs(gl[3] - e0) / e0),
                energy_first_step_rel=float(abs(g0[3] - e0) / e0),
                particles_conserved=bool(np.all(alive == w.n)),
                pairs_per_step=float(r["counters"][:, 1].mean()),
                collided_fraction=float(2 * r["counters"][:, 1].mean() / w.n))


def _tanh_width(x, n, x_s, lo, hi):
    """Width of a shock front: least-squares fit of
    n(x) = lo + (hi - lo) (1 - tanh((x - c) / d)) / 2 near x_s; returns the
    10-90% rise distance 2 atanh(0.8) d."""
    from scipy.optimize import curve_fit

    def model(x, c, d):
        return lo + (hi - lo) * 0.5 * (1.0 - np.tanh((x - c) / d))
    (c, d), _ = curve_fit(model, x, n, p0=(x_s, 0.005), maxfev=20000)
    return float(2.0 * math.atanh(0.8) * abs(d)), float(c)


def sod(precision, n=4_000_000, steps=500, kn=1e-3, planar=False, seed=1, rank_time=False, pair_random=False,
        free=False):
    """free: no collisions (sigma = 0), the free-streaming limit of Sec. 5."""
    from oracle import analytic as A
    from paper_1210_8084_amd import workloads as W
    if planar:
        w = W.sod2d(n=n, ncell=1000, nobin=200, dt=1.134e-4, kn=kn, seed=seed)
    else:
        w = W.sod(n=n, ncell=1000, nobin=200, dt=1.134e-4, kn=kn, seed=seed)
    if free:
        w.params["sigma"] = 0.0
    f = 2 if planar else 3
    r = _run(w, precision, steps, progress=100, rank_time=rank_time, pair_random=pair_random)
    t = steps * w.params["dt"]
    M = r["moments"]
    nob = w.grid["nobin"][0]
    # o-bin volume: length x cross-section (an area in space, a width in the plane)
    vol = (1.0 / nob) * (w.info["side"] if planar else 0.05 * 0.05)
    n_ = M[:, 0] / vol
    # p = n T + virial / (f V), T = m sum (v - vbar)^2 / (f count)
    kin = M[:, 4:4 + f].sum(axis=1) / f
    vir = M[:, 7:7 + f].sum(axis=1) / f
    p_kin = kin / vol
    p_tot = (kin + vir) / vol
    xc = (np.arange(nob) + 0.5) / nob
    nl, nr = w.info["n_left"], w.info["n_right"]
    tl, tr = w.info["t_left"], w.info["t_right"]
    rho, u, p = A.sod_profile(xc, t, (nl, 0.0, nl * tl), (nr, 0.0, nr * tr), gamma=w.info["gamma"])
    # Shock front: the exact shock speed and post-shock density, and the
    # 10-90% width of a tanh fit to a fine density profile (bins of half a
    # mean free path) within 0.02 of the exact front.
    g_ = w.info["gamma"]
    left, right = (nl, 0.0, nl * tl), (nr, 0.0, nr * tr)
    ps, _ = A.riemann_star(left, right, g_)
    a_r = math.sqrt(g_ * nr * tr / nr)
    x_s = 0.5 + t * a_r * math.sqrt((g_ + 1.0) / (2.0 * g_) * ps / (nr * tr) + (g_ - 1.0) / (2.0 * g_))
    q = ps / (nr * tr)
    n2 = nr * (q + (g_ - 1.0) / (g_ + 1.0)) / ((g_ - 1.0) / (g_ + 1.0) * q + 1.0)
    lam = w.info.get("lam", kn)
    width = x_fit = None
    if not free and lam <= 4e-3:  # at least ten bins in the window; no front to fit without collisions
        fe = np.arange(x_s - 0.02, x_s + 0.02 + 1e-12, 0.5 * lam)
        fc, _ = np.histogram(r["state"]["x"], bins=fe)
        fn = fc / ((fe[1] - fe[0]) * (w.info["side"] if planar else 0.05 * 0.05))
        width, x_fit = _tanh_width(0.5 * (fe[1:] + fe[:-1]), fn, x_s, nr, n2)
    return dict(workload=f"{w.name} n={n} kn={kn}", steps=steps, t=t, wall_s=r["wall"],
                cells=r["cells"], speed_bound=r["speed_bound"], status=r["status"],
                rank="random partners" if pair_random else "contact time" if rank_time else "closest approach",
                shock_x_exact=x_s, shock_x_fit=x_fit, shock_width=width,
                shock_width_mfp=None if width is None else width / lam,
                l1_density=float(np.mean(np.abs(n_ - rho)) / nl),
                l1_pressure_kinetic=float(np.mean(np.abs(p_kin - p)) / (nl * tl)),
                l1_pressure_with_virial=float(np.mean(np.abs(p_tot - p)) / (nl * tl)),
                profile_density=(n_ / nl).round(4).tolist(), analytic_density=(rho / nl).round(4).tolist(),
                **_conservation(w, r))


def noh(precision, n=8_000_000, steps=800, planar=False, seed=1, kn=1e-3, ncell=256, free=False):
    """ncell below 256 keeps the particles per c-bin of the 8M run at
    n = 8M (ncell / 256)^2, with dt scaled to move the inflow the same
    fraction of a c-bin."""
    from oracle import analytic as A
    from paper_1210_8084_amd import workloads as W
    w = (W.noh2d if planar else W.noh)(n=n, steps=steps, seed=seed, kn=kn, ncell=ncell, dt=7.5e-4 * 256 / ncell)
    if free:
        w.params["sigma"] = 0.0
    f = 2 if planar else 3
    r = _run(w, precision, steps, progress=200)
    t = steps * w.params["dt"]
    st = r["state"]
    rad = np.sqrt(st["x"] ** 2 + st["y"] ** 2)
    edges = np.arange(0.0, 0.4 + 1e-12, 0.01)
    cnt, _ = np.histogram(rad, bins=edges)
    area = math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    n_ = cnt / (area * (1.0 if planar else w.info["h"]))
    rc = 0.5 * (edges[1:] + edges[:-1])
    gamma = w.info["gamma"]
    na, _, _, rs = A.noh_profile(rc, t, n0=w.info["n0"], v0=1.0, gamma=gamma, d=2)
    inside = rc < rs * 0.8
    # Shocked gas at rest with internal energy v0^2 / 2 per mass: T = m v0^2 / f.
    core = rad < 0.8 * rs
    t_core = None
    if core.sum() > 100:
        dv2 = sum((st[k][core] - st[k][core].mean()) ** 2 for k in ("vx", "vy", "vz")[:f])
        t_core = float(w.params["mass"] * dv2.mean() / f)
    return dict(workload=f"{w.name} n={n}", steps=steps, t=t, wall_s=r["wall"],
                cells=r["cells"], speed_bound=r["speed_bound"], status=r["status"], r_shock=rs,
                l1_density=float(np.mean(np.abs(n_ - na)) / w.info["n0"]),
                shocked_density_over_n0=float(np.mean(n_[inside]) / w.info["n0"]) if inside.any() else None,
                analytic_shocked=((gamma + 1.0) / (gamma - 1.0)) ** 2,
                shocked_temperature=t_core, analytic_shocked_temperature=w.params["mass"] * 1.0 / f,
                profile_density=(n_ / w.info["n0"]).round(3).tolist(), analytic_density=(na / w.info["n0"]).round(3).tolist(),
                **_conservation(w, r))


def noh3d(precision, n=8_000_000, steps=160, seed=1):
    """Spherical Noh: radial number density against the analytic solution
    with d = 3 (jump ((gamma + 1) / (gamma - 1))^3 = 64), and the shocked
    temperature m v0^2 / f."""
    from oracle import analytic as A
    from paper_1210_8084_amd import workloads as W
    w = W.noh3d(n=n, steps=steps, seed=seed)
    r = _run(w, precision, steps, progress=40)
    t = steps * w.params["dt"]
    st = r["state"]
    rad = np.sqrt(st["x"] ** 2 + st["y"] ** 2 + st["z"] ** 2)
    edges = np.arange(0.0, 0.4 + 1e-12, 0.01)
    cnt, _ = np.histogram(rad, bins=edges)
    vol = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    n_ = cnt / vol
    rc = 0.5 * (edges[1:] + edges[:-1])
    gamma = w.info["gamma"]
    na, _, _, rs = A.noh_profile(rc, t, n0=w.info["n0"], v0=1.0, gamma=gamma, d=3)
    inside = rc < rs * 0.8
    core = rad < 0.8 * rs
    t_core = None
    if core.sum() > 100:
        dv2 = sum((st[k][core] - st[k][core].mean()) ** 2 for k in ("vx", "vy", "vz"))
        t_core = float(w.params["mass"] * dv2.mean() / 3.0)
    return dict(workload=f"{w.name} n={n}", steps=steps, t=t, wall_s=r["wall"],
                cells=r["cells"], speed_bound=r["speed_bound"], status=r["status"], r_shock=rs,
                l1_density=float(np.mean(np.abs(n_ - na)) / w.info["n0"]),
                shocked_density_over_n0=float(np.mean(n_[inside]) / w.info["n0"]) if inside.any() else None,
                analytic_shocked=((gamma + 1.0) / (gamma - 1.0)) ** 3,
                shocked_temperature=t_core, analytic_shocked_temperature=w.params["mass"] * 1.0 / 3.0,
                profile_density=(n_ / w.info["n0"]).round(3).tolist(), analytic_density=(na / w.info["n0"]).round(3).tolist(),
                **_conservation(w, r))


def sedov(precision, n=16_000_000, steps=600, planar=False, seed=1, rank_time=False, pair_random=False,
          kn=1e-3, free=False):
    from oracle import analytic as A
    from paper_1210_8084_amd import workloads as W
    w = (W.sedov2d if planar else W.sedov)(n=n, steps=steps, seed=seed, kn=kn)
    if free:
        w.params["sigma"] = 0.0
    r = _run(w, precision, steps, progress=200, rank_time=rank_time, pair_random=pair_random)
    t = steps * w.params["dt"]
    st = r["state"]
    j = 2 if planar else 3
    rad = np.sqrt(sum((st[k] - 0.5) ** 2 for k in ("x", "y", "z")[:j]))
    edges = np.arange(0.0, 0.5 + 1e-12, 0.01)
    cnt, _ = np.histogram(rad, bins=edges)
    if planar:
        vol = math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    else:
        vol = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    rho = cnt * w.params["mass"] / vol
    rc = 0.5 * (edges[1:] + edges[:-1])
    ra, _, _, R = A.sedov_profile(rc, t, energy=w.info["energy"], rho0=1.0, gamma=w.info["gamma"], j=j)
    peak = int(np.argmax(rho))
    # Front width: 10-90% of the rise from rho0 to the peak on the outer flank
    # of a fine radial profile (shells of a fifth of the coarse ones).
    fe = np.arange(0.0, 0.5 + 1e-12, 0.002)
    fc, _ = np.histogram(rad, bins=fe)
    fv = math.pi * (fe[1:] ** 2 - fe[:-1] ** 2) if planar else 4.0 / 3.0 * math.pi * (fe[1:] ** 3 - fe[:-1] ** 3)
    fr = fc * w.params["mass"] / fv
    frc = 0.5 * (fe[1:] + fe[:-1])
    k = int(np.argmax(fr))
    top = fr[k]

    def outer_cross(level):
        for i in range(k, len(fr) - 1):
            if fr[i] >= level > fr[i + 1]:
                return frc[i] + (fr[i] - level) / (fr[i] - fr[i + 1]) * (frc[i + 1] - frc[i])
        return float("nan")
    width = float(outer_cross(1.0 + 0.1 * (top - 1.0)) - outer_cross(1.0 + 0.9 * (top - 1.0)))
    lam = w.info.get("lam", 1e-3)
    return dict(workload=f"{w.name} n={n}", steps=steps, t=t, wall_s=r["wall"],
                cells=r["cells"], speed_bound=r["speed_bound"], status=r["status"], r_shock_analytic=R,
                rank="random partners" if pair_random else "contact time" if rank_time else "closest approach",
                central_density=float(rho[rc < 0.05].mean()),
                front_width=width, front_width_mfp=width / lam,
                r_density_peak=float(rc[peak]), peak_density=float(rho[peak]),
                l1_density=float(np.mean(np.abs(rho - ra))),
                profile_density=rho.round(3).tolist(), analytic_density=ra.round(3).tolist(),
                **_conservation(w, r))


# ---------------------------------------------------------------- Sec. 5, Sec. 4.1
MFP_OVER_DX = (1e-3, 1.0, 10.0, 30.0, 100.0, float("inf"))  # inf: free streaming (sigma = 0)


def mfp_sweep(precision, quick=False, problems=("sod2d", "noh2d", "sedov2d")):
    """The mean-free-path study of Sec. 5: the 2D Sod, Noh and Sedov problems
    with lambda = 1e-3 (continuum), 1, 10, 30 and 100 c-bin widths and
    without collisions (free streaming).  Sizes: Sod 1M particles on 1000
    c-bins (dx = 1e-3), Noh 2M on 128^2 (dx = 1/64, the particles per c-bin
    of the 8M run), Sedov 4M on 800^2 (dx = 1.25e-3)."""
    out = {}
    for name in problems:
        for m in MFP_OVER_DX:
            free = m == float("inf")
            tag = f"{name}_mfp_{'free' if free else f'{m:g}dx'}"
            print(f"== {tag}", flush=True)
            if name == "sod2d":
                kn = (m if not free else 1.0) * 1e-3
                res = sod(precision, n=250_000 if quick else 1_000_000, steps=500, kn=kn, planar=True, free=free)
            elif name == "noh2d":
                kn = (m if not free else 1.0) * 2.0 / 128
                res = noh(precision, n=500_000 if quick else 2_000_000, steps=400, planar=True, kn=kn, ncell=128,
                          free=free)
            else:
                kn = (m if not free else 1.0) * 1.25e-3
                res = sedov(precision, n=1_000_000 if quick else 4_000_000, steps=600, planar=True, kn=kn,
                            free=free)
            res["lambda_over_dx"] = None if free else m
            brief = {k: v for k, v in res.items() if not k.startswith(("profile", "analytic_density"))}
            print(json.dumps(brief), flush=True)
            out[tag] = res
    return out


def equilibration2d(precision, lam_over_dx, n=20_000_000, ncell=1000, steps=400, sample=200_000, every=2):
    """Sec. 4.1 in its own setup: N particles of speed 10 in random in-plane
    directions, periodic [0,4]^2 on ncell^2 c-bins, dt = dx / 60.  Per step:
    the fraction of particles that collide; every `every` steps, the
    Kolmogorov-Smirnov distance between the speeds of a fixed subsample and
    the 2D Maxwell-Boltzmann (Rayleigh) law of the same mean energy,
    F(v) = 1 - exp(-v^2 / <v^2>)."""
    import torch
    from paper_1210_8084_amd import tpkmc as T
    from paper_1210_8084_amd import workloads as W
    w = W.equilibration2d(n=n, lam_over_dx=lam_over_dx, ncell=ncell, steps=steps)
    g, p = w.grid, w.params
    eng = T.Engine(max_particles=w.n, max_cells=T.ncells(g) + 1, max_obins=T.nobins(g), precision=precision)
    dst = T.to_device(w.state, precision)
    cnt = torch.zeros((steps, 8), dtype=torch.int64, device="cuda")
    idx = torch.arange(0, w.n, max(1, w.n // sample), device="cuda")
    v2mean = float(np.mean(w.state["vx"] ** 2 + w.state["vy"] ** 2))
    ks = []
    t0 = time.perf_counter()
    for s in range(steps):
        o = T.DeviceOutputs(counters=cnt[s:s + 1], globals=None, moments=None, pairs=None, pair_cap=0)
        eng.step(dst, g, dict(p, step=s), o)  # caller order kept: the subsample is the same particles
        if (s + 1) % every == 0 or s == 0:
            vx = dst["vx"].index_select(0, idx).double()
            vy = dst["vy"].index_select(0, idx).double()
            v = torch.sqrt(vx * vx + vy * vy).cpu().numpy()
            v.sort()
            F = 1.0 - np.exp(-v * v / v2mean)
            emp_hi = np.arange(1, len(v) + 1) / len(v)
            emp_lo = np.arange(0, len(v)) / len(v)
            ks.append((s + 1, float(max(np.max(np.abs(emp_hi - F)), np.max(np.abs(emp_lo - F))))))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c = cnt.cpu().numpy().view(np.uint64)
    eng.close()
    frac = 2.0 * c[:, 1].astype(np.float64) / w.n
    noise = 1.63 / math.sqrt(len(idx))  # KS critical value at the 1% level
    settled = next((st for st, d in ks if d < 2.0 * noise), None)
    return dict(workload=f"equilibration2d n={n} ncell={ncell}^2 lambda={lam_over_dx:g}dx", steps=steps,
                wall_s=wall, collided_fraction_first=float(frac[0]),
                collided_fraction_mean=float(frac[min(10, steps - 1):].mean()),
                collided_fraction_last=float(frac[-1]), ks_threshold=2.0 * noise,
                steps_to_maxwell_boltzmann=settled, ks=[(st, round(d, 4)) for st, d in ks[::5]],
                particles_conserved=bool(np.all(c[:, 0] == w.n)))


KN = None  # Knudsen number of the 3D Sod tube (--kn)


def _one(name, prec, quick, seed):
    planar = name.endswith("2d")
    base = name[:-2] if name.endswith(("2d", "3d")) else name
    if base == "sod":
        return sod(prec, n=400_000 if quick else 4_000_000, steps=100 if quick else 500, planar=planar, seed=seed,
                   kn=KN if KN is not None else 1e-3)
    if base == "noh" and name.endswith("3d"):
        return noh3d(prec, n=800_000 if quick else 8_000_000, steps=160, seed=seed)
    if base == "noh":
        return noh(prec, n=800_000 if quick else 8_000_000, steps=200 if quick else 800, planar=planar, seed=seed)
    n_full = 4_000_000 if planar else 16_000_000
    return sedov(prec, n=n_full // 8 if quick else n_full, steps=150 if quick else 600, planar=planar, seed=seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="smaller sizes and fewer steps")
    ap.add_argument("--only", default="sod,noh,sedov,sod2d,noh2d,sedov2d,noh3d")
    ap.add_argument("--seeds", default="1", help="comma-separated workload seeds; with several, the "
                    "report adds the mean and spread of L1 and of the FP32 - FP64 difference")
    ap.add_argument("--rank-compare", action="store_true",
                    help="partners by closest approach against by earliest contact and against random "
                    "partners inside each c-bin (FP32): collided fraction, L1 density and shock width of the "
                    "Sod tube and the Sedov blast")
    ap.add_argument("--mfp-sweep", action="store_true",
                    help="Sec. 5: 2D Sod, Noh and Sedov at lambda = 1e-3, 1, 10, 30, 100 c-bin widths and "
                         "free streaming (FP32)")
    ap.add_argument("--equilibration", action="store_true",
                    help="Sec. 4.1: 2D equilibration at lambda = 1e-3, 1 and 10 c-bin widths (FP32)")
    ap.add_argument("--kn", type=float, default=None, help="Knudsen number of the 3D Sod tube (--only sod)")
    args = ap.parse_args()
    from paper_1210_8084_amd import tpkmc as T
    seeds = [int(v) for v in args.seeds.split(",")]
    report = {}
    if args.mfp_sweep or args.equilibration:
        if args.equilibration:
            for m in (1e-3, 1.0, 10.0):
                print(f"== equilibration2d lambda={m:g}dx", flush=True)
                res = equilibration2d(T.FP32, m, n=2_000_000 if args.quick else 20_000_000,
                                      ncell=316 if args.quick else 1000)
                report[f"equilibration2d_{m:g}dx"] = res
                print(json.dumps(res), flush=True)
        if args.mfp_sweep:
            report.update(mfp_sweep(T.FP32, quick=args.quick))
        if args.out:
            with open(args.out, "w") as f:
                json.dump(report, f, indent=1)
        return
    if args.rank_compare:
        keys = ("rank", "collided_fraction", "l1_density", "shock_width_mfp", "front_width_mfp", "peak_density",
                "energy_rel_drift")
        for name in ("sod", "sedov"):
            for rule in ("distance", "time", "random"):
                kw = dict(rank_time=rule == "time", pair_random=rule == "random")
                print(f"== {name} {rule}", flush=True)
                if name == "sod":
                    res = sod(T.FP32, n=400_000 if args.quick else 4_000_000, steps=100 if args.quick else 500, **kw)
                else:
                    res = sedov(T.FP32, n=2_000_000 if args.quick else 16_000_000, steps=150 if args.quick else 600,
                                **kw)
                report[f"{name}_{rule}"] = res
                print(json.dumps({k: res[k] for k in keys if k in res}), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(report, f, indent=1)
        return
    global KN
    KN = args.kn
    for name in args.only.split(","):
        diffs, l1 = [], {"fp32": [], "fp64": []}
        for seed in seeds:
            for prec, label in ((T.FP32, "fp32"), (T.FP64, "fp64")):
                print(f"== {name} {label} seed {seed}", flush=True)
                res = _one(name, prec, args.quick, seed)
                key = f"{name}_{label}" if len(seeds) == 1 else f"{name}_{label}_seed{seed}"
                report[key] = res
                l1[label].append(res["l1_density"])
                brief = {k: v for k, v in res.items() if not k.startswith(("profile", "analytic_density"))}
                print(json.dumps(brief), flush=True)
            diffs.append(l1["fp32"][-1] - l1["fp64"][-1])
            print(f"{name} seed {seed}: L1 density FP32 - FP64 = {diffs[-1]:.3e}", flush=True)
        if len(seeds) == 1:
            report[f"{name}_fp32_minus_fp64_l1_density"] = diffs[0]
        else:
            summ = dict(seeds=seeds, l1_fp32_mean=float(np.mean(l1["fp32"])), l1_fp64_mean=float(np.mean(l1["fp64"])),
                        l1_fp64_spread=float(np.std(l1["fp64"], ddof=1)),
                        diff_mean=float(np.mean(diffs)), diff_spread=float(np.std(diffs, ddof=1)),
                        diff_mean_stderr=float(np.std(diffs, ddof=1) / math.sqrt(len(diffs))))
            report[f"{name}_seed_summary"] = summ
            print(f"{name}: " + json.dumps(summ), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
