"""Seeded synthetic initial states for the collision step.

This module only draws initial conditions (positions, velocities, ids) and
derives the input parameters of each workload; it contains none of the
step's arithmetic, so both the GPU library and the CPU oracle can be fed
from it.  The workload shapes follow the paper's test problems (Sec. 4):
a Sod shock tube, a cylindrical Noh implosion, a Sedov point blast and the
Maxwell-Boltzmann equilibration box, in units m = 1 (Sedov: m = 1/N) and
k_B = 1, with pressure p = n T and temperature T = m <c^2> / 3.

The cross section of a workload follows from its Knudsen number: the mean
free path is lambda = Kn * L with L the problem's length scale, and
lambda = 1 / (sigma n) (Sec. 2.4) with n the mean number density over the
occupied volume.

Every state is a dict of contiguous float64 arrays ``x y z vx vy vz``, a
uint32 ``id`` and a uint8 ``alive``; grids and params are plain dicts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

REFLECT, PERIODIC, ABSORB = 0, 1, 2
FP64, FP32 = 0, 1


@dataclass
class Workload:
    name: str
    state: dict
    grid: dict
    params: dict
    steps: int
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.state["x"])


def sigma_from_kn(kn: float, length: float, n_mean: float) -> float:
    """sigma = 1 / (n lambda) with lambda = Kn * length."""
    return 1.0 / (n_mean * kn * length)


def mean_speed(temperature: float, mass: float = 1.0) -> float:
    """Mean speed of a 3D Maxwellian, sqrt(8 T / (pi m))."""
    return math.sqrt(8.0 * temperature / (math.pi * mass))


def make_state(x, y, z, vx, vy, vz, ids=None):
    n = len(x)
    st = {k: np.ascontiguousarray(v, dtype=np.float64)
          for k, v in zip(("x", "y", "z", "vx", "vy", "vz"), (x, y, z, vx, vy, vz))}
    st["id"] = (np.arange(n, dtype=np.uint32) if ids is None
                else np.ascontiguousarray(ids, dtype=np.uint32))
    st["alive"] = np.ones(n, dtype=np.uint8)
    return st


def copy_state(st, dtype=np.float64):
    out = {k: np.array(st[k], dtype=dtype) for k in ("x", "y", "z", "vx", "vy", "vz")}
    if st.get("mass") is not None:
        out["mass"] = np.array(st["mass"], dtype=dtype)
    out["id"] = st["id"].copy()
    out["alive"] = st["alive"].copy() if st.get("alive") is not None else np.ones(len(st["x"]), np.uint8)
    return out


def shuffle_state(st, seed: int):
    """Same particles in a random array order (ids travel with them)."""
    perm = np.random.default_rng(seed).permutation(len(st["x"]))
    return {k: np.ascontiguousarray(v[perm]) for k, v in st.items()}


def grid(lo, hi, ncell, bc, nobin=None):
    return dict(lo=tuple(float(v) for v in lo), hi=tuple(float(v) for v in hi),
                ncell=tuple(int(v) for v in ncell), bc=tuple(int(v) for v in bc),
                nobin=tuple(int(v) for v in (nobin if nobin is not None else ncell)))


def params(sigma, dt, mass=1.0, seed=1, step=0, instance=0):
    return dict(sigma=float(sigma), dt=float(dt), mass=float(mass), seed=int(seed),
                step=int(step), instance=int(instance))


def _isotropic(rng, n):
    v = rng.normal(size=(3, n))
    v /= np.sqrt((v * v).sum(axis=0))
    return v


def sod(n=100_000, seed=1, kn=1e-3, ncell=200, nobin=200, dt=None, steps=100,
        t_left=1.25, t_right=1.0, density_ratio=8.0, side=0.05):
    """Sod shock tube in a thin periodic box [0,1] x [0,side]^2.

    The left half holds density_ratio times the right half's density, both
    Maxwellian with zero mean flow; T_l / T_r = 1.25 gives p_l / p_r = 10
    (Sec. 4.2, the Sod ratios).  Without an explicit dt, dt = 0.2 mean
    collision times, tau = lambda / <|v|> with the particle-weighted T."""
    rng = np.random.default_rng(seed)
    n_left = int(round(n * density_ratio / (density_ratio + 1.0)))
    n_right = n - n_left
    x = np.concatenate([rng.uniform(0.0, 0.5, n_left), rng.uniform(0.5, 1.0, n_right)])
    y = rng.uniform(0.0, side, n)
    z = rng.uniform(0.0, side, n)
    vl = rng.normal(0.0, math.sqrt(t_left), size=(3, n_left))
    vr = rng.normal(0.0, math.sqrt(t_right), size=(3, n_right))
    vl -= vl.mean(axis=1, keepdims=True)
    vr -= vr.mean(axis=1, keepdims=True)
    v = np.concatenate([vl, vr], axis=1)
    volume = 1.0 * side * side
    n_mean = n / volume
    lam = kn * 1.0
    sigma = sigma_from_kn(kn, 1.0, n_mean)
    t_mean = (n_left * t_left + n_right * t_right) / n
    tau = lam / mean_speed(t_mean)
    if dt is None:
        dt = 0.2 * tau
    g = grid((0, 0, 0), (1.0, side, side), (ncell, 1, 1), (REFLECT, PERIODIC, PERIODIC), (nobin, 1, 1))
    st = make_state(x, y, z, v[0], v[1], v[2])
    info = dict(kn=kn, lam=lam, n_mean=n_mean, n_left=n_left / (0.5 * volume),
                n_right=n_right / (0.5 * volume), t_left=t_left, t_right=t_right, tau=tau,
                gamma=5.0 / 3.0)
    return Workload("sod", st, g, params(sigma, dt, seed=seed), steps, info)


def noh(n=8_000_000, seed=1, kn=1e-3, ncell=256, nobin=None, dt=7.5e-4, steps=800,
        thermal=1e-3, v0=1.0):
    """Cylindrical Noh implosion (Sec. 4.3): uniform density in a cylinder of
    radius 1, radial inflow speed v0 plus a cold Maxwellian, periodic along
    a thin axial extent h = 2 / ncell."""
    rng = np.random.default_rng(seed)
    h = 2.0 / ncell
    rad = np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    x, y = rad * np.cos(th), rad * np.sin(th)
    z = rng.uniform(0.0, h, n)
    vt = rng.normal(0.0, thermal, size=(3, n))
    vx = -v0 * np.cos(th) + vt[0]
    vy = -v0 * np.sin(th) + vt[1]
    vz = vt[2]
    n0 = n / (math.pi * h)
    sigma = sigma_from_kn(kn, 1.0, n0)
    nb = ncell if nobin is None else nobin
    g = grid((-1, -1, 0), (1, 1, h), (ncell, ncell, 1), (REFLECT, REFLECT, PERIODIC), (nb, nb, 1))
    st = make_state(x, y, z, vx, vy, vz)
    info = dict(kn=kn, lam=kn, n0=n0, v0=v0, h=h, gamma=5.0 / 3.0, geometry=2)
    return Workload("noh", st, g, params(sigma, dt, seed=seed), steps, info)


def noh3d(n=8_000_000, seed=1, kn=1e-3, ncell=128, nobin=None, dt=None, steps=160, thermal=1e-3, v0=1.0):
    """Spherical Noh implosion (Sec. 4.3, the 3D run; gamma = 5/3, density
    jump 64): uniform ball of radius 1 in the box [-1, 1]^3 with reflecting
    walls, radial inflow speed v0 plus a cold Maxwellian.  Without an explicit
    dt, dt moves an inflowing particle a quarter c-bin."""
    rng = np.random.default_rng(seed)
    rad = rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    d = _isotropic(rng, n)
    x, y, z = rad * d[0], rad * d[1], rad * d[2]
    vt = rng.normal(0.0, thermal, size=(3, n))
    v = -v0 * d + vt
    n0 = n / (4.0 / 3.0 * math.pi)
    sigma = sigma_from_kn(kn, 1.0, n0)
    if dt is None:
        dt = 0.25 * (2.0 / ncell) / v0
    nb = ncell if nobin is None else nobin
    g = grid((-1, -1, -1), (1, 1, 1), (ncell,) * 3, (REFLECT,) * 3, (nb,) * 3)
    st = make_state(x, y, z, v[0], v[1], v[2])
    info = dict(kn=kn, lam=kn, n0=n0, v0=v0, gamma=5.0 / 3.0, f=3, geometry=3)
    return Workload("noh3d", st, g, params(sigma, dt, seed=seed), steps, info)


def sedov(n=16_000_000, seed=1, kn=1e-3, ncell=128, nobin=64, steps=600, blast_fraction=1e-3,
          energy=1.0, cold_ratio=1e-3):
    """Sedov point blast (Sec. 4.4) in the unit cube with reflecting walls:
    mass m = 1/N (rho_0 = 1); the blast_fraction * N particles nearest the
    centre carry the energy as isotropic velocities of equal speed, the rest
    move isotropically at cold_ratio times that speed.  dt moves the fastest
    particle half a c-bin."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(3, n))
    m = 1.0 / n
    nb = max(1, int(round(blast_fraction * n)))
    r2 = ((pos - 0.5) ** 2).sum(axis=0)
    blast = np.argpartition(r2, nb - 1)[:nb]
    vb = math.sqrt(2.0 * energy / (nb * m))
    speed = np.full(n, cold_ratio * vb)
    speed[blast] = vb
    v = _isotropic(rng, n) * speed
    w = 1.0 / ncell
    dt = 0.5 * w / vb
    sigma = sigma_from_kn(kn, 1.0, float(n))
    g = grid((0, 0, 0), (1, 1, 1), (ncell,) * 3, (REFLECT,) * 3, (nobin,) * 3)
    st = make_state(pos[0], pos[1], pos[2], v[0], v[1], v[2])
    info = dict(kn=kn, lam=kn, n0=float(n), rho0=1.0, energy=energy, v_blast=vb, n_blast=nb,
                gamma=5.0 / 3.0, geometry=3)
    return Workload("sedov", st, g, params(sigma, dt, mass=m, seed=seed), steps, info)


def equilibration(n=200_000, seed=1, lam_over_dx=1e-3, ncell=(32, 32, 32), box=4.0, speed=10.0,
                  dt_over_dx=1.0 / 60.0, steps=50):
    """Maxwell-Boltzmann equilibration (Sec. 4.1): every particle starts with
    the same speed in a random direction, in a periodic box."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(3, n))
    v = _isotropic(rng, n) * speed
    dx = box / ncell[0]
    volume = box ** 3
    lam = lam_over_dx * dx
    sigma = 1.0 / ((n / volume) * lam)
    dt = dt_over_dx * dx
    g = grid((0, 0, 0), (box,) * 3, ncell, (PERIODIC,) * 3)
    st = make_state(pos[0], pos[1], pos[2], v[0], v[1], v[2])
    info = dict(lam=lam, dx=dx, speed=speed)
    return Workload("equilibration", st, g, params(sigma, dt, seed=seed), steps, info)


def equilibration2d(n=20_000_000, seed=1, lam_over_dx=1e-3, ncell=1000, box=4.0, speed=10.0,
                    dt_over_dx=1.0 / 60.0, steps=400):
    """Maxwell-Boltzmann equilibration of a two-dimensional gas (Sec. 4.1, the
    paper's own setup): N particles uniform in the periodic square
    [0, box]^2 of the plane z = 0 on ncell^2 c-bins, every one at the same
    speed in a random in-plane direction, dt = dt_over_dx * dx.  sigma is a
    length, 1 / (n lambda) with n the number per area and lambda =
    lam_over_dx * dx."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(2, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    dx = box / ncell
    lam = lam_over_dx * dx
    sigma = 1.0 / ((n / (box * box)) * lam)
    dt = dt_over_dx * dx
    g = grid((0, 0, -0.5), (box, box, 0.5), (ncell, ncell, 1), (PERIODIC,) * 3)
    z, vz = _in_plane(n)
    st = make_state(pos[0], pos[1], z, speed * np.cos(th), speed * np.sin(th), vz)
    info = dict(lam=lam, dx=dx, speed=speed, lam_over_dx=lam_over_dx, f=2)
    return Workload("equilibration2d", st, g, dict(params(sigma, dt, seed=seed), planar=True), steps, info)


def mean_speed_2d(temperature: float, mass: float = 1.0) -> float:
    """Mean speed of a 2D Maxwellian, sqrt(pi T / (2 m))."""
    return math.sqrt(math.pi * temperature / (2.0 * mass))


def _in_plane(n, z=0.0):
    return np.full(n, float(z)), np.zeros(n)


def sod2d(n=100_000, seed=1, kn=1e-3, ncell=200, nobin=200, dt=None, steps=100,
          t_left=1.25, t_right=1.0, density_ratio=8.0, side=0.05):
    """Sod shock tube of a two-dimensional gas (Sec. 4.2, the 2D run; f = 2,
    gamma = 2) in the strip [0,1] x [0,side] of the plane z = 0: reflecting
    ends, periodic along y.  sigma is a length, 1 / (n lambda) with n the
    number per area."""
    rng = np.random.default_rng(seed)
    n_left = int(round(n * density_ratio / (density_ratio + 1.0)))
    n_right = n - n_left
    x = np.concatenate([rng.uniform(0.0, 0.5, n_left), rng.uniform(0.5, 1.0, n_right)])
    y = rng.uniform(0.0, side, n)
    vl = rng.normal(0.0, math.sqrt(t_left), size=(2, n_left))
    vr = rng.normal(0.0, math.sqrt(t_right), size=(2, n_right))
    vl -= vl.mean(axis=1, keepdims=True)
    vr -= vr.mean(axis=1, keepdims=True)
    v = np.concatenate([vl, vr], axis=1)
    area = 1.0 * side
    n_mean = n / area
    lam = kn * 1.0
    sigma = sigma_from_kn(kn, 1.0, n_mean)
    t_mean = (n_left * t_left + n_right * t_right) / n
    tau = lam / mean_speed_2d(t_mean)
    if dt is None:
        dt = 0.2 * tau
    g = grid((0, 0, -0.5), (1.0, side, 0.5), (ncell, 1, 1), (REFLECT, PERIODIC, PERIODIC), (nobin, 1, 1))
    z, vz = _in_plane(n)
    st = make_state(x, y, z, v[0], v[1], vz)
    info = dict(kn=kn, lam=lam, n_mean=n_mean, n_left=n_left / (0.5 * area),
                n_right=n_right / (0.5 * area), t_left=t_left, t_right=t_right, tau=tau,
                gamma=2.0, f=2, side=side)
    return Workload("sod2d", st, g, dict(params(sigma, dt, seed=seed), planar=True), steps, info)


def noh2d(n=8_000_000, seed=1, kn=1e-3, ncell=256, nobin=None, dt=7.5e-4, steps=800,
          thermal=1e-3, v0=1.0):
    """Cylindrical Noh implosion of a two-dimensional gas (Sec. 4.3, the 2D
    run; f = 2, gamma = 2, density jump 9): uniform disk of radius 1 in the
    plane z = 0, radial inflow speed v0 plus a cold 2D Maxwellian."""
    rng = np.random.default_rng(seed)
    rad = np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    x, y = rad * np.cos(th), rad * np.sin(th)
    vt = rng.normal(0.0, thermal, size=(2, n))
    vx = -v0 * np.cos(th) + vt[0]
    vy = -v0 * np.sin(th) + vt[1]
    n0 = n / math.pi
    sigma = sigma_from_kn(kn, 1.0, n0)
    nb = ncell if nobin is None else nobin
    g = grid((-1, -1, -0.5), (1, 1, 0.5), (ncell, ncell, 1), (REFLECT, REFLECT, PERIODIC), (nb, nb, 1))
    z, vz = _in_plane(n)
    st = make_state(x, y, z, vx, vy, vz)
    info = dict(kn=kn, lam=kn, n0=n0, v0=v0, gamma=2.0, f=2, geometry=2)
    return Workload("noh2d", st, g, dict(params(sigma, dt, seed=seed), planar=True), steps, info)


def sedov2d(n=4_000_000, seed=1, kn=1e-3, ncell=800, nobin=200, steps=600, blast_fraction=1e-3,
            energy=1.0, cold_ratio=1e-3):
    """Point blast in a two-dimensional gas (Sec. 4.4, the 2D run; f = 2,
    gamma = 2, cylindrical similarity solution) in the unit square with
    reflecting walls, mass 1/N (areal density 1).  dt moves the fastest
    particle half a c-bin."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(2, n))
    m = 1.0 / n
    nb = max(1, int(round(blast_fraction * n)))
    r2 = ((pos - 0.5) ** 2).sum(axis=0)
    blast = np.argpartition(r2, nb - 1)[:nb]
    vb = math.sqrt(2.0 * energy / (nb * m))
    speed = np.full(n, cold_ratio * vb)
    speed[blast] = vb
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    w = 1.0 / ncell
    dt = 0.5 * w / vb
    sigma = sigma_from_kn(kn, 1.0, float(n))
    g = grid((0, 0, -0.5), (1, 1, 0.5), (ncell, ncell, 1), (REFLECT, REFLECT, PERIODIC), (nobin, nobin, 1))
    z, vz = _in_plane(n)
    st = make_state(pos[0], pos[1], z, speed * np.cos(th), speed * np.sin(th), vz)
    info = dict(kn=kn, lam=kn, n0=float(n), rho0=1.0, energy=energy, v_blast=vb, n_blast=nb,
                gamma=2.0, f=2, geometry=2)
    return Workload("sedov2d", st, g, dict(params(sigma, dt, mass=m, seed=seed), planar=True), steps, info)


def random_plane(n=2000, seed=1, ncell=(6, 5), bc=(REFLECT, PERIODIC), hi=(1.0, 0.8), speed=1.0,
                 d_over_w=0.6, dt_over=0.4, nobin=None):
    """Small two-dimensional box for parity tests: uniform positions in the
    plane z = 0, Gaussian in-plane velocities; D = d_over_w * (smallest
    c-bin width), sigma = 2 D."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, hi[0], n)
    y = rng.uniform(0.0, hi[1], n)
    v = rng.normal(0.0, speed, size=(2, n))
    wmin = min(hi[0] / ncell[0], hi[1] / ncell[1])
    sigma = 2.0 * d_over_w * wmin
    dt = dt_over * wmin / speed
    nb = (ncell[0], ncell[1]) if nobin is None else nobin
    g = grid((0, 0, -0.5), (hi[0], hi[1], 0.5), (ncell[0], ncell[1], 1), (bc[0], bc[1], PERIODIC),
             (nb[0], nb[1], 1))
    z, vz = _in_plane(n)
    st = make_state(x, y, z, v[0], v[1], vz)
    return Workload("random_plane", st, g, dict(params(sigma, dt, seed=seed), planar=True), 1, {})


def random_box(n=2000, seed=1, ncell=(6, 5, 4), bc=(REFLECT, PERIODIC, PERIODIC), lo=(0, 0, 0),
               hi=(1.0, 0.8, 0.6), speed=1.0, d_over_w=0.6, dt_over=0.4, nobin=None):
    """Small generic box for parity tests: uniform positions, Gaussian
    velocities; sigma chosen so that D = d_over_w * (smallest c-bin width)
    and dt so that the typical particle moves dt_over * (that width)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    pos = rng.uniform(lo[:, None], hi[:, None], size=(3, n))
    v = rng.normal(0.0, speed, size=(3, n))
    wmin = float(np.min((hi - lo) / np.asarray(ncell)))
    dmax = d_over_w * wmin
    sigma = math.pi * dmax * dmax
    dt = dt_over * wmin / speed
    g = grid(lo, hi, ncell, bc, nobin)
    st = make_state(pos[0], pos[1], pos[2], v[0], v[1], v[2])
    return Workload("random_box", st, g, params(sigma, dt, seed=seed), 1, dict(d=dmax))


def batched(n_inst=64, seed=1, n_min=50_000, n_max=2_000_000, kn_min=1e-3, kn_max=1e-1,
            scale=1.0):
    """Ensemble of independent instances: type k mod 3 (Sod, Noh, Sedov),
    log-uniform particle counts and Knudsen numbers.  c-bins are scaled with
    the particle count to keep the parent workload's particles per c-bin.
    ``scale`` multiplies every particle count (for small test ensembles)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        nk = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) * scale))
        nk = max(nk, 64)
        kn = math.exp(rng.uniform(math.log(kn_min), math.log(kn_max)))
        kind = k % 3
        if kind == 0:
            # Sod: 4M particles on 1000 c-bins in the parent workload.
            nc = max(3, int(round(1000 * nk / 4_000_000)))
            w = sod(n=nk, seed=seed * 1000 + k, kn=kn, ncell=nc, nobin=max(1, nc // 5) if nc >= 5 else nc,
                    dt=1.134e-4 * (1000 / nc), steps=100)
        elif kind == 1:
            # Noh: 8M particles on 256^2 c-bins.
            nc = max(3, int(round(256 * math.sqrt(nk / 8_000_000))))
            w = noh(n=nk, seed=seed * 1000 + k, kn=kn, ncell=nc, dt=7.5e-4 * (256 / nc), steps=100)
        else:
            # Sedov: 16M particles on 128^3 c-bins.
            nc = max(3, int(round(128 * (nk / 16_000_000) ** (1.0 / 3.0))))
            w = sedov(n=nk, seed=seed * 1000 + k, kn=kn, ncell=nc, nobin=max(1, nc // 2), steps=100)
        w.params["seed"] = seed * 1000 + k
        w.params["instance"] = k
        w.info["kind"] = ("sod", "noh", "sedov")[kind]
        out.append(w)
    return out
