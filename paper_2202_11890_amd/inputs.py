"""Seeded synthetic inputs for two vertically stacked 2D domains.

This module only builds input states: it holds none of the solver's
arithmetic (no fluxes, no time stepping) and imports neither the HIP binding
nor the CPU oracle, so both can consume the same arrays.

Background (per domain d): pressure p0 = 1/gamma, temperature T_d, density
rho_d = gamma p0 / T_d (equation of state p = rho T / gamma), at rest.
Perturbation: p = p0 (1 + A exp(-r^2 / w^2)) with r the x-periodic distance
to a seeded centre (x_c, z_c); density follows isentropically,
rho = rho_d (p / p0)^(1/gamma).  Values are point values at cell centres.
Arrays are float64 [4, nz, nx] = (rho, rho u, rho w, rho E).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    nz_lower: int
    nz_upper: int
    lx: float = 10.0            # x in (-lx/2, lx/2), periodic
    lz_lower: float = 5.0       # lower domain z in (-lz_lower, 0)
    lz_upper: float = 5.0       # upper domain z in (0, lz_upper)
    fast_is_lower: bool = True
    n_buffer: int = 4
    base: int = 2               # base Runge-Kutta: 2 (RK2 of Table 1) or 3 (SSP-RK3)
    m: int = 2                  # rate ratio
    steps: int = 100
    gamma: float = 1.4
    prandtl: float = 0.72
    mu_lower: float = 1e-3
    mu_upper: float = 1e-3
    gravity: float = 0.0
    t_lower: float = 16.0       # fast domain: 4x sound speed
    t_upper: float = 1.0
    amplitude: float = 1e-2
    width: float = 0.5
    seed: int = 0
    cfl: float = 0.5
    dnum: float = 0.25
    extra: dict = field(default_factory=dict, compare=False)

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dz_lower(self) -> float:
        return self.lz_lower / self.nz_lower

    @property
    def dz_upper(self) -> float:
        return self.lz_upper / self.nz_upper

    @property
    def s(self) -> int:
        return self.base

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def small() -> Workload:
    """64x32 cells per domain, MPRK with the RK2 base, m = 2, 100 slow steps."""
    return Workload("two-domain 2D CNS 64x32 x2, MPRK2 m=2", nx=64, nz_lower=32, nz_upper=32,
                    base=2, m=2, steps=100, n_buffer=4, seed=0)


def large() -> Workload:
    """1024x512 cells per domain, 4 buffer rows, SSP-RK3 base, m = 4, 1000 slow steps."""
    return Workload("two-domain 2D CNS 1024x512 x2, MPRK3 m=4", nx=1024, nz_lower=512,
                    nz_upper=512, base=3, m=4, steps=1000, n_buffer=4, seed=1)


def ensemble(n: int = 64, seed0: int = 100):
    """Batched ensemble: n independent two-domain problems of the small and
    large workloads' setup, member i seeded with seed0 + i: nx uniform in
    [128, 512], nz uniform in [64, 256] (the same for both domains),
    perturbation amplitude log-uniform in [1e-3, 1e-1], viscosity log-uniform
    in [1e-4, 1e-2] (both domains), m uniform in {2, 4, 8}; RK2 base, 4
    buffer rows, 500 slow steps."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        nx = int(rng.integers(128, 513))
        nz = int(rng.integers(64, 257))
        amp = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
        mu = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        m = int(rng.choice([2, 4, 8]))
        out.append(Workload("ensemble member %d" % i, nx=nx, nz_lower=nz, nz_upper=nz, base=2, m=m,
                            steps=500, n_buffer=4, mu_lower=mu, mu_upper=mu, amplitude=amp,
                            seed=seed0 + i))
    return out


def serving_requests(n: int, rate: float, seed: int = 7):
    """Serving workload: n requests with Poisson arrivals at `rate` per second
    (exponential gaps), as (arrival_seconds, Workload): nx log-uniform in
    [64, 1024] with nz = nx/2 per domain, 50..500 slow steps, m in {2, 4},
    RK2 base, seeded perturbation."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        nx = int(round(np.exp(rng.uniform(np.log(64), np.log(1024)))))
        nx = max(64, min(1024, nx))
        nz = max(8, nx // 2)
        steps = int(rng.integers(50, 501))
        m = int(rng.choice([2, 4]))
        w = Workload("request %d" % i, nx=nx, nz_lower=nz, nz_upper=nz, base=2, m=m, steps=steps,
                     n_buffer=4, seed=10_000 + seed * 1000 + i)
        out.append((t, w))
    return out


def centre(w: Workload):
    rng = np.random.default_rng(w.seed)
    xc = rng.uniform(-w.lx / 2, w.lx / 2)
    zc = rng.uniform(-0.7 * w.lz_lower, 0.7 * w.lz_upper)
    return float(xc), float(zc)


def _domain(w: Workload, lower: bool, xc: float, zc: float) -> np.ndarray:
    nz = w.nz_lower if lower else w.nz_upper
    dz = w.dz_lower if lower else w.dz_upper
    z0 = -w.lz_lower if lower else 0.0
    T = w.t_lower if lower else w.t_upper
    g = w.gamma
    p0 = 1.0 / g
    rho0 = g * p0 / T
    x = -w.lx / 2 + (np.arange(w.nx) + 0.5) * w.dx
    z = z0 + (np.arange(nz) + 0.5) * dz
    ddx = np.abs(x - xc)
    ddx = np.minimum(ddx, w.lx - ddx)
    r2 = ddx[None, :] ** 2 + (z[:, None] - zc) ** 2
    p = p0 * (1.0 + w.amplitude * np.exp(-r2 / w.width ** 2))
    rho = rho0 * (p / p0) ** (1.0 / g)
    q = np.zeros((4, nz, w.nx))
    q[0] = rho
    q[3] = p / (g - 1.0)
    return q


def initial_state(w: Workload):
    """(q_lower, q_upper) as float64 numpy arrays."""
    xc, zc = centre(w)
    return _domain(w, True, xc, zc), _domain(w, False, xc, zc)


def random_state(w: Workload, seed: int, amp: float = 0.05):
    """Random smooth-free physical states (used for small brute-force checks):
    rho, T within +-amp relative of the background, |u|, |w| <= amp * a."""
    rng = np.random.default_rng(seed)
    out = []
    for lower in (True, False):
        nz = w.nz_lower if lower else w.nz_upper
        T0 = w.t_lower if lower else w.t_upper
        g = w.gamma
        rho0 = 1.0 / T0
        rho = rho0 * (1 + amp * rng.uniform(-1, 1, (nz, w.nx)))
        T = T0 * (1 + amp * rng.uniform(-1, 1, (nz, w.nx)))
        a = np.sqrt(T)
        u = amp * a * rng.uniform(-1, 1, (nz, w.nx))
        v = amp * a * rng.uniform(-1, 1, (nz, w.nx))
        p = rho * T / g
        q = np.zeros((4, nz, w.nx))
        q[0] = rho
        q[1] = rho * u
        q[2] = rho * v
        q[3] = p / (g - 1) + 0.5 * rho * (u * u + v * v)
        out.append(q)
    return out[0], out[1]


def uniform_state(w: Workload, rho: float, u: float, wv: float, p: float):
    g = w.gamma
    res = []
    for nz in (w.nz_lower, w.nz_upper):
        q = np.zeros((4, nz, w.nx))
        q[0] = rho
        q[1] = rho * u
        q[2] = rho * wv
        q[3] = p / (g - 1) + 0.5 * rho * (u * u + wv * wv)
        res.append(q)
    return res[0], res[1]


# ---- 3D (two stacked domains, x and y periodic) -------------------------------
@dataclass(frozen=True)
class Workload3:
    name: str
    nx: int
    ny: int
    nz_lower: int
    nz_upper: int
    lx: float = 10.0
    ly: float = 10.0
    lz_lower: float = 1.25      # fast domain below: dz_lower = dz_upper / 4 at equal nz
    lz_upper: float = 5.0
    fast_is_lower: bool = True
    n_buffer: int = 5
    base: int = 3
    m: int = 4
    steps: int = 200
    gamma: float = 1.4
    prandtl: float = 0.72
    mu_lower: float = 1e-3
    mu_upper: float = 1e-3
    gravity: float = 0.0
    t_lower: float = 1.0
    t_upper: float = 1.0
    amplitude: float = 1e-3
    kmax: int = 4
    seed: int = 3
    cfl: float = 0.5
    dnum: float = 0.25

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def dz_lower(self) -> float:
        return self.lz_lower / self.nz_lower

    @property
    def dz_upper(self) -> float:
        return self.lz_upper / self.nz_upper

    def with_(self, **kw) -> "Workload3":
        return replace(self, **kw)


def large3d() -> Workload3:
    """256 x 256 x 128 cells per domain, slow domain 5 high above a fast domain
    1.25 high (dz_fast = dz_slow / 4), SSP-RK3 base, m = 4, 200 slow steps."""
    return Workload3("two-domain 3D CNS 256x256x128 x2, MPRK3 m=4", nx=256, ny=256, nz_lower=128,
                     nz_upper=128)


def small3d() -> Workload3:
    """A 3D case the oracle finishes in seconds: 24 x 20 x 12 below, x 10 above."""
    return Workload3("two-domain 3D CNS 24x20x(12+10)", nx=24, ny=20, nz_lower=12, nz_upper=10,
                     lz_lower=1.25 * 12 / 10, lz_upper=5.0, m=2, n_buffer=5, steps=10,
                     amplitude=2e-2, seed=5)


def initial_state3(w: Workload3):
    """Uniform background (rho = 1/T, p = 1/gamma, at rest) plus random-phase
    velocity perturbations: each of u, v, w is a sum of cos(kx x + ky y + phase)
    over integer wavenumbers 1 <= |k| <= kmax (k in units of 2 pi / L), seeded
    phases, scaled so the largest |component| is the amplitude (times the
    local sound speed); w is multiplied by sin(pi zeta), zeta the height within
    its domain, so it vanishes at the walls and at the interface."""
    rng = np.random.default_rng(w.seed)
    ks = [(a, b) for a in range(-w.kmax, w.kmax + 1) for b in range(-w.kmax, w.kmax + 1)
          if 0 < a * a + b * b <= w.kmax * w.kmax]
    x = -w.lx / 2 + (np.arange(w.nx) + 0.5) * w.dx
    y = -w.ly / 2 + (np.arange(w.ny) + 0.5) * w.dy
    X, Y = np.meshgrid(x, y)
    fields = []
    for _ in range(3):
        ph = rng.uniform(0, 2 * np.pi, len(ks))
        f = np.zeros_like(X)
        for (a, b), p in zip(ks, ph):
            f += np.cos(2 * np.pi * a * X / w.lx + 2 * np.pi * b * Y / w.ly + p)
        fields.append(f / np.abs(f).max())
    out = []
    for lower in (True, False):
        nz = w.nz_lower if lower else w.nz_upper
        lz = w.lz_lower if lower else w.lz_upper
        T = w.t_lower if lower else w.t_upper
        g = w.gamma
        p0 = 1.0 / g
        rho = g * p0 / T
        a = np.sqrt(T)
        zeta = (np.arange(nz) + 0.5) / nz
        q = np.zeros((5, nz, w.ny, w.nx))
        u = w.amplitude * a * fields[0][None]
        v = w.amplitude * a * fields[1][None]
        ww = w.amplitude * a * fields[2][None] * np.sin(np.pi * zeta)[:, None, None]
        u = np.broadcast_to(u, (nz, w.ny, w.nx))
        v = np.broadcast_to(v, (nz, w.ny, w.nx))
        q[0] = rho
        q[1] = rho * u
        q[2] = rho * v
        q[3] = rho * ww
        q[4] = p0 / (g - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww)
        out.append(q)
    return out[0], out[1]


def random_state3(w: Workload3, seed: int, amp: float = 0.05):
    """Random physical 3D states: rho, T within +-amp of the background,
    |u|, |v|, |w| <= amp a."""
    rng = np.random.default_rng(seed)
    out = []
    for lower in (True, False):
        nz = w.nz_lower if lower else w.nz_upper
        T0 = w.t_lower if lower else w.t_upper
        g = w.gamma
        shp = (nz, w.ny, w.nx)
        rho = (1.0 / T0) * (1 + amp * rng.uniform(-1, 1, shp))
        T = T0 * (1 + amp * rng.uniform(-1, 1, shp))
        a = np.sqrt(T)
        vel = [amp * a * rng.uniform(-1, 1, shp) for _ in range(3)]
        q = np.zeros((5,) + shp)
        q[0] = rho
        for c in range(3):
            q[1 + c] = rho * vel[c]
        q[4] = rho * T / g / (g - 1) + 0.5 * rho * sum(v * v for v in vel)
        out.append(q)
    return out[0], out[1]


def uniform_state3(w: Workload3, rho: float, u: float, v: float, wv: float, p: float):
    out = []
    for nz in (w.nz_lower, w.nz_upper):
        q = np.zeros((5, nz, w.ny, w.nx))
        q[0] = rho
        q[1] = rho * u
        q[2] = rho * v
        q[3] = rho * wv
        q[4] = p / (w.gamma - 1) + 0.5 * rho * (u * u + v * v + wv * wv)
        out.append(q)
    return out[0], out[1]
