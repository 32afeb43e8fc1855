"""Seeded synthetic workloads (positions, velocities, masses).

This module draws random numbers and lays them out; it contains none of the
Barnes-Hut arithmetic.  Both the GPU library's tests and benchmark and the CPU
oracle take their inputs from here.

The paper's workload is a thin self-gravitating planetary ring around a
central planet (Sec. 2 and Table 1: ring radius 1e5 km, width 100 km,
1e7 particles per process).  The generators below produce dimensionless
stand-ins for it (G = 1, ring radius ~1) plus Plummer spheres for the
batched case.  All generators use numpy's PCG64 (np.random.default_rng).
"""
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class System:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.size)

    def pos(self):
        return self.x, self.y, self.z

    def vel(self):
        return self.vx, self.vy, self.vz


def ring(n, seed, r_in=1.0, r_out=1.1, z_sigma=1e-3, central_mass=0.0, v_disp=1e-4, G=1.0):
    """Thin ring: r uniform in [r_in, r_out], phi uniform, z ~ N(0, z_sigma).

    Equal masses 1/n.  With central_mass > 0 the velocities are circular
    Keplerian about the origin, sqrt(G M / r_cyl) along phi-hat, plus an
    isotropic Gaussian dispersion v_disp per Cartesian component; otherwise
    the velocities are the dispersion alone.
    """
    rng = np.random.default_rng(seed)
    r = r_in + (r_out - r_in) * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    z = rng.normal(0.0, z_sigma, n)
    x = r * np.cos(phi)
    y = r * np.sin(phi)
    dv = rng.normal(0.0, v_disp, (3, n))
    if central_mass > 0.0:
        vc = np.sqrt(G * central_mass / np.hypot(x, y))
        vx = -vc * np.sin(phi) + dv[0]
        vy = vc * np.cos(phi) + dv[1]
    else:
        vx, vy = dv[0].copy(), dv[1].copy()
    vz = dv[2].copy()
    m = np.full(n, 1.0 / n)
    return System(x, y, z, vx, vy, vz, m)


def plummer(n, seed, a=1.0, M=1.0, r_max=10.0, G=1.0):
    """Plummer sphere by the Aarseth, Henon & Wielen (1974) recipe.

    Radii from the inverted cumulative mass, r = a (u^(-2/3) - 1)^(-1/2),
    redrawn while r > r_max; speeds q * v_esc(r) with q drawn by rejection
    from g(q) = q^2 (1 - q^2)^(7/2); isotropic directions; masses M / n.
    """
    rng = np.random.default_rng(seed)
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        u = rng.random(todo.size)
        rr = a / np.sqrt(np.maximum(u, 1e-300) ** (-2.0 / 3.0) - 1.0)
        ok = (rr <= r_max) & np.isfinite(rr)
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]

    def iso(k):
        cz = 2.0 * rng.random(k) - 1.0
        ph = 2.0 * math.pi * rng.random(k)
        sz = np.sqrt(1.0 - cz * cz)
        return sz * np.cos(ph), sz * np.sin(ph), cz

    ux, uy, uz = iso(n)
    q = np.empty(n)
    todo = np.arange(n)
    gmax = 0.1
    while todo.size:
        qq = rng.random(todo.size)
        gg = gmax * rng.random(todo.size)
        ok = gg < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * G * M) * (r * r + a * a) ** -0.25
    vx_, vy_, vz_ = iso(n)
    v = q * vesc
    return System(r * ux, r * uy, r * uz, v * vx_, v * vy_, v * vz_, np.full(n, M / n))


def force_sample(n, seed, k=4096):
    """Sorted indices of the particles whose force error is measured."""
    rng = np.random.default_rng(seed + 1000)
    k = min(k, n)
    return np.sort(rng.choice(n, k, replace=False))


# --------------------------------------------------------------------------
# The five workloads.  Sizes and parameters follow the problem statement of
# the benchmark; seeds: ring cases 0, 1, 3; batched Plummer spheres 2.
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    systems: list
    theta: float
    eps: float
    n_leaf: int = 8
    n_grp: int = 64
    G: float = 1.0
    central_mass: float = 0.0
    dt: float = 0.0
    n_steps: int = 0
    rebuild_every: int = 1
    extra: dict = field(default_factory=dict)


def workload(idx, n=None):
    """Workload idx in 0..4; n overrides the particle count (for small tests)."""
    if idx == 0:
        n = n or 4096
        return Workload("ring4k_fp64_single_force", [ring(n, 0)], theta=0.5, eps=1e-3, n_grp=64)
    if idx == 1:
        n = n or 1 << 20
        return Workload("ring1m_fp32_10steps", [ring(n, 1, central_mass=1.0)], theta=0.5, eps=1e-4,
                        n_grp=256, central_mass=1.0, dt=1e-3, n_steps=10, rebuild_every=1)
    if idx == 2:
        rng = np.random.default_rng(2)
        nk = np.rint(np.exp(rng.uniform(math.log(1e3), math.log(2e5), 64))).astype(int)
        if n is not None:                      # scale the whole batch down for tests
            nk = np.maximum(16, (nk * n // max(1, nk.sum())).astype(int))
        systems = [plummer(int(k), 200 + s) for s, k in enumerate(nk)]
        return Workload("plummer64_batched_20steps", systems, theta=0.6, eps=1e-2, n_grp=0,
                        dt=2.0 ** -8, n_steps=20, rebuild_every=1)
    if idx in (3, 4):
        n = n or 1 << 24
        sysm = ring(n, 3, r_in=1.0, r_out=1.2, z_sigma=5e-4, central_mass=1.0)
        return Workload("ring16m_reuse4_32steps" if idx == 3 else "ring16m_learned",
                        [sysm], theta=0.5, eps=1e-4, n_grp=256, central_mass=1.0, dt=1e-3,
                        n_steps=32, rebuild_every=4)
    raise ValueError(idx)
