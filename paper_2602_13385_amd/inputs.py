"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no part of the method's arithmetic (no basis functions, no
coefficients, no host-potential forces): it only draws particle positions,
velocities, masses, orbit initial conditions and target tracks from textbook
distributions with numpy's PCG64 generator, so both sides are fed identical
inputs.  The paper's own initial conditions (King W0 = 5 clusters drawn with
COSMIC, Milky-Way globular-cluster orbits) are not available; these recipes
stand in for them with the same shapes and sizes.

Units: G = M = a = 1 (N-body units) unless stated otherwise.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 13385

R_MIN = 1e-6  # no particle is placed closer than this to the expansion centre


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng, n):
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(ph), s * np.sin(ph), mu])


def _push_out(pos):
    r = np.sqrt((pos * pos).sum(0))
    small = r < R_MIN
    if small.any():
        pos[:, small] *= (R_MIN / np.maximum(r[small], 1e-300))
        # exactly-zero radii get a fixed direction
        zero = small & (r == 0.0)
        pos[0, zero] = R_MIN
    return pos


@dataclass
class Particles:
    pos: np.ndarray  # (3, n) float64
    vel: np.ndarray  # (3, n) float64
    mass: np.ndarray  # (n,) float64

    @property
    def n(self):
        return self.mass.shape[0]

    def state(self):
        return np.concatenate([self.pos, self.vel], axis=0)


def plummer(n: int, seed: int, M: float = 1.0, a: float = 1.0, G: float = 1.0,
            centre_com: bool = True) -> Particles:
    """Plummer sphere (Aarseth, Henon & Wielen 1974 recipe), equal masses."""
    rng = _rng(seed)
    X = rng.uniform(0.0, 1.0, n)
    X = np.clip(X, 1e-300, 1.0 - 1e-15)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = r * _isotropic(rng, n)
    # speed fraction q = v / v_esc from g(q) = q^2 (1 - q^2)^(7/2) by rejection
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    vel = (q * vesc) * _isotropic(rng, n)
    mass = np.full(n, M / n)
    if centre_com and n > 0:
        pos -= pos.mean(axis=1, keepdims=True)
        vel -= vel.mean(axis=1, keepdims=True)
    return Particles(_push_out(pos), vel, mass)


def hernquist(n: int, seed: int, M: float = 1.0, a: float = 1.0, sigma_v: float = 0.3) -> Particles:
    """Hernquist sphere positions (inverse cumulative mass), Gaussian velocities."""
    rng = _rng(seed)
    X = rng.uniform(0.0, 1.0, n)
    X = np.clip(X, 1e-300, 1.0 - 1e-12)
    sx = np.sqrt(X)
    r = a * sx / (1.0 - sx)
    pos = r * _isotropic(rng, n)
    vel = rng.normal(0.0, sigma_v, (3, n))
    mass = np.full(n, M / n)
    return Particles(_push_out(pos), vel, mass)


def uniform_ball(n: int, seed: int, radius: float = 2.0) -> Particles:
    """Uniform ball, for edge cases and small parity tests."""
    rng = _rng(seed)
    r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    pos = r * _isotropic(rng, n)
    vel = rng.normal(0.0, 0.3, (3, n))
    mass = rng.uniform(0.5, 1.5, n) / max(n, 1)
    return Particles(_push_out(pos), vel, mass)


def quadrature_sphere(profile: str, alpha: float, nr: int = 48, nmu: int = 24, nphi: int = 24,
                      M: float = 1.0, a: float = 1.0) -> Particles:
    """Deterministic 'quadrature particles' for a spherical profile.

    Nodes: radius r = a ((1+u)/(1-u))^alpha on Gauss nodes u in (-1, 1),
    Gauss-Legendre in cos(theta), uniform in phi; masses = rho dV times the
    weights.  For the Hernquist profile with alpha = 1 Gauss-Legendre nodes are
    used in u; for the Plummer profile with alpha = 1/2 Gauss-Chebyshev nodes of
    the second kind, for which sums of mass x polynomial(u) are exact."""
    if profile == "hernquist":
        u, wu = np.polynomial.legendre.leggauss(nr)
        rho = lambda r: M * a / (2.0 * math.pi * r * (r + a) ** 3)
    elif profile == "plummer":
        k = np.arange(1, nr + 1)
        u = np.cos(k * math.pi / (nr + 1))
        wu = math.pi / (nr + 1) * np.sin(k * math.pi / (nr + 1)) ** 2
        wu = wu / np.sqrt(1.0 - u * u)  # convert to weights for the plain measure du
        rho = lambda r: 3.0 * M / (4.0 * math.pi * a ** 3) * (1.0 + (r / a) ** 2) ** -2.5
    else:
        raise ValueError(profile)
    t = (1.0 + u) / (1.0 - u)
    r = a * t ** alpha
    drdu = a * alpha * t ** (alpha - 1.0) * 2.0 / (1.0 - u) ** 2
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    ph = (np.arange(nphi) + 0.5) * 2.0 * math.pi / nphi
    wph = np.full(nphi, 2.0 * math.pi / nphi)
    R, MU, PH = np.meshgrid(r, mu, ph, indexing="ij")
    W = (wu * rho(r) * r * r * drdu)[:, None, None] * wmu[None, :, None] * wph[None, None, :]
    S = np.sqrt(1.0 - MU * MU)
    pos = np.stack([R * S * np.cos(PH), R * S * np.sin(PH), R * MU]).reshape(3, -1)
    mass = W.reshape(-1)
    vel = np.zeros_like(pos)
    return Particles(pos, vel, mass)


# ----------------------------------------------------------------------------
# workload recipes (seed = SEED_BASE + config index)
# ----------------------------------------------------------------------------
# circular speed of the logarithmic halo psi = v0^2/2 ln(r^2 + rc^2) with
# v0 = 1.5, rc = 1 at R = 20: v0 R / sqrt(R^2 + rc^2)
LOG_VC_20 = 1.5 * 20.0 / math.sqrt(401.0)


@dataclass
class Workload:
    name: str
    nmax: int
    lmax: int
    dt: float
    nsteps: int
    clusters: list = field(default_factory=list)  # list of Particles
    centres: list = field(default_factory=list)  # list of (6,) arrays R, V
    host: list = field(default_factory=list)  # list of (kind_name, params)
    alpha: float = 1.0
    b: float = 1.0
    G: float = 1.0
    extra: dict = field(default_factory=dict)


def config1(n: int = 10_000) -> Workload:
    """Isolated Plummer, N = 1e4, nmax = 6, lmax = 4, 100 steps of dt = 0.01."""
    p = plummer(n, SEED_BASE + 1)
    return Workload("isolated-plummer-N1e4-n6l4", 6, 4, 0.01, 100, [p], [np.zeros(6)], [])


def config2(n: int = 100_000) -> Workload:
    """Plummer N = 1e5 on a circular orbit R = 20 in a logarithmic halo."""
    p = plummer(n, SEED_BASE + 2)
    c = np.array([20.0, 0.0, 0.0, 0.0, LOG_VC_20, 0.0])
    return Workload("plummer-N1e5-n10l6-log-host", 10, 6, 0.005, 10_000, [p], [c],
                    [("log", (1.5, 1.0, 0.0))])


def config3(n: int = 1_000_000) -> Workload:
    """Hernquist N = 1e6, nmax = 16, lmax = 10, single step (no host)."""
    p = hernquist(n, SEED_BASE + 3)
    return Workload("hernquist-N1e6-n16l10", 16, 10, 0.005, 1, [p], [np.zeros(6)], [])


# composite host for config 4 (G = 1, length unit kpc, v_c(20) ~ 1.5):
# Hernquist bulge + Miyamoto-Nagai disk + NFW halo
CONFIG4_HOST = [("hernquist", (1.11955, 1.0, 0.0)),
                ("mn", (11.8372, 3.0, 0.28)),
                ("nfw", (124.107, 15.626, 0.0))]


BATCHED_ORBITS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                              "tests", "golden", "batched_orbits.txt")


def batched_orbit_speeds(path: str = BATCHED_ORBITS) -> np.ndarray:
    """Apocentre speeds of the batched workload's orbits: a stored table (the
    speeds whose orbits, integrated in the composite host, have the drawn
    eccentricities; written once by tests/golden/make_batched_orbits.py)."""
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return np.array([float(r[3]) for r in rows])


def config4(nclust: int = 10, nmin: float = 2e4, nmax_n: float = 5e5,
            orbit_speeds="stored") -> Workload:
    """10 Plummer progenitors, N log-uniform in [2e4, 5e5], eccentric orbits:
    e ~ U(0.1, 0.7) and r_apo ~ U(15, 40), an isotropic orbital plane, the
    start at apocentre with the tangential speed of the stored table
    (orbit_speeds=None leaves the speeds zero, for the script that finds them)."""
    rng = _rng(SEED_BASE + 4)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax_n), nclust))).astype(int)
    es = rng.uniform(0.1, 0.7, nclust)
    rapo = rng.uniform(15.0, 40.0, nclust)
    speeds = batched_orbit_speeds() if orbit_speeds == "stored" else np.zeros(nclust)
    assert len(speeds) == nclust
    clusters, centres, planes = [], [], []
    for i in range(nclust):
        clusters.append(plummer(int(ns[i]), SEED_BASE + 400 + i))
        nrm = _isotropic(rng, 1)[:, 0]  # orbital-plane normal
        # apocentre direction perpendicular to the normal
        tmp = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(nrm, tmp)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        planes.append((e1, e2))
        centres.append(np.concatenate([rapo[i] * e1, speeds[i] * e2]))
    return Workload("batched-10-plummer-n10l6-composite-host", 10, 6, 0.005, 1000, clusters,
                    centres, list(CONFIG4_HOST),
                    extra={"e_target": es, "r_apo": rapo, "plane": planes})


def config5(n: int = 100_000) -> Workload:
    """Adjoint workload: Plummer N = 1e5 in an NFW host, 2000 steps."""
    p = plummer(n, SEED_BASE + 5)
    c = np.array([20.0, 0.0, 0.0, 0.1, 1.4, 0.3])
    track = target_track(SEED_BASE + 5)
    return Workload("adjoint-plummer-N1e5-n10l6-nfw", 10, 6, 0.005, 2000, [p], [c],
                    [("nfw", (232.98, 20.0, 0.0))], extra={"track": track, "checkpoint": 100})


def target_track(seed: int, npts: int = 200, radius: float = 20.0, jitter: float = 0.2) -> np.ndarray:
    """Seeded target stream track: a tilted arc of radius ~20 plus N(0, jitter^2)."""
    rng = _rng(seed + 1000)
    ph = np.linspace(0.0, 1.5 * math.pi, npts)
    rr = radius * (1.0 + 0.05 * np.sin(3.0 * ph))
    pts = np.stack([rr * np.cos(ph), rr * np.sin(ph), 2.0 * np.sin(ph)], axis=1)
    return pts + rng.normal(0.0, jitter, pts.shape)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
