"""Seeded synthetic initial conditions for the gravity workloads.

This module only draws inputs. It holds none of the force, tree or integrator
arithmetic, so both the GPU library and the CPU oracle can be fed from it
without sharing any of the method's code.

Workload shapes follow the paper's gravity experiments (uniform random clouds,
Section "GPU-parallel octree") and its rubble-pile aggregation scenes (Section
"The asteroid aggregation problem"), in N-body units (G = 1).

All generators use numpy's PCG64 with an explicit seed and return float64
arrays: positions and velocities as (N, 3) C-contiguous, masses and softening
lengths as (N,).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Scene",
    "uniform_ball",
    "uniform_cube",
    "plummer",
    "rubble_pile",
    "batched_scenes",
    "perturbed_target",
    "two_body_circular",
]


@dataclass
class Scene:
    """One synthetic scene. ``eps`` is None when the softening is uniform."""

    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    eps: np.ndarray | None
    softening: float
    name: str

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _ball_points(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    # radius * u^(1/3) gives a uniform density inside the ball; the direction
    # is an isotropic Gaussian draw normalised to unit length.
    u = rng.random(n)
    d = rng.standard_normal((n, 3))
    norm = np.sqrt((d * d).sum(axis=1))
    norm[norm == 0.0] = 1.0
    return np.ascontiguousarray(d / norm[:, None] * (radius * np.cbrt(u))[:, None])


def uniform_ball(n: int, seed: int = 11, radius: float = 1.0, softening: float = 1e-3,
                 total_mass: float = 1.0) -> Scene:
    """Uniform sphere of radius ``radius``, equal masses ``total_mass/n``, at rest."""
    rng = _rng(seed)
    pos = _ball_points(rng, n, radius)
    mass = np.full(n, total_mass / max(n, 1), dtype=np.float64)
    vel = np.zeros((n, 3), dtype=np.float64)
    return Scene(pos, vel, mass, None, softening, f"uniform_ball(n={n},seed={seed})")


def uniform_cube(n: int, seed: int = 12, side: float = 2.0, softening: float = 1e-3,
                 total_mass: float = 1.0) -> Scene:
    """Uniform random cube centred on the origin, as in the paper's timing runs."""
    rng = _rng(seed)
    pos = np.ascontiguousarray((rng.random((n, 3)) - 0.5) * side)
    mass = np.full(n, total_mass / max(n, 1), dtype=np.float64)
    vel = np.zeros((n, 3), dtype=np.float64)
    return Scene(pos, vel, mass, None, softening, f"uniform_cube(n={n},seed={seed})")


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    # uniform directions on the unit sphere by (cos theta, phi) sampling
    cz = 2.0 * rng.random(n) - 1.0
    ph = 2.0 * math.pi * rng.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def plummer(n: int, seed: int = 22, a: float = 1.0, total_mass: float = 1.0,
            rmax: float = 10.0, softening: float = 1e-3) -> Scene:
    """Plummer sphere sampled the Aarseth-Henon-Wielen (1974) way, in G = 1 units.

    Radii come from inverting the cumulative mass profile, redrawn beyond
    ``rmax``; speeds are q * v_esc with q drawn by rejection from
    g(q) = q^2 (1 - q^2)^(7/2); directions are isotropic; the cloud is moved
    to its centre-of-mass frame.
    """
    rng = _rng(seed)
    r = np.empty(n)
    filled = 0
    while filled < n:
        x = rng.random(n - filled)
        x = x[x > 0.0]
        rr = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr <= rmax]
        take = min(rr.size, n - filled)
        r[filled:filled + take] = rr[:take]
        filled += take
    pos = _isotropic(rng, n) * (a * r)[:, None]
    q = np.empty(n)
    filled = 0
    while filled < n:
        m = 2 * (n - filled) + 16
        x = rng.random(m)
        y = 0.1 * rng.random(m)
        ok = y < x * x * (1.0 - x * x) ** 3.5
        xs = x[ok]
        take = min(xs.size, n - filled)
        q[filled:filled + take] = xs[:take]
        filled += take
    vesc = math.sqrt(2.0 * total_mass / a) * (1.0 + r * r) ** (-0.25)
    vel = _isotropic(rng, n) * (q * vesc)[:, None]
    mass = np.full(n, total_mass / n)
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    return Scene(np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass, None,
                 softening, f"plummer(n={n},seed={seed})")


def rubble_pile(n: int, seed: int = 33, radius: float = 1.0, median_r: float = 1e-3,
                sigma: float = 0.3, virial_frac: float = 0.1, omega: float = 0.2,
                total_mass: float = 1.0) -> Scene:
    """Rubble-pile aggregation cloud in G = 1 units.

    Body centres are uniform in a ball of ``radius``; body radii are lognormal
    (median ``median_r``, log-sigma ``sigma``); masses scale as r^3 and sum to
    ``total_mass``; velocities are isotropic Gaussian in the centre-of-mass
    frame, scaled so the mass-weighted rms speed is ``virial_frac`` times the
    virial speed sqrt(3 G M / (5 R)) of a uniform sphere, plus solid-body spin
    ``omega`` about z. Each body's softening length is its radius.
    """
    rng = _rng(seed)
    pos = _ball_points(rng, n, radius)
    rad = median_r * np.exp(sigma * rng.standard_normal(n))
    mass = rad ** 3
    mass *= total_mass / mass.sum()
    vel = rng.standard_normal((n, 3))
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    vrms = math.sqrt(float((mass * (vel * vel).sum(1)).sum() / mass.sum()))
    target = virial_frac * math.sqrt(0.6 * total_mass / radius)
    vel *= target / vrms
    vel[:, 0] += -omega * pos[:, 1]
    vel[:, 1] += omega * pos[:, 0]
    return Scene(np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass,
                 np.ascontiguousarray(rad), 0.0, f"rubble_pile(n={n},seed={seed})")


def batched_scenes(n_scenes: int = 256, seed: int = 44, n_lo: int = 1024,
                   n_hi: int = 65536, softening: float = 1e-3) -> list[Scene]:
    """Independent uniform-ball scenes with N log-uniform in [n_lo, n_hi]."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_scenes))).astype(np.int64)
    return [uniform_ball(int(ns[s]), seed=4400 + s, softening=softening) for s in range(n_scenes)]


def perturbed_target(pos: np.ndarray, seed: int = 56, scale: float = 0.01) -> np.ndarray:
    """x_target = x + scale * xi with xi ~ N(0, I)."""
    rng = _rng(seed)
    return np.ascontiguousarray(pos + scale * rng.standard_normal(pos.shape))


def two_body_circular(m1: float = 0.6, m2: float = 0.4, sep: float = 1.0) -> Scene:
    """Two bodies on a circular orbit about their barycentre (G = 1, no softening)."""
    mt = m1 + m2
    pos = np.array([[-m2 / mt * sep, 0.0, 0.0], [m1 / mt * sep, 0.0, 0.0]])
    w = math.sqrt(mt / sep ** 3)
    vel = np.array([[0.0, -m2 / mt * sep * w, 0.0], [0.0, m1 / mt * sep * w, 0.0]])
    return Scene(pos, vel, np.array([m1, m2]), None, 0.0, "two_body_circular")
