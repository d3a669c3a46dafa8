"""Seeded synthetic workloads for exact grid DBSCAN.

This module only draws point sets and parameters.  It holds none of the
clustering arithmetic, so both the CPU oracle's tests and the GPU path's
tests and benchmark can take their inputs from here without sharing any
code with each other.

The shapes follow the paper's experimental section (Section 5.1): integer
coordinates, seed-spreader data (a random walk that emits points uniformly
in a ball around its current location and restarts at a random location
with a small probability) and Gaussian-blob data with uniform noise.  The
paper's own SS-simden / SS-varden files and its real data sets are not
available; these generators stand in for their shapes.

Every generator returns an ``int32`` array of shape ``(n, d)``; callers pass
it on as ``float32`` (every value is an integer of magnitude below 2**24,
so the conversion is exact).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One clustering problem: a generator recipe plus eps and MinPts."""

    name: str
    n: int
    d: int
    eps: int
    minpts: int
    seed: int
    kind: str            # "blobs" or "spreader"
    domain: int          # coordinates are clipped to [0, domain]
    # blob parameters
    n_blobs: int = 0
    sigma: float = 0.0               # isotropic sigma (if sigma_range is None)
    sigma_range: tuple | None = None  # per-axis log-uniform sigma range
    noise_frac: float = 0.0
    # spreader parameters
    pts_per_step: int = 0
    step_len: float = 0.0
    ball_radius: float = 0.0
    restart_p: float = 0.0
    radius_levels: int = 1   # >1: each walk segment scales its ball and step by 2**k, k < levels

    def with_n(self, n: int) -> "Workload":
        """Same recipe at a different size (used for small parity cases)."""
        return dataclasses.replace(self, n=int(n), name=f"{self.name}@n={n}")


# The five workloads of the benchmark plan plus the n=10M, d=3 headline one.
WORKLOADS = {
    "cfg0": Workload("cfg0", n=10_000, d=2, eps=100, minpts=10, seed=20221014,
                     kind="blobs", domain=10_000, n_blobs=10, sigma=200.0,
                     noise_frac=0.10),
    "cfg1": Workload("cfg1", n=2_000_000, d=3, eps=200, minpts=100, seed=20221015,
                     kind="spreader", domain=100_000, pts_per_step=100,
                     step_len=50.0, ball_radius=100.0, restart_p=0.001,
                     noise_frac=0.0001),
    "cfg2": Workload("cfg2", n=10_000_000, d=5, eps=5000, minpts=20, seed=20221016,
                     kind="blobs", domain=1_000_000, n_blobs=100,
                     sigma_range=(2000.0, 20000.0), noise_frac=0.01),
    "cfg4": Workload("cfg4", n=20_000_000, d=3, eps=150, minpts=50, seed=20221018,
                     kind="spreader", domain=100_000, pts_per_step=300,
                     step_len=50.0, ball_radius=100.0, restart_p=0.001,
                     noise_frac=0.0001),
    "H": Workload("H", n=10_000_000, d=3, eps=200, minpts=100, seed=20221019,
                  kind="spreader", domain=100_000, pts_per_step=100,
                  step_len=50.0, ball_radius=100.0, restart_p=0.001,
                  noise_frac=0.0001),
}

BATCH_SEED_BASE = 20221017
BATCH_COUNT = 256


def _ball(rng: np.random.Generator, m: int, d: int, radius: float) -> np.ndarray:
    """m points uniform in the d-ball of the given radius (centred at 0)."""
    g = rng.standard_normal((m, d))
    g /= np.maximum(np.linalg.norm(g, axis=1, keepdims=True), 1e-300)
    r = radius * rng.random(m) ** (1.0 / d)
    return g * r[:, None]


def _spreader(w: Workload, rng: np.random.Generator) -> np.ndarray:
    n_noise = int(round(w.noise_frac * w.n))
    n_walk = w.n - n_noise
    steps = -(-n_walk // w.pts_per_step)
    L = float(w.domain)
    loc = rng.random(w.d) * L
    dirs = rng.standard_normal((steps, w.d))
    dirs /= np.maximum(np.linalg.norm(dirs, axis=1, keepdims=True), 1e-300)
    restart = rng.random(steps) < w.restart_p
    jumps = rng.random((steps, w.d)) * L
    # variable density: a segment between restarts spreads its points over a
    # ball (and moves by a step) 2**k times the base size; the extra draws
    # come from a stream of their own so one-level recipes are unchanged
    scale = np.ones(steps)
    if w.radius_levels > 1:
        seg = np.cumsum(restart)
        k = np.random.default_rng(w.seed + 1).integers(0, w.radius_levels, size=int(seg[-1]) + 1)
        scale = np.exp2(k[seg])
    centres = np.empty((steps, w.d))
    for s in range(steps):
        if restart[s]:
            loc = jumps[s].copy()
        centres[s] = loc
        loc = loc + w.step_len * scale[s] * dirs[s]
        # reflect at the walls of the domain
        loc = np.where(loc < 0.0, -loc, loc)
        loc = np.where(loc > L, 2.0 * L - loc, loc)
    owner = np.repeat(np.arange(steps), w.pts_per_step)[:n_walk]
    walk = centres[owner] + _ball(rng, n_walk, w.d, w.ball_radius) * scale[owner, None]
    noise = rng.random((n_noise, w.d)) * L
    return np.concatenate([walk, noise], axis=0)


def _blobs(w: Workload, rng: np.random.Generator) -> np.ndarray:
    n_noise = int(round(w.noise_frac * w.n))
    n_blob = w.n - n_noise
    L = float(w.domain)
    centres = rng.random((w.n_blobs, w.d)) * L
    if w.sigma_range is not None:
        lo, hi = w.sigma_range
        sig = np.exp(rng.uniform(math.log(lo), math.log(hi), (w.n_blobs, w.d)))
    else:
        sig = np.full((w.n_blobs, w.d), w.sigma)
    counts = rng.multinomial(n_blob, np.full(w.n_blobs, 1.0 / w.n_blobs))
    owner = np.repeat(np.arange(w.n_blobs), counts)
    pts = centres[owner] + rng.standard_normal((n_blob, w.d)) * sig[owner]
    noise = rng.random((n_noise, w.d)) * L
    return np.concatenate([pts, noise], axis=0)


def make_points(w: Workload | str, n: int | None = None) -> np.ndarray:
    """Draw the workload's points: int32 array (n, d), rows in random order."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    if n is not None:
        w = w.with_n(n)
    rng = np.random.default_rng(w.seed)
    if w.kind == "spreader":
        x = _spreader(w, rng)
    elif w.kind == "blobs":
        x = _blobs(w, rng)
    else:
        raise ValueError(f"unknown workload kind {w.kind!r}")
    x = np.clip(np.rint(x), 0, w.domain).astype(np.int32)
    perm = rng.permutation(x.shape[0])
    return np.ascontiguousarray(x[perm])


def batch_workloads(count: int = BATCH_COUNT, seed_base: int = BATCH_SEED_BASE):
    """The heterogeneous batch: per instance n log-uniform in [1e3, 1e6],
    d in {2, 3}, Gaussian blobs plus 10% noise in [0, 1e4]^d, integer eps in
    [50, 300] and integer MinPts in [5, 50]."""
    out = []
    for i in range(count):
        seed = seed_base * 1000 + i
        rng = np.random.default_rng(seed)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e6)))))
        d = int(rng.integers(2, 4))
        eps = int(rng.integers(50, 301))
        minpts = int(rng.integers(5, 51))
        out.append(Workload(f"batch{i}", n=n, d=d, eps=eps, minpts=minpts,
                            seed=seed + 7, kind="blobs", domain=10_000,
                            n_blobs=10, sigma=200.0, noise_frac=0.10))
    return out


# The paper's sweeps (Section 5.2): seed-spreader data in [0, 1e5]^d with
# similar (simden) or variable (varden) cluster density, d in {2, 3, 5, 7},
# 2M points unless n is the swept quantity.  Defaults: eps 2000, MinPts 100.
SWEEP_DIMS = (2, 3, 5, 7)
SWEEP_KINDS = ("simden", "varden")
SWEEP_EPS = (500, 1000, 2000, 3000, 4000, 5000)
SWEEP_MINPTS = (10, 25, 50, 75, 100)
SWEEP_N = (100_000, 500_000, 2_000_000, 5_000_000, 10_000_000)
SWEEP_DEFAULT = {"n": 2_000_000, "eps": 2000, "minpts": 100}


def sweep_workload(kind: str, d: int, n: int = SWEEP_DEFAULT["n"], eps: int = SWEEP_DEFAULT["eps"],
                   minpts: int = SWEEP_DEFAULT["minpts"]) -> Workload:
    """Seed-spreader data of the sweeps.  The spreader emits 100 points
    uniformly in a ball of radius 100 around its location, then moves
    50 d in a random direction; it jumps to a uniform random location about
    ten times over the whole set (so about ten walks, whatever n), and 1e-4
    of the points are uniform noise.  varden gives each walk a ball radius
    and step of 1, 2, 4 or 8 times the base.  The points depend on
    (kind, d, n) only, so an eps or MinPts sweep clusters one point set."""
    if kind not in SWEEP_KINDS:
        raise ValueError(f"unknown sweep kind {kind!r}")
    seed = 20221100 + 100 * SWEEP_KINDS.index(kind) + 10 * d + SWEEP_N.index(n) if n in SWEEP_N else \
        20221200 + 10 * d + SWEEP_KINDS.index(kind) + n
    return Workload(f"ss-{kind}-{d}d@n={n}", n=int(n), d=int(d), eps=int(eps), minpts=int(minpts), seed=seed,
                    kind="spreader", domain=100_000, pts_per_step=100, step_len=50.0 * d, ball_radius=100.0,
                    restart_p=min(1.0, 10.0 * 100 / max(n, 1)), noise_frac=1e-4,
                    radius_levels=4 if kind == "varden" else 1)


def sweep_name(w: Workload) -> str:
    """Key of a sweep point: 'ss-<kind>-<d>d/n=<n>/eps=<eps>/minpts=<minpts>'."""
    return f"{w.name.split('@')[0]}/n={w.n}/eps={w.eps}/minpts={w.minpts}"


def sweep_from_name(key: str) -> Workload:
    """Inverse of sweep_name."""
    head, *fields = key.split("/")
    _, kind, dd = head.split("-")
    kv = dict(f.split("=") for f in fields)
    return sweep_workload(kind, int(dd[:-1]), int(kv["n"]), int(kv["eps"]), int(kv["minpts"]))


def random_small(seed: int, n: int, d: int, domain: int) -> np.ndarray:
    """Uniform integer points, for tiny brute-force cases."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, domain + 1, size=(n, d), dtype=np.int64).astype(np.int32)
