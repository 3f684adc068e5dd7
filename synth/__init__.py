"""Seeded synthetic workloads: moving point sets in [0,1]^d, d in {2, 3}.

This module is shared by the CPU oracle and the GPU path as their common input.
It holds no part of the certificate method (no distances, no clearances, no
cells): it only draws positions.  Every trajectory is produced in float64 with a
counter-based Philox generator and rounded once per frame to float32; both sides
consume the same float32 arrays, so there is no cross-device RNG parity to keep.

Layout: a trajectory is a float32 array of shape [T+1, d, N] (structure of
arrays per frame: all x, then all y, then all z), frame 0 being the start.

The paper names its motion families without defining them (Section 3, the list
of ten families, and Table 1 for the names).  The five used here follow
these definitions:

* ``uniform_brownian``: start uniform in [0,1]^d; each step adds a Gaussian
  displacement of per-axis scale eps/sqrt(d), its Euclidean length clipped to eps.
* ``ring_rotation``: a ring of radius 0.4 about the box centre (in the z = 0.5
  plane for d = 3) with static Gaussian thickness 1e-3; each step rotates the set
  rigidly about the centre by the angle that moves radius 0.45 (beyond the
  ring's support) by eps/2, and adds Brownian jitter clipped to eps/2, so eps
  bounds every step.
* ``adversarial_crossing``: two Gaussian blobs (sigma 0.05) centred at x = 0.45
  and x = 0.55 translate toward each other by eps per step along x (they cross
  after 0.05/eps steps).
* ``clustered_drift``: 64 Gaussian clusters (sigma 0.01) with centres uniform in
  [0.2, 0.8]^d, each translating rigidly by eps along its own fixed random unit
  direction.
* ``shear_band``: start uniform; each step moves a point by ((y - 0.5) * eps) along x.

The other five families of the paper's list (``EXTRA_FAMILIES``, used by the
failure audit) are read as follows; in d = 3 the planar ones keep a static
z = 0.5 + N(0, 1e-3^2) layer:

* ``vortex``: start uniform in the disc of radius 0.45 about the centre; each step
  rotates a point about the centre with linear speed eps * exp(-r / 0.15) (a fast
  core, a slow rim: differential rotation), so no point moves more than eps.
* ``filament``: points on the closed three-lobed curve r(theta) = 0.3 + 0.08 sin(3
  theta) about the centre, each with a fixed radial offset N(0, 2e-3^2); each step
  advances theta by eps / (2 * 0.46) for every point (flow along the curve; 0.46
  bounds the curve's speed |dp/dtheta|, so a step moves at most eps / 2).
* ``split_merge``: one Gaussian cluster (sigma 0.05) at the centre; the points of
  one half move by eps per step along a fixed random unit direction u, the other
  half along -u, for the first half of the trajectory, then both halves return.
* ``grid_jitter``: the first n points of a regular lattice with ceil(n^(1/d))
  points per axis (cell-centred), in random order; each step adds Brownian jitter
  clipped to eps (a near-lattice scene: many near-equal distances).
* ``spiral``: an Archimedean spiral r = 0.05 + 0.4 * theta / (6 pi) over three
  turns with Gaussian thickness 1e-3, rotated rigidly about the centre by the
  angle that moves radius 0.46 by eps / 2 per step, plus Brownian jitter clipped
  to eps / 2, the step clipped to eps (jitter lets points drift past 0.46).

Point indices are a random permutation of the generation order, so an index
carries no spatial information in any family.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FAMILIES = (
    "uniform_brownian",
    "ring_rotation",
    "adversarial_crossing",
    "clustered_drift",
    "shear_band",
)

EXTRA_FAMILIES = (
    "vortex",
    "filament",
    "split_merge",
    "grid_jitter",
    "spiral",
)


def rng(*key: int) -> np.random.Generator:
    """Philox stream keyed by a tuple of non-negative integers."""
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(list(key))))


def _clip_norm(delta: np.ndarray, bound: float) -> np.ndarray:
    """Scale columns of delta [d, n] whose Euclidean length exceeds ``bound``."""
    norm = np.sqrt(np.sum(delta * delta, axis=0))
    scale = np.where(norm > bound, bound / np.maximum(norm, 1e-300), 1.0)
    return delta * scale


def _brownian(g: np.random.Generator, d: int, n: int, bound: float) -> np.ndarray:
    return _clip_norm(g.standard_normal((d, n)) * (bound / math.sqrt(d)), bound)


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32)


@dataclass
class Trajectory:
    family: str
    d: int
    n: int
    eps: float
    frames: np.ndarray  # float32 [T+1, d, n]

    @property
    def steps(self) -> int:
        return self.frames.shape[0] - 1


def _planar(g: np.random.Generator, d: int, n: int, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    p = np.empty((d, n))
    p[0] = x
    p[1] = y
    if d == 3:
        p[2] = 0.5 + 1e-3 * g.standard_normal(n)
    return p


def initial_positions(family: str, n: int, d: int, g: np.random.Generator):
    """Frame-0 positions (float64 [d, n]) and per-family motion parameters."""
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    params: dict = {}
    if family in ("uniform_brownian", "shear_band"):
        p = g.random((d, n))
    elif family == "ring_rotation":
        theta = g.random(n) * (2.0 * math.pi)
        radius = 0.4 + 1e-3 * g.standard_normal(n)
        p = np.empty((d, n))
        p[0] = 0.5 + radius * np.cos(theta)
        p[1] = 0.5 + radius * np.sin(theta)
        if d == 3:
            p[2] = 0.5 + 1e-3 * g.standard_normal(n)
    elif family == "adversarial_crossing":
        na = n // 2
        side = np.zeros(n)
        side[:na] = 1.0
        side[na:] = -1.0
        mu = np.full((d, n), 0.5)
        mu[0] = np.where(side > 0, 0.45, 0.55)
        p = mu + 0.05 * g.standard_normal((d, n))
        params["side"] = side  # +1 moves toward +x, -1 toward -x
    elif family == "clustered_drift":
        k = 64
        centres = 0.2 + 0.6 * g.random((d, k))
        label = np.arange(n) % k
        p = centres[:, label] + 0.01 * g.standard_normal((d, n))
        u = g.standard_normal((d, k))
        u /= np.sqrt(np.sum(u * u, axis=0))
        params["label"] = label
        params["direction"] = u
    elif family == "vortex":
        r = 0.45 * np.sqrt(g.random(n))
        theta = g.random(n) * (2.0 * math.pi)
        p = _planar(g, d, n, 0.5 + r * np.cos(theta), 0.5 + r * np.sin(theta))
    elif family == "filament":
        theta = g.random(n) * (2.0 * math.pi)
        params["offset"] = 2e-3 * g.standard_normal(n)
        params["theta"] = theta
        r = 0.3 + 0.08 * np.sin(3.0 * theta) + params["offset"]
        p = _planar(g, d, n, 0.5 + r * np.cos(theta), 0.5 + r * np.sin(theta))
    elif family == "split_merge":
        p = 0.5 + 0.05 * g.standard_normal((d, n))
        u = g.standard_normal(d)
        params["direction"] = u / math.sqrt(float(np.sum(u * u)))
        params["side"] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    elif family == "grid_jitter":
        m = int(math.ceil(n ** (1.0 / d) - 1e-9))
        while m ** d < n:
            m += 1
        idx = np.arange(n)
        p = np.empty((d, n))
        for k in range(d):
            p[k] = ((idx // (m ** k)) % m + 0.5) / m
    elif family == "spiral":
        s = g.random(n)
        theta = s * (6.0 * math.pi)
        r = 0.05 + 0.4 * s + 1e-3 * g.standard_normal(n)
        p = _planar(g, d, n, 0.5 + r * np.cos(theta), 0.5 + r * np.sin(theta))
    else:
        raise ValueError(f"unknown family {family!r}")
    perm = g.permutation(n)
    p = p[:, perm]
    for key in ("side", "label", "offset", "theta"):
        if key in params:
            params[key] = params[key][perm]
    return p, params


def make_trajectory(family: str, n: int, d: int, steps: int, eps: float, seed) -> Trajectory:
    """Seeded trajectory of ``steps`` transitions; ``seed`` is an int or a tuple of ints."""
    key = seed if isinstance(seed, tuple) else (seed,)
    g = rng(*key)
    p64, params = initial_positions(family, n, d, g)
    frames = np.empty((steps + 1, d, n), dtype=np.float32)
    frames[0] = _f32(p64)
    centre = 0.5
    omega = (0.5 * eps) / 0.45
    c, s = math.cos(omega), math.sin(omega)
    for t in range(steps):
        cur = frames[t].astype(np.float64)
        if family == "uniform_brownian":
            nxt = cur + _brownian(g, d, n, eps)
        elif family == "ring_rotation":
            x = cur[0] - centre
            y = cur[1] - centre
            nxt = cur.copy()
            nxt[0] = centre + (c * x - s * y)
            nxt[1] = centre + (s * x + c * y)
            nxt += _brownian(g, d, n, 0.5 * eps)
        elif family == "adversarial_crossing":
            nxt = cur.copy()
            nxt[0] += params["side"] * eps
        elif family == "clustered_drift":
            nxt = cur + eps * params["direction"][:, params["label"]]
        elif family == "shear_band":
            nxt = cur.copy()
            nxt[0] += (cur[1] - 0.5) * eps
        elif family == "vortex":
            x = cur[0] - centre
            y = cur[1] - centre
            r = np.sqrt(x * x + y * y)
            ang = eps * np.exp(-r / 0.15) / np.maximum(r, 1e-9)
            ang = np.minimum(ang, 1.0)  # the chord 2 r sin(a/2) stays below r a <= eps
            ca, sa = np.cos(ang), np.sin(ang)
            nxt = cur.copy()
            nxt[0] = centre + (ca * x - sa * y)
            nxt[1] = centre + (sa * x + ca * y)
        elif family == "filament":
            params["theta"] = params["theta"] + eps / (2.0 * 0.46)
            th = params["theta"]
            r = 0.3 + 0.08 * np.sin(3.0 * th) + params["offset"]
            nxt = cur.copy()
            nxt[0] = centre + r * np.cos(th)
            nxt[1] = centre + r * np.sin(th)
        elif family == "split_merge":
            sign = 1.0 if t < steps // 2 else -1.0
            nxt = cur + (sign * eps) * params["direction"][:, None] * params["side"][None, :]
        elif family == "grid_jitter":
            nxt = cur + _brownian(g, d, n, eps)
        elif family == "spiral":
            x = cur[0] - centre
            y = cur[1] - centre
            a = (0.5 * eps) / 0.46
            ca, sa = math.cos(a), math.sin(a)
            rot = np.zeros_like(cur)
            rot[0] = (ca * x - sa * y) - x
            rot[1] = (sa * x + ca * y) - y
            # jitter accumulates, so a point may drift past radius 0.46: the whole
            # step is clipped to eps
            nxt = cur + _clip_norm(rot + _brownian(g, d, n, 0.5 * eps), eps)
        else:  # pragma: no cover - rejected by initial_positions
            raise ValueError(family)
        frames[t + 1] = _f32(nxt)
    return Trajectory(family, d, n, eps, frames)


# --- the workload configurations -------------------------------------------------

def plane_1k(steps: int = 50) -> Trajectory:
    """N = 1000 uniform points in the unit square, Brownian steps clipped to 1e-3."""
    return make_trajectory("uniform_brownian", 1000, 2, steps, 1e-3, 1)


def cube_16k(family: str, n: int = 16000, steps: int = 200) -> Trajectory:
    """N = 16000 points in the unit cube, eps = 5e-4, one of the five families."""
    return make_trajectory(family, n, 3, steps, 5e-4, 2000 + FAMILIES.index(family))


@dataclass
class BatchSpec:
    n: np.ndarray       # int64 [scenes]
    d: np.ndarray       # int32 [scenes]
    family: list        # str per scene


def batch_spec(scenes: int = 512, lo: int = 500, hi: int = 20000, seed: int = 4000) -> BatchSpec:
    """Scene sizes log-uniform in [lo, hi], d uniform over {2, 3}, family uniform."""
    g = rng(seed)
    n = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), scenes))).astype(np.int64)
    d = np.where(g.random(scenes) < 0.5, 2, 3).astype(np.int32)
    fam = [FAMILIES[int(k)] for k in g.integers(0, len(FAMILIES), scenes)]
    return BatchSpec(n, d, fam)


def batch_trajectories(spec: BatchSpec, steps: int, eps: float = 5e-4, seed: int = 4000):
    """One trajectory per scene, scene s keyed by (seed, s)."""
    return [make_trajectory(spec.family[s], int(spec.n[s]), int(spec.d[s]), steps, eps, (seed, s))
            for s in range(len(spec.n))]


def concat_frame(trajs, t: int) -> np.ndarray:
    """Concatenate frame t of every scene: scene s's block is [d_s][N_s] SoA."""
    return np.concatenate([tr.frames[t].reshape(-1) for tr in trajs]).astype(np.float32)


# --- the frontier-fraction sweep (one large scene, one transition per point) ---------

def sweep_start(n: int = 1 << 20, seed: int = 3000) -> np.ndarray:
    """N points uniform in the unit square, float32 [2, N]."""
    return _f32(rng(seed).random((2, n)))


def sweep_centre(seed: int = 3000) -> np.ndarray:
    """Centre of the moving disc, uniform in [0.1, 0.9]^2."""
    return 0.1 + 0.8 * rng(seed, 1).random(2)


def sweep_motion(p0: np.ndarray, eps: float, mode: str, seed: int = 3000, radius: float = 0.05) -> np.ndarray:
    """One transition of the sweep: Brownian steps clipped to eps for the points inside
    a disc of the given radius ("localized"), or for the same number of points drawn
    uniformly at random ("diffuse"); every other point stays put."""
    g = rng(seed, 2)
    p = p0.astype(np.float64)
    c = sweep_centre(seed)
    inside = np.flatnonzero((p[0] - c[0]) ** 2 + (p[1] - c[1]) ** 2 <= radius * radius)
    if mode == "localized":
        movers = inside
    elif mode == "diffuse":
        movers = np.sort(g.choice(p.shape[1], inside.size, replace=False))
    else:
        raise ValueError(mode)
    p[:, movers] += _brownian(g, 2, movers.size, eps)
    return _f32(p)


def sweep_lists(p0: np.ndarray, count: int, seed: int = 3000):
    """Forced frontiers of equal size: the ``count`` points nearest the disc centre
    (localized) and ``count`` points drawn uniformly (diffuse), ascending int32."""
    g = rng(seed, 3)
    c = sweep_centre(seed)
    r2 = (p0[0].astype(np.float64) - c[0]) ** 2 + (p0[1].astype(np.float64) - c[1]) ** 2
    local = np.sort(np.argpartition(r2, count - 1)[:count]).astype(np.int32)
    diffuse = np.sort(g.choice(p0.shape[1], count, replace=False)).astype(np.int32)
    return local, diffuse


# --- large scenes generated on the device (scaling runs) ---------------------------

def device_uniform(n: int, d: int, seed: int, device="cuda"):
    """N points uniform in the unit box, float32 [d, N], drawn on the device by a
    seeded torch generator (for sizes whose host generation would dominate)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.rand((d, n), generator=g, device=device, dtype=torch.float32)


def device_brownian_step(p, eps: float, seed: int):
    """One Brownian transition of device positions: per-axis Gaussian of scale
    eps/sqrt(d), each displacement's Euclidean length clipped to 0.999 * eps (the
    margin keeps the binary32 step within eps)."""
    import torch
    d = p.shape[0]
    g = torch.Generator(device=p.device)
    g.manual_seed(int(seed))
    delta = torch.randn(p.shape, generator=g, device=p.device, dtype=torch.float32) * (eps / math.sqrt(d))
    norm = torch.sqrt((delta * delta).sum(0, keepdim=True))
    scale = torch.clamp((0.999 * eps) / torch.clamp(norm, min=1e-30), max=1.0)
    return (p + delta * scale).contiguous()
