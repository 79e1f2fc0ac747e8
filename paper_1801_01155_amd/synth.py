"""Seeded synthetic inputs: streamline sets, cameras and transfer functions.

This module only *produces inputs*. It holds none of the rendering method's
arithmetic (no grid set-up, no voxelization, no ray generation, no shading);
both the HIP library and the CPU oracle consume what it returns.

Streamlines stand in for the paper's flow datasets (Results section, dataset
list): they are RK4 integral curves of the ABC flow

    u(x) = (A sin z + C cos y,  B sin x + A cos z,  C sin y + B cos x),
    A = sqrt(3), B = sqrt(2), C = 1,

optionally plus eight seeded divergence-free sinusoidal modes
``0.1 * e_m * sin(k_m . x + phi_m)`` (``e_m`` orthogonal to ``k_m``).
Vertices are emitted in world coordinates as float32, the paper's "original
geometry" format (Memory statistics section: 3 floats per vertex); mapping
them into grid coordinates is the method's first step and lives on each side.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

ABC_A = math.sqrt(3.0)
ABC_B = math.sqrt(2.0)
ABC_C = 1.0
RK4_DT = 0.01


@dataclass
class LineSet:
    xyz: np.ndarray        # float32 [V, 3] world coordinates
    curve_off: np.ndarray  # int64 [C + 1]
    attr: np.ndarray       # uint8 [C]: round(255 * importance)

    @property
    def n_curves(self) -> int:
        return int(self.curve_off.shape[0] - 1)

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])


def _perturbation(rng: np.random.Generator, n_modes: int = 8):
    ks, es = [], []
    while len(ks) < n_modes:
        k = rng.integers(-3, 4, size=3).astype(np.float64)
        if not k.any():
            continue
        e = rng.normal(size=3)
        e -= k * (e @ k) / (k @ k)
        n = np.linalg.norm(e)
        if n < 1e-6:
            continue
        ks.append(k)
        es.append(e / n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return np.array(ks), np.array(es), phi


def _velocity(x: np.ndarray, modes) -> np.ndarray:
    px, py, pz = x[:, 0], x[:, 1], x[:, 2]
    u = np.empty_like(x)
    u[:, 0] = ABC_A * np.sin(pz) + ABC_C * np.cos(py)
    u[:, 1] = ABC_B * np.sin(px) + ABC_A * np.cos(pz)
    u[:, 2] = ABC_C * np.sin(py) + ABC_B * np.cos(px)
    if modes is not None:
        ks, es, phi = modes
        s = np.sin(x @ ks.T + phi)            # [n, m]
        u += 0.1 * (s @ es)
    return u


def abc_lineset(n_curves: int, n_vertices: int, seed: int,
                perturb: bool = False, chunk: int = 1 << 14, workers: int = 0) -> LineSet:
    """RK4 (dt = 0.01, fp64) streamlines of the (perturbed) ABC flow.

    Seeds are uniform in [0, 2 pi]^3 from ``numpy.random.default_rng(seed)``;
    draw order: seeds, perturbation modes (if any), per-curve importance.
    Curves are integrated in fixed chunks of ``chunk`` curves, spread over
    ``workers`` threads (0: up to 8); the result does not depend on the
    number of threads.
    """
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, 2.0 * math.pi, size=(n_curves, 3))
    modes = _perturbation(rng) if perturb else None
    importance = rng.uniform(0.0, 1.0, size=n_curves)
    attr = np.rint(255.0 * importance).astype(np.uint8)

    xyz = np.empty((n_curves, n_vertices, 3), dtype=np.float32)
    h = RK4_DT

    def integrate(c0):
        x = seeds[c0:c0 + chunk].copy()
        xyz[c0:c0 + chunk, 0] = x
        for i in range(1, n_vertices):
            k1 = _velocity(x, modes)
            k2 = _velocity(x + 0.5 * h * k1, modes)
            k3 = _velocity(x + 0.5 * h * k2, modes)
            k4 = _velocity(x + h * k3, modes)
            x = x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            xyz[c0:c0 + chunk, i] = x

    starts = list(range(0, n_curves, chunk))
    nw = workers if workers > 0 else min(8, os.cpu_count() or 1)
    if nw > 1 and len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(nw, len(starts))) as ex:
            list(ex.map(integrate, starts))
    else:
        for c0 in starts:
            integrate(c0)
    curve_off = np.arange(n_curves + 1, dtype=np.int64) * n_vertices
    return LineSet(xyz.reshape(-1, 3), curve_off, attr)


# ----------------------------------------------------------------------------
# Cameras: (eye, forward, right, up) as float32; right/up are the half-extent
# vectors of the image plane (not unit vectors).
# ----------------------------------------------------------------------------

@dataclass
class Camera:
    eye: tuple
    forward: tuple
    right: tuple
    up: tuple
    width: int
    height: int
    orthographic: bool = False

    def as_arrays(self):
        f = lambda v: np.asarray(v, dtype=np.float32)
        return f(self.eye), f(self.forward), f(self.right), f(self.up)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def look_camera(grid, width: int, height: int, view_dir, orthographic: bool,
                dist_factor: float = None, fov_deg: float = 40.0) -> Camera:
    """Camera looking at the grid centre from direction ``view_dir``.

    Perspective: eye at centre + 2.6 R * w, vertical field of view 40 deg.
    Orthographic: eye at centre + 2 R * w, image half-height 0.9 R.
    World up is +z (falls back to +y when looking along z).
    """
    g = np.asarray(grid, dtype=np.float64)
    R = float(g.max())
    c = g / 2.0
    w = _unit(view_dir)
    F = -w
    zup = np.array([0.0, 0.0, 1.0])
    if abs(F @ zup) > 0.999:
        zup = np.array([0.0, 1.0, 0.0])
    r = _unit(np.cross(F, zup))
    u = np.cross(r, F)
    aspect = width / height
    if orthographic:
        d = 2.0 * R if dist_factor is None else dist_factor * R
        eye = c + d * w
        Rv = 0.9 * R * aspect * r
        Uv = 0.9 * R * u
    else:
        d = 2.6 * R if dist_factor is None else dist_factor * R
        eye = c + d * w
        t = math.tan(math.radians(fov_deg) / 2.0)
        Rv = t * aspect * r
        Uv = t * u
    t32 = lambda v: tuple(float(x) for x in np.asarray(v, dtype=np.float32))
    return Camera(t32(eye), t32(F), t32(Rv), t32(Uv), width, height, orthographic)


def default_camera(grid, width, height, orthographic=False) -> Camera:
    return look_camera(grid, width, height, (1.0, 0.8, 0.6), orthographic)


def orbit_cameras(grid, n: int, seed: int, width: int, height: int,
                  orthographic: bool = False):
    """``n`` seeded random views on a sphere around the grid centre."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        v = rng.normal(size=3)
        cams.append(look_camera(grid, width, height, v, orthographic))
    return cams


# ----------------------------------------------------------------------------
# Transfer functions: straight-alpha RGBA [256][4], indexed by the 1-byte
# per-line attribute.
# ----------------------------------------------------------------------------

def _ramp_rgb(x: np.ndarray) -> np.ndarray:
    # blue -> cyan -> yellow -> red
    stops = np.array([[0.10, 0.20, 0.90], [0.10, 0.80, 0.90],
                      [0.95, 0.90, 0.20], [0.90, 0.15, 0.10]])
    pos = x * (len(stops) - 1)
    i = np.clip(np.floor(pos).astype(int), 0, len(stops) - 2)
    f = (pos - i)[:, None]
    return stops[i] * (1 - f) + stops[i + 1] * f


def lut_importance_alpha(a_min: float = 0.02, a_max: float = 0.5) -> np.ndarray:
    """alpha = a_min + (a_max - a_min) * attr / 255, colour ramp over attr."""
    x = np.arange(256, dtype=np.float64) / 255.0
    lut = np.empty((256, 4), dtype=np.float32)
    lut[:, :3] = _ramp_rgb(x)
    lut[:, 3] = a_min + (a_max - a_min) * x
    return lut


def lut_constant(rgb=(0.8, 0.8, 0.8), alpha: float = 1.0) -> np.ndarray:
    lut = np.empty((256, 4), dtype=np.float32)
    lut[:, :3] = np.asarray(rgb, dtype=np.float32)
    lut[:, 3] = alpha
    return lut


def lut_ramp(alpha: float = 1.0) -> np.ndarray:
    x = np.arange(256, dtype=np.float64) / 255.0
    lut = np.empty((256, 4), dtype=np.float32)
    lut[:, :3] = _ramp_rgb(x)
    lut[:, 3] = alpha
    return lut


# ----------------------------------------------------------------------------
# Workloads (sizes of the paper-scale synthetic stand-ins)
# ----------------------------------------------------------------------------

WORKLOADS = {
    # 1000 x 64 vertices, 64^3, N=32, r=0.4, opaque, 256x256 orthographic
    "small": dict(n_curves=1000, n_vertices=64, seed=1, perturb=False,
                  grid=64, bins=32, radius=0.4, opaque=True,
                  width=256, height=256, orthographic=True),
    # 100k x 200 vertices, 256^3, transparent, alpha in [0.02, 0.5], 1080p
    "scale": dict(n_curves=100_000, n_vertices=200, seed=2, perturb=True,
                  grid=256, bins=32, radius=0.4, opaque=False,
                  width=1920, height=1080, orthographic=False),
    # 1M x 100 vertices, 512^3, LoD + AO (16 cones) + soft shadow, 1080p
    "gi": dict(n_curves=1_000_000, n_vertices=100, seed=3, perturb=True,
               grid=512, bins=32, radius=0.4, opaque=False,
               width=1920, height=1080, orthographic=False),
}

LIGHT_DIR = tuple(float(x) for x in _unit((-0.4, -0.3, -0.87)).astype(np.float32))


def batch_workload_spec(seed: int = 4, n_sets: int = 8, n_views: int = 64,
                        min_segments: float = 1e6, max_segments: float = 20e6,
                        vertices_per_curve: int = 100):
    """Sets and views of the batching workload.

    Sets: n_seg_i = min * (max/min)^(i/(n_sets-1)) input segments as curves
    of 100 vertices; grids 128^3 (i < 3), 256^3 (i < 6), else 512^3; even sets
    opaque, odd transparent. Views: area log-uniform in [256^2, 1920*1080],
    aspect 1:1, 4:3 or 16:9, view k on set k mod n_sets, seeded orbit cameras.
    """
    rng = np.random.default_rng(seed)
    sets = []
    for i in range(n_sets):
        nseg = min_segments * (max_segments / min_segments) ** (i / max(1, n_sets - 1))
        n_curves = max(1, int(round(nseg / (vertices_per_curve - 1))))
        grid = 128 if i < 3 else (256 if i < 6 else 512)
        sets.append(dict(n_curves=n_curves, n_vertices=vertices_per_curve, seed=100 + i,
                         perturb=True, grid=grid, opaque=(i % 2 == 0)))
    views = []
    lo, hi = np.log(256.0 * 256.0), np.log(1920.0 * 1080.0)
    for k in range(n_views):
        area = float(np.exp(rng.uniform(lo, hi)))
        aspect = [1.0, 4.0 / 3.0, 16.0 / 9.0][int(rng.integers(0, 3))]
        h = max(16, int(round(np.sqrt(area / aspect))))
        w = max(16, int(round(h * aspect)))
        direction = rng.normal(size=3)
        views.append(dict(set=k % n_sets, width=w, height=h, direction=tuple(direction)))
    return sets, views


SERVE_RESOLUTIONS = ((512, 512), (1280, 720), (1920, 1080))


def serve_workload_spec(seed: int = 5, n_requests: int = 2000,
                        set_segments=(1e6, 5e6, 20e6, 50e6), grids=(256, 256, 512, 512),
                        vertices_per_curve: int = 100):
    """Resident sets and the request stream of the serving workload.

    Sets: curves of 100 vertices with the given input-segment counts and
    grids (perturbed flow, seeds 200 + i). Requests: set uniform over the
    sets, resolution uniform over 512^2, 1280x720 and 1920x1080,
    transparency and AO shading each on with probability 1/2, direction of a
    random orbit camera. Arrival times are drawn by the caller per rate.
    """
    rng = np.random.default_rng(seed)
    sets = []
    for i, (nseg, g) in enumerate(zip(set_segments, grids)):
        n_curves = max(1, int(round(nseg / (vertices_per_curve - 1))))
        sets.append(dict(n_curves=n_curves, n_vertices=vertices_per_curve, seed=200 + i,
                         perturb=True, grid=g))
    reqs = []
    for _ in range(n_requests):
        s = int(rng.integers(0, len(sets)))
        w, h = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        transparent = bool(rng.integers(0, 2))
        ao = bool(rng.integers(0, 2))
        direction = tuple(rng.normal(size=3))
        reqs.append(dict(set=s, width=w, height=h, transparent=transparent, ao=ao,
                         direction=direction))
    return sets, reqs
