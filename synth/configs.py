"""Named synthetic workloads shaped like the paper's setting (Sec. 3.1, Sec. 4).

The paper evaluates on an unspecified controlled scene and on a CO3D sequence;
neither is available, so these seeded analytic scenes stand in for them.

* ``tiny``      - 32^3 grid, one sphere, 4 ring views at 80x60 (unit tests).
* ``sphere64``  - one sphere r=0.30 m, 64^3 grid of 1.5 cm voxels, +-3 voxel band,
                  truncation 4 voxels, 8 ring views at 160x120 (fx=fy=150) on a 1.0 m ring.
* ``union256``  - union of 3 spheres, a rounded box and a torus (seeded), 256^3 grid of
                  4 mm voxels, +-4 voxel band, truncation 5 voxels, 40 hemisphere views
                  at 640x480 (fx=fy=525) on a 1.2 m hemisphere.
* ``union512``  - the same generator on a 512^3 grid of 2 mm voxels, 120 views.
* ``union512s`` - as union512 with 16 spheres, 6 rounded boxes and 6 tori (a larger band).
* ``union1024`` - the union512 scene, views and depth maps on a 1024^3 grid of 1 mm voxels
                  (a band of several million voxels, far beyond the 256 MB Infinity Cache).
* ``sphere512`` - the sphere64 scene on a 512^3 grid of 2 mm voxels (tests of the 512^3 walk).
* ``union128``  - the union generator on a 128^3 grid of 8 mm voxels, 24 views at 320x240
                  (training scenes of the warm start).
* ``batchsphere`` - sphere64-type scenes whose voxel size is chosen so the band has a
                  seeded log-uniform target size (the uneven multi-scene batch).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np

from .cameras import Camera, ring_poses, hemisphere_poses, sphere_candidates
from .render import render_depth, add_depth_noise
from .scenes import single_sphere, random_union


@dataclasses.dataclass
class Workload:
    name: str
    G: int
    h: float
    origin: tuple
    tau: float
    band: float            # band half-width in metres (|TSDF| <= band)
    cam: Camera
    poses: np.ndarray      # [T][3][4] float64 camera-to-world
    depth: np.ndarray      # [T][H][W] float32 z-depth, 0 = no return
    noise: tuple = (0.0012, 0.0019, 0.4)   # sigma(z) = a + c (z - z0)^2
    lam: float = 10.0
    eps: float = 1e-6
    lam_b: float = 0.0
    tol: float = 1e-8
    probes: int = 16
    probe_seed: int = 0
    n_cand: int = 512
    cand_radius: float = 1.2
    ray_cam: Camera = Camera.centred(160, 120, 150.0, 150.0)
    scene: Optional[object] = None

    @property
    def T(self) -> int:
        return int(self.poses.shape[0])

    def candidates(self) -> np.ndarray:
        return sphere_candidates(self.n_cand, self.cand_radius)


def _cached_depth(name, seed, render):
    """Rendered noisy depth, kept in $BF_SYNTH_CACHE (if set) as <name>_<seed>.npy
    so that repeated runs (profilers) skip the ray casting."""
    cache = os.environ.get("BF_SYNTH_CACHE")
    if not cache:
        return render()
    path = os.path.join(cache, f"{name}_{seed}.npy")
    if os.path.exists(path):
        return np.load(path)
    depth = render()
    os.makedirs(cache, exist_ok=True)
    np.save(path, depth)
    return depth


def _grid(G: int, h: float):
    o = -G * h / 2.0
    return (o, o, o)


def sphere_workload(name, G, h, beta, trunc, cam, n_views, ring_radius, noise_seed,
                    radius=0.30, device="cpu", **kw) -> Workload:
    scene = single_sphere(radius)
    poses = ring_poses(n_views, ring_radius)
    depth = _cached_depth(name, noise_seed, lambda: add_depth_noise(
        render_depth(scene, cam, poses, device=device), noise_seed))
    return Workload(name=name, G=G, h=h, origin=_grid(G, h), tau=trunc * h, band=beta * h,
                    cam=cam, poses=poses, depth=depth, scene=scene, **kw)


def union_workload(name, G, h, n_views, scene_seed, noise_seed, device="cpu",
                   width=640, height=480, f=525.0, radius=1.2, beta=4, trunc=5, primitives=None, **kw) -> Workload:
    scene = random_union(scene_seed, **(primitives or {}))
    cam = Camera.centred(width, height, f, f)
    poses = hemisphere_poses(n_views, radius)
    depth = _cached_depth(name, noise_seed, lambda: add_depth_noise(
        render_depth(scene, cam, poses, device=device), noise_seed))
    return Workload(name=name, G=G, h=h, origin=_grid(G, h), tau=trunc * h, band=beta * h,
                    cam=cam, poses=poses, depth=depth, scene=scene, **kw)


def batch_target_size(s: int) -> float:
    """Seeded log-uniform band-size target in [2e4, 8e5] for batch scene ``s``."""
    rng = np.random.default_rng((0xBA7C, int(s)))
    return float(math.exp(rng.uniform(math.log(2e4), math.log(8e5))))


# Fraction of a sphere's 7-voxel shell that the 8 ring views bring into the band
# (the polar caps are never seen and the band is |TSDF| <= 3h); measured 0.466-0.476
# over batch scenes of 10k-350k voxels.
RING_BAND_FRACTION = 0.47


def batch_sphere(s: int, device="cpu") -> Workload:
    """Sphere scene whose voxel edge h makes the measured band about
    batch_target_size(s) voxels: h^2 = f 4 pi r^2 7 / N with the observed
    fraction f = RING_BAND_FRACTION of the sphere's shell."""
    n_target = batch_target_size(s)
    h = math.sqrt(RING_BAND_FRACTION * 4.0 * math.pi * 0.3 ** 2 * 7.0 / n_target)
    G = int(math.ceil(0.96 / h))
    return sphere_workload(f"batchsphere{s}", G, h, 3, 4, Camera.centred(160, 120, 150.0, 150.0),
                           8, 1.0, s, device=device, probes=64, tol=1e-6, probe_seed=s)


def train_sphere(s: int, device="cpu") -> Workload:
    """Sphere scene with a seeded radius in [0.15, 0.35] m and voxel edge in
    [12, 20] mm, 8 ring views at 160x120 (training scenes of the warm start)."""
    rng = np.random.default_rng((0x7EA1, int(s)))
    radius = float(rng.uniform(0.15, 0.35))
    h = float(rng.uniform(0.012, 0.020))
    G = int(math.ceil(0.96 / h))
    return sphere_workload(f"trainsphere{s}", G, h, 3, 4, Camera.centred(160, 120, 150.0, 150.0), 8, 1.0, s,
                           radius=radius, device=device, probes=64, tol=1e-6)


def regrid(wl: Workload, name: str, G: int, h: float) -> Workload:
    """The same scene, views and depth maps on another grid: G^3 voxels of edge h
    centred at the origin, with the band half-width and truncation scaled to
    keep their size in voxels."""
    return dataclasses.replace(wl, name=name, G=G, h=h, origin=_grid(G, h), tau=wl.tau / wl.h * h,
                               band=wl.band / wl.h * h)


def make_workload(name: str, device="cpu", seed: int = 0) -> Workload:
    if name == "tiny":
        return sphere_workload("tiny", 32, 0.03, 3, 4, Camera.centred(80, 60, 75.0, 75.0), 4, 1.0,
                               seed, device=device, probes=8)
    if name == "sphere64":
        return sphere_workload("sphere64", 64, 0.015, 3, 4, Camera.centred(160, 120, 150.0, 150.0),
                               8, 1.0, seed, device=device, probes=16, tol=1e-8)
    if name == "sphere512":  # a 512^3 grid (8-voxel bricks) that the oracle can still walk whole
        return sphere_workload("sphere512", 512, 0.002, 3, 4, Camera.centred(160, 120, 150.0, 150.0),
                               8, 1.0, seed, device=device, probes=8, tol=1e-6)
    if name == "union128":
        return union_workload("union128", 128, 0.008, 24, seed, seed, device=device,
                              width=320, height=240, f=262.5, tol=1e-6, probes=16)
    if name == "union256":
        return union_workload("union256", 256, 0.004, 40, seed, seed, device=device,
                              tol=1e-6, probes=32)
    if name == "union512":
        return union_workload("union512", 512, 0.002, 120, seed, seed, device=device,
                              tol=1e-6, probes=32)
    if name == "union1024":  # the 512^3 full pass's scene and views on a 1024^3 grid of 1 mm voxels
        return regrid(make_workload("union512", device=device, seed=seed), "union1024", 1024, 0.001)
    if name == "union512s":  # the 512^3 pass with more primitives (which mostly occlude each other)
        return union_workload("union512s", 512, 0.002, 120, seed, seed, device=device, tol=1e-6, probes=32,
                              primitives=dict(n_spheres=16, n_boxes=6, n_tori=6))
    if name.startswith("batchsphere"):
        return batch_sphere(int(name[len("batchsphere"):]), device=device)
    if name.startswith("trainsphere"):
        return train_sphere(int(name[len("trainsphere"):]), device=device)
    raise KeyError(name)


WORKLOADS = ("tiny", "sphere64", "union128", "union256", "union512")
