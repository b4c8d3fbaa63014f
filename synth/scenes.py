"""Analytic signed-distance scenes used to render synthetic depth.

The scene is only a source of ground-truth depth; the fused field never calls
these functions.  SDFs are evaluated in float64 with torch so that the renderer
can run on the CPU (small test scenes) or on a GPU (full-size workloads).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import torch


def _on(prim, name: str, p: torch.Tensor) -> torch.Tensor:
    """Attribute `name` of a primitive as a tensor on p's device and dtype,
    converted once per device (the renderer evaluates every primitive at every
    sphere-tracing step)."""
    cache = prim.__dict__.setdefault("_tensors", {})
    key = (name, p.device, p.dtype)
    t = cache.get(key)
    if t is None:
        t = torch.as_tensor(np.asarray(getattr(prim, name)), dtype=p.dtype, device=p.device)
        cache[key] = t
    return t


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


@dataclasses.dataclass
class Sphere:
    centre: np.ndarray
    radius: float

    def bound(self) -> float:
        return self.radius

    def sdf(self, p: torch.Tensor) -> torch.Tensor:
        return torch.linalg.vector_norm(p - _on(self, "centre", p), dim=-1) - self.radius


@dataclasses.dataclass
class RoundedBox:
    centre: np.ndarray
    rot: np.ndarray          # local -> world rotation
    half: np.ndarray         # half extents (including the rounding)
    rounding: float

    def bound(self) -> float:
        return float(np.linalg.norm(self.half))

    @property
    def core(self) -> np.ndarray:
        return self.half - self.rounding

    def sdf(self, p: torch.Tensor) -> torch.Tensor:
        q = (p - _on(self, "centre", p)) @ _on(self, "rot", p)  # world -> local
        b = _on(self, "core", p)
        d = q.abs() - b
        outside = torch.linalg.vector_norm(d.clamp(min=0.0), dim=-1)
        inside = d.max(dim=-1).values.clamp(max=0.0)
        return outside + inside - self.rounding


@dataclasses.dataclass
class Torus:
    centre: np.ndarray
    rot: np.ndarray
    major: float
    minor: float

    def bound(self) -> float:
        return self.major + self.minor

    def sdf(self, p: torch.Tensor) -> torch.Tensor:
        q = (p - _on(self, "centre", p)) @ _on(self, "rot", p)
        ring = torch.sqrt(q[..., 0] ** 2 + q[..., 2] ** 2) - self.major
        return torch.sqrt(ring * ring + q[..., 1] ** 2) - self.minor


@dataclasses.dataclass
class Scene:
    prims: List[object]

    def bound(self) -> float:
        return max(float(np.linalg.norm(p.centre)) + p.bound() for p in self.prims)

    def sdf(self, p: torch.Tensor) -> torch.Tensor:
        d = self.prims[0].sdf(p)
        for prim in self.prims[1:]:
            d = torch.minimum(d, prim.sdf(p))
        return d


def single_sphere(radius: float = 0.30, centre=(0.0, 0.0, 0.0)) -> Scene:
    return Scene([Sphere(np.asarray(centre, dtype=np.float64), float(radius))])


def random_union(seed: int, n_spheres: int = 3, n_boxes: int = 1, n_tori: int = 1,
                 size_lo: float = 0.05, size_hi: float = 0.25, half_cube: float = 0.5) -> Scene:
    """Union of spheres, rounded boxes and tori with seeded sizes and poses.

    Sizes are uniform in [size_lo, size_hi]: sphere radius, box half extents,
    torus major radius.  The box rounding is 0.2 x its smallest half extent and
    the torus minor radius is U(0.2, 0.5) x its major radius.  Each primitive's
    bounding sphere lies inside the cube [-half_cube, half_cube]^3.
    """
    rng = np.random.default_rng((0xB5F, int(seed)))
    prims: List[object] = []

    def centre_for(bound: float) -> np.ndarray:
        lim = max(half_cube - bound, 0.0)
        return rng.uniform(-lim, lim, size=3)

    for _ in range(n_spheres):
        r = rng.uniform(size_lo, size_hi)
        prims.append(Sphere(centre_for(r), float(r)))
    for _ in range(n_boxes):
        half = rng.uniform(size_lo, size_hi, size=3)
        rot = _random_rotation(rng)
        box = RoundedBox(np.zeros(3), rot, half, 0.2 * float(half.min()))
        box.centre = centre_for(box.bound())
        prims.append(box)
    for _ in range(n_tori):
        major = rng.uniform(size_lo, size_hi)
        minor = rng.uniform(0.2, 0.5) * major
        rot = _random_rotation(rng)
        tor = Torus(np.zeros(3), rot, float(major), float(minor))
        tor.centre = centre_for(tor.bound())
        prims.append(tor)
    return Scene(prims)


def surface_points(scene: Scene, n: int, seed: int, shell: float = 0.01, device="cpu") -> np.ndarray:
    """n seeded points on the scene's surface (the zero set of its SDF), the
    ground truth of the geometry metrics.

    Candidates are uniform in the scene's bounding cube and kept inside the
    shell |sdf| < shell, so they are spread about evenly by area; each is
    moved by Newton steps p <- p - f(p) grad f / |grad f|^2 (for the exact
    SDFs here one step lands on the nearest surface point of the active
    primitive) and kept when |f| <= 1e-9 afterwards, which drops points that
    landed inside another primitive of the union.
    """
    rng = np.random.default_rng((0x5F3, int(seed)))
    bound = scene.bound()
    out, have = [], 0
    while have < n:
        cand = rng.uniform(-bound, bound, size=(max(4 * n, 65536), 3))
        with torch.no_grad():
            f = scene.sdf(torch.as_tensor(cand, dtype=torch.float64, device=device)).cpu().numpy()
        p = torch.as_tensor(cand[np.abs(f) < shell], dtype=torch.float64, device=device)
        for _ in range(3):
            p = p.detach().requires_grad_(True)
            f = scene.sdf(p)
            (g,) = torch.autograd.grad(f.sum(), p)
            p = p - (f / (g * g).sum(dim=-1).clamp(min=1e-30)).unsqueeze(-1) * g
        with torch.no_grad():
            ok = scene.sdf(p).abs() <= 1e-9
        pts = p.detach()[ok].cpu().numpy()
        out.append(pts)
        have += len(pts)
    return np.ascontiguousarray(np.concatenate(out)[:n])
