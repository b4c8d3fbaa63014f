"""Ray-cast z-depth of an analytic scene and seeded heteroscedastic noise.

Each pixel's ray is o + s * R (u'/fx, v'/fy, 1): with the camera-frame direction
normalised to z = 1 the ray parameter s is the camera-z depth directly.  The
ray is sphere-traced against the scene SDF inside the scene's bounding sphere.
Missed pixels get depth 0 (no return).
"""
from __future__ import annotations

import sys

import numpy as np
import torch

from .cameras import Camera


def sigma_depth(z, a: float = 0.0012, c: float = 0.0019, z0: float = 0.4):
    """Sensor noise standard deviation (metres) used to simulate depth."""
    return a + c * (z - z0) ** 2


def _ray_dirs(cam: Camera, device, dtype=torch.float64) -> torch.Tensor:
    rows = torch.arange(cam.height, dtype=dtype, device=device)
    cols = torch.arange(cam.width, dtype=dtype, device=device)
    v, u = torch.meshgrid(rows, cols, indexing="ij")
    d = torch.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, torch.ones_like(u)], dim=-1)
    return d.reshape(-1, 3)


@torch.no_grad()
def render_depth(scene, cam: Camera, poses: np.ndarray, device="cpu",
                 max_steps: int = 256, hit_eps: float = 1e-7) -> np.ndarray:
    """Noise-free z-depth maps, float64 [T][H][W]; 0 where the ray misses."""
    poses = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    dcam = _ray_dirs(cam, device)
    bound = scene.bound() + 1e-3
    out = np.zeros((poses.shape[0], cam.height, cam.width), dtype=np.float64)
    for t, pose in enumerate(poses):
        if poses.shape[0] >= 40 and t % 20 == 0:
            print(f"[render] view {t}/{poses.shape[0]}", file=sys.stderr, flush=True)
        rot = torch.as_tensor(pose[:, :3], dtype=torch.float64, device=device)
        org = torch.as_tensor(pose[:, 3], dtype=torch.float64, device=device)
        d = dcam @ rot.T
        dn = torch.linalg.vector_norm(d, dim=-1)
        # Entry/exit of the bounding sphere |o + s d| = bound.
        a2 = (d * d).sum(-1)
        b2 = 2.0 * (d @ org)
        c2 = float(org @ org) - bound * bound
        disc = b2 * b2 - 4.0 * a2 * c2
        hit_bs = disc > 0
        sq = torch.sqrt(disc.clamp(min=0.0))
        s = ((-b2 - sq) / (2.0 * a2)).clamp(min=0.0)
        s_far = (-b2 + sq) / (2.0 * a2)
        depth = torch.zeros_like(s)
        idx = torch.nonzero(hit_bs & (s_far > 0), as_tuple=False).squeeze(1)
        s = s[idx]
        s_far = s_far[idx]
        dd = d[idx]
        dnn = dn[idx]
        for _ in range(max_steps):
            if idx.numel() == 0:
                break
            p = org + s.unsqueeze(1) * dd
            dist = scene.sdf(p)
            hit = dist < hit_eps * (1.0 + s)
            depth[idx[hit]] = s[hit]
            keep = (~hit) & (s <= s_far)
            s = (s + dist / dnn)[keep]
            idx, s_far, dd, dnn = idx[keep], s_far[keep], dd[keep], dnn[keep]
        out[t] = depth.reshape(cam.height, cam.width).cpu().numpy()
    return out


def add_depth_noise(depth: np.ndarray, seed: int, a: float = 0.0012, c: float = 0.0019,
                    z0: float = 0.4) -> np.ndarray:
    """D = z + N(0, sigma(z)^2) on valid pixels, as float32; invalid pixels stay 0."""
    rng = np.random.default_rng(int(seed))
    noise = rng.standard_normal(depth.shape)
    valid = depth > 0
    noisy = np.where(valid, depth + sigma_depth(depth, a, c, z0) * noise, 0.0)
    noisy = np.where(noisy > 0, noisy, 0.0)
    return noisy.astype(np.float32)
