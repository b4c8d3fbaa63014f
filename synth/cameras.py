"""Pinhole cameras and pose rigs (OpenCV convention: x right, y down, z forward).

A pose is the 3x4 camera-to-world matrix [R | t] of Sec. 3.1 (T_{w<-c}); the
columns of R are the camera axes in world coordinates and t is the optical
centre.  Depth values produced for these cameras are camera-z depth, which is
what the back-projection of eq. (2) implies (the third entry of K^-1 u~ is 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @staticmethod
    def centred(width: int, height: int, fx: float, fy: float) -> "Camera":
        # Pixel centres sit on integers, so the principal point of a centred
        # camera is ((W-1)/2, (H-1)/2).
        return Camera(width, height, float(fx), float(fy), (width - 1) / 2.0, (height - 1) / 2.0)


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world 3x4 pose looking from ``eye`` at ``target``."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(fwd @ up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0]) if abs(fwd[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    pose = np.empty((3, 4), dtype=np.float64)
    pose[:, 0] = right
    pose[:, 1] = down
    pose[:, 2] = fwd
    pose[:, 3] = eye
    return pose


def ring_poses(n: int, radius: float, z: float = 0.0) -> np.ndarray:
    """``n`` poses on a horizontal ring at angles 2*pi*k/n, looking at the origin."""
    out = np.empty((n, 3, 4), dtype=np.float64)
    for k in range(n):
        a = 2.0 * math.pi * k / n
        out[k] = look_at((radius * math.cos(a), radius * math.sin(a), z))
    return out


def _fibonacci(n: int, hemisphere: bool) -> np.ndarray:
    golden = math.pi * (3.0 - math.sqrt(5.0))
    pts = np.empty((n, 3), dtype=np.float64)
    for i in range(n):
        if hemisphere:
            zc = 1.0 - (i + 0.5) / n
        else:
            zc = 1.0 - (2.0 * i + 1.0) / n
        r = math.sqrt(max(0.0, 1.0 - zc * zc))
        phi = i * golden
        pts[i] = (r * math.cos(phi), r * math.sin(phi), zc)
    return pts


def hemisphere_poses(n: int, radius: float) -> np.ndarray:
    """``n`` poses on the upper hemisphere (Fibonacci lattice), looking at the origin."""
    return np.stack([look_at(radius * p) for p in _fibonacci(n, True)])


def sphere_candidates(n: int, radius: float) -> np.ndarray:
    """``n`` candidate poses on a full sphere (Fibonacci lattice), looking at the origin.

    Next-best-view candidates are generated here, once, on the host, and passed
    to every scorer as input, so no transcendental function is evaluated by the
    scorers themselves.
    """
    return np.stack([look_at(radius * p) for p in _fibonacci(n, False)])
