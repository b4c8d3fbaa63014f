"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package holds no arithmetic of the fusion method itself: it builds analytic
scenes, camera rigs, ray-cast z-depth maps with the heteroscedastic depth noise
model of the paper's observation model (Sec. 3.5, eq. 5), and next-best-view
candidate poses.  Everything it returns is plain numpy (or torch on a chosen
device for the depth renderer) and is handed unchanged to both sides.
"""
from .cameras import look_at, Camera
from .scenes import surface_points
from .configs import Workload, make_workload
