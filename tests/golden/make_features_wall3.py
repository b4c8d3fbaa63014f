"""Writes features_wall3.txt: the 12 learned-start input features of a plus-shaped
band on a 4^3 grid (0.25 m voxels, low corner -0.5 m) seen by five
fronto-parallel views from (0, 0, -2) along +z whose walls lie at camera
depths 2.1, 2.2, 2.25, 1.6 and 2.45 m (each rounded to float32, as the depth maps hold
them).  Tau = 0.5 m.  Noise sigma(D) = 0.0012 + 0.0019 (D - 0.4)^2.

Everything is derived from the definitions with exact rational arithmetic
(fractions.Fraction); only the two logarithms are taken in double at the end.
No oracle code is used.

Features of a voxel with camera depth Z (= its centre's z + 2):
  y_t = min(D_t - Z, tau) for each view with D_t - Z >= -tau; W = n_obs = #views kept
  0 TSDF/h = mean(y)/h     1 log(1 + W)     2 deg/6     3 n_obs/T
  4 mean y/h   5 (mean y^2 - mean(y)^2)/h^2   6 mean sigma/h   7 min sigma/h
  8 log(1 + h^2 sum 1/sigma^2)
  9-11 (TSDF(+a) - TSDF(-a)) / (2h) along x, y, z, with the voxel's own TSDF
       where that neighbour is not in the band.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np

H = Fr(1, 4)
TAU = Fr(1, 2)
VIEWS = [Fr(float(np.float32(d))) for d in (2.1, 2.2, 2.25, 1.6, 2.45)]
CENTRE = (1, 2, 2)
OFFS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))
CELLS = [CENTRE] + [tuple(c + d for c, d in zip(CENTRE, o)) for o in OFFS]


def sigma(D):
    e = D - Fr(2, 5)
    return Fr(12, 10000) + Fr(19, 10000) * e * e


def voxel_obs(c):
    Z = Fr(-1, 2) + (c[2] + Fr(1, 2)) * H + 2  # camera z of the voxel centre
    ys, sig = [], []
    for D in VIEWS:
        d = D - Z
        if d < -TAU:
            continue
        ys.append(min(d, TAU))
        sig.append(sigma(D))
    return ys, sig


def tsdf(c):
    ys, _ = voxel_obs(c)
    return sum(ys, Fr(0)) / len(ys)


def features(c):
    ys, sig = voxel_obs(c)
    n = len(ys)
    my = sum(ys, Fr(0)) / n
    vy = sum((y * y for y in ys), Fr(0)) / n - my * my
    lam = sum((1 / (s * s) for s in sig), Fr(0))
    inband = set(CELLS)
    deg = sum(tuple(a + d for a, d in zip(c, o)) in inband for o in OFFS)
    out = [tsdf(c) / H, math.log(1 + n), Fr(deg, 6), Fr(n, len(VIEWS)), my / H, vy / (H * H),
           sum(sig, Fr(0)) / n / H, min(sig) / H, math.log(float(1 + lam * H * H))]
    for a in range(3):
        m = tuple(x - (1 if i == a else 0) for i, x in enumerate(c))
        p = tuple(x + (1 if i == a else 0) for i, x in enumerate(c))
        tm = tsdf(m) if m in inband else tsdf(c)
        tp = tsdf(p) if p in inband else tsdf(c)
        out.append((tp - tm) / (2 * H))
    return [float(v) for v in out]


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "features_wall3.txt")
    with open(path, "w") as fh:
        fh.write("# Learned-start features of a plus-shaped band under five wall views;\n")
        fh.write("# derived by hand (exact rationals) in make_features_wall3.py.  Columns:\n")
        fh.write("# i j k  TSDF/h log(1+W) deg/6 n_obs/T mean_y/h var_y/h^2 mean_sigma/h min_sigma/h "
                 "log(1+Lambda h^2) dx dy dz\n")
        for c in CELLS:
            fh.write(" ".join(str(v) for v in c) + " " + " ".join(repr(v) for v in features(c)) + "\n")


if __name__ == "__main__":
    main()
