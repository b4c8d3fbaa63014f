"""Shared helpers of the GPU parity tests: run the library and the oracle on the
same seeded synthetic workload."""
from __future__ import annotations

import functools

import numpy as np
import torch

import oracle as O
import paper_2602_19697_amd as bf
from synth import make_workload

DEV = torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def workload(name, seed=0):
    return make_workload(name, seed=seed)


@functools.lru_cache(maxsize=None)
def oracle_ref(name, seed=0):
    return O.full_pipeline(workload(name, seed), with_acc=True)


def to_dev(wl):
    depth = torch.from_numpy(np.ascontiguousarray(wl.depth)).to(DEV)
    poses = torch.from_numpy(np.ascontiguousarray(wl.poses)).to(DEV)
    return depth, poses


def gpu_system(ctx, wl, keep_dense=False, lam=None, eps=None, lam_b=None):
    depth, poses = to_dev(wl)
    g = bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band)
    band = ctx.bf_build_band(g, wl.cam, depth, poses, keep_dense=keep_dense)
    sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, bf.noise_struct(*wl.noise),
                           wl.lam if lam is None else lam, wl.eps if eps is None else eps,
                           wl.lam_b if lam_b is None else lam_b)
    return band, sys_, depth, poses


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def morton_to_linear(G, P):
    """Index map: linear (k*G+j)*G+i -> Morton position in the P^3 dense cube."""
    i, j, k = np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij")
    i, j, k = i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(), k.transpose(2, 1, 0).ravel()
    key = np.zeros(i.shape, dtype=np.uint64)
    for b in range(11):
        key |= ((i >> b) & 1).astype(np.uint64) << np.uint64(3 * b)
        key |= ((j >> b) & 1).astype(np.uint64) << np.uint64(3 * b + 1)
        key |= ((k >> b) & 1).astype(np.uint64) << np.uint64(3 * b + 2)
    return key.astype(np.int64)
