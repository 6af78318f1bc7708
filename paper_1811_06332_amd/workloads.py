"""Seeded synthetic particle systems shared by the GPU path's tests, the
benchmark and the oracle's tests.

This module only draws positions and charges with numpy's ``default_rng``; it
contains none of the method's arithmetic.  The paper measures on no dataset
(its only measurements are single operator calls, Table 1), so these recipes
stand in for the workloads: a uniform cube, a Plummer sphere and a Hernquist
cluster, with the sizes, charges and seeds listed in ``CONFIGS``.
"""
from __future__ import annotations

import math

import numpy as np


def uniform_cube(n: int, seed: int, qlo: float = 0.5, qhi: float = 1.5):
    """x ~ U[0,1)^3, q ~ U(qlo, qhi).  Returns (xyz [n,3] f64, q [n] f64)."""
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3))
    q = rng.uniform(qlo, qhi, n)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(q)


def _isotropic(rng, r):
    u = rng.uniform(-1.0, 1.0, r.size)
    phi = rng.uniform(0.0, 2.0 * math.pi, r.size)
    s = np.sqrt(np.maximum(0.0, 1.0 - u * u))
    return np.stack([r * s * np.cos(phi), r * s * np.sin(phi), r * u], axis=1)


def plummer(n: int, seed: int, rcut: float = 20.0):
    """Plummer sphere, scale radius 1, radius truncated at rcut by drawing the
    enclosed-mass fraction X ~ U(0, M(rcut)) with M(r) = r^3/(r^2+1)^{3/2} and
    inverting r = (X^{-2/3} - 1)^{-1/2}; isotropic directions; q = 1/n."""
    rng = np.random.default_rng(seed)
    mcut = rcut ** 3 / (rcut ** 2 + 1.0) ** 1.5
    X = rng.uniform(0.0, mcut, n)
    X = np.maximum(X, 1e-300)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    xyz = _isotropic(rng, r)
    q = np.full(n, 1.0 / n)
    return np.ascontiguousarray(xyz), q


def hernquist(n: int, seed: int, rcut: float = 50.0):
    """Hernquist cluster, scale 1, cut at rcut: M(r) = r^2/(r+1)^2, so
    r = sqrt(X)/(1 - sqrt(X)) with X ~ U(0, M(rcut)); isotropic; q = 1/n."""
    rng = np.random.default_rng(seed)
    mcut = (rcut / (rcut + 1.0)) ** 2
    X = rng.uniform(0.0, mcut, n)
    s = np.sqrt(X)
    r = s / (1.0 - s)
    xyz = _isotropic(rng, r)
    q = np.full(n, 1.0 / n)
    return np.ascontiguousarray(xyz), q


def batched_systems(nsys: int = 256, base_seed: int = 2000, nmin: float = 1e4, nmax: float = 5e5):
    """Uneven batch: N_i = round(exp(U(ln nmin, ln nmax))) drawn from seed
    base_seed-1; system i uses seed base_seed+i; even i -> uniform cube with
    q ~ U(0.5,1.5), odd i -> Plummer with q = 1/N_i; p_i = (4,6,8)[i % 3]."""
    rng = np.random.default_rng(base_seed - 1)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nsys))).astype(np.int64)
    out = []
    for i in range(nsys):
        if i % 2 == 0:
            xyz, q = uniform_cube(int(ns[i]), base_seed + i)
        else:
            xyz, q = plummer(int(ns[i]), base_seed + i)
        out.append((xyz, q, (4, 6, 8)[i % 3]))
    return out


# The five workloads.  "tree" names the octree the configuration asks for.
CONFIGS = {
    0: dict(name="uniform4096_p4_d3_fp64", n=4096, kind="cube", seed=1000, qlo=0.5, qhi=1.5,
            p=4, tree="uniform", depth=3),
    1: dict(name="plummer1M_p8_adaptive64", n=1 << 20, kind="plummer", seed=1001,
            p=8, tree="adaptive", leaf_max=64),
    2: dict(name="uniform16M_p10_d7", n=1 << 24, kind="cube", seed=1002, qlo=-1.0, qhi=1.0,
            p=10, tree="uniform", depth=7),
    4: dict(name="hernquist4M_learned_p", n=1 << 22, kind="hernquist", seed=1005,
            p=10, tree="adaptive", leaf_max=64),
}


def make(cfg: dict, n: int | None = None, seed: int | None = None):
    """Draw the particles of a configuration (optionally with another n/seed)."""
    n = cfg["n"] if n is None else n
    seed = cfg["seed"] if seed is None else seed
    if cfg["kind"] == "cube":
        return uniform_cube(n, seed, cfg.get("qlo", 0.5), cfg.get("qhi", 1.5))
    if cfg["kind"] == "plummer":
        return plummer(n, seed)
    if cfg["kind"] == "hernquist":
        return hernquist(n, seed)
    raise ValueError(cfg["kind"])
