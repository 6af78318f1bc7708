"""FP64 GPU path against the FP64 oracle: potential, gradient and the M and L
expansions of every level, element by element, relative error <= 1e-12."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import oracle_columns, rel  # noqa: E402
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def gpu_fmm(xyz, q, p, depth, lo=(0.0, 0.0, 0.0), side=1.0, precision="fp64", levels=()):
    import torch
    from paper_1811_06332_amd import ctfmm as F
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.ascontiguousarray(xyz)).to(dev)
    Q = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    f = F.FMM(p, depth, precision, lo, side)
    try:
        phi, grad = f.evaluate(X, Q, sync=True)
        exps = {l: (f.expansions(l, "M"), f.expansions(l, "L")) for l in levels}
    finally:
        f.close()
    return phi.cpu().numpy(), grad.cpu().numpy(), exps


def check(xyz, q, p, depth, lo=(0.0, 0.0, 0.0), side=1.0, expansions=True):
    print(f"[case] n={len(q)} p={p} depth={depth} lo={lo} side={side}", flush=True)
    levels = tuple(range(2, depth + 1)) if expansions else ()
    pg, gg, ex = gpu_fmm(xyz, q, p, depth, lo, side, levels=levels)
    if expansions and depth >= 2:
        po, go, Mo, Lo = oracle.fmm_uniform(xyz, q, p, depth, lo, side, dump=True)
        cols = oracle_columns(oracle, p)
        for l in levels:
            Mg, Lg = ex[l]
            assert rel(Mg, Mo[l][:, cols]) <= TOL, ("M", l, rel(Mg, Mo[l][:, cols]))
            assert rel(Lg, Lo[l][:, cols]) <= TOL, ("L", l, rel(Lg, Lo[l][:, cols]))
    else:
        po, go = oracle.fmm_uniform(xyz, q, p, depth, lo, side)
    eP, eF = rel(pg, po), rel(gg, go)
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e}", flush=True)
    assert eP <= TOL and eF <= TOL, (eP, eF)
    return pg, gg


def test_config0_against_oracle_and_direct_sum():
    cfg = W.CONFIGS[0]
    xyz, q = W.make(cfg)
    pg, gg = check(xyz, q, cfg["p"], cfg["depth"])
    pd, gd = oracle.direct(xyz, q)
    # the approximation itself: truncation level at p = 4
    assert rel(pg, pd) < 5e-4 and rel(gg, gd) < 5e-3


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5, 6, 7, 8, 9, 10])
def test_orders(p):
    xyz, q = W.uniform_cube(1531, 300 + p, -1.0, 1.0)
    check(xyz, q, p, 3, expansions=(p in (1, 7, 10)))


@pytest.mark.parametrize("depth", [0, 1, 2, 4])
def test_depths(depth):
    n = {0: 200, 1: 500, 2: 2000, 4: 9000}[depth]
    xyz, q = W.uniform_cube(n, 400 + depth)
    check(xyz, q, 5, depth, expansions=(depth == 2))


def test_clustered_empty_leaves_and_crowded_leaf():
    rng = np.random.default_rng(7)
    a = rng.random((300, 3)) * 0.2            # > 64 particles in one depth-2 leaf
    b = 0.6 + rng.random((50, 3)) * 0.05      # a second cluster; most leaves empty
    xyz = np.vstack([a, b])
    q = rng.uniform(-1, 1, len(xyz))
    check(xyz, q, 6, 2)
    check(xyz, q, 4, 3)


def test_boundaries_coincident_and_outside():
    rng = np.random.default_rng(8)
    xyz = rng.random((400, 3))
    xyz[:20] = np.floor(xyz[:20] * 8) / 8       # exactly on cell faces
    xyz[20:25] = xyz[30:35]                     # coincident pairs
    xyz[40] = [1.0, 1.0, 1.0]                   # upper corner (clamped into the last leaf)
    xyz[41] = [-0.01, 0.5, 0.5]                 # slightly outside (clamped)
    q = rng.uniform(0.5, 1.5, 400)
    check(xyz, q, 5, 3)


def test_shifted_root_box():
    rng = np.random.default_rng(9)
    lo, side = (-1.0, -2.0, 0.5), 3.0
    xyz = np.array(lo) + rng.random((1200, 3)) * side
    q = rng.uniform(-1, 1, 1200)
    check(xyz, q, 7, 3, lo, side)


def test_tiny_inputs():
    for n in (1, 2, 3):
        xyz, q = W.uniform_cube(n, 10 + n)
        check(xyz, q, 4, 3, expansions=False)


def test_zero_particles_is_noop():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    f = F.FMM(4, 3)
    X = torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")
    Q = torch.zeros((0,), dtype=torch.float64, device="cuda:0")
    phi, grad = f.evaluate(X, Q, sync=True)
    assert phi.numel() == 0 and grad.numel() == 0
    f.close()


def test_context_reuse_and_growth():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    f = F.FMM(6, 3)
    try:
        for n, seed in ((500, 1), (3000, 2), (800, 3)):
            xyz, q = W.uniform_cube(n, seed)
            phi, grad = f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
            po, go = oracle.fmm_uniform(xyz, q, 6, 3)
            assert rel(phi.cpu().numpy(), po) <= TOL and rel(grad.cpu().numpy(), go) <= TOL
    finally:
        f.close()


def test_nonfinite_coordinate_is_reported():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.uniform_cube(100, 5)
    xyz[3, 1] = np.nan
    f = F.FMM(4, 3)
    try:
        f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda())
        with pytest.raises(F.CtfmmError) as e:
            F.ctfmm_sync(f.ctx)
        assert e.value.status == F.CTFMM_EINVAL
    finally:
        f.close()
