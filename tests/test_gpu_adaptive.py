"""Adaptive octree on the GPU against the adaptive FP64 oracle.

The tree and its U/V/W/X lists are integer work: their sizes must equal the
oracle's exactly (node count, leaves, depth, and the number of entries of
every list), as must the automatic root cube.  Potential and gradient in
FP64 must match the oracle within 1e-12 (normwise relative).  The FP32 and
BF16x3 M2L modes must stay within a relative force error of 1e-6 of FP64."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import MAXREL_FP64, MAXREL_MIXED, compare_trees, maxrel, rel  # noqa: E402
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def gpu_adaptive(xyz, q, p, leaf_max, precision="fp64", lo=None, side=None):
    import torch
    from paper_1811_06332_amd import ctfmm as F
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.ascontiguousarray(xyz)).to(dev)
    Q = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    f = F.FMM(p, 0, precision, root_lo=lo if lo is not None else (0.0, 0.0, 0.0), root_side=side,
              tree="adaptive", leaf_max=leaf_max)
    try:
        phi, grad = f.evaluate(X, Q, sync=True)
        st = f.tree_stats()
    finally:
        f.close()
    return phi.cpu().numpy(), grad.cpu().numpy(), st


def two_density(n, seed):
    """A uniform cube with a dense clump in one corner (levels differ by many)."""
    rng = np.random.default_rng(seed)
    a = rng.random((n // 2, 3))
    b = 0.8 + 0.01 * rng.random((n - n // 2, 3))
    return np.ascontiguousarray(np.concatenate([a, b])), rng.uniform(0.5, 1.5, n)


def coincident(n, seed):
    """Half the particles on one point: the leaf holding them reaches the
    deepest level; pairs at zero distance contribute nothing."""
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3))
    xyz[: n // 2] = (0.3, 0.6, 0.2)
    return xyz, rng.uniform(0.5, 1.5, n)


CASES = {
    "plummer3000_p4_leaf24": (lambda: W.plummer(3000, 7), 4, 24),
    "plummer3000_p8_leaf24": (lambda: W.plummer(3000, 7), 8, 24),
    "hernquist2500_p10_leaf32": (lambda: W.hernquist(2500, 11), 10, 32),
    "two_density4000_p6_leaf16": (lambda: two_density(4000, 12), 6, 16),
    "cube2000_p3_leaf8": (lambda: W.uniform_cube(2000, 13), 3, 8),
    "plummer400_p2_leaf1": (lambda: W.plummer(400, 14), 2, 1),
    "plummer1500_p0_leaf4": (lambda: W.plummer(1500, 15), 0, 4),
    "plummer1500_p1_leaf4": (lambda: W.plummer(1500, 15), 1, 4),
    "coincident300_p3_leaf8": (lambda: coincident(300, 16), 3, 8),
    "root_leaf50_p4": (lambda: W.plummer(50, 17), 4, 64),
    "single_particle": (lambda: (np.array([[0.1, 0.2, 0.3]]), np.array([2.0])), 4, 64),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_adaptive_fp64_matches_oracle(name):
    make, p, leaf = CASES[name]
    xyz, q = make()
    print(f"[case] adaptive {name} n={len(q)} p={p} leaf_max={leaf}", flush=True)
    pg, gg, st = gpu_adaptive(xyz, q, p, leaf)
    po, go, info = oracle.fmm_adaptive(xyz, q, p, leaf, stats=True, nthreads=len(os.sched_getaffinity(0)))
    got = dict(nodes=st["nodes"], leaves=st["leaves"], max_level=st["max_level"], V=st["v_pairs"],
               U=st["u_pairs"], W=st["w_pairs"], X=st["x_pairs"])
    want = {k: info[k] for k in got}
    print(f"[case] gpu lists {got}", flush=True)
    assert got == want, (got, want)
    assert tuple(st["root_lo"]) == tuple(info["root_lo"]) and st["root_side"] == info["root_side"]
    eP, eF = rel(pg, po), rel(gg, go)
    mP, mF = maxrel(pg, po), maxrel(gg, go)
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e} worst particle {mP:.3e} {mF:.3e}", flush=True)
    assert eP <= TOL and eF <= TOL, (eP, eF)
    assert mP <= MAXREL_FP64 and mF <= MAXREL_FP64, (mP, mF)


@pytest.mark.parametrize("name", sorted(CASES))
def test_adaptive_tree_and_lists_exact(name):
    """Integer work, bit-exact: the GPU's tree (nodes, leaves, parents, the
    particles of every leaf) and every U, V, W and X list equal the
    oracle's entry by entry."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    make, p, leaf = CASES[name]
    xyz, q = make()
    f = F.FMM(p, 0, "fp64", root_side=None, tree="adaptive", leaf_max=leaf)
    try:
        print(f"[case] adaptive tree {name}", flush=True)
        f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
        tg = f.tree_copy()
    finally:
        f.close()
    sizes = compare_trees(tg, oracle.adaptive_tree(xyz, leaf))
    print(f"[case] equal entry by entry: {sizes}", flush=True)


def test_adaptive_explicit_root_box_clamps():
    """A given root cube smaller than the particle cloud: outside particles
    are clamped into the boundary cells, as in the oracle."""
    xyz, q = W.plummer(2000, 18)
    lo, side = (-2.0, -2.0, -2.0), 4.0
    print(f"[case] adaptive explicit box n={len(q)}", flush=True)
    pg, gg, st = gpu_adaptive(xyz, q, 5, 16, lo=lo, side=side)
    po, go, info = oracle.fmm_adaptive(xyz, q, 5, 16, lo=lo, side=side, stats=True)
    assert (st["nodes"], st["v_pairs"], st["u_pairs"], st["w_pairs"]) == (info["nodes"], info["V"], info["U"],
                                                                             info["W"])
    assert rel(pg, po) <= TOL and rel(gg, go) <= TOL


def test_adaptive_repeat_and_regrow():
    """The same context on a small, a larger, then the small input again:
    workspace growth keeps results identical to fresh evaluations."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    a = W.plummer(1500, 19)
    b = two_density(6000, 20)
    f = F.FMM(6, 0, "fp64", root_side=None, tree="adaptive", leaf_max=16)
    outs = []
    try:
        for xyz, q in (a, b, a):
            print(f"[case] adaptive reuse n={len(q)}", flush=True)
            phi, grad = f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
            outs.append((phi.cpu().numpy(), grad.cpu().numpy()))
    finally:
        f.close()
    assert np.array_equal(outs[0][0], outs[2][0]) and np.array_equal(outs[0][1], outs[2][1])
    po, go = oracle.fmm_adaptive(b[0], b[1], 6, 16)
    assert rel(outs[1][0], po) <= TOL and rel(outs[1][1], go) <= TOL


def test_adaptive_workspace_not_assumed_zero():
    """Workspace from the caching allocator holds whatever was freed before:
    poison the cache with NaN, then every context must still match the
    oracle (padding and partial sums are written, never assumed zero)."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    cases = [(W.plummer(1500, 19), 6, "fp64"), (two_density(6000, 20), 6, "fp64"), (two_density(6000, 20), 8, "fp32")]
    for (xyz, q), p, prec in cases:
        junk = [torch.full((1 << k,), float("nan"), dtype=torch.float64, device="cuda") for k in range(10, 25)]
        del junk
        print(f"[case] adaptive poisoned workspace n={len(q)} p={p} {prec}", flush=True)
        f = F.FMM(p, 0, prec, root_side=None, tree="adaptive", leaf_max=16)
        try:
            phi, grad = f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
        finally:
            f.close()
        phi, grad = phi.cpu().numpy(), grad.cpu().numpy()
        assert np.all(np.isfinite(phi)) and np.all(np.isfinite(grad))
        po, go = oracle.fmm_adaptive(xyz, q, p, 16)
        tol = TOL if prec == "fp64" else 1e-6
        assert rel(phi, po) <= tol and rel(grad, go) <= tol, (p, prec, rel(phi, po), rel(grad, go))


def test_adaptive_decays_to_direct_sum():
    """The approximation itself: error against the direct sum falls with p."""
    xyz, q = W.plummer(4000, 21)
    pd, gd = oracle.direct(xyz, q)
    errs = []
    for p in (2, 4, 6, 8):
        print(f"[case] adaptive decay p={p}", flush=True)
        pg, gg, _ = gpu_adaptive(xyz, q, p, 32)
        errs.append(rel(gg, gd))
    print(f"[case] e_F vs direct {errs}", flush=True)
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 5e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("p", [4, 8, 10])
def test_adaptive_mixed_precision_force_error(precision, p):
    xyz, q = W.plummer(30000, 22)
    print(f"[case] adaptive {precision} p={p}", flush=True)
    p64, g64, _ = gpu_adaptive(xyz, q, p, 64, "fp64")
    pm, gm, _ = gpu_adaptive(xyz, q, p, 64, precision)
    eF, eP = rel(gm, g64), rel(pm, p64)
    print(f"[case] e_F={eF:.3e} e_phi={eP:.3e}", flush=True)
    assert eF <= 1e-6 and eP <= 1e-6


def test_config1_fullsize_sampled():
    """Plummer N = 2^20, p = 8, leaf <= 64, in the launch configuration the
    benchmark times, in FP64, FP32 (the headline mode) and BF16x3, against the
    oracle on sampled particles (the oracle's upward pass is complete; its
    downward pass covers the sampled leaves' paths): FP64 within 1e-12
    normwise and 1e-10 per particle, the mixed modes within a relative force
    error of 1e-6; and the lists' sizes against the oracle's exactly."""
    cfg = W.CONFIGS[1]
    xyz, q = W.make(cfg)
    n = len(q)
    print(f"[case] config1 fullsize n={n}", flush=True)
    res = {prec: gpu_adaptive(xyz, q, cfg["p"], cfg["leaf_max"], precision=prec)
           for prec in ("fp64", "fp32", "bf16x3")}
    pg, gg, st = res["fp64"]
    rng = np.random.default_rng(78)
    idx = np.unique(np.concatenate([rng.choice(n, 46, replace=False), [0, n - 1]]))
    print(f"[case] oracle on {len(idx)} sampled particles", flush=True)
    po, go, info = oracle.fmm_adaptive(xyz, q, cfg["p"], cfg["leaf_max"], targets=idx, stats=True,
                                       nthreads=len(os.sched_getaffinity(0)))
    got = dict(nodes=st["nodes"], leaves=st["leaves"], max_level=st["max_level"], V=st["v_pairs"],
               U=st["u_pairs"], W=st["w_pairs"], X=st["x_pairs"])
    print(f"[case] gpu lists {got}", flush=True)
    assert got == {k: info[k] for k in got}
    eP, eF = rel(pg[idx], po), rel(gg[idx], go)
    print(f"[case] fp64 e_phi={eP:.3e} e_grad={eF:.3e} max {maxrel(gg[idx], go):.3e}", flush=True)
    assert eP <= TOL and eF <= TOL
    assert maxrel(pg[idx], po) <= MAXREL_FP64 and maxrel(gg[idx], go) <= MAXREL_FP64
    for prec in ("fp32", "bf16x3"):
        pm, gm, _ = res[prec]
        eP, eF = rel(pm[idx], po), rel(gm[idx], go)
        print(f"[case] {prec} e_phi={eP:.3e} e_grad={eF:.3e} max {maxrel(gm[idx], go):.3e}", flush=True)
        assert eP <= 1e-6 and eF <= 1e-6
        assert maxrel(gm[idx], go) <= MAXREL_MIXED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("targets", [32, 64, 128])
def test_adaptive_every_m2l_tile_shape(precision, targets):
    """Each M2L tile shape the tuner may pick gives the oracle's result."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.plummer(6000, 23)
    p = 8
    print(f"[case] adaptive tile {targets} {precision}", flush=True)
    f = F.FMM(p, 0, precision, root_side=None, tree="adaptive", leaf_max=32)
    try:
        try:
            f.set_m2l_tile(p, targets)
        except F.CtfmmError as e:
            assert e.status == F.CTFMM_EUNSUPPORTED
            pytest.skip(f"tile of {targets} targets does not fit this device's LDS in {precision}")
        phi, grad = f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
        assert f.m2l_tile(p) == targets
    finally:
        f.close()
    po, go = oracle.fmm_adaptive(xyz, q, p, 32)
    tol = TOL if precision == "fp64" else 1e-6
    eP, eF = rel(phi.cpu().numpy(), po), rel(grad.cpu().numpy(), go)
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e}", flush=True)
    assert eP <= tol and eF <= tol


def test_adaptive_tile_tuner_picks_a_shape():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.plummer(20000, 24)
    f = F.FMM(6, 0, "fp32", root_side=None, tree="adaptive", leaf_max=64)
    try:
        assert f.m2l_tile(6) == 0
        print("[case] adaptive tile tuner", flush=True)
        f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
        chosen = f.m2l_tile(6)
        print(f"[case] tuner chose {chosen}", flush=True)
        assert chosen in (32, 64, 128)
    finally:
        f.close()


def test_adaptive_timing_stats_deferred():
    """With timing on, a fixed-order evaluation returns before its timings are
    read; they are added at the next call or when the statistics are read.
    Three timed evaluations count three times the tree's M2L pairs, every
    phase time is positive, and a reset drops an evaluation still pending."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.plummer(3000, 7)
    print("[case] adaptive timing stats plummer3000 p=6 leaf_max=24", flush=True)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.ascontiguousarray(xyz)).to(dev)
    Q = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    f = F.FMM(6, 0, "fp32", root_side=None, tree="adaptive", leaf_max=24)
    try:
        f.evaluate(X, Q, sync=True)
        F.ctfmm_set_timing(f.ctx, True)
        f.evaluate(X, Q)  # pending when the statistics are reset
        F.ctfmm_reset_stats(f.ctx)
        for _ in range(3):
            f.evaluate(X, Q)
        st, ts = f.stats(), f.tree_stats()
        assert st["evaluations"] == 3
        assert st["m2l_pairs"] == 3 * ts["v_pairs"] and ts["v_pairs"] > 0
        for k in ("ms_total", "ms_tree", "ms_p2m", "ms_m2m", "ms_m2l", "ms_l2l", "ms_near"):
            assert st[k] > 0.0, (k, st[k])
        parts = sum(st[k] for k in ("ms_tree", "ms_p2m", "ms_m2m", "ms_convert", "ms_m2l", "ms_p2l", "ms_l2l",
                                    "ms_near"))
        assert abs(parts - st["ms_total"]) <= 1e-3 * st["ms_total"] + 0.05, (parts, st["ms_total"])
        # a second read adds nothing
        assert f.stats()["m2l_pairs"] == st["m2l_pairs"]
    finally:
        f.close()
