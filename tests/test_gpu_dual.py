"""Dual-tree traversal with the theta MAC (Appendix C) on the GPU against the
FP64 oracle.

The traversal is integer work: the centres of the geometric mode, and the
accepted (M2L) and direct leaf pairs of every mode, must equal the oracle's
entry by entry (nodes matched by level and Morton prefix).  Potential and
gradient in FP64 must match the oracle within 1e-10 (largest relative
difference per particle) and 1e-12 (normwise).  Mutual M2L conserves the
total force to rounding."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import MAXREL_FP64, maxrel, node_codes, rel  # noqa: E402
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def gpu_dual(xyz, q, p, leaf_max, theta, centre, copy=False, f32=False):
    import torch
    from paper_1811_06332_amd import ctfmm as F
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.ascontiguousarray(xyz)).to(dev)
    Q = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    f = F.FMM(p, 0, "fp64", root_side=None, tree="dual", leaf_max=leaf_max, theta=theta, centre=centre)
    try:
        if f32:
            phi, grad = f.evaluate_f32(X.float(), Q.float(), sync=True)
            if centre == "ap":
                phi = None
        else:
            phi, grad = f.evaluate(X, Q, sync=True)
        out = {"phi": None if phi is None else phi.cpu().double().numpy(), "grad": grad.cpu().double().numpy(),
               "stats": f.tree_stats()}
        if copy:
            out["tree"] = f.tree_copy()
            out["dual"] = f.dual_copy()
    finally:
        f.close()
    return out


def check_parity(g, xyz, q, p, leaf_max, theta, centre):
    po, go, info = oracle.fmm_dual(xyz, q, p, leaf_max, theta, centre, stats=True)
    st = g["stats"]
    assert st["v_pairs"] == 2 * info["m2l_pairs"]
    assert st["nodes"] == info["nodes"] and st["leaves"] == info["leaves"]
    assert maxrel(g["grad"], go) < MAXREL_FP64 and rel(g["grad"], go) < TOL
    if centre != "ap":
        assert maxrel(g["phi"], po) < MAXREL_FP64 and rel(g["phi"], po) < TOL
    else:
        assert g["phi"] is None
    return po, go


def two_density(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n // 2, 3))
    b = 0.8 + 0.01 * rng.random((n - n // 2, 3))
    return np.ascontiguousarray(np.concatenate([a, b])), rng.uniform(0.5, 1.5, n)


CASES = {
    "plummer3000_p4_leaf16_t05": (lambda: W.plummer(3000, 7), 4, 16, 0.5),
    "plummer3000_p8_leaf24_t06": (lambda: W.plummer(3000, 7), 8, 24, 0.6),
    "hernquist2500_p10_leaf32_t07": (lambda: W.hernquist(2500, 11), 10, 32, 0.7),
    "two_density4000_p6_leaf12_t05": (lambda: two_density(4000, 12), 6, 12, 0.5),
    "uniform2000_p7_leaf8_t08": (lambda: (np.random.default_rng(13).random((2000, 3)),
                                          np.random.default_rng(14).uniform(0.5, 1.5, 2000)), 7, 8, 0.8),
    "plummer1500_p0_leaf4_t05": (lambda: W.plummer(1500, 15), 0, 4, 0.5),
    "plummer1500_p1_leaf4_t04": (lambda: W.plummer(1500, 15), 1, 4, 0.4),
}


@pytest.mark.parametrize("centre", ["geometric", "mass", "ap"])
@pytest.mark.parametrize("case", list(CASES))
def test_dual_fp64_parity(case, centre):
    mk, p, leaf, theta = CASES[case]
    xyz, q = mk()
    g = gpu_dual(xyz, q, p, leaf, theta, centre)
    check_parity(g, xyz, q, p, leaf, theta, centre)


@pytest.mark.parametrize("centre", ["geometric", "mass", "ap"])
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_dual_traversal_exact(centre, theta):
    """Centres, radii and both pair lists against the oracle's traversal."""
    xyz, q = W.plummer(2500, 21)
    leaf = 10
    g = gpu_dual(xyz, q, 3, leaf, theta, centre, copy=True)
    t, d = g["tree"], g["dual"]
    ot = oracle.adaptive_tree(xyz, leaf)
    od = oracle.dual_pairs(xyz, q, leaf, theta, centre)
    cg = node_codes(t["level"], t["key"])
    co = node_codes(ot["level"], ot["key"])
    assert len(cg) == len(co) and set(cg.tolist()) == set(co.tolist())
    pos = {int(c): i for i, c in enumerate(cg)}
    perm = np.array([pos[int(c)] for c in co])  # oracle node -> GPU node
    zg = d["zr"][perm]
    if centre == "geometric":
        assert np.array_equal(zg, od["zr"])
    else:
        assert np.allclose(zg, od["zr"], rtol=1e-14, atol=1e-15 * np.abs(od["zr"]).max())
    # directed M2L entries (target, source) as node codes
    a, b = od["m2l"][:, 0], od["m2l"][:, 1]
    ref = np.concatenate([np.stack([co[b], co[a]], 1), np.stack([co[a], co[b]], 1)])
    got = np.stack([cg[d["m2l"][:, 0]], cg[d["m2l"][:, 1]]], 1)
    assert len(got) == len(ref) == g["stats"]["v_pairs"]
    assert np.array_equal(np.unique(got, axis=0), np.unique(ref, axis=0))
    assert len(np.unique(got, axis=0)) == len(got)
    refp = np.stack([co[od["p2p"][:, 0]], co[od["p2p"][:, 1]]], 1)
    gotp = np.stack([cg[d["p2p"][:, 0]], cg[d["p2p"][:, 1]]], 1)
    assert len(gotp) == len(refp)
    assert np.array_equal(np.unique(gotp, axis=0), np.unique(refp, axis=0))
    # the GPU lists come sorted by (target, source)
    assert np.all(np.diff(d["m2l"][:, 0].astype(np.int64) * len(cg) + d["m2l"][:, 1]) > 0)


def test_dual_theta0_is_direct():
    xyz, q = W.plummer(3000, 22)
    pd, gd = oracle.direct(xyz, q)
    for centre in ("geometric", "mass"):
        g = gpu_dual(xyz, q, 6, 16, 0.0, centre)
        assert g["stats"]["v_pairs"] == 0
        assert maxrel(g["phi"], pd) < 1e-12 and maxrel(g["grad"], gd) < 1e-12


@pytest.mark.parametrize("centre", ["geometric", "mass", "ap"])
def test_dual_momentum_and_accuracy(centre):
    """Newton's third law to rounding; the error against the direct sum falls
    with p."""
    xyz, q = W.plummer(20000, 23)
    tg = np.arange(0, 20000, 97)
    pd, gd = oracle.direct(xyz, q, targets=tg)
    errs = []
    for p in (2, 5, 8):
        g = gpu_dual(xyz, q, p, 32, 0.5, centre)
        f = q[:, None] * g["grad"]
        assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(f).sum(), (centre, p)
        errs.append(rel(g["grad"][tg], gd))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-4, errs


def test_dual_deterministic():
    xyz, q = W.plummer(30000, 24)
    a = gpu_dual(xyz, q, 6, 32, 0.6, "mass")
    b = gpu_dual(xyz, q, 6, 32, 0.6, "mass")
    assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["grad"], b["grad"])


def test_dual_edge_cases():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    # one particle, two particles, coincident particles (deepest level)
    for xyz, q in ((np.array([[0.1, 0.2, 0.3]]), np.array([2.0])),
                   (np.array([[0.1, 0.2, 0.3], [0.4, -0.2, 0.9]]), np.array([1.0, 3.0]))):
        g = gpu_dual(xyz, q, 5, 1, 0.5, "geometric")
        pd, gd = oracle.direct(xyz, q)
        assert np.allclose(g["phi"], pd, rtol=1e-14, atol=0) and np.allclose(g["grad"], gd, rtol=1e-14, atol=0)
    rng = np.random.default_rng(25)
    xyz = rng.random((600, 3))
    xyz[:200] = (0.3, 0.6, 0.2)
    q = rng.uniform(0.5, 1.5, 600)
    for centre in ("geometric", "ap"):
        g = gpu_dual(xyz, q, 5, 8, 0.6, centre)
        check_parity(g, xyz, q, 5, 8, 0.6, centre)
    # AP: phi must be NULL, charges positive
    dev = torch.device("cuda:0")
    f = F.FMM(4, 0, "fp64", root_side=None, tree="dual", leaf_max=8, theta=0.5, centre="ap")
    try:
        X = torch.from_numpy(rng.random((100, 3))).to(dev)
        Q = torch.ones(100, dtype=torch.float64, device=dev)
        with pytest.raises(F.CtfmmError) as e:
            F.ctfmm_evaluate(f.ctx, X, Q, torch.empty(100, dtype=torch.float64, device=dev),
                             torch.empty((100, 3), dtype=torch.float64, device=dev))
        assert e.value.status == F.CTFMM_EINVAL
        Q[7] = -1.0
        with pytest.raises(F.CtfmmError) as e:
            f.evaluate(X, Q, sync=True)
        assert e.value.status == F.CTFMM_EINVAL
        Q[7] = 1.0
        _, g = f.evaluate(X, Q, sync=True)  # the context still works
        assert torch.isfinite(g).all()
        with pytest.raises(F.CtfmmError):
            f.set_mac(1.5, "mass")
    finally:
        f.close()


def test_dual_f32_entry_point():
    xyz, q = W.plummer(4000, 26)
    g = gpu_dual(xyz, q, 5, 16, 0.5, "mass", f32=True)
    x32, q32 = xyz.astype(np.float32).astype(np.float64), q.astype(np.float32).astype(np.float64)
    po, go = oracle.fmm_dual(x32, q32, 5, 16, 0.5, "mass")
    assert rel(g["grad"], go) < 1e-6 and rel(g["phi"], po) < 1e-6


def test_dual_fullsize_properties():
    """The headline workload (Plummer N = 2^20, p = 8, leaves <= 64) through
    the dual tree at theta 0.5, as bench.py times it, checked by properties
    that hold at any size: every directed M2L entry has its reverse; on the
    exported centres and radii every accepted pair passes the criterion and
    every direct pair of distinct leaves fails it, and no pair is both; the
    total force vanishes to rounding; and on sampled particles the error
    against the direct sum stays at the truncation level."""
    cfg = W.CONFIGS[1]
    xyz, q = W.make(cfg)
    n = len(q)
    print(f"[case] dual fullsize n={n}", flush=True)
    g = gpu_dual(xyz, q, cfg["p"], cfg["leaf_max"], 0.5, "geometric", copy=True)
    d, t = g["dual"], g["tree"]
    zr, m, pp = d["zr"], d["m2l"].astype(np.int64), d["p2p"].astype(np.int64)
    nn = len(zr)
    key, rkey = m[:, 0] * nn + m[:, 1], m[:, 1] * nn + m[:, 0]
    assert np.array_equal(np.sort(key), np.sort(rkey))

    def mac(a, b):
        dx, dy, dz = (zr[b, k] - zr[a, k] for k in range(3))
        return 0.5 * np.sqrt((dx * dx + dy * dy) + dz * dz) > zr[a, 3] + zr[b, 3]

    assert np.all(mac(m[:, 0], m[:, 1]))
    other = pp[pp[:, 0] != pp[:, 1]]
    assert not np.any(mac(other[:, 0], other[:, 1]))
    assert np.all(t["leaf"][pp[:, 0]] == 1) and np.all(t["leaf"][pp[:, 1]] == 1)
    assert len(np.intersect1d(key, other[:, 0] * nn + other[:, 1])) == 0
    f = q[:, None] * g["grad"]
    mom = np.abs(f.sum(0)).max() / np.abs(f).sum()
    rng = np.random.default_rng(79)
    idx = np.unique(np.concatenate([rng.choice(n, 62, replace=False), [0, n - 1]]))
    pd, gd = oracle.direct(xyz, q, targets=idx, nthreads=len(os.sched_getaffinity(0)))
    eP, eF = rel(g["phi"][idx], pd), rel(g["grad"][idx], gd)
    print(f"[case] entries {len(m)} direct {len(pp)} momentum {mom:.2e} vs direct: e_phi={eP:.2e} "
          f"e_grad={eF:.2e}", flush=True)
    assert mom < 1e-12
    assert eP < 1e-4 and eF < 1e-3
