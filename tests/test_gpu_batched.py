"""Many independent systems in one batched call (adaptive trees, one forest
per expansion order, numeric passes replayed from a captured HIP graph).

Every system of the batch must match the adaptive oracle run on that system
alone: FP64 within 1e-12, list sizes exactly (summed over the batch).  The
graph replays must reproduce the eager result bit for bit, with eager work
and synchronisation between the replays.  FP32 M2L stays within a relative
force error of 1e-6 of FP64."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import rel  # noqa: E402
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def small_batch(sizes, seed0):
    """Systems in the recipe of the uneven batch (even i: cube, odd i:
    Plummer; p = (4, 6, 8)[i % 3]) with the given sizes."""
    systems = []
    for i, n in enumerate(sizes):
        xyz, q = W.uniform_cube(n, seed0 + i) if i % 2 == 0 else W.plummer(n, seed0 + i)
        systems.append((xyz, q, (4, 6, 8)[i % 3]))
    return systems


def concat(systems):
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s[1]) for s in systems])
    xyz = np.ascontiguousarray(np.concatenate([s[0] for s in systems]))
    q = np.ascontiguousarray(np.concatenate([s[1] for s in systems]))
    orders = np.array([s[2] for s in systems], dtype=np.int32)
    return offs, orders, xyz, q


def run_batch(systems, precision="fp64", leaf_max=64, repeats=1, between=None):
    import torch
    from paper_1811_06332_amd import ctfmm as F
    offs, orders, xyz, q = concat(systems)
    X = torch.from_numpy(xyz).cuda()
    Q = torch.from_numpy(q).cuda()
    f = F.FMM(int(orders.max()), 0, precision, root_side=None, tree="adaptive", leaf_max=leaf_max)
    outs = []
    try:
        for r in range(repeats):
            phi, grad = f.evaluate_batched(offs, orders, X, Q, sync=True)
            outs.append((phi.cpu().numpy(), grad.cpu().numpy()))
            if between is not None:
                between(r)
        st, ts = f.stats(), f.tree_stats()
    finally:
        f.close()
    return offs, outs, st, ts


def test_batched_fp64_matches_oracle_per_system():
    systems = small_batch([900, 2500, 400, 1800, 3000, 700, 60], 300)
    print(f"[case] batched fp64 sizes={[len(s[1]) for s in systems]}", flush=True)
    offs, outs, st, ts = run_batch(systems, leaf_max=24)
    phi, grad = outs[0]
    tot = dict(nodes=0, V=0, U=0, W=0, X=0)
    for i, (xyz, q, p) in enumerate(systems):
        po, go, info = oracle.fmm_adaptive(xyz, q, p, 24, stats=True)
        a, b = offs[i], offs[i + 1]
        eP, eF = rel(phi[a:b], po), rel(grad[a:b], go)
        print(f"[case] system {i} n={len(q)} p={p} e_phi={eP:.3e} e_grad={eF:.3e}", flush=True)
        assert eP <= TOL and eF <= TOL, (i, eP, eF)
        for k in tot:
            tot[k] += info[k]
    got = dict(nodes=ts["nodes"], V=ts["v_pairs"], U=ts["u_pairs"], W=ts["w_pairs"], X=ts["x_pairs"])
    assert got == tot, (got, tot)


def test_batched_graph_replays_match_eager():
    """Call 1 runs eagerly, call 2 captures the graph, calls 2-5 launch it;
    torch work and a synchronisation run between the calls."""
    import torch
    systems = small_batch([1500, 800, 2200, 1200], 400)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")

    def between(r):
        scratch.add_(float(r + 1)).mul_(0.5)
        torch.cuda.synchronize()

    print("[case] batched graph replays", flush=True)
    offs, outs, st, _ = run_batch(systems, leaf_max=32, repeats=5, between=between)
    assert st["graph_launches"] == 4, st["graph_launches"]
    for r in range(1, 5):
        assert np.array_equal(outs[r][0], outs[0][0]) and np.array_equal(outs[r][1], outs[0][1]), r


def test_batched_signature_change_recaptures():
    """A different batch after a captured one runs eagerly and is still right."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    a = small_batch([1000, 1400, 600], 500)
    b = small_batch([700, 2000], 600)
    f = F.FMM(8, 0, "fp64", root_side=None, tree="adaptive", leaf_max=32)
    try:
        for systems in (a, a, a, b):
            offs, orders, xyz, q = concat(systems)
            print(f"[case] batched reuse sizes={[len(s[1]) for s in systems]}", flush=True)
            phi, grad = f.evaluate_batched(offs, orders, torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(),
                                           sync=True)
        phi, grad = phi.cpu().numpy(), grad.cpu().numpy()
        for i, (xyz, q, p) in enumerate(b):
            po, go = oracle.fmm_adaptive(xyz, q, p, 32)
            assert rel(phi[offs[i]:offs[i + 1]], po) <= TOL and rel(grad[offs[i]:offs[i + 1]], go) <= TOL
        assert f.stats()["graph_launches"] == 2
    finally:
        f.close()


def test_batched_fp32_force_error():
    systems = small_batch([20000, 35000, 12000, 50000, 8000, 26000], 700)
    print("[case] batched fp32 vs fp64", flush=True)
    _, o64, _, _ = run_batch(systems, "fp64")
    _, o32, _, _ = run_batch(systems, "fp32")
    eF, eP = rel(o32[0][1], o64[0][1]), rel(o32[0][0], o64[0][0])
    print(f"[case] e_F={eF:.3e} e_phi={eP:.3e}", flush=True)
    assert eF <= 1e-6 and eP <= 1e-6


def test_config3_fullsize_fp32_sampled_systems():
    """The uneven batch at full size (256 systems, N log-uniform in
    [1e4, 5e5], p in {4, 6, 8}) in FP32, as the benchmark runs it; the three
    smallest systems against the FP64 oracle (relative force error 1e-6)."""
    systems = W.batched_systems()
    sizes = np.array([len(s[1]) for s in systems])
    print(f"[case] config3 fullsize nsys={len(systems)} total={sizes.sum()}", flush=True)
    offs, outs, st, ts = run_batch(systems, "fp32")
    phi, grad = outs[0]
    for i in np.argsort(sizes)[:3]:
        xyz, q, p = systems[i]
        po, go = oracle.fmm_adaptive(xyz, q, p, 64, nthreads=len(os.sched_getaffinity(0)))
        a, b = offs[i], offs[i + 1]
        eP, eF = rel(phi[a:b], po), rel(grad[a:b], go)
        print(f"[case] system {i} n={len(q)} p={p} e_phi={eP:.3e} e_grad={eF:.3e}", flush=True)
        assert eF <= 1e-6 and eP <= 1e-6
