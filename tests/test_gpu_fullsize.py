"""Full-size parity: the benchmark workload (N = 2^24 uniform, q ~ U(-1,1),
depth 7, p = 10) in the launch configuration bench.py times, checked on a
sample of particles the oracle computes one by one (its upward pass is
complete; its downward pass covers only the sampled leaves' paths)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import rel  # noqa: E402
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _sample(n, rng, k=48):
    """k particles: random ones plus the first and last in input order."""
    return np.unique(np.concatenate([rng.choice(n, k - 2, replace=False), [0, n - 1]]))


def test_fullsize_fp64_sampled():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    cfg = W.CONFIGS[2]
    xyz, q = W.make(cfg)
    n = len(q)
    print(f"[case] fullsize fp64 n={n} p={cfg['p']} depth={cfg['depth']}", flush=True)
    f = F.FMM(cfg["p"], cfg["depth"], "fp64")
    try:
        phi, grad = f.evaluate(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), sync=True)
        phi = phi.cpu().numpy(); grad = grad.cpu().numpy()
    finally:
        f.close()
    idx = _sample(n, np.random.default_rng(77))
    print(f"[case] oracle on {len(idx)} sampled particles", flush=True)
    po, go = oracle.fmm_uniform(xyz, q, cfg["p"], cfg["depth"], targets=idx,
                                nthreads=len(os.sched_getaffinity(0)))
    eP, eF = rel(phi[idx], po), rel(grad[idx], go)
    worst = float(np.max(np.linalg.norm(grad[idx] - go, axis=1) / np.linalg.norm(go, axis=1)))
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e} worst particle grad={worst:.3e}", flush=True)
    assert eP <= 1e-12 and eF <= 1e-12 and worst <= 1e-10
