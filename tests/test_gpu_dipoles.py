"""Point dipoles (Appendix B.1) on the GPU: the uniform FMM with charges and
dipoles against the FP64 oracle with the same dipoles (1e-12 in FP64, 1e-6
with FP32 and BF16x3 M2L), over several orders and depths, and against the
direct sum (truncation level, falling with p)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
from helpers import MAXREL_FP64, MAXREL_MIXED, maxrel, rel  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(n, seed, scale=0.01):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rng.uniform(-1, 1, n), scale * rng.normal(size=(n, 3))


def _gpu(xyz, q, dip, p, depth, precision="fp64"):
    import torch
    from paper_1811_06332_amd import ctfmm as F
    f = F.FMM(p, depth, precision)
    try:
        phi, grad = f.evaluate_dipoles(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(),
                                       torch.from_numpy(np.ascontiguousarray(dip)).cuda(), sync=True)
    finally:
        f.close()
    return phi.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("p,depth", [(0, 2), (1, 2), (4, 3), (7, 3), (10, 2), (6, 4)])
def test_dipoles_fp64_match_oracle(p, depth):
    xyz, q, dip = _case(3000, 60 + p)
    print(f"[case] dipoles p={p} depth={depth}", flush=True)
    pg, gg = _gpu(xyz, q, dip, p, depth)
    po, go = oracle.fmm_uniform_dipoles(xyz, q, dip, p, depth)
    eP, eF, mP, mF = rel(pg, po), rel(gg, go), maxrel(pg, po), maxrel(gg, go)
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e} worst {mP:.3e} {mF:.3e}", flush=True)
    assert eP <= 1e-12 and eF <= 1e-12
    assert mP <= MAXREL_FP64 and mF <= MAXREL_FP64


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_dipoles_mixed_precision(precision):
    xyz, q, dip = _case(4000, 70)
    print(f"[case] dipoles {precision}", flush=True)
    pg, gg = _gpu(xyz, q, dip, 8, 3, precision)
    po, go = oracle.fmm_uniform_dipoles(xyz, q, dip, 8, 3)
    eP, eF = rel(pg, po), rel(gg, go)
    print(f"[case] e_phi={eP:.3e} e_grad={eF:.3e}", flush=True)
    assert eP <= 1e-6 and eF <= 1e-6
    assert maxrel(gg, go) <= MAXREL_MIXED


def test_dipoles_only_decay_to_direct_sum():
    """Pure dipoles (no charges): the error against the direct sum falls with
    p; the dipoles' far field is carried by the multipoles alone."""
    xyz, _, dip = _case(2000, 71, 1.0)
    q = np.zeros(len(xyz))
    pd, gd = oracle.direct_dipoles(xyz, q, dip)
    errs = []
    for p in (2, 4, 6, 8):
        pg, gg = _gpu(xyz, q, dip, p, 3)
        errs.append(rel(gg, gd))
    print(f"[case] dipole-only e_grad vs direct {errs}", flush=True)
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-3


def test_dipoles_need_the_uniform_tree():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q, dip = _case(100, 72)
    f = F.FMM(4, 0, "fp64", root_side=None, tree="adaptive", leaf_max=16)
    try:
        with pytest.raises(F.CtfmmError) as e:
            f.evaluate_dipoles(torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda(), torch.from_numpy(dip).cuda())
        assert e.value.status == F.CTFMM_EUNSUPPORTED
    finally:
        f.close()
