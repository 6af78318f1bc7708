"""The C-ABI boundary on the GPU: the FP32 entry points against the FP64
ones on the same (FP32-representable) inputs, and the workspace allocator
(torch's caching allocator behind the binding, a failing allocator giving
ENOMEM instead of a crash)."""
import ctypes as C
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from paper_1811_06332_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tree", ["uniform", "adaptive"])
def test_f32_entry_is_the_f64_path_rounded(tree):
    """ctfmm_evaluate_f32 widens its inputs, runs the FP64-interface path and
    rounds the outputs: bit-identical to rounding ctfmm_evaluate's outputs on
    the widened inputs."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.plummer(5000, 41) if tree == "adaptive" else W.uniform_cube(5000, 42)
    x32 = torch.from_numpy(xyz.astype(np.float32)).cuda()
    q32 = torch.from_numpy(q.astype(np.float32)).cuda()
    kw = dict(root_side=None, tree="adaptive", leaf_max=32) if tree == "adaptive" else {}
    f = F.FMM(6, 3, "fp32", **kw)
    try:
        print(f"[case] f32 entry {tree}", flush=True)
        p32, g32 = f.evaluate_f32(x32, q32, sync=True)
        p64, g64 = f.evaluate(x32.double(), q32.double(), sync=True)
    finally:
        f.close()
    assert torch.equal(p32, p64.float()) and torch.equal(g32, g64.float())


def test_batched_f32_entry_is_the_f64_path_rounded():
    import torch
    from paper_1811_06332_amd import ctfmm as F
    systems = [W.plummer(3000, 43), W.uniform_cube(2000, 44), W.plummer(4000, 45)]
    orders = [4, 6, 8]
    xyz = np.concatenate([s[0] for s in systems]).astype(np.float32)
    q = np.concatenate([s[1] for s in systems]).astype(np.float32)
    offs = np.cumsum([0] + [len(s[1]) for s in systems])
    x32, q32 = torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda()
    f = F.FMM(8, 0, "fp32", root_side=None, tree="adaptive", leaf_max=64)
    try:
        print("[case] batched f32 entry", flush=True)
        p32, g32 = f.evaluate_batched_f32(offs, orders, x32, q32, sync=True)
        p64, g64 = f.evaluate_batched(offs, orders, x32.double(), q32.double(), sync=True)
    finally:
        f.close()
    assert torch.equal(p32, p64.float()) and torch.equal(g32, g64.float())


def test_workspace_comes_from_torch():
    """The binding routes the library's workspace to torch's caching
    allocator: it shows in torch's accounting while the context lives and
    is returned when it is destroyed."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    xyz, q = W.plummer(20000, 46)
    X, Q = torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    f = F.FMM(8, 0, "fp32", root_side=None, tree="adaptive", leaf_max=64)
    try:
        phi, grad = f.evaluate(X, Q, sync=True)
        held = torch.cuda.memory_allocated() - base
    finally:
        f.close()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated() - base
    print(f"[case] torch-held workspace {held / 2**20:.1f} MiB, after destroy {after / 2**20:.1f} MiB", flush=True)
    # the operators alone are several MiB; phi and grad (0.6 MiB) stay allocated
    assert held > 4 * 2**20
    assert after <= phi.numel() * 8 + grad.numel() * 8 + 2**20


def test_failing_allocator_gives_enomem():
    """An allocator that returns NULL: rebuilding the tables through it fails
    with ENOMEM; one that fails after the tables fails the evaluation with
    ENOMEM; the context stays usable after hipMalloc is restored."""
    import torch
    from paper_1811_06332_amd import ctfmm as F
    lib = F.load()
    calls = {"n": 0, "limit": 0}
    live = {}

    def _alloc(nbytes, user, stream):
        calls["n"] += 1
        if calls["n"] > calls["limit"]:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(ptr, user, stream):
        live.pop(int(ptr), None)

    af, ff = F.ALLOC_FN(_alloc), F.FREE_FN(_free)
    xyz, q = W.plummer(3000, 47)
    X, Q = torch.from_numpy(xyz).cuda(), torch.from_numpy(q).cuda()
    f = F.FMM(6, 0, "fp64", root_side=None, tree="adaptive", leaf_max=32, torch_alloc=False)
    try:
        print("[case] allocator returning NULL", flush=True)
        st = lib.ctfmm_set_allocator(C.c_void_p(f.ctx), C.cast(af, C.c_void_p), C.cast(ff, C.c_void_p), None)
        assert st == F.CTFMM_ENOMEM and F.ctfmm_last_error(f.ctx)
        # enough for the tables, then nothing
        calls["n"], calls["limit"] = 0, 64
        assert lib.ctfmm_set_allocator(C.c_void_p(f.ctx), C.cast(af, C.c_void_p), C.cast(ff, C.c_void_p),
                                       None) == F.CTFMM_OK
        tables = calls["n"]
        calls["limit"] = tables
        print(f"[case] allocator failing after the {tables} table allocations", flush=True)
        with pytest.raises(F.CtfmmError) as e:
            f.evaluate(X, Q, sync=True)
        assert e.value.status == F.CTFMM_ENOMEM
        # back to hipMalloc: the context works again
        F.ctfmm_set_allocator(f.ctx, None, None)
        phi, grad = f.evaluate(X, Q, sync=True)
        assert torch.isfinite(phi).all() and torch.isfinite(grad).all()
    finally:
        f.close()
    assert not live  # everything the library took was handed back
