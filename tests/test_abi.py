"""The C-ABI library loads and exports every symbol include/ctfmm.h declares;
argument checks that return before any device call (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_1811_06332_amd import ctfmm as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ctfmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ctfmm_[a-z0-9_]+)\s*\(", src)) - {"ctfmm_alloc_fn", "ctfmm_free_fn"})


def test_library_exports_every_declared_symbol():
    lib = F.load()
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(F.EXPORTED)


def test_version_and_defaults():
    assert F.ctfmm_version() == 4
    prm = F.ctfmm_default_params()
    assert (prm.order_p, prm.depth, prm.ws, prm.precision, prm.root_side) == (4, 3, 1, 0, 1.0)
    assert (prm.tree, prm.leaf_max) == (F.CTFMM_TREE_UNIFORM, 64)


@pytest.mark.parametrize("field,value,status", [
    ("order_p", 11, F.CTFMM_EUNSUPPORTED), ("order_p", -1, F.CTFMM_EINVAL), ("depth", 10, F.CTFMM_EINVAL),
    ("ws", 2, F.CTFMM_EINVAL), ("root_side", 0.0, F.CTFMM_EINVAL), ("root_side", float("nan"), F.CTFMM_EINVAL),
    ("tree", 7, F.CTFMM_EUNSUPPORTED),
    # adaptive tree: leaf_max >= 1; root_side <= 0 is the automatic cube but must be finite
    ("adaptive:leaf_max", 0, F.CTFMM_EINVAL), ("adaptive:root_side", float("inf"), F.CTFMM_EINVAL),
    ("adaptive:order_p", 11, F.CTFMM_EUNSUPPORTED),
    # dual tree: FP64 only, adaptive-tree parameter rules
    ("dual:precision", 1, F.CTFMM_EUNSUPPORTED), ("dual:precision", 2, F.CTFMM_EUNSUPPORTED),
    ("dual:leaf_max", 0, F.CTFMM_EINVAL), ("dual:order_p", 11, F.CTFMM_EUNSUPPORTED),
])
def test_create_rejects_bad_params(field, value, status):
    lib = F.load()
    prm = F.ctfmm_default_params()
    if field.startswith("adaptive:") or field.startswith("dual:"):
        prm.tree = F.CTFMM_TREE_ADAPTIVE if field.startswith("adaptive:") else F.CTFMM_TREE_DUAL
        field = field.split(":", 1)[1]
    setattr(prm, field, value)
    h = C.c_void_p()
    assert lib.ctfmm_create(C.byref(prm), None, C.byref(h)) == status
    assert h.value is None
    assert F.ctfmm_last_error()


def test_null_arguments():
    lib = F.load()
    assert lib.ctfmm_create(None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_evaluate(None, 1, None, None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_evaluate_f32(None, 1, None, None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_evaluate_batched(None, 1, None, None, None, None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_evaluate_batched_f32(None, 1, None, None, None, None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_set_allocator(None, None, None, None) == F.CTFMM_EINVAL
    assert lib.ctfmm_sync(None) == F.CTFMM_EINVAL
    assert lib.ctfmm_default_params(None) == F.CTFMM_EINVAL
    assert lib.ctfmm_set_mac(None, 0.5, 0) == F.CTFMM_EINVAL
    assert lib.ctfmm_copy_dual(None, None) == F.CTFMM_EINVAL
    lib.ctfmm_destroy(None)


def test_splitmix64_reference_values():
    """The order-map hash of the tests is SplitMix64: its first outputs from
    state 0 are the published ones."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import numpy as np
    from helpers import splitmix64
    golden = 0x9E3779B97F4A7C15
    outs = [int(splitmix64(np.uint64((k * golden) & 0xFFFFFFFFFFFFFFFF))) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
