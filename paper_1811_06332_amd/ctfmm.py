"""Python binding of libctfmm (argument marshalling only).

Every function here forwards to the C ABI of ``include/ctfmm.h`` under the
same name; all arithmetic runs in the library's HIP kernels.  PyTorch
provides device memory and the stream.  There is no fallback: if the built
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libctfmm.so")

CTFMM_OK, CTFMM_EINVAL, CTFMM_ENOMEM, CTFMM_EDEVICE, CTFMM_EUNSUPPORTED = 0, 1, 2, 3, 4
CTFMM_TREE_UNIFORM, CTFMM_TREE_ADAPTIVE, CTFMM_TREE_DUAL = 0, 1, 2
TREES = {"uniform": CTFMM_TREE_UNIFORM, "adaptive": CTFMM_TREE_ADAPTIVE, "dual": CTFMM_TREE_DUAL}
CENTRES = {"geometric": 0, "mass": 1, "ap": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
CTFMM_P_MAX = 10
CTFMM_DEPTH_MAX = 9
CTFMM_ADAPTIVE_LEVEL_MAX = 21

EXPORTED = ["ctfmm_version", "ctfmm_default_params", "ctfmm_create", "ctfmm_set_allocator",
            "ctfmm_evaluate", "ctfmm_evaluate_dipoles", "ctfmm_evaluate_f32", "ctfmm_evaluate_batched",
            "ctfmm_evaluate_batched_f32",
            "ctfmm_copy_expansions", "ctfmm_copy_tree", "ctfmm_tree_stats", "ctfmm_set_m2l_tile",
            "ctfmm_get_m2l_tile", "ctfmm_set_order_table", "ctfmm_set_order_hash", "ctfmm_set_order_model",
            "ctfmm_set_mac", "ctfmm_copy_dual",
            "ctfmm_mlp_forward", "ctfmm_mlp_backward", "ctfmm_mlp_backward_noalloc", "ctfmm_mlp_train",
            "ctfmm_mlp_labels", "ctfmm_mlp_samples", "ctfmm_set_timing", "ctfmm_stats", "ctfmm_reset_stats",
            "ctfmm_sync", "ctfmm_last_error", "ctfmm_destroy"]


class CtfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ctfmm status {status}: {msg}")
        self.status = status


class ctfmm_params(C.Structure):
    _fields_ = [("order_p", C.c_int32), ("tree", C.c_int32), ("depth", C.c_int32), ("ws", C.c_int32),
                ("precision", C.c_int32), ("leaf_max", C.c_int32), ("root_lo", C.c_double * 3),
                ("root_side", C.c_double)]


class ctfmm_stats_t(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_tree", C.c_double), ("ms_p2m", C.c_double),
                ("ms_m2m", C.c_double), ("ms_m2l", C.c_double), ("ms_l2l", C.c_double),
                ("ms_near", C.c_double), ("ms_convert", C.c_double), ("ms_p2l", C.c_double),
                ("ms_numeric", C.c_double), ("evaluations", C.c_int64), ("m2l_launches", C.c_int64),
                ("m2l_pairs", C.c_int64), ("p2p_leaf_pairs", C.c_int64), ("graph_launches", C.c_int64),
                ("m2l_order_pairs", C.c_int64 * 11)]


class ctfmm_tree_copy_t(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("particles", C.c_int64), ("u_len", C.c_int64), ("v_len", C.c_int64),
                ("w_len", C.c_int64), ("x_len", C.c_int64), ("key", C.c_void_p), ("level", C.c_void_p),
                ("leaf", C.c_void_p), ("parent", C.c_void_p), ("pb", C.c_void_p), ("pe", C.c_void_p),
                ("perm", C.c_void_p), ("u_off", C.c_void_p), ("u_list", C.c_void_p), ("w_off", C.c_void_p),
                ("w_list", C.c_void_p), ("x_off", C.c_void_p), ("x_list", C.c_void_p), ("v_pairs", C.c_void_p)]


class ctfmm_dual_copy_t(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("m2l", C.c_int64), ("p2p", C.c_int64), ("zr", C.c_void_p),
                ("m2l_pairs", C.c_void_p), ("p2p_pairs", C.c_void_p)]


class ctfmm_tree_stats_t(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("leaves", C.c_int64), ("max_level", C.c_int64), ("v_pairs", C.c_int64),
                ("u_pairs", C.c_int64), ("w_pairs", C.c_int64), ("x_pairs", C.c_int64),
                ("root_lo", C.c_double * 3), ("root_side", C.c_double)]


_lib = None


def load():
    """Load libctfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1811_06332_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ctfmm_version.restype = C.c_int
        L.ctfmm_default_params.argtypes = [C.POINTER(ctfmm_params)]
        L.ctfmm_create.argtypes = [C.POINTER(ctfmm_params), vp, C.POINTER(vp)]
        L.ctfmm_set_allocator.argtypes = [vp, vp, vp, vp]
        L.ctfmm_evaluate.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ctfmm_evaluate_f32.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ctfmm_evaluate_dipoles.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ctfmm_evaluate_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.ctfmm_evaluate_batched_f32.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.ctfmm_copy_expansions.argtypes = [vp, i32, i32, vp, C.c_size_t]
        L.ctfmm_tree_stats.argtypes = [vp, C.POINTER(ctfmm_tree_stats_t)]
        L.ctfmm_copy_tree.argtypes = [vp, C.POINTER(ctfmm_tree_copy_t)]
        L.ctfmm_set_m2l_tile.argtypes = [vp, i32, i32]
        L.ctfmm_set_order_table.argtypes = [vp, vp]
        L.ctfmm_set_order_hash.argtypes = [vp, C.c_uint64, i32]
        L.ctfmm_set_order_model.argtypes = [vp, vp, vp, C.c_double, C.c_double]
        L.ctfmm_set_mac.argtypes = [vp, C.c_double, i32]
        L.ctfmm_copy_dual.argtypes = [vp, C.POINTER(ctfmm_dual_copy_t)]
        L.ctfmm_mlp_forward.argtypes = [vp, i64, vp, vp, i32, vp]
        L.ctfmm_mlp_backward.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ctfmm_mlp_backward_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ctfmm_mlp_train.argtypes = [vp, i64, vp, vp, vp, i32, i32, C.c_float, vp]
        L.ctfmm_mlp_labels.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ctfmm_mlp_samples.argtypes = [vp, i64, vp, vp, i64, C.c_uint64, vp, vp]
        L.ctfmm_get_m2l_tile.argtypes = [vp, i32, C.POINTER(C.c_int32)]
        L.ctfmm_set_timing.argtypes = [vp, i32]
        L.ctfmm_stats.argtypes = [vp, C.POINTER(ctfmm_stats_t)]
        L.ctfmm_reset_stats.argtypes = [vp]
        L.ctfmm_sync.argtypes = [vp]
        L.ctfmm_last_error.argtypes = [vp]
        L.ctfmm_last_error.restype = C.c_char_p
        L.ctfmm_destroy.argtypes = [vp]
        L.ctfmm_destroy.restype = None
        for name in EXPORTED:
            if name not in ("ctfmm_version", "ctfmm_last_error", "ctfmm_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != CTFMM_OK:
        msg = load().ctfmm_last_error(ctx)
        raise CtfmmError(status, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- C names

def ctfmm_version() -> int:
    return load().ctfmm_version()


def ctfmm_default_params() -> ctfmm_params:
    prm = ctfmm_params()
    _check(load().ctfmm_default_params(C.byref(prm)))
    return prm


def ctfmm_create(prm: ctfmm_params, stream: int | None = None):
    """Returns the context handle (an int).  `stream` is a hipStream_t as an
    int (torch.cuda.Stream.cuda_stream); None = torch's current stream."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    h = C.c_void_p()
    _check(load().ctfmm_create(C.byref(prm), C.c_void_p(stream), C.byref(h)))
    return h.value


def _io_check(n, dtype, xyz, q, phi, grad):
    for t, shape in ((xyz, (n, 3)), (q, (n,)), (phi, (n,)), (grad, (n, 3))):
        if t is None:
            continue
        if not t.is_cuda or str(t.dtype) != dtype or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"tensors must be contiguous cuda {dtype} of shapes [n,3], [n], [n], [n,3]")


def ctfmm_evaluate(ctx, xyz, q, phi=None, grad=None):
    """xyz: cuda float64 [n,3] contiguous; q: cuda float64 [n]; phi [n] and
    grad [n,3] cuda float64 outputs (either may be None)."""
    n = int(q.shape[0])
    _io_check(n, "torch.float64", xyz, q, phi, grad)
    _check(load().ctfmm_evaluate(C.c_void_p(ctx), n, _ptr(xyz), _ptr(q), _ptr(phi), _ptr(grad)), C.c_void_p(ctx))


def ctfmm_evaluate_dipoles(ctx, xyz, q, dip, phi=None, grad=None):
    """As ctfmm_evaluate with point dipoles dip: cuda float64 [n,3]."""
    n = int(q.shape[0])
    _io_check(n, "torch.float64", xyz, q, phi, grad)
    _io_check(n, "torch.float64", dip, None, None, None)
    _check(load().ctfmm_evaluate_dipoles(C.c_void_p(ctx), n, _ptr(xyz), _ptr(q), _ptr(dip), _ptr(phi), _ptr(grad)),
           C.c_void_p(ctx))


def ctfmm_evaluate_f32(ctx, xyz, q, phi=None, grad=None):
    """As ctfmm_evaluate with cuda float32 inputs and outputs."""
    n = int(q.shape[0])
    _io_check(n, "torch.float32", xyz, q, phi, grad)
    _check(load().ctfmm_evaluate_f32(C.c_void_p(ctx), n, _ptr(xyz), _ptr(q), _ptr(phi), _ptr(grad)),
           C.c_void_p(ctx))


def _batch_args(offsets, orders):
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ords = np.ascontiguousarray(orders, dtype=np.int32)
    if off.size != ords.size + 1:
        raise ValueError("offsets must have nsys+1 entries")
    return off, ords


def ctfmm_evaluate_batched(ctx, offsets, orders, xyz, q, phi=None, grad=None):
    """offsets: host int64 [nsys+1]; orders: host int32 [nsys]; xyz, q, phi,
    grad as in ctfmm_evaluate for the concatenated systems."""
    off, ords = _batch_args(offsets, orders)
    n = int(q.shape[0])
    _io_check(n, "torch.float64", xyz, q, phi, grad)
    _check(load().ctfmm_evaluate_batched(C.c_void_p(ctx), int(ords.size), C.c_void_p(off.ctypes.data),
                                         C.c_void_p(ords.ctypes.data), _ptr(xyz), _ptr(q), _ptr(phi), _ptr(grad)),
           C.c_void_p(ctx))


def ctfmm_evaluate_batched_f32(ctx, offsets, orders, xyz, q, phi=None, grad=None):
    """As ctfmm_evaluate_batched with cuda float32 inputs and outputs."""
    off, ords = _batch_args(offsets, orders)
    n = int(q.shape[0])
    _io_check(n, "torch.float32", xyz, q, phi, grad)
    _check(load().ctfmm_evaluate_batched_f32(C.c_void_p(ctx), int(ords.size), C.c_void_p(off.ctypes.data),
                                             C.c_void_p(ords.ctypes.data), _ptr(xyz), _ptr(q), _ptr(phi),
                                             _ptr(grad)), C.c_void_p(ctx))


# ---------------------------------------------------------------- allocator

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def torch_allocator():
    """(alloc, free) callbacks that take the library's device workspace from
    torch's caching allocator on the stream the library passes.  A failed
    allocation returns NULL (the library then reports ENOMEM).  Keep the
    returned objects alive as long as a context uses them."""
    import torch

    def _alloc(nbytes, user, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # out of memory: the library reports ENOMEM
            return None

    def _free(ptr, user, stream):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:  # interpreter shutdown: the memory goes with the process
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


def ctfmm_set_allocator(ctx, alloc=None, free=None) -> None:
    """alloc/free: ALLOC_FN/FREE_FN callbacks (None restores hipMalloc)."""
    _check(load().ctfmm_set_allocator(C.c_void_p(ctx), C.cast(alloc, C.c_void_p) if alloc else None,
                                      C.cast(free, C.c_void_p) if free else None, None), C.c_void_p(ctx))


def ctfmm_copy_expansions(ctx, level: int, which: int, out) -> None:
    """out: host numpy float64 array with 8**level * (p+1)**2 elements."""
    _check(load().ctfmm_copy_expansions(C.c_void_p(ctx), level, which, C.c_void_p(out.ctypes.data), out.size),
           C.c_void_p(ctx))


def ctfmm_copy_tree(ctx) -> dict:
    """The adaptive tree and lists of the last evaluate as numpy arrays
    (keys of include/ctfmm.h's ctfmm_tree_copy_t)."""
    import numpy as np
    io = ctfmm_tree_copy_t()
    _check(load().ctfmm_copy_tree(C.c_void_p(ctx), C.byref(io)), C.c_void_p(ctx))
    nn, n = int(io.nodes), int(io.particles)
    out = {"key": np.zeros(nn, np.uint64), "v_pairs": np.zeros((max(int(io.v_len), 1), 2), np.int32)}
    for name in ("level", "leaf", "parent", "pb", "pe"):
        out[name] = np.zeros(nn, np.int32)
    out["perm"] = np.zeros(n, np.int32)
    for L, ln in (("u", io.u_len), ("w", io.w_len), ("x", io.x_len)):
        out[L + "_off"] = np.zeros(nn + 1, np.int32)
        out[L + "_list"] = np.zeros(max(int(ln), 1), np.int32)
    for name, arr in out.items():
        setattr(io, name, arr.ctypes.data)
    _check(load().ctfmm_copy_tree(C.c_void_p(ctx), C.byref(io)), C.c_void_p(ctx))
    out["v_pairs"] = out["v_pairs"][: int(io.v_len)]
    for L, ln in (("u", io.u_len), ("w", io.w_len), ("x", io.x_len)):
        out[L + "_list"] = out[L + "_list"][: int(ln)]
    return out


def ctfmm_tree_stats(ctx) -> dict:
    st = ctfmm_tree_stats_t()
    _check(load().ctfmm_tree_stats(C.c_void_p(ctx), C.byref(st)), C.c_void_p(ctx))
    out = {name: getattr(st, name) for name, _ in ctfmm_tree_stats_t._fields_ if name != "root_lo"}
    out["root_lo"] = tuple(st.root_lo)
    return out


def ctfmm_set_m2l_tile(ctx, p: int, targets: int) -> None:
    _check(load().ctfmm_set_m2l_tile(C.c_void_p(ctx), p, targets), C.c_void_p(ctx))


def ctfmm_get_m2l_tile(ctx, p: int) -> int:
    v = C.c_int32()
    _check(load().ctfmm_get_m2l_tile(C.c_void_p(ctx), p, C.byref(v)), C.c_void_p(ctx))
    return v.value


MLP_NIN, MLP_NOUT, MLP_NPARAM = 12, 9, 5577


def mlp_init_params(seed: int):
    """Starting parameters of the order network (flat layout of
    CTFMM_MLP_NPARAM): He-uniform weights, zero biases, float32."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((MLP_NIN, 64), (64, 64), (64, MLP_NOUT)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def _f32dev(t, shape=None):
    if t is None or not t.is_cuda or str(t.dtype) != "torch.float32" or not t.is_contiguous():
        raise ValueError("expected a contiguous cuda float32 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return _ptr(t)


def ctfmm_set_order_table(ctx, order_r2) -> None:
    import numpy as np
    if order_r2 is None:
        _check(load().ctfmm_set_order_table(C.c_void_p(ctx), None), C.c_void_p(ctx))
        return
    tab = np.ascontiguousarray(order_r2, dtype=np.int32)
    assert tab.size == 28
    _check(load().ctfmm_set_order_table(C.c_void_p(ctx), C.c_void_p(tab.ctypes.data)), C.c_void_p(ctx))


def ctfmm_set_order_hash(ctx, seed: int, pmin: int) -> None:
    _check(load().ctfmm_set_order_hash(C.c_void_p(ctx), int(seed), int(pmin)), C.c_void_p(ctx))


def ctfmm_set_mac(ctx, theta: float, centre: int) -> None:
    _check(load().ctfmm_set_mac(C.c_void_p(ctx), float(theta), int(centre)), C.c_void_p(ctx))


def ctfmm_copy_dual(ctx) -> dict:
    """The dual-tree traversal of the last evaluate as numpy arrays: zr
    (nodes, 4), m2l (entries, 2) = (target, source), p2p (entries, 2) =
    (leaf, partner), both sorted."""
    import numpy as np
    io = ctfmm_dual_copy_t()
    _check(load().ctfmm_copy_dual(C.c_void_p(ctx), C.byref(io)), C.c_void_p(ctx))
    out = {"zr": np.zeros((int(io.nodes), 4)), "m2l": np.zeros((max(int(io.m2l), 1), 2), np.int32),
           "p2p": np.zeros((max(int(io.p2p), 1), 2), np.int32)}
    io.zr, io.m2l_pairs, io.p2p_pairs = out["zr"].ctypes.data, out["m2l"].ctypes.data, out["p2p"].ctypes.data
    _check(load().ctfmm_copy_dual(C.c_void_p(ctx), C.byref(io)), C.c_void_p(ctx))
    out["m2l"] = out["m2l"][: int(io.m2l)]
    out["p2p"] = out["p2p"][: int(io.p2p)]
    return out


def ctfmm_set_order_model(ctx, params, norm, target_rel_err: float, margin: float) -> None:
    import numpy as np
    if params is None:
        _check(load().ctfmm_set_order_model(C.c_void_p(ctx), None, None, 1.0, 0.0), C.c_void_p(ctx))
        return
    prm = np.ascontiguousarray(params, dtype=np.float32)
    nrm = np.ascontiguousarray(norm, dtype=np.float32)
    assert prm.size == MLP_NPARAM and nrm.size == 2 * MLP_NIN
    _check(load().ctfmm_set_order_model(C.c_void_p(ctx), C.c_void_p(prm.ctypes.data), C.c_void_p(nrm.ctypes.data),
                                        float(target_rel_err), float(margin)), C.c_void_p(ctx))


def ctfmm_mlp_forward(ctx, x, params, y, precision: int = 0) -> None:
    n = int(x.shape[0])
    _check(load().ctfmm_mlp_forward(C.c_void_p(ctx), n, _f32dev(x, (n, MLP_NIN)), _f32dev(params, (MLP_NPARAM,)),
                                    precision, _f32dev(y, (n, MLP_NOUT))), C.c_void_p(ctx))


def ctfmm_mlp_backward(ctx, x, t, params, grad, loss) -> None:
    n = int(x.shape[0])
    _check(load().ctfmm_mlp_backward(C.c_void_p(ctx), n, _f32dev(x, (n, MLP_NIN)), _f32dev(t, (n, MLP_NOUT)),
                                     _f32dev(params, (MLP_NPARAM,)), _f32dev(grad, (MLP_NPARAM,)),
                                     _f32dev(loss, (1,))), C.c_void_p(ctx))


def ctfmm_mlp_backward_noalloc(ctx, x, t, params, grad, loss) -> None:
    """As ctfmm_mlp_backward, with the library's fixed scratch (n <= 4096)."""
    n = int(x.shape[0])
    _check(load().ctfmm_mlp_backward_noalloc(C.c_void_p(ctx), n, _f32dev(x, (n, MLP_NIN)), _f32dev(t, (n, MLP_NOUT)),
                                             _f32dev(params, (MLP_NPARAM,)), _f32dev(grad, (MLP_NPARAM,)),
                                             _f32dev(loss, (1,))), C.c_void_p(ctx))


def ctfmm_mlp_train(ctx, x, t, params, steps: int, batch: int, lr: float):
    """Trains params (cuda float32, in place); returns the per-step losses."""
    import numpy as np
    n = int(x.shape[0])
    losses = np.zeros(steps, dtype=np.float32)
    _check(load().ctfmm_mlp_train(C.c_void_p(ctx), n, _f32dev(x, (n, MLP_NIN)), _f32dev(t, (n, MLP_NOUT)),
                                  _f32dev(params, (MLP_NPARAM,)), steps, batch, float(lr),
                                  C.c_void_p(losses.ctypes.data)), C.c_void_p(ctx))
    return losses


def ctfmm_mlp_labels(ctx, M, v, x, y) -> None:
    """M: cuda float64 [n,121]; v: host int array [n,3]; x, y: cuda float32."""
    import numpy as np
    n = int(M.shape[0])
    vv = np.ascontiguousarray(v, dtype=np.int32).reshape(n, 3)
    if not M.is_cuda or str(M.dtype) != "torch.float64" or not M.is_contiguous() or tuple(M.shape) != (n, 121):
        raise ValueError("M must be contiguous cuda float64 [n,121]")
    _check(load().ctfmm_mlp_labels(C.c_void_p(ctx), n, _ptr(M), C.c_void_p(vv.ctypes.data),
                                   _f32dev(x, (n, MLP_NIN)), _f32dev(y, (n, MLP_NOUT))), C.c_void_p(ctx))


def ctfmm_mlp_samples(ctx, xyz, q, nsamp: int, seed: int, x, y) -> None:
    n = int(q.shape[0])
    _check(load().ctfmm_mlp_samples(C.c_void_p(ctx), n, _ptr(xyz), _ptr(q), nsamp, seed,
                                    _f32dev(x, (nsamp, MLP_NIN)), _f32dev(y, (nsamp, MLP_NOUT))), C.c_void_p(ctx))


def ctfmm_set_timing(ctx, on: bool) -> None:
    _check(load().ctfmm_set_timing(C.c_void_p(ctx), 1 if on else 0), C.c_void_p(ctx))


def ctfmm_stats(ctx) -> dict:
    st = ctfmm_stats_t()
    _check(load().ctfmm_stats(C.c_void_p(ctx), C.byref(st)), C.c_void_p(ctx))
    out = {name: getattr(st, name) for name, _ in ctfmm_stats_t._fields_}
    out["m2l_order_pairs"] = list(st.m2l_order_pairs)
    return out


def ctfmm_reset_stats(ctx) -> None:
    _check(load().ctfmm_reset_stats(C.c_void_p(ctx)), C.c_void_p(ctx))


def ctfmm_sync(ctx) -> None:
    _check(load().ctfmm_sync(C.c_void_p(ctx)), C.c_void_p(ctx))


def ctfmm_last_error(ctx=None) -> str:
    m = load().ctfmm_last_error(None if ctx is None else C.c_void_p(ctx))
    return m.decode() if m else ""


def ctfmm_destroy(ctx) -> None:
    load().ctfmm_destroy(C.c_void_p(ctx))


# ---------------------------------------------------------------- convenience

class FMM:
    """A context bound to torch's current stream on the current device, its
    device workspace taken from torch's caching allocator (torch_alloc=False:
    hipMalloc).

    tree="uniform": octree of the given depth over the cube (root_lo, root_side).
    tree="adaptive": leaves of at most leaf_max particles; depth is ignored and
    root_side=None (or <= 0) selects the automatic root cube.
    tree="dual": the same octree driven by the dual-tree traversal with the
    acceptance parameter theta and the expansion centres ("geometric",
    "mass" or "ap"; the AP variant gives the gradient only)."""

    def __init__(self, p: int, depth: int = 0, precision: str = "fp64", root_lo=(0.0, 0.0, 0.0),
                 root_side: float | None = 1.0, stream: int | None = None, tree: str = "uniform",
                 leaf_max: int = 64, torch_alloc: bool = True, theta: float = 0.5, centre: str = "geometric"):
        prm = ctfmm_default_params()
        prm.order_p, prm.depth, prm.precision = p, depth, PRECISIONS[precision]
        prm.tree, prm.leaf_max = TREES[tree], leaf_max
        prm.root_lo[0], prm.root_lo[1], prm.root_lo[2] = root_lo
        prm.root_side = 0.0 if root_side is None else root_side
        self.p, self.depth, self.tree = p, depth, tree
        self.ctx = None
        self._alloc = None
        self.ctx = ctfmm_create(prm, stream)
        if torch_alloc:
            self._alloc = torch_allocator()
            ctfmm_set_allocator(self.ctx, *self._alloc)
        self.centre = centre
        if tree == "dual":
            ctfmm_set_mac(self.ctx, theta, CENTRES[centre])

    def set_mac(self, theta: float, centre: str = "geometric") -> None:
        ctfmm_set_mac(self.ctx, theta, CENTRES[centre])
        self.centre = centre

    def dual_copy(self) -> dict:
        return ctfmm_copy_dual(self.ctx)

    def tree_stats(self) -> dict:
        return ctfmm_tree_stats(self.ctx)

    def tree_copy(self) -> dict:
        return ctfmm_copy_tree(self.ctx)

    def evaluate(self, xyz, q, phi=None, grad=None, sync=False):
        """phi and grad (allocated if None); the AP variant returns phi None"""
        import torch
        n = int(q.shape[0])
        if phi is None and not (self.tree == "dual" and self.centre == "ap"):
            phi = torch.empty(n, dtype=torch.float64, device=q.device)
        if grad is None:
            grad = torch.empty((n, 3), dtype=torch.float64, device=q.device)
        ctfmm_evaluate(self.ctx, xyz, q, phi, grad)
        if sync:
            ctfmm_sync(self.ctx)
        return phi, grad

    def evaluate_dipoles(self, xyz, q, dip, phi=None, grad=None, sync=False):
        import torch
        n = int(q.shape[0])
        if phi is None:
            phi = torch.empty(n, dtype=torch.float64, device=q.device)
        if grad is None:
            grad = torch.empty((n, 3), dtype=torch.float64, device=q.device)
        ctfmm_evaluate_dipoles(self.ctx, xyz, q, dip, phi, grad)
        if sync:
            ctfmm_sync(self.ctx)
        return phi, grad

    def evaluate_f32(self, xyz, q, phi=None, grad=None, sync=False):
        import torch
        n = int(q.shape[0])
        if phi is None:
            phi = torch.empty(n, dtype=torch.float32, device=q.device)
        if grad is None:
            grad = torch.empty((n, 3), dtype=torch.float32, device=q.device)
        ctfmm_evaluate_f32(self.ctx, xyz, q, phi, grad)
        if sync:
            ctfmm_sync(self.ctx)
        return phi, grad

    def evaluate_batched_f32(self, offsets, orders, xyz, q, phi=None, grad=None, sync=False):
        import torch
        n = int(q.shape[0])
        if phi is None:
            phi = torch.empty(n, dtype=torch.float32, device=q.device)
        if grad is None:
            grad = torch.empty((n, 3), dtype=torch.float32, device=q.device)
        ctfmm_evaluate_batched_f32(self.ctx, offsets, orders, xyz, q, phi, grad)
        if sync:
            ctfmm_sync(self.ctx)
        return phi, grad

    def evaluate_batched(self, offsets, orders, xyz, q, phi=None, grad=None, sync=False):
        import torch
        n = int(q.shape[0])
        if phi is None:
            phi = torch.empty(n, dtype=torch.float64, device=q.device)
        if grad is None:
            grad = torch.empty((n, 3), dtype=torch.float64, device=q.device)
        ctfmm_evaluate_batched(self.ctx, offsets, orders, xyz, q, phi, grad)
        if sync:
            ctfmm_sync(self.ctx)
        return phi, grad

    def stats(self) -> dict:
        return ctfmm_stats(self.ctx)

    def set_order_table(self, order_r2) -> None:
        ctfmm_set_order_table(self.ctx, order_r2)

    def set_order_hash(self, seed: int, pmin: int) -> None:
        ctfmm_set_order_hash(self.ctx, seed, pmin)

    def set_order_model(self, params, norm, target_rel_err: float, margin: float) -> None:
        ctfmm_set_order_model(self.ctx, params, norm, target_rel_err, margin)

    def set_m2l_tile(self, p: int, targets: int) -> None:
        ctfmm_set_m2l_tile(self.ctx, p, targets)

    def m2l_tile(self, p: int) -> int:
        return ctfmm_get_m2l_tile(self.ctx, p)

    def expansions(self, level: int, which: str):
        import numpy as np
        out = np.zeros((8 ** level, (self.p + 1) ** 2))
        ctfmm_copy_expansions(self.ctx, level, {"M": 0, "L": 1}[which], out)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            ctfmm_destroy(self.ctx)
            self.ctx = None
        self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
