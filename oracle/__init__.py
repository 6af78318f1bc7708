"""Plain FP64 CPU oracle for the Cartesian traceless FMM (arXiv 1811.06332).

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
anything in this package; only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` do.  It shares no code with the GPU path.

This module is argument marshalling (numpy <-> ctypes) around
``ctfmm_oracle.c``; every operator is computed there, in full symmetric
storage, from the paper's equations (see the header of that file).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no intrinsics, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-Wall",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i32, i64, d = C.c_int, C.c_int64, C.c_double
        L.oracle_nfull.argtypes = [i32]; L.oracle_nfull.restype = i32
        L.oracle_full_index.argtypes = [i32, i32, i32]; L.oracle_full_index.restype = i32
        L.oracle_detracer_T.argtypes = [i32, _dp, _dp]
        L.oracle_detracer_D.argtypes = [i32, _dp, _dp]
        L.oracle_dtensor.argtypes = [i32, _dp, _dp]
        L.oracle_p2m.argtypes = [i32, _dp, i64, _dp, _dp, _dp]
        L.oracle_m2m.argtypes = [i32, _dp, _dp, _dp]
        L.oracle_m2l.argtypes = [i32, _dp, _dp, _dp]
        L.oracle_m2l_with_D.argtypes = [i32, _dp, _dp, _dp]
        L.oracle_l2l.argtypes = [i32, _dp, _dp, _dp]
        L.oracle_l2p.argtypes = [i32, _dp, _dp, _dp, _dp]
        L.oracle_direct.argtypes = [i64, _dp, _dp, i64, C.c_void_p, _dp, _dp, i32]
        L.oracle_fmm_uniform.argtypes = [i64, _dp, _dp, i32, i32, _dp, d, i64, C.c_void_p,
                                         _dp, _dp, C.c_void_p, C.c_void_p, i32]
        L.oracle_fmm_uniform.restype = i32
        L.oracle_fmm_uniform_dipoles.argtypes = [i64, _dp, _dp, _dp, i32, i32, _dp, d, i64, C.c_void_p,
                                                 _dp, _dp, i32]
        L.oracle_fmm_uniform_dipoles.restype = i32
        L.oracle_direct_dipoles.argtypes = [i64, _dp, _dp, _dp, i64, C.c_void_p, _dp, _dp, i32]
        L.oracle_p2m_dipole.argtypes = [i32, _dp, i64, _dp, _dp, _dp]
        L.oracle_max_threads.restype = i32
        L.oracle_fmm_adaptive.argtypes = [i64, _dp, _dp, i32, i32, _dp, d, i64, C.c_void_p, _dp, _dp,
                                          C.c_void_p, C.c_void_p, i32]
        L.oracle_fmm_adaptive.restype = i32
        L.oracle_auto_root.argtypes = [i64, _dp, _dp, C.c_void_p]
        L.oracle_fmm_adaptive_orders.argtypes = [i64, _dp, _dp, i32, i32, _dp, d, i64, C.c_void_p, _dp, _dp,
                                                 C.c_void_p, C.c_void_p, i32, C.c_void_p]
        L.oracle_fmm_adaptive_orders.restype = i32
        L.oracle_fmm_adaptive_pair_orders.argtypes = [i64, _dp, _dp, i32, i32, _dp, d, i64, C.c_void_p, _dp, _dp,
                                                      C.c_void_p, C.c_void_p, i32, C.c_void_p]
        L.oracle_fmm_adaptive_pair_orders.restype = i32
        L.oracle_fmm_dual.argtypes = [i64, _dp, _dp, i32, i32, d, i32, _dp, d, i64, C.c_void_p, _dp, _dp,
                                      C.c_void_p, C.c_void_p, i32]
        L.oracle_fmm_dual.restype = i32
        L.oracle_dual_pairs.argtypes = [i64, _dp, _dp, i32, d, i32, _dp, d, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
        L.oracle_dual_pairs.restype = i32
        L.oracle_adaptive_tree.argtypes = [i64, _dp, i32, _dp, d, C.c_void_p] + [C.c_void_p] * 15
        L.oracle_adaptive_tree.restype = i32
        _lib_handle = L
    return _lib_handle


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# ---------------------------------------------------------------- indexing

def nfull(p: int) -> int:
    """C(p+3,3): components of a full symmetric polytensor of ranks 0..p."""
    return _lib().oracle_nfull(p)


def full_index(a: int, b: int, c: int) -> int:
    """Slot of multi-index (a,b,c) in the oracle's full storage."""
    return _lib().oracle_full_index(a, b, c)


def multi_indices(p: int):
    """All multi-indices of rank <= p, in the oracle's storage order."""
    out = [None] * nfull(p)
    for n in range(p + 1):
        for a in range(n + 1):
            for b in range(n - a + 1):
                out[full_index(a, b, n - a - b)] = (a, b, n - a - b)
    return out


# ---------------------------------------------------------------- operators

def detracer_T(p, A):
    A = _vec(A, nfull(p)); out = np.zeros_like(A)
    _lib().oracle_detracer_T(p, A, out)
    return out


def detracer_D(p, A):
    A = _vec(A, nfull(p)); out = np.zeros_like(A)
    _lib().oracle_detracer_D(p, A, out)
    return out


def dtensor(p, r):
    out = np.zeros(nfull(p))
    _lib().oracle_dtensor(p, _vec(r, 3), out)
    return out


def p2m(p, z, xyz, q):
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    M = np.zeros(nfull(p))
    _lib().oracle_p2m(p, _vec(z, 3), xyz.shape[0], np.ascontiguousarray(xyz.ravel()), q, M)
    return M


def p2m_dipole(p, z, xyz, dip):
    """Multipole (full storage) of point dipoles dip [n,3] at xyz about z."""
    xyz = _vec(xyz).reshape(-1, 3); dip = _vec(dip).reshape(-1, 3)
    M = np.zeros(nfull(p))
    _lib().oracle_p2m_dipole(p, _vec(z, 3), xyz.shape[0], np.ascontiguousarray(xyz.ravel()),
                             np.ascontiguousarray(dip.ravel()), M)
    return M


def direct_dipoles(xyz, q, dip, targets=None, nthreads=0):
    """O(N^2) potential and gradient of charges q and point dipoles dip [n,3]."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0]); dip = _vec(dip).reshape(-1, 3)
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    _lib().oracle_direct_dipoles(n, np.ascontiguousarray(xyz.ravel()), q, np.ascontiguousarray(dip.ravel()), nt, tp,
                                 phi, grad, nthreads)
    del keep
    return phi, grad.reshape(-1, 3)


def fmm_uniform_dipoles(xyz, q, dip, p, depth, lo=(0.0, 0.0, 0.0), side=1.0, targets=None, nthreads=0):
    """Uniform FMM of charges q and point dipoles dip [n,3] (see
    oracle_fmm_uniform_dipoles)."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0]); dip = _vec(dip).reshape(-1, 3)
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    rc = _lib().oracle_fmm_uniform_dipoles(n, np.ascontiguousarray(xyz.ravel()), q, np.ascontiguousarray(dip.ravel()),
                                           p, depth, _vec(lo, 3), float(side), nt, tp, phi, grad, nthreads)
    del keep
    if rc != 0:
        raise RuntimeError(f"oracle_fmm_uniform_dipoles failed with code {rc}")
    return phi, grad.reshape(-1, 3)


def m2m(p, d, M):
    out = np.zeros(nfull(p))
    _lib().oracle_m2m(p, _vec(d, 3), _vec(M, nfull(p)), out)
    return out


def m2l(p, r, M):
    out = np.zeros(nfull(p))
    _lib().oracle_m2l(p, _vec(r, 3), _vec(M, nfull(p)), out)
    return out


def m2l_with_D(p, M, D):
    out = np.zeros(nfull(p))
    _lib().oracle_m2l_with_D(p, _vec(M, nfull(p)), _vec(D, nfull(p)), out)
    return out


def l2l(p, d, L):
    out = np.zeros(nfull(p))
    _lib().oracle_l2l(p, _vec(d, 3), _vec(L, nfull(p)), out)
    return out


def l2p(p, rb, L):
    phi = np.zeros(1); grad = np.zeros(3)
    _lib().oracle_l2p(p, _vec(rb, 3), _vec(L, nfull(p)), phi, grad)
    return phi[0], grad


def direct(xyz, q, targets=None, nthreads=0):
    """O(N^2) potential and gradient at `targets` (particle indices; all if None)."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    _lib().oracle_direct(n, np.ascontiguousarray(xyz.ravel()), q, nt, tp, phi, grad, nthreads)
    del keep
    return phi, grad.reshape(-1, 3)


def fmm_uniform(xyz, q, p, depth, lo=(0.0, 0.0, 0.0), side=1.0, targets=None,
                dump=False, nthreads=0):
    """Full FMM on a uniform octree (see oracle_fmm_uniform in ctfmm_oracle.c).

    Returns (phi, grad) at `targets` (all particles, input order, if None);
    with dump=True also (M, L): lists over levels 0..depth of arrays
    [8**l, nfull(p)] (cells row-major, x fastest), full storage.
    """
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    nf = nfull(p)
    Md = Ld = None
    if dump:
        tot = sum(8 ** l for l in range(depth + 1)) * nf
        Md = np.zeros(tot); Ld = np.zeros(tot)
    rc = _lib().oracle_fmm_uniform(n, np.ascontiguousarray(xyz.ravel()), q, p, depth,
                                   _vec(lo, 3), float(side), nt, tp, phi, grad,
                                   None if Md is None else Md.ctypes.data,
                                   None if Ld is None else Ld.ctypes.data, nthreads)
    del keep
    if rc != 0:
        raise RuntimeError(f"oracle_fmm_uniform failed with code {rc}")
    grad = grad.reshape(-1, 3)
    if not dump:
        return phi, grad
    Ms, Ls, off = [], [], 0
    for l in range(depth + 1):
        c = 8 ** l * nf
        Ms.append(Md[off:off + c].reshape(8 ** l, nf))
        Ls.append(Ld[off:off + c].reshape(8 ** l, nf))
        off += c
    return phi, grad, Ms, Ls


def auto_root(xyz):
    """The automatic root cube of the adaptive tree: (lo[3], side)."""
    xyz = _vec(xyz).reshape(-1, 3)
    lo = np.zeros(3); side = np.zeros(1)
    _lib().oracle_auto_root(xyz.shape[0], np.ascontiguousarray(xyz.ravel()), lo, side.ctypes.data)
    return lo, float(side[0])


def fmm_adaptive(xyz, q, p, leaf_max, lo=None, side=0.0, targets=None, nthreads=0, stats=False,
                 order_r2=None, v_orders=None):
    """Full FMM on the adaptive octree (see oracle_fmm_adaptive).  lo/side
    None/0 selects the automatic root cube.  With stats=True also returns a
    dict of tree and list sizes and the root box.  order_r2 (28 ints, index
    |v|^2) sets the M2L order of every V-list pair by its offset (see
    oracle_fmm_adaptive_orders); v_orders (one per V-list entry, in the
    V_list order of adaptive_tree) sets it pair by pair (see
    oracle_fmm_adaptive_pair_orders)."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    st = np.zeros(8, dtype=np.int64); root = np.zeros(4)
    lo_arr = _vec(lo if lo is not None else (0.0, 0.0, 0.0), 3)
    args = (n, np.ascontiguousarray(xyz.ravel()), q, p, leaf_max, lo_arr, float(side) if lo is not None else 0.0,
            nt, tp, phi, grad, st.ctypes.data, root.ctypes.data, nthreads)
    if v_orders is not None:
        vo = np.ascontiguousarray(np.asarray(v_orders, dtype=np.int8))
        rc = _lib().oracle_fmm_adaptive_pair_orders(*args, vo.ctypes.data)
    elif order_r2 is None:
        rc = _lib().oracle_fmm_adaptive(*args)
    else:
        otab = np.ascontiguousarray(np.asarray(order_r2, dtype=np.int32))
        assert otab.size == 28
        rc = _lib().oracle_fmm_adaptive_orders(*args, otab.ctypes.data)
    del keep
    if rc != 0:
        raise RuntimeError(f"oracle_fmm_adaptive failed with code {rc}")
    grad = grad.reshape(-1, 3)
    if not stats:
        return phi, grad
    names = ["nodes", "leaves", "max_level", "V", "U", "W", "X"]
    info = {k: int(v) for k, v in zip(names, st[:7])}
    info["root_lo"] = root[:3].copy(); info["root_side"] = float(root[3])
    return phi, grad, info


DUAL_CENTRES = {"geometric": 0, "mass": 1, "ap": 2}


def fmm_dual(xyz, q, p, leaf_max, theta, centre="geometric", lo=None, side=0.0, targets=None, nthreads=0,
             stats=False):
    """The FMM driven by the dual-tree traversal with the theta MAC (see
    oracle_fmm_dual); centre "geometric", "mass" or "ap" (centre of mass,
    dipole dropped, gradient only: phi comes back as None)."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    n = xyz.shape[0]
    if targets is None:
        nt, tp, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt, tp = keep.size, keep.ctypes.data
    phi = np.zeros(nt); grad = np.zeros(3 * nt)
    st = np.zeros(8, dtype=np.int64); root = np.zeros(4)
    lo_arr = _vec(lo if lo is not None else (0.0, 0.0, 0.0), 3)
    rc = _lib().oracle_fmm_dual(n, np.ascontiguousarray(xyz.ravel()), q, p, leaf_max, float(theta),
                                DUAL_CENTRES[centre], lo_arr, float(side) if lo is not None else 0.0,
                                nt, tp, phi, grad, st.ctypes.data, root.ctypes.data, nthreads)
    del keep
    if rc != 0:
        raise RuntimeError(f"oracle_fmm_dual failed with code {rc}")
    grad = grad.reshape(-1, 3)
    if centre == "ap":
        phi = None
    if not stats:
        return phi, grad
    info = dict(zip(["nodes", "leaves", "max_level", "m2l_pairs", "direct_pairs"], (int(v) for v in st[:5])))
    return phi, grad, info


def dual_pairs(xyz, q, leaf_max, theta, centre="geometric", lo=None, side=0.0):
    """The traversal's integer result (see oracle_dual_pairs): dict with
    m2l (k, 2) accepted pairs in traversal order, p2p (k, 2) ordered direct
    pairs, zr (nodes, 4) centres and radii; node numbers as adaptive_tree."""
    xyz = _vec(xyz).reshape(-1, 3); q = _vec(q, xyz.shape[0])
    n = xyz.shape[0]
    lo_arr = _vec(lo if lo is not None else (0.0, 0.0, 0.0), 3)
    sd = float(side) if lo is not None else 0.0
    args = (n, np.ascontiguousarray(xyz.ravel()), q, leaf_max, float(theta), DUAL_CENTRES[centre], lo_arr, sd)
    sizes = np.zeros(3, dtype=np.int64)
    rc = _lib().oracle_dual_pairs(*args, sizes.ctypes.data, None, None, None)
    if rc != 0:
        raise RuntimeError(f"oracle_dual_pairs failed with code {rc}")
    m2l = np.zeros((int(sizes[1]), 2), dtype=np.int32)
    p2p = np.zeros((int(sizes[2]), 2), dtype=np.int32)
    zr = np.zeros((int(sizes[0]), 4))
    rc = _lib().oracle_dual_pairs(*args, sizes.ctypes.data, m2l.ctypes.data, p2p.ctypes.data, zr.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_dual_pairs failed with code {rc}")
    return {"m2l": m2l, "p2p": p2p, "zr": zr}


def adaptive_tree(xyz, leaf_max, lo=None, side=0.0):
    """The adaptive tree and U/V/W/X lists of fmm_adaptive (see
    oracle_adaptive_tree): a dict of numpy arrays level, key, leaf, parent,
    pb, pe (per node, the oracle's numbering), order (input index of each
    sorted position) and, for L in U, V, W, X, L_off [nodes+1] and L_list."""
    xyz = _vec(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    flat = np.ascontiguousarray(xyz.ravel())
    lo_arr = _vec(lo if lo is not None else (0.0, 0.0, 0.0), 3)
    sd = float(side) if lo is not None else 0.0
    sizes = np.zeros(6, dtype=np.int64)
    L = _lib()
    nulls = [None] * 15
    rc = L.oracle_adaptive_tree(n, flat, leaf_max, lo_arr, sd, sizes.ctypes.data, *nulls)
    if rc != 0:
        raise RuntimeError(f"oracle_adaptive_tree failed with code {rc}")
    nn = int(sizes[0])
    out = {"level": np.zeros(nn, np.int32), "key": np.zeros(nn, np.uint64), "leaf": np.zeros(nn, np.int32),
           "parent": np.zeros(nn, np.int32), "pb": np.zeros(nn, np.int64), "pe": np.zeros(nn, np.int64),
           "order": np.zeros(n, np.int64)}
    for k, name in enumerate("UVWX"):
        out[name + "_off"] = np.zeros(nn + 1, np.int64)
        out[name + "_list"] = np.zeros(max(int(sizes[2 + k]), 1), np.int32)
    args = [out[k].ctypes.data for k in ("level", "key", "leaf", "parent", "pb", "pe", "order")]
    for name in "UVWX":
        args += [out[name + "_off"].ctypes.data, out[name + "_list"].ctypes.data]
    rc = L.oracle_adaptive_tree(n, flat, leaf_max, lo_arr, sd, sizes.ctypes.data, *args)
    if rc != 0:
        raise RuntimeError(f"oracle_adaptive_tree failed with code {rc}")
    for k, name in enumerate("UVWX"):
        out[name + "_list"] = out[name + "_list"][: int(sizes[2 + k])]
    return out


def max_threads() -> int:
    return _lib().oracle_max_threads()
