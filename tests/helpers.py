"""Shared test helpers: index bookkeeping between the oracle's full storage
and the library's independent traceless components (no FMM arithmetic)."""
from __future__ import annotations

import numpy as np


def independent_indices(p):
    """(nx,ny,nz) of the library's (p+1)^2 independent components, in its
    documented order: by rank, then n_z in {0,1}, then n_x descending."""
    out = []
    for n in range(p + 1):
        for a in range(n, -1, -1):
            out.append((a, n - a, 0))
        for a in range(n - 1, -1, -1):
            out.append((a, n - 1 - a, 1))
    return out


def oracle_columns(oracle, p):
    return np.array([oracle.full_index(*m) for m in independent_indices(p)])


def rel(a, b):
    """Normwise relative error ||a - b||_2 / ||b||_2 over all particles."""
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def maxrel(a, b):
    """Worst particle: max_b |a_b - ref_b| / RMS_b |ref_b|, for potentials
    ([n]) or gradients ([n,3], |.| the Euclidean norm of each row).  A
    handful of wrong particles that a normwise error over many particles
    would hide shows up here."""
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        a = a[:, None]; b = b[:, None]
    d = np.linalg.norm(a - b, axis=1)
    rms = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    return float(d.max() / (rms if rms > 0 else 1.0)) if d.size else 0.0


# per-particle bounds beside the normwise gates (1e-12 in FP64, 1e-6 with
# FP32 or BF16x3 M2L): the worst particle may carry more than the average
MAXREL_FP64 = 1e-10
MAXREL_MIXED = 1e-4


def node_codes(level, key):
    """One int64 per node: level in the top bits, the Morton prefix below
    (unique per node of one tree, equal between two builds of it)."""
    return (np.asarray(level, dtype=np.int64) << 58) | np.asarray(key, dtype=np.uint64).astype(np.int64)


def compare_trees(gpu, ora):
    """Entry-by-entry comparison of the GPU's adaptive tree and lists
    (ctfmm_copy_tree) with the oracle's (oracle.adaptive_tree): the same
    nodes, leaves, parents, particles of every node (as sets: the order of
    equal keys is free), and U, V, W, X lists (as sets per node; no
    duplicates).  Returns a dict of sizes."""
    cg = node_codes(gpu["level"], gpu["key"])
    co = node_codes(ora["level"], ora["key"])
    assert len(np.unique(cg)) == len(cg) and len(cg) == len(co)
    og, oo = np.argsort(cg), np.argsort(co)
    assert np.array_equal(cg[og], co[oo]), "node sets differ"
    # oracle node index -> gpu node index
    o2g = np.empty(len(co), dtype=np.int64)
    o2g[oo] = og
    assert np.array_equal(gpu["leaf"][o2g], ora["leaf"])
    par = ora["parent"].astype(np.int64)
    assert np.array_equal(gpu["parent"][o2g], np.where(par >= 0, o2g[np.maximum(par, 0)], -1))
    assert np.array_equal(gpu["pb"][o2g], ora["pb"]) and np.array_equal(gpu["pe"][o2g], ora["pe"])
    perm_g, perm_o = gpu["perm"].astype(np.int64), ora["order"]
    for i in np.nonzero(ora["leaf"])[0]:
        b, e = ora["pb"][i], ora["pe"][i]
        assert np.array_equal(np.sort(perm_g[b:e]), np.sort(perm_o[b:e])), i

    def pairs(off, lst, mapping=None):
        off = np.asarray(off, dtype=np.int64)
        tgt = np.repeat(np.arange(len(off) - 1), np.diff(off))
        src = np.asarray(lst, dtype=np.int64)
        if mapping is not None:
            tgt, src = mapping[tgt], mapping[src]
        return tgt, src

    def canon(tgt, src):
        a = cg[tgt] if tgt.size else tgt
        b = cg[src] if src.size else src
        order = np.lexsort((b, a))
        return np.stack([a[order], b[order]])

    sizes = {}
    for L in "uwx":
        tg, sg = pairs(gpu[L + "_off"], gpu[L + "_list"])
        to, so = pairs(ora[L.upper() + "_off"], ora[L.upper() + "_list"], o2g)
        A, B = canon(tg, sg), canon(to, so)
        assert A.shape == B.shape and np.array_equal(A, B), f"{L.upper()} lists differ"
        assert not np.any(np.all(A[:, 1:] == A[:, :-1], axis=0)), f"duplicate {L.upper()} entries"
        sizes[L.upper()] = A.shape[1]
    vg = gpu["v_pairs"].astype(np.int64)
    to, so = pairs(ora["V_off"], ora["V_list"], o2g)
    A, B = canon(vg[:, 0], vg[:, 1]), canon(to, so)
    assert A.shape == B.shape and np.array_equal(A, B), "V lists differ"
    sizes["V"] = A.shape[1]
    sizes["nodes"] = len(cg)
    return sizes


# ---------------------------------------------------------------- per-pair orders

CLASSES_R2 = [4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 17, 18, 19, 22, 27]
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(z):
    """SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) on
    uint64 arrays (numpy arithmetic wraps modulo 2^64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hashed_orders(level, key, cls, seed, pmin, p, sys=0):
    """The order map of ctfmm_set_order_hash for cells (level, key) of system
    sys in distance class cls."""
    z = splitmix64(np.uint64(seed) ^ np.asarray(key, dtype=np.uint64))
    z = splitmix64(z ^ np.asarray(level, dtype=np.uint64))
    z = splitmix64(z ^ (np.uint64(16) * np.uint64(sys) + np.asarray(cls, dtype=np.uint64)))
    return (pmin + (z % np.uint64(p - pmin + 1))).astype(np.int64)


def tile_max_v_orders(tree, tt, seed, pmin, p):
    """Order of every V-list entry of an (oracle) adaptive tree under the
    rule of the GPU's M2L tiles: the targets of one level and one octant,
    in Morton order, are grouped tt at a time; all pairs of one tile at one
    offset v run at the largest order any of them asks for, each pair
    asking for the map's order of its source cell in the class of |v|^2."""
    level = np.asarray(tree["level"], dtype=np.int64)
    key = np.asarray(tree["key"], dtype=np.uint64)
    nn = len(level)
    coords = np.zeros((nn, 3), dtype=np.int64)
    for l in range(int(level.max()) + 1):
        for d in range(3):
            coords[:, d] |= ((key >> np.uint64(3 * l + d)).astype(np.int64) & 1) << l
    coords[level == 0] = 0
    # the tile of every node of level >= 2
    tile = np.full(nn, -1, dtype=np.int64)
    nt = 0
    for l in range(2, int(level.max()) + 1):
        for o in range(8):
            sel = np.nonzero((level == l) & ((key & np.uint64(7)).astype(np.int64) == o))[0]
            sel = sel[np.argsort(key[sel])]
            tile[sel] = nt + np.arange(len(sel)) // tt
            nt += (len(sel) + tt - 1) // tt
    off = np.asarray(tree["V_off"], dtype=np.int64)
    tgt = np.repeat(np.arange(nn), np.diff(off))
    src = np.asarray(tree["V_list"], dtype=np.int64)
    v = coords[src] - coords[tgt]
    r2 = np.sum(v * v, axis=1)
    cls = np.searchsorted(CLASSES_R2, r2)
    assert np.array_equal(np.asarray(CLASSES_R2)[cls], r2)
    want = hashed_orders(level[src], key[src], cls, seed, pmin, p)
    group = (tile[tgt] * 343) + (v[:, 0] + 3) + 7 * (v[:, 1] + 3) + 49 * (v[:, 2] + 3)
    gmax = {}
    for g, w in zip(group.tolist(), want.tolist()):
        if gmax.get(g, -1) < w:
            gmax[g] = w
    return np.array([gmax[g] for g in group.tolist()], dtype=np.int8)
