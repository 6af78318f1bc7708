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
