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
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))
