"""The operator tables the GPU path is built from, checked against the oracle.

The generator (paper_1811_06332_amd/gen/gen_operators.py) derives, in exact
rational arithmetic, every table the HIP kernels use: the detracer rows of
P2M (Eq. P2M with Eq. Detracer), the per-particle P2M terms (Eq. Detracer3),
the M2M and L2L octant matrices in scaled variables (Eq. M2M, Eq. L2L) and the
M2L contraction of independent components (Eq. M2L).  The GPU parity tests
see them only through whole evaluations; here each table is compared, entry
range by entry range, with the oracle's own operators (which share no code
with the generator) at every rank up to the largest compiled order, on random
inputs.  The comparison goes through the generator's rationals rounded to
FP64, as the kernels use them.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle

GEN_DIR = os.path.join(os.path.dirname(__file__), "..", "paper_1811_06332_amd", "gen")
sys.path.insert(0, GEN_DIR)
import gen_operators as G  # noqa: E402

G.DET = G.detracer_rows()
P = G.PMAX
RTOL = 1e-12


def _oracle_ind(full_vec, p=P):
    """The independent components (generator order) of an oracle full-storage vector."""
    return np.array([full_vec[oracle.full_index(*m)] for m in G.IND if G.rank(m) <= p])


def _rank_arr(p=P):
    return np.array([G.rank(m) for m in G.IND if G.rank(m) <= p])


def _close(a, b, rtol=RTOL):
    scale = np.abs(b).max()
    assert scale > 0
    err = np.abs(a - b).max() / scale
    assert err <= rtol, err


def _cluster(rng, centre, half, n):
    return np.asarray(centre) + rng.uniform(-half, half, (n, 3)), rng.uniform(-1.0, 1.0, n)


def test_detracer_rows_and_p2m_terms_match_oracle_p2m():
    """M~_n = sum_f DET[n][f] S_f, S_f = sum_a q_a u_a^f, u = z - x (h = 1), and the
    per-particle terms of Eq. Detracer3 both reproduce the oracle's P2M at every
    independent component of ranks 0..PMAX."""
    rng = np.random.default_rng(11)
    z = np.array([0.1, -0.2, 0.3])
    xyz, q = _cluster(rng, z, 0.5, 23)
    ref = _oracle_ind(oracle.p2m(P, z, xyz, q))
    u = z - xyz
    S = np.array([np.sum(q * u[:, 0] ** f[0] * u[:, 1] ** f[1] * u[:, 2] ** f[2]) for f in G.FULL])
    det = np.array([sum(float(w) * S[f] for f, w in row.items()) for row in G.DET])
    _close(det, ref)
    r2 = np.sum(u * u, axis=1)
    terms = np.array([sum(float(c) * np.sum(q * u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** d * r2 ** e)
                          for (c, a, b, d, e) in row) for row in G.p2m_terms()])
    _close(terms, ref)


def test_detracer_rows_by_rank_match_the_rows():
    """The straight-line rows emitted per rank use only full slots of that rank (the
    one-thread-per-leaf P2M sums the moments rank by rank)."""
    for N in range(P + 1):
        f0 = N * (N + 1) * (N + 2) // 6
        f1 = f0 + (N + 1) * (N + 2) // 2
        for i in range(N * N, (N + 1) * (N + 1)):
            assert all(f0 <= f < f1 for f in G.DET[i]), (N, i)


@pytest.mark.parametrize("octant", range(8))
def test_m2m_octant_matrix_matches_oracle(octant):
    """Parent M~ = A_o child M~ (M~_n = M_n / h^|n|) for the child of octant o
    (centre offset (2 o_d - 1) h_P / 4): the oracle's P2M of the same particles
    about the child and about the parent centre, at every rank up to PMAX."""
    rng = np.random.default_rng(100 + octant)
    hp, hc = 1.0, 0.5
    zp = np.array([0.25, -0.5, 0.125])
    sig = np.array([2 * ((octant >> d) & 1) - 1 for d in range(3)])
    zc = zp + sig * hp / 4
    xyz, q = _cluster(rng, zc, hc / 2, 17)
    rk = _rank_arr()
    mc = _oracle_ind(oracle.p2m(P, zc, xyz, q)) / hc ** rk
    mp = _oracle_ind(oracle.p2m(P, zp, xyz, q)) / hp ** rk
    A = G.m2m_matrix(octant)
    got = np.array([sum(float(v) * mc[j] for j, v in row.items()) for row in A])
    _close(got, mp)


@pytest.mark.parametrize("octant", range(8))
def test_l2l_octant_matrix_matches_oracle(octant):
    """Child L~ = B_o parent L~ (L~_n = L_n h^(|n|+1)) against the oracle's L2L
    (a Taylor shift by the child's centre offset) of a local expansion made by
    the oracle's M2L from a distant cluster."""
    rng = np.random.default_rng(200 + octant)
    hp, hc = 1.0, 0.5
    zp = np.array([-0.3, 0.2, 0.1])
    sig = np.array([2 * ((octant >> d) & 1) - 1 for d in range(3)])
    d = sig * hp / 4
    zs = zp + np.array([4.0, -3.0, 2.5])
    xyz, q = _cluster(rng, zs, 0.5, 9)
    M = oracle.p2m(P, zs, xyz, q)
    Lp = oracle.m2l(P, zp - zs, M)
    Lc = oracle.l2l(P, d, Lp)
    rk = _rank_arr()
    lp = _oracle_ind(Lp) * hp ** (rk + 1)
    lc = _oracle_ind(Lc) * hc ** (rk + 1)
    B = G.l2l_matrix(octant)
    got = np.array([sum(float(v) * lp[j] for j, v in row.items()) for row in B])
    _close(got, lc)


@pytest.mark.parametrize("r", [(2.0, 0.0, 0.0), (3.0, -1.0, 2.0), (-1.5, 2.5, -2.0)])
def test_m2l_contraction_matches_oracle(r):
    """L_n = sum_j K[n][j] M_j with K[n][j] = sum_i c[n,j,i] D_i(r) (independent
    components only, pairs with |n| + |j| <= PMAX) against the oracle's M2L,
    which contracts full tensors."""
    rng = np.random.default_rng(300)
    xyz, q = _cluster(rng, (0.0, 0.0, 0.0), 0.5, 11)
    M = oracle.p2m(P, (0.0, 0.0, 0.0), xyz, q)
    ref = _oracle_ind(oracle.m2l(P, r, M))
    Dind = _oracle_ind(oracle.dtensor(P, r))
    Mind = _oracle_ind(M)
    c = G.m2l_contraction()
    got = np.zeros(len(G.IND))
    for (n, j), terms in c.items():
        got[n] += sum(float(v) * Dind[i] for i, v in terms.items()) * Mind[j]
    _close(got, ref)


def test_expansion_of_dependent_components_matches_the_trace():
    """Every full component of a traceless tensor from its independent ones
    (expand) equals the oracle's full traceless tensor at that component."""
    rng = np.random.default_rng(400)
    xyz, q = _cluster(rng, (0.0, 0.0, 0.0), 0.5, 13)
    M = oracle.p2m(P, (0.0, 0.0, 0.0), xyz, q)
    Mind = _oracle_ind(M)
    full = np.array([sum(e * Mind[j] for j, e in G.expand(m).items()) for m in G.FULL])
    ref = np.array([M[oracle.full_index(*m)] for m in G.FULL])
    _close(full, ref)


def test_planted_table_mistakes_are_caught(monkeypatch):
    """Each comparison above rejects a small mistake planted in the table it
    checks: one detracer coefficient off by 1e-6, the M2M matrix of the
    opposite octant, the L2L row of one component without its top-rank terms,
    one M2L contraction term dropped, and a sign flipped in the expansion of a
    dependent component."""
    from fractions import Fraction

    def rejects(fn, *args):
        with pytest.raises(AssertionError):
            fn(*args)

    k = next(iter(G.DET[40]))
    G.DET[40][k] += Fraction(1, 10 ** 6)
    try:
        rejects(test_detracer_rows_and_p2m_terms_match_oracle_p2m)
    finally:
        G.DET[40][k] -= Fraction(1, 10 ** 6)
    m2m = G.m2m_matrix
    monkeypatch.setattr(G, "m2m_matrix", lambda o: m2m(7 - o))
    rejects(test_m2m_octant_matrix_matches_oracle, 2)
    monkeypatch.setattr(G, "m2m_matrix", m2m)
    l2l = G.l2l_matrix

    def l2l_short(o):
        B = l2l(o)
        B[3] = {j: v for j, v in B[3].items() if G.rank(G.IND[j]) < P}
        return B

    monkeypatch.setattr(G, "l2l_matrix", l2l_short)
    rejects(test_l2l_octant_matrix_matches_oracle, 1)
    monkeypatch.setattr(G, "l2l_matrix", l2l)
    contraction = G.m2l_contraction

    def contraction_short():
        c = contraction()
        t = dict(c[(10, 20)])
        t.pop(next(iter(t)))
        c[(10, 20)] = t
        return c

    monkeypatch.setattr(G, "m2l_contraction", contraction_short)
    rejects(test_m2l_contraction_matches_oracle, (3.0, -1.0, 2.0))
    monkeypatch.setattr(G, "m2l_contraction", contraction)
    expand = G.expand
    monkeypatch.setattr(G, "expand", lambda m: {j: -v for j, v in expand(m).items()} if m == (1, 1, 2) else expand(m))
    rejects(test_expansion_of_dependent_components_matches_the_trace)
