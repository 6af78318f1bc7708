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


def _build_full(p, Lind):
    """The full coefficients as the kernels build them (the generated slot
    table, then the trace-condition passes), in FP64."""
    ind, passes = G.l2p_build_tables(p)
    C = [None] * len(G.l2p_horner_layout(p))
    for j, (slot, w) in enumerate(ind):
        C[slot] = float(w) * Lind[j]
    for ps in passes:
        for d, s1, s2, a, b in ps:
            assert C[s1] is not None and C[s2] is not None and C[d] is None
        for d, s1, s2, a, b in ps:
            C[d] = float(a) * C[s1] + float(b) * C[s2]
    assert all(c is not None for c in C)
    return C


def _horner_eval(p, Lind, r):
    """Run the generated nested-Horner L2P (its straight-line operations) on the
    full coefficients built as the kernels build them."""
    ops = G.l2p_horner_ops(p)
    C = _build_full(p, Lind)
    env = {"x": r[0], "y": r[1], "z": r[2]}
    val = lambda v: 0.0 if v is None else (C[v[1]] if isinstance(v, tuple) else env[v])
    for op in ops[:-1]:
        dst, acc, var, add = op
        env[dst] = (0.0 if acc is None else env[acc] * env[var]) + val(add)
    return [val(v) for v in ops[-1][1:]]


@pytest.mark.parametrize("p", [0, 1, 2, 5, 8, P])
def test_horner_l2p_matches_oracle_l2p(p):
    """The nested-Horner L2P (the full coefficients L_n / n! from the generated
    weights, then the generated Horner operations) gives the oracle's L2P
    potential and gradient (Eq. L2P) at points of the leaf, h = 1."""
    rng = np.random.default_rng(500 + p)
    xyz, q = _cluster(rng, (5.0, -4.0, 3.0), 0.5, 7)
    M = oracle.p2m(p, (5.0, -4.0, 3.0), xyz, q)
    Lfull = oracle.m2l(p, (-5.0, 4.0, -3.0), M)
    Lind = _oracle_ind(Lfull, p)
    for _ in range(4):
        r = rng.uniform(-0.5, 0.5, 3)
        phi, grad = oracle.l2p(p, r, Lfull)
        got = _horner_eval(p, Lind, r)
        _close(np.array(got), np.array([phi, *grad]), 1e-12)


def test_horner_layout_covers_each_full_component_once():
    """The Horner order visits every full component of rank <= p exactly once."""
    for p in range(P + 1):
        lay = G.l2p_horner_layout(p)
        assert len(lay) == len(set(lay)) == (p + 1) * (p + 2) * (p + 3) // 6
        assert all(G.rank(m) <= p for m in lay)


@pytest.mark.parametrize("p", [2, 7, P])
def test_trace_recursion_build_matches_the_direct_expansion(p):
    """The pass-by-pass build of the full coefficients (slot table plus trace
    condition) equals L_n / n! with L_n written directly through the
    independent components (expand), at every slot; each pass reads only slots
    written before it (checked inside the build)."""
    rng = np.random.default_rng(600 + p)
    Lind = rng.normal(size=(p + 1) ** 2)
    direct = np.array([sum(float(w) * Lind[j] for j, w in row.items()) for row in G.l2p_full_table(p)])
    _close(np.array(_build_full(p, Lind)), direct, 1e-13)


def test_planted_table_mistakes_are_caught(monkeypatch):
    """Each comparison above rejects a small mistake planted in the table it
    checks: one detracer coefficient off by 1e-6, the M2M matrix of the
    opposite octant, the L2L row of one component without its top-rank terms,
    one M2L contraction term dropped, a sign flipped in the expansion of a
    dependent component, one term dropped from a full coefficient of the
    Horner L2P, a sign flipped in its trace-condition build, and a y step of
    its Horner scheme taken in z."""
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
    monkeypatch.setattr(G, "expand", expand)
    table = G.l2p_full_table

    def table_short(p):
        t = table(p)
        k = G.l2p_horner_layout(p).index((0, 1, 4))
        t[k] = dict(list(t[k].items())[:-1])
        return t

    monkeypatch.setattr(G, "l2p_full_table", table_short)
    rejects(test_trace_recursion_build_matches_the_direct_expansion, 7)
    monkeypatch.setattr(G, "l2p_full_table", table)
    build = G.l2p_build_tables

    def build_wrong_beta(p):
        ind, passes = build(p)
        d, s1, s2, a, b = passes[1][3]
        passes[1][3] = (d, s1, s2, a, -b)
        return ind, passes

    monkeypatch.setattr(G, "l2p_build_tables", build_wrong_beta)
    rejects(test_horner_l2p_matches_oracle_l2p, 8)
    monkeypatch.setattr(G, "l2p_build_tables", build)
    ops = G.l2p_horner_ops

    def ops_swapped(p):
        o = ops(p)
        i = next(i for i, op in enumerate(o) if op[2] == "y" and op[1] is not None)
        dst, acc, var, add = o[i]
        o[i] = (dst, acc, "z", add)
        return o

    monkeypatch.setattr(G, "l2p_horner_ops", ops_swapped)
    rejects(test_horner_l2p_matches_oracle_l2p, 5)
