"""Pins for the FP64 oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own formulas.

Each ``pin_*`` function takes an oracle module (``oracle`` or a mutant built
from a patched copy of its source) and raises AssertionError when the oracle
disagrees.  ``tests/test_oracle_pins.py`` runs them on the real oracle;
``tests/test_oracle_mutants.py`` plants plausible mistakes in copies of the
oracle and checks that at least one pin fails for each.
"""
from __future__ import annotations

import functools
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


def rel(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


# --------------------------------------------------------------- helpers

def _trace_residual(o, p, A):
    """max over ranks n >= 2 and k (|k| = n-2) of |A_{k+2x}+A_{k+2y}+A_{k+2z}|,
    relative to max |A| of that rank (Appendix A: one-fold trace)."""
    mi = o.multi_indices(p)
    pos = {m: i for i, m in enumerate(mi)}
    worst = 0.0
    for n in range(2, p + 1):
        scale = max(abs(A[pos[m]]) for m in mi if sum(m) == n) or 1.0
        for k in mi:
            if sum(k) != n - 2:
                continue
            a, b, c = k
            t = A[pos[(a + 2, b, c)]] + A[pos[(a, b + 2, c)]] + A[pos[(a, b, c + 2)]]
            worst = max(worst, abs(t) / scale)
    return worst


def _contract(o, p, n, A, B):
    """n-fold contraction of the rank-n parts: sum_{|k|=n} n!/k! A_k B_k."""
    s = 0.0
    for i, k in enumerate(o.multi_indices(p)):
        if sum(k) == n:
            s += math.factorial(n) / (math.factorial(k[0]) * math.factorial(k[1]) * math.factorial(k[2])) * A[i] * B[i]
    return s


def _outer_powers(o, p, r):
    """the full polytensor r^n (all ranks <= p): component n is rx^a ry^b rz^c."""
    return np.array([r[0] ** a * r[1] ** b * r[2] ** c for (a, b, c) in o.multi_indices(p)])


@functools.lru_cache(maxsize=None)
def _sympy_grad_table(maxrank):
    import sympy as sp
    x, y, z = sp.symbols("x y z", real=True)
    f = 1 / sp.sqrt(x * x + y * y + z * z)
    table = {}
    for n in range(maxrank + 1):
        for a in range(n + 1):
            for b in range(n - a + 1):
                c = n - a - b
                e = f
                if a: e = sp.diff(e, x, a)
                if b: e = sp.diff(e, y, b)
                if c: e = sp.diff(e, z, c)
                table[(a, b, c)] = sp.lambdify((x, y, z), e, "math")
    return table


# --------------------------------------------------------------- pins

def pin_storage_table(o):
    """Appendix table of element counts: full storage C(p+3,3) and the
    (p+1)^2 independent traceless components (those with n_z <= 1)."""
    for row in _read_golden("storage_table.txt"):
        p, full_p, full_tot, tl_p, tl_tot, _ = (int(v) for v in row.split())
        assert o.nfull(p) == full_tot, (p, o.nfull(p), full_tot)
        mi = o.multi_indices(p)
        assert len(set(mi)) == full_tot
        assert sum(1 for m in mi if sum(m) == p) == full_p
        assert sum(1 for m in mi if m[2] <= 1) == tl_tot
        assert sum(1 for m in mi if m[2] <= 1 and sum(m) == p) == tl_p


def pin_dtensor_sympy(o):
    """D_k(r) = grad^k (1/r) (Eq. traceless grad) against SymPy's symbolic
    derivatives, every component of rank <= 5 plus all of rank 7."""
    table = _sympy_grad_table(7)
    rng = np.random.default_rng(11)
    for _ in range(3):
        r = rng.uniform(-2.0, 2.0, 3)
        r[0] += 2.5
        D = o.dtensor(7, r)
        for i, m in enumerate(o.multi_indices(7)):
            if sum(m) <= 5 or sum(m) == 7:
                ref = table[m](*r)
                scale = math.factorial(sum(m)) / np.linalg.norm(r) ** (sum(m) + 1)
                assert abs(D[i] - ref) <= 1e-12 * scale, (m, D[i], ref)


def pin_dtensor_excerpt(o):
    """Rank-2 diagonal of the traceless gradient as printed in the M2L
    optimisation example (Sec. 2.2)."""
    import sympy as sp
    x, y, z, h, u = sp.symbols("x y z h u")
    rng = np.random.default_rng(12)
    for _ in range(4):
        r = rng.uniform(-1.5, 1.5, 3)
        hv = float(r @ r); uv = hv ** -0.5
        D = o.dtensor(2, r)
        for row in _read_golden("dtensor_rank2_excerpt.txt"):
            lhs, rhs = row.split("=")
            idx = tuple(int(v) for v in lhs.split())
            val = float(sp.sympify(rhs).subs({x: r[0], y: r[1], z: r[2], h: hv, u: uv}))
            assert abs(D[o.full_index(*idx)] - val) <= 1e-13 * abs(uv ** 3) * 3, (idx, val)


def pin_detracer_invariants(o):
    """Appendix A: D[A] is traceless, D D = D, T T = (2n-1)!! T, and the
    detracer exchange theorem A.n.T[B] = T[A].n.B, on random symmetric A, B."""
    p = 6
    rng = np.random.default_rng(13)
    A = rng.standard_normal(o.nfull(p))
    B = rng.standard_normal(o.nfull(p))
    DA = o.detracer_D(p, A)
    assert _trace_residual(o, p, DA) < 1e-13
    assert rel(o.detracer_D(p, DA), DA) < 1e-13
    TA = o.detracer_T(p, A)
    TTA = o.detracer_T(p, TA)
    mi = o.multi_indices(p)
    dfact = [1.0] * (2 * p + 2)
    for n in range(p + 1):
        f = 1.0
        for i in range(2 * n - 1, 1, -2):
            f *= i
        dfact[n] = f
    for i, m in enumerate(mi):
        n = sum(m)
        assert abs(TTA[i] - dfact[n] * TA[i]) <= 1e-11 * max(1.0, abs(dfact[n] * TA[i]))
    TB = o.detracer_T(p, B)
    for n in range(p + 1):
        l = _contract(o, p, n, A, TB)
        r = _contract(o, p, n, TA, B)
        assert abs(l - r) <= 1e-11 * max(1.0, abs(l)), (n, l, r)
    # a traceless input is a fixed point of D
    assert rel(o.detracer_D(p, o.detracer_D(p, B)), o.detracer_D(p, B)) < 1e-13


def pin_detracer_vs_gradient(o):
    """Eq. traceless grad relates the general detracer (Eq. Detracer) applied
    to the polytensor r^n and the derivatives of 1/r:
    T[r^n]_n = (-1)^n r^(2n+1) grad^n r^-1, with the derivatives from SymPy."""
    p = 6
    table = _sympy_grad_table(p)
    r = np.array([0.7, -1.1, 0.4])
    T = o.detracer_T(p, _outer_powers(o, p, r))
    rn = np.linalg.norm(r)
    for i, m in enumerate(o.multi_indices(p)):
        n = sum(m)
        ref = (-1) ** n * rn ** (2 * n + 1) * table[m](*r)
        assert abs(T[i] - ref) <= 1e-11 * max(1.0, abs(ref)), (m, T[i], ref)


def pin_m2l_listing(o):
    """The printed symbolic L_x of M2L at p = 3 (Sec. 2.2): exactly the listed
    terms with weights 1/m!, nothing else."""
    p = 3
    terms = {}
    for row in _read_golden("m2l_Lx_p3.txt"):
        v = row.split()
        m = tuple(int(t) for t in v[0:3]); k = tuple(int(t) for t in v[3:6])
        terms[m] = (k, float(v[6]))
    mi = o.multi_indices(p)
    lx = o.full_index(1, 0, 0)
    rng = np.random.default_rng(14)
    D = rng.standard_normal(o.nfull(p))
    for j, m in enumerate(mi):
        M = np.zeros(o.nfull(p)); M[j] = 1.0
        L = o.m2l_with_D(p, M, D)
        if m in terms:
            k, w = terms[m]
            assert abs(L[lx] - w * D[o.full_index(*k)]) < 1e-15, (m, L[lx])
        else:
            assert L[lx] == 0.0, m


def pin_single_particle_at_centre(o):
    """A charge at the expansion centre has M = q delta_{n,0}; its M2L is then
    L_n = q grad^n(1/r) exactly (SymPy derivatives)."""
    p = 6
    q = 1.7
    z = np.array([0.3, 0.2, 0.9])
    M = o.p2m(p, z, z[None, :], np.array([q]))
    e0 = np.zeros(o.nfull(p)); e0[0] = q
    assert rel(M, e0) < 1e-15
    r = np.array([2.1, -0.4, 1.3])
    L = o.m2l(p, r, M)
    table = _sympy_grad_table(p)
    for i, m in enumerate(o.multi_indices(p)):
        ref = q * table[m](*r)
        assert abs(L[i] - ref) <= 1e-12 * max(1e-3, abs(ref)), (m, L[i], ref)


def _cluster_case(o, p):
    rng = np.random.default_rng(15)
    src = rng.random((20, 3)) * 0.5
    zA = np.array([0.25, 0.25, 0.25])
    q = rng.uniform(0.5, 1.5, 20)
    zB = np.array([1.25, 0.25, 0.25])
    xb = zB + np.array([0.05, -0.1, 0.12])
    M = o.p2m(p, zA, src, q)
    L = o.m2l(p, zB - zA, M)
    f, g = o.l2p(p, xb - zB, L)
    d = xb - src
    r = np.linalg.norm(d, axis=1)
    fe = float((q / r).sum())
    ge = -(q[:, None] * d / r[:, None] ** 3).sum(0)
    return abs(f - fe) / fe, rel(g, ge)


def pin_far_field_vs_direct(o):
    """P2M -> M2L -> L2P reproduces the brute-force sum over 20 sources, with
    the error falling as p grows (truncation of Eq. phi expansion)."""
    prev = None
    errs = []
    for p in (2, 4, 6, 8, 10):
        eP, eF = _cluster_case(o, p)
        errs.append((p, eP, eF))
        if prev is not None:
            assert eF < prev, errs
        prev = eF
    assert errs[0][2] < 0.2 and errs[-1][2] < 5e-4 and errs[-1][1] < 1e-5, errs


def pin_m2m_exact(o):
    """M2M(P2M at z) equals P2M at the shifted centre z' (the paper's own
    self-check, Sec. 2.2): the shift is exact."""
    p = 8
    rng = np.random.default_rng(16)
    x = rng.random((15, 3)) * 0.5
    q = rng.uniform(-1, 1, 15)
    z = np.array([0.25, 0.25, 0.25])
    zp = np.array([0.5, 0.5, 0.5])
    M = o.p2m(p, z, x, q)
    Ms = o.m2m(p, z - zp, M)
    Mref = o.p2m(p, zp, x, q)
    assert rel(Ms, Mref) < 1e-13, rel(Ms, Mref)


def pin_l2l_exact(o):
    """L2L is a Taylor shift of the degree-p local polynomial, so evaluating
    after the shift equals evaluating before it (Eq. L2L, Eq. L2P)."""
    p = 7
    rng = np.random.default_rng(17)
    L = rng.standard_normal(o.nfull(p))
    d = np.array([0.1, -0.2, 0.15])
    Ls = o.l2l(p, d, L)
    for _ in range(3):
        x = rng.uniform(-0.3, 0.3, 3)
        f0, g0 = o.l2p(p, x, L)
        f1, g1 = o.l2p(p, x - d, Ls)
        assert abs(f0 - f1) <= 1e-12 * max(1.0, abs(f0))
        assert rel(g1, g0) < 1e-12


def pin_traceless_outputs(o):
    """P2M, M2M, M2L and L2L outputs are totally traceless (Appendix B)."""
    p = 7
    rng = np.random.default_rng(18)
    x = rng.random((12, 3)) * 0.4
    q = rng.uniform(0.5, 1.5, 12)
    M = o.p2m(p, np.array([0.2, 0.2, 0.2]), x, q)
    assert _trace_residual(o, p, M) < 1e-13
    M2 = o.m2m(p, np.array([-0.2, -0.2, -0.2]), M)
    assert _trace_residual(o, p, M2) < 1e-13
    L = o.m2l(p, np.array([1.5, 0.5, -0.5]), M2)
    assert _trace_residual(o, p, L) < 1e-12
    L2 = o.l2l(p, np.array([0.1, 0.05, -0.1]), L)
    assert _trace_residual(o, p, L2) < 1e-12


def pin_laplace(o):
    """The local expansion's potential is harmonic: central differences of
    the L2P gradient give a Laplacian that is tiny next to its diagonal terms."""
    p = 8
    rng = np.random.default_rng(19)
    x = rng.random((10, 3)) * 0.5
    q = rng.uniform(0.5, 1.5, 10)
    M = o.p2m(p, np.array([0.25, 0.25, 0.25]), x, q)
    L = o.m2l(p, np.array([1.2, 0.3, 0.6]), M)
    h = 1e-4
    pt = np.array([0.05, -0.08, 0.1])
    lap = 0.0; diag = 0.0
    for i in range(3):
        e = np.zeros(3); e[i] = h
        gp = o.l2p(p, pt + e, L)[1][i]
        gm = o.l2p(p, pt - e, L)[1][i]
        d2 = (gp - gm) / (2 * h)
        lap += d2; diag += abs(d2)
    assert abs(lap) < 1e-6 * diag, (lap, diag)


def pin_direct_two_body(o):
    """Eq. PhiAB for two charges, with self pairs excluded and coincident
    pairs contributing nothing."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0], [0.3, 0.4, 0.0]])
    q = np.array([2.0, 3.0, 5.0])
    phi, grad = o.direct(xyz, q)
    d = 0.5
    assert abs(phi[0] - (3.0 + 5.0) / d) < 1e-14
    assert abs(phi[1] - 2.0 / d) < 1e-14 and abs(phi[2] - 2.0 / d) < 1e-14
    g1 = -2.0 * np.array([0.3, 0.4, 0.0]) / d ** 3
    assert rel(grad[1], g1) < 1e-14
    g0 = -(8.0) * np.array([-0.3, -0.4, 0.0]) / d ** 3
    assert rel(grad[0], g0) < 1e-14


def pin_fmm_shallow_is_direct(o):
    """With depth <= 1 every leaf is adjacent to every other, so the FMM is
    the near field alone and equals the direct sum."""
    rng = np.random.default_rng(20)
    xyz = rng.random((300, 3)); q = rng.uniform(-1, 1, 300)
    pd, gd = o.direct(xyz, q)
    for depth in (0, 1):
        pf, gf = o.fmm_uniform(xyz, q, 4, depth)
        assert rel(pf, pd) < 1e-13 and rel(gf, gd) < 1e-13


def pin_fmm_vs_direct_decay(o):
    """Full FMM (uniform octree, ws=1) against the O(N^2) sum: the relative
    errors fall monotonically with p and are at the truncation level."""
    from paper_1811_06332_amd.workloads import uniform_cube
    xyz, q = uniform_cube(1024, 21)
    pd, gd = o.direct(xyz, q)
    prev = None
    errs = []
    for p in (2, 4, 6, 8):
        pf, gf = o.fmm_uniform(xyz, q, p, 3)
        eP, eF = rel(pf, pd), rel(gf, gd)
        errs.append((p, eP, eF))
        if prev is not None:
            assert eF < prev[1] and eP < prev[0], errs
        prev = (eP, eF)
    assert errs[0][2] < 3e-2 and errs[-1][2] < 1e-3, errs


def pin_fmm_sampled(o):
    """Evaluating a sample of targets gives exactly the full run's values."""
    from paper_1811_06332_amd.workloads import uniform_cube
    xyz, q = uniform_cube(2000, 22)
    pf, gf = o.fmm_uniform(xyz, q, 5, 3)
    idx = np.array([3, 17, 999, 1500, 1999])
    ps, gs = o.fmm_uniform(xyz, q, 5, 3, targets=idx)
    assert np.array_equal(ps, pf[idx]) and np.array_equal(gs, gf[idx])


def pin_m2m_then_m2l(o):
    """M2L from a parent expansion obtained by M2M agrees with M2L from the
    child expansion up to truncation, with the gap shrinking as p grows."""
    rng = np.random.default_rng(23)
    x = rng.random((16, 3)) * 0.25 + 0.25  # inside the child [0.25,0.5)^3
    q = rng.uniform(0.5, 1.5, 16)
    zc = np.array([0.375, 0.375, 0.375]); zp = np.array([0.5, 0.5, 0.5])
    zB = np.array([2.5, 0.5, 0.5])
    prev = None
    for p in (4, 8, 12):
        Mc = o.p2m(p, zc, x, q)
        Mp = o.m2m(p, zc - zp, Mc)
        L1 = o.m2l(p, zB - zc, Mc)
        L2 = o.m2l(p, zB - zp, Mp)
        f1, g1 = o.l2p(p, np.zeros(3), L1)
        f2, g2 = o.l2p(p, np.zeros(3), L2)
        e = rel(g2, g1)
        if prev is not None:
            assert e < prev, (p, e, prev)
        prev = e
    assert prev < 1e-6


def pin_fmm_expansion_centres(o):
    """Expansions sit at the geometric cell centres (Appendix C): a charge
    placed at the centre of its leaf gives that leaf M = q delta_{n,0}, and
    its parent's M equals a P2M about the parent's geometric centre."""
    depth, p = 3, 4
    h = 1.0 / 2 ** depth
    leaves = [(1, 2, 3), (6, 5, 0)]
    xyz = np.array([[(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h] for (i, j, k) in leaves])
    q = np.array([1.5, -0.75])
    _, _, Ms, _ = o.fmm_uniform(xyz, q, p, depth, dump=True)
    n1 = 2 ** depth
    for (i, j, k), x, qq in zip(leaves, xyz, q):
        M = Ms[depth][i + n1 * (j + n1 * k)]
        ref = np.zeros(o.nfull(p)); ref[o.full_index(0, 0, 0)] = qq
        assert rel(M, ref) < 1e-14, (i, j, k)
        I, J, K = i // 2, j // 2, k // 2
        zp = np.array([(I + 0.5) * 2 * h, (J + 0.5) * 2 * h, (K + 0.5) * 2 * h])
        Mp = Ms[depth - 1][I + (n1 // 2) * (J + (n1 // 2) * K)]
        assert rel(Mp, o.p2m(p, zp, x[None, :], np.array([qq]))) < 1e-13


def _lattice_cube(depth, per_leaf, seed):
    """per_leaf random particles inside every leaf of a uniform depth-`depth` grid"""
    rng = np.random.default_rng(seed)
    n1 = 2 ** depth
    cells = np.array([(i, j, k) for k in range(n1) for j in range(n1) for i in range(n1)], float)
    xyz = ((cells[:, None, :] + rng.random((len(cells), per_leaf, 3))) / n1).reshape(-1, 3)
    return xyz, rng.uniform(-1, 1, len(xyz))


def pin_adaptive_equals_uniform_when_tree_is_uniform(o):
    """With exactly leaf_max particles in every depth-3 cell the adaptive tree
    is the uniform depth-3 octree: its V/U lists are the ws=1 lists (counts
    checked by brute force over cell pairs), W and X are empty, and the
    result equals the uniform FMM."""
    xyz, q = _lattice_cube(3, 8, 31)
    pa, ga, info = o.fmm_adaptive(xyz, q, 5, 8, lo=(0.0, 0.0, 0.0), side=1.0, stats=True)
    pu, gu = o.fmm_uniform(xyz, q, 5, 3)
    assert rel(pa, pu) < 1e-13 and rel(ga, gu) < 1e-13
    cnt_v = 0
    for l in (2, 3):
        n1 = 2 ** l
        cells = [(i, j, k) for i in range(n1) for j in range(n1) for k in range(n1)]
        for a in cells:
            for b in cells:
                par_adj = max(abs(a[d] // 2 - b[d] // 2) for d in range(3)) <= 1
                adj = max(abs(a[d] - b[d]) for d in range(3)) <= 1
                cnt_v += par_adj and not adj
    n1 = 8
    cnt_u = sum(1 for a in range(n1 ** 3) for b in range(n1 ** 3)
                if max(abs((a >> 0) % 8 - (b >> 0) % 8), abs((a // 8) % 8 - (b // 8) % 8), abs(a // 64 - b // 64)) <= 1)
    assert info["V"] == cnt_v and info["U"] == cnt_u and info["W"] == 0 and info["X"] == 0, info
    assert info["leaves"] == 512 and info["max_level"] == 3


def pin_adaptive_vs_direct_decay(o):
    """Adaptive FMM (U, V, W, X lists) on a Plummer sphere against the O(N^2)
    sum: the W and X lists are exercised and the errors fall with p."""
    from paper_1811_06332_amd.workloads import plummer
    xyz, q = plummer(2500, 41)
    pd, gd = o.direct(xyz, q)
    prev = None
    errs = []
    for p in (2, 4, 6, 8):
        pa, ga, info = o.fmm_adaptive(xyz, q, p, 24, stats=True)
        eP, eF = rel(pa, pd), rel(ga, gd)
        errs.append((p, eP, eF))
        if prev is not None:
            assert eF < prev[1] and eP < prev[0], errs
        prev = (eP, eF)
    assert info["W"] > 0 and info["X"] > 0 and info["max_level"] >= 5, info
    assert errs[0][2] < 0.1 and errs[-1][2] < 1e-3, errs


def pin_adaptive_two_density(o):
    """A dense small cluster beside a sparse background (leaves at very
    different levels, large W and X lists): the adaptive FMM stays at the
    truncation level against the direct sum."""
    rng = np.random.default_rng(43)
    xyz = np.vstack([rng.random((600, 3)), 0.41 + 0.03 * rng.random((900, 3))])
    q = rng.uniform(0.5, 1.5, len(xyz))
    pd, gd = o.direct(xyz, q)
    pa, ga, info = o.fmm_adaptive(xyz, q, 8, 12, stats=True)
    assert info["W"] > 0 and info["X"] > 0
    assert rel(pa, pd) < 1e-4 and rel(ga, gd) < 2e-3, (rel(pa, pd), rel(ga, gd), info)


def pin_order_table(o):
    """M2L orders per offset class (|v|^2) in the adaptive FMM: the table that
    keeps order p everywhere reproduces the fixed-order FMM bit for bit; the
    error against the direct sum grows as the table's order falls; lowering
    only the farthest class (|v|^2 = 27) costs less accuracy than lowering
    only the nearest (|v|^2 = 4), since the expansion converges faster with
    distance."""
    from paper_1811_06332_amd.workloads import plummer
    xyz, q = plummer(1500, 44)
    p = 8
    pf, gf = o.fmm_adaptive(xyz, q, p, 16)
    full = np.full(28, p, dtype=np.int32)
    pt, gt = o.fmm_adaptive(xyz, q, p, 16, order_r2=full)
    assert np.array_equal(pf, pt) and np.array_equal(gf, gt)
    pd, gd = o.direct(xyz, q)
    errs = []
    for pp in (2, 4, 6):
        pt, gt = o.fmm_adaptive(xyz, q, p, 16, order_r2=np.full(28, pp, dtype=np.int32))
        errs.append(rel(gt, gd))
    assert errs[0] > errs[1] > errs[2] > rel(gf, gd), errs
    far = full.copy(); far[27] = 2
    near = full.copy(); near[4] = 2
    _, gfar = o.fmm_adaptive(xyz, q, p, 16, order_r2=far)
    _, gnear = o.fmm_adaptive(xyz, q, p, 16, order_r2=near)
    assert 0.0 < rel(gfar, gf) < rel(gnear, gf), (rel(gfar, gf), rel(gnear, gf))
    # class membership: |v|^2 of a ws=1 pair is a sum of three squares of
    # integers in [-3, 3] with at least one of magnitude >= 2; lowering one
    # such class alone changes the result, lowering an empty class does not
    occupied = sorted({a * a + b * b + c * c for a in range(4) for b in range(4) for c in range(4)
                       if max(a, b, c) >= 2})
    assert occupied == [4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 17, 18, 19, 22, 27]
    for k in range(4, 28):
        tab = full.copy(); tab[k] = p - 2
        _, gk = o.fmm_adaptive(xyz, q, p, 16, order_r2=tab)
        if k in occupied:
            assert rel(gk, gf) > 1e-14, k
        else:
            assert np.array_equal(gk, gf), k


def pin_auto_root_hand_boxes(o):
    """The automatic root cube on boxes worked out by hand: centred on the
    bounding box, side = largest extent * (1 + 2^-20), side 1 when all
    points coincide; every point then lies strictly inside the cube."""
    # extents (4, 1, 0.5): side 4 (1 + 2^-20) = 4.000003814697265625, centre (1, 0.5, 2.25)
    lo, side = o.auto_root(np.array([[-1.0, 0.0, 2.0], [3.0, 1.0, 2.5], [0.0, 0.25, 2.1]]))
    assert side == 4.000003814697265625
    assert tuple(lo) == (-1.0000019073486328125, -1.5000019073486328125, 0.2499980926513671875)
    # extents (0, 0, 6): the z extent decides; the cube is centred on (7, -3, 0)
    lo, side = o.auto_root(np.array([[7.0, -3.0, -3.0], [7.0, -3.0, 3.0]]))
    assert side == 6.00000572204589843750
    assert tuple(lo) == (3.99999713897705078125, -6.00000286102294921875, -3.00000286102294921875)
    # all points on one spot: side 1 (1 + 2^-20) around it
    lo, side = o.auto_root(np.array([[0.5, 0.5, 0.5]] * 3))
    assert side == 1.00000095367431640625 and tuple(lo) == (-0.000000476837158203125,) * 3
    from paper_1811_06332_amd.workloads import plummer
    xyz, _ = plummer(3000, 45)
    lo, side = o.auto_root(xyz)
    assert np.all(xyz > lo) and np.all(xyz < lo + side)


def _tree_by_definition(xyz, leaf_max):
    """The adaptive tree built from its definition (not the oracle's code):
    cells at level l are the 2^l-grid cells of the root cube; a cell is a
    node if it holds a particle and its parent is a node holding more than
    leaf_max particles (down to level 21).  Returns {(l, ix, iy, iz):
    (sorted particle indices, leaf)} and the root box."""
    mn, mx = xyz.min(0), xyz.max(0)
    side = float((mx - mn).max())
    side = (side if side > 0 else 1.0) * (1.0 + 2.0 ** -20)
    lo = (mn + mx) * 0.5 - side * 0.5
    D = 21
    c = np.clip(np.floor((xyz - lo) / side * 2.0 ** D), 0, 2 ** D - 1).astype(np.int64)
    nodes = {}
    todo = [(0, (0, 0, 0), np.arange(len(xyz)))]
    while todo:
        l, (i, j, k), idx = todo.pop()
        leaf = len(idx) <= leaf_max or l >= D
        nodes[(l, i, j, k)] = (np.sort(idx), leaf)
        if not leaf:
            sub = c[idx] >> (D - l - 1)
            for ch in {tuple(r) for r in sub}:
                todo.append((l + 1, ch, idx[np.all(sub == ch, axis=1)]))
    return nodes, lo, side


def _lists_by_definition(nodes):
    """U, V, W, X of every node by brute force over node pairs:
    V(B): same-level cells not adjacent to B whose parents are adjacent or equal;
    U(B), B a leaf: the leaves whose closed cubes touch B's (B included);
    W(B), B a leaf: finer cells not adjacent to B whose parent is adjacent to B;
    X(B): the cells C with B in W(C)."""
    D = 21
    keys = list(nodes)

    def span(n):
        l, i, j, k = n
        s = 1 << (D - l)
        return [(i * s, (i + 1) * s), (j * s, (j + 1) * s), (k * s, (k + 1) * s)]

    def touch(a, b):
        return all(x0 <= y1 and y0 <= x1 for (x0, x1), (y0, y1) in zip(span(a), span(b)))

    def parent(n):
        l, i, j, k = n
        return (l - 1, i >> 1, j >> 1, k >> 1)

    U, V, W = {n: set() for n in keys}, {n: set() for n in keys}, {n: set() for n in keys}
    for b in keys:
        leaf_b = nodes[b][1]
        for a in keys:
            if a[0] == b[0] and b[0] >= 2 and touch(parent(a), parent(b)) and not touch(a, b):
                V[b].add(a)
            if leaf_b and nodes[a][1] and touch(a, b):
                U[b].add(a)
            if leaf_b and a[0] > b[0] and not touch(a, b) and touch(parent(a), b):
                W[b].add(a)
    X = {n: set() for n in keys}
    for b in keys:
        for a in W[b]:
            X[a].add(b)
    return U, V, W, X


def _decode_key(level, key):
    ix = iy = iz = 0
    for l in range(level):
        ix |= ((key >> (3 * l)) & 1) << l
        iy |= ((key >> (3 * l + 1)) & 1) << l
        iz |= ((key >> (3 * l + 2)) & 1) << l
    return (level, ix, iy, iz)


def pin_adaptive_tree_and_lists_by_definition(o):
    """The oracle's adaptive tree (nodes, leaves, parents, particles of every
    leaf) and every U/V/W/X list equal, entry by entry, the ones built from
    their definitions by brute force, on a cluster with leaves at several
    levels (W and X non-empty)."""
    from paper_1811_06332_amd.workloads import plummer
    for xyz, leaf_max in ((plummer(700, 46)[0], 6), (np.vstack([np.random.default_rng(47).random((200, 3)),
                                                                0.3 + 0.02 * np.random.default_rng(48).random((250, 3))]),
                                                     5)):
        nodes, lo, side = _tree_by_definition(xyz, leaf_max)
        U, V, W, X = _lists_by_definition(nodes)
        t = o.adaptive_tree(xyz, leaf_max)
        name = [_decode_key(int(l), int(k)) for l, k in zip(t["level"], t["key"])]
        assert sorted(name) == sorted(nodes)
        for i, nm in enumerate(name):
            idx, leaf = nodes[nm]
            assert bool(t["leaf"][i]) == leaf, nm
            par = int(t["parent"][i])
            assert (par < 0 and nm[0] == 0) or name[par] == (nm[0] - 1, nm[1] >> 1, nm[2] >> 1, nm[3] >> 1)
            got = np.sort(t["order"][t["pb"][i]:t["pe"][i]])
            assert np.array_equal(got, idx), nm
            for L, ref in (("U", U), ("V", V), ("W", W), ("X", X)):
                ent = t[L + "_list"][t[L + "_off"][i]:t[L + "_off"][i + 1]]
                assert len(ent) == len(set(ent.tolist())), (L, nm)
                assert {name[e] for e in ent} == ref[nm], (L, nm)
        assert sum(len(v) for v in W.values()) > 0 and max(n[0] for n in nodes) >= 4


def pin_pair_orders(o):
    """M2L orders given pair by pair: all at p reproduce the fixed order bit
    for bit, and the orders an |v|^2 table gives each V pair (worked out
    here from the exported tree) reproduce the table mode bit for bit."""
    from paper_1811_06332_amd.workloads import plummer
    xyz, q = plummer(1500, 49)
    p, leaf = 7, 16
    t = o.adaptive_tree(xyz, leaf)
    nv = int(t["V_off"][-1])
    pf, gf = o.fmm_adaptive(xyz, q, p, leaf)
    pa, ga = o.fmm_adaptive(xyz, q, p, leaf, v_orders=np.full(nv, p, dtype=np.int8))
    assert np.array_equal(pf, pa) and np.array_equal(gf, ga)
    tab = np.array([p] * 4 + [3, 0, 6, p, 2, 7, 1, 5, 4, 2, 3, p, p, 1, 6, 0, p, p, 5, p, p, p, p, 2], dtype=np.int32)
    coords = np.array([_decode_key(int(l), int(k))[1:] for l, k in zip(t["level"], t["key"])])
    tgt = np.repeat(np.arange(len(t["level"])), np.diff(t["V_off"]))
    d = coords[tgt] - coords[t["V_list"]]
    vo = tab[np.sum(d * d, axis=1)].astype(np.int8)
    pt, gt = o.fmm_adaptive(xyz, q, p, leaf, order_r2=tab)
    pv, gv = o.fmm_adaptive(xyz, q, p, leaf, v_orders=vo)
    assert np.array_equal(pt, pv) and np.array_equal(gt, gv)
    assert rel(gt, gf) > 1e-8


def _dipoles_as_charge_pairs(xyz, dip, eps):
    """Each point dipole p at x as charges +s at x + d/2 and -s at x - d/2
    with d = eps p/|p| and s = |p|/eps (s d = p): the definition of a point
    dipole in the limit eps -> 0 (Appendix B.1)."""
    norm = np.linalg.norm(dip, axis=1, keepdims=True)
    d = eps * dip / norm
    return np.vstack([xyz + d / 2, xyz - d / 2]), np.concatenate([norm[:, 0] / eps, -norm[:, 0] / eps])


def pin_dipole_direct_is_charge_pair_limit(o):
    """The direct sum over point dipoles equals that over the charge pairs
    they are the limit of, to O(eps^2)."""
    rng = np.random.default_rng(50)
    tgt = rng.random((40, 3))
    xd, dip = rng.random((30, 3)), rng.normal(size=(30, 3))
    n_t = len(tgt)
    pd, gd = o.direct_dipoles(np.vstack([tgt, xd]), np.zeros(n_t + 30), np.vstack([np.zeros((n_t, 3)), dip]),
                              targets=np.arange(n_t))
    errs = []
    for eps in (1e-3, 1e-4):
        xc, qc = _dipoles_as_charge_pairs(xd, dip, eps)
        pc, gc = o.direct(np.vstack([tgt, xc]), np.concatenate([np.zeros(n_t), qc]), targets=np.arange(n_t))
        errs.append((rel(pd, pc), rel(gd, gc)))
    assert errs[1][0] < 1e-5 and errs[1][1] < 1e-5, errs
    assert errs[1][0] < 0.02 * errs[0][0] and errs[1][1] < 0.02 * errs[0][1], errs  # second order


def pin_dipole_p2m_is_charge_pair_limit(o):
    """The multipole of point dipoles (a pure dipole moved by M2M) equals the
    P2M of the charge pairs they are the limit of, to O(eps^2), and its
    expansion reproduces the direct dipole field far away, better with p."""
    rng = np.random.default_rng(51)
    z = np.array([0.5, 0.5, 0.5])
    xd, dip = 0.5 + 0.3 * (rng.random((12, 3)) - 0.5), rng.normal(size=(12, 3))
    for p in (1, 4, 7):
        M = o.p2m_dipole(p, z, xd, dip)
        errs = []
        for eps in (1e-2, 1e-3):
            xc, qc = _dipoles_as_charge_pairs(xd, dip, eps)
            errs.append(rel(M, o.p2m(p, z, xc, qc)))
        # second order in eps (exact at p = 1: a charge pair has no rank-1 error)
        assert errs[1] < 1e-5 and (errs[0] < 1e-10 or errs[1] < 0.05 * errs[0]), (p, errs)
    tgt = np.array([[3.2, -1.7, 2.9], [-2.5, 3.1, 0.4]])
    pd, gd = o.direct_dipoles(np.vstack([tgt, xd]), np.zeros(14), np.vstack([np.zeros((2, 3)), dip]),
                              targets=np.arange(2))
    prev = None
    for p in (2, 4, 6, 8):
        M = o.p2m_dipole(p, z, xd, dip)
        got = []
        for t in tgt:
            L = o.m2l(p, t - z, M)
            f, g = o.l2p(p, np.zeros(3), L)
            got.append((f, g))
        e = rel([f for f, _ in got], pd) + rel([g for _, g in got], gd)
        assert prev is None or e < prev, (p, e, prev)
        prev = e
    assert prev < 1e-6


def pin_dipole_fmm_vs_direct_decay(o):
    """The uniform FMM with charges and point dipoles against the direct sum:
    the errors fall with p."""
    rng = np.random.default_rng(52)
    xyz = rng.random((400, 3))
    q, dip = rng.uniform(-1, 1, 400), 0.01 * rng.normal(size=(400, 3))
    pd, gd = o.direct_dipoles(xyz, q, dip)
    errs = []
    for p in (2, 4, 6, 8):
        pf, gf = o.fmm_uniform_dipoles(xyz, q, dip, p, 3)
        errs.append((rel(pf, pd), rel(gf, gd)))
    for a, b in zip(errs, errs[1:]):
        assert b[0] < a[0] and b[1] < a[1], errs
    assert errs[-1][1] < 1e-3, errs
    # dipoles matter: without them the result is far off
    pc, gc = o.fmm_uniform(xyz, q, 8, 3)
    assert rel(gc, gd) > 100 * errs[-1][1]


# ------------------------------------------------------------ dual-tree traversal with the theta MAC

def _dual_case(seed, n=600):
    """a Plummer sphere (leaves at several levels)"""
    from paper_1811_06332_amd.workloads import plummer
    xyz, q = plummer(n, seed)
    return xyz, q


def pin_dual_theta0_is_direct(o):
    """theta = 0 accepts no pair: every centre mode gives the direct sum."""
    xyz, q = _dual_case(60, 500)
    pd, gd = o.direct(xyz, q)
    for centre in ("geometric", "mass", "ap"):
        pf, gf, info = o.fmm_dual(xyz, q, 6, 8, 0.0, centre, stats=True)
        assert info["m2l_pairs"] == 0
        assert rel(gf, gd) < 1e-13, centre
        if centre != "ap":
            assert rel(pf, pd) < 1e-13, centre


def pin_dual_vs_direct_decay(o):
    """The error against the direct sum falls with p at fixed theta and with
    theta at fixed p, in every centre mode."""
    xyz, q = _dual_case(61, 1500)
    pd, gd = o.direct(xyz, q)
    for centre in ("geometric", "mass", "ap"):
        errs = []
        for p in (2, 4, 6, 8):
            pf, gf = o.fmm_dual(xyz, q, p, 12, 0.5, centre)
            errs.append(rel(gf, gd) + (rel(pf, pd) if pf is not None else 0.0))
        assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), (centre, errs)
        assert errs[-1] < 3e-4, (centre, errs)
        et = [rel(o.fmm_dual(xyz, q, 4, 12, th, centre)[1], gd) for th in (0.3, 0.5, 0.7)]
        assert et[0] < et[1] < et[2], (centre, et)


def pin_dual_momentum_conserved(o):
    """Mutual interactions: the total force sum_b q_b grad phi_b vanishes to
    rounding (Newton's third law), while a single one-way translation would
    leave an error of the size of the truncation error."""
    xyz, q = _dual_case(62, 1200)
    pd, gd = o.direct(xyz, q)
    for centre in ("geometric", "mass", "ap"):
        for p in (2, 5):
            _, gf = o.fmm_dual(xyz, q, p, 10, 0.7, centre)
            f = q[:, None] * gf
            assert np.abs(f.sum(0)).max() < 1e-13 * np.abs(f).sum(), (centre, p)
            assert rel(gf, gd) > 1e-6  # the expansions are really used


def _dual_by_definition(o, xyz, q, theta, centre, t):
    """Centres, radii and the dual-tree traversal written out here from the
    definitions (numpy centres, recursion in Python) on the exported tree."""
    nn = len(t["level"])
    lo, side = o.auto_root(xyz)
    lo = np.asarray(lo, dtype=np.float64)
    zr = np.zeros((nn, 4))
    child = [[] for _ in range(nn)]
    for i in range(nn):
        par = int(t["parent"][i])
        if par >= 0:
            child[par].append(i)
    for i in range(nn):
        idx = t["order"][t["pb"][i]:t["pe"][i]]
        l, ix, iy, iz = _decode_key(int(t["level"][i]), int(t["key"][i]))
        h = side / 2.0 ** l
        z = lo + (np.array([ix, iy, iz]) + 0.5) * h
        if centre != "geometric" and q[idx].sum() > 0:
            z = (q[idx, None] * xyz[idx]).sum(0) / q[idx].sum()
        zr[i, :3] = z
        zr[i, 3] = np.sqrt(((xyz[idx] - z) ** 2).sum(1)).max()
    key = {i: _decode_key(int(t["level"][i]), int(t["key"][i])) for i in range(nn)}
    for i in range(nn):  # children in octant order
        child[i].sort(key=lambda c: (key[c][1] & 1) | ((key[c][2] & 1) << 1) | ((key[c][3] & 1) << 2))
    leaf = t["leaf"].astype(bool)
    m2l, p2p = [], {i: [] for i in range(nn)}

    def walk(a, b):
        if a == b:
            if leaf[a]:
                p2p[a].append(a)
                return
            for x, ca in enumerate(child[a]):
                for cb in child[a][x:]:
                    walk(ca, cb)
            return
        d = np.sqrt(((zr[b, :3] - zr[a, :3]) ** 2).sum())
        if theta * d > zr[a, 3] + zr[b, 3]:
            m2l.append((a, b))
            return
        if leaf[a] and leaf[b]:
            p2p[a].append(b)
            p2p[b].append(a)
            return
        if not leaf[a] and (leaf[b] or zr[a, 3] >= zr[b, 3]):
            for c in child[a]:
                walk(c, b)
        else:
            for c in child[b]:
                walk(a, c)

    walk(0, 0)
    return zr, m2l, p2p


def pin_dual_traversal_by_definition(o):
    """The oracle's centres, radii, accepted pairs and direct pairs equal the
    ones worked out here from the definitions (same order), every accepted
    pair passes the MAC and every direct pair fails it, and together they
    cover every ordered particle pair exactly once."""
    for seed, n, leaf_max, theta in ((63, 400, 6, 0.5), (64, 300, 4, 0.8)):
        xyz, q = _dual_case(seed, n)
        for centre in ("geometric", "mass", "ap"):
            t = o.adaptive_tree(xyz, leaf_max)
            got = o.dual_pairs(xyz, q, leaf_max, theta, centre)
            zr, m2l, p2p = _dual_by_definition(o, xyz, q, theta, centre, t)
            assert np.allclose(got["zr"], zr, rtol=1e-14, atol=1e-14), centre
            assert [tuple(r) for r in got["m2l"].tolist()] == m2l, centre
            ref = [(i, c) for i in range(len(zr)) for c in p2p[i]]
            assert [tuple(r) for r in got["p2p"].tolist()] == ref, centre
            cover = np.zeros((n, n), dtype=np.int32)
            parts = [t["order"][t["pb"][i]:t["pe"][i]] for i in range(len(zr))]
            for a, b in m2l:
                cover[np.ix_(parts[b], parts[a])] += 1
                cover[np.ix_(parts[a], parts[b])] += 1
            for b, c in ref:
                cover[np.ix_(parts[b], parts[c])] += 1
            assert np.all(cover == 1), centre
            assert len(m2l) > 50, centre


def pin_dual_ap_is_centre_of_mass_ft(o):
    """About the centre of mass the dipole of positive charges vanishes, so
    the AP variant (dipole dropped, gradient only) gives the gradient of the
    fully traceless expansion about the same centres to rounding."""
    xyz, q = _dual_case(65, 1000)
    z = (q[:, None] * xyz).sum(0) / q.sum()
    M = o.p2m(4, z, xyz, q)
    assert np.abs(M[1:4]).max() < 1e-14 * np.abs(M).max()
    for p in (1, 3, 6):
        _, gm = o.fmm_dual(xyz, q, p, 8, 0.6, "mass")
        _, ga = o.fmm_dual(xyz, q, p, 8, 0.6, "ap")
        assert rel(ga, gm) < 1e-12, p


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
