"""Operator generator for the GPU path (build time only).

Builds the Cartesian traceless FMM operators of Coles & Bieri (arXiv
1811.06332, Sec. 2 and Appendices A-B) in exact rational arithmetic, reduces
them to the independent traceless components, and emits HIP source:

  * the independent basis: the (p+1)^2 components with n_z in {0,1} of each
    traceless polytensor (Appendix B: dependent elements follow from the
    trace, e.g. A_zz = -A_xx - A_yy);
  * the expansion of every full component into independent ones;
  * P2M per particle in the compact form of Eq. (Detracer3):
    D[u^n]_n = sum_m f_{n,m}/(2n-1)!! |u|^{2m} u^{n-2m}, u = -(x - z)/h;
  * M2M (Eq. M2M) and L2L (Eq. L2L) for the eight octant shifts of an
    octree, in scaled variables M~_n = M_n / h^|n|, L~_n = L_n h^(|n|+1);
    with those scalings the shift is a constant rational matrix per octant;
  * the M2L contraction (Eq. M2L) reduced to independent components:
    L~_n = sum_j K_v[n,j] M~_j with K_v[n,j] = sum_i c[n,j,i] D_i(v),
    D_i the independent components of the traceless gradient at v;
  * straight-line, common-subexpression-eliminated code for the traceless
    gradient D_k(r) = (-1)^k r^{-2k-1} T[r^k]_k (Eq. traceless grad with
    Eq. Detracer3), optimised as the paper's second stage does: constants
    factored, CSE over all components of the operator together and iterated
    until it stops improving, powers expanded into products, rationals
    turned into floating-point literals.

Usage: python gen_operators.py OUTDIR   (writes ctfmm_gen.h)
"""
from __future__ import annotations

import os
import sys
from fractions import Fraction
from math import comb, factorial

PMAX = 10


# ------------------------------------------------------------------ indices

def ind_list(p=PMAX):
    """independent components, ordered by rank, then n_z, then n_x descending"""
    out = []
    for n in range(p + 1):
        for a in range(n, -1, -1):
            out.append((a, n - a, 0))
        for a in range(n - 1, -1, -1):
            out.append((a, n - 1 - a, 1))
    return out


def full_list(p=PMAX):
    out = []
    for n in range(p + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


IND = ind_list()
FULL = full_list()
IND_POS = {m: i for i, m in enumerate(IND)}
FULL_POS = {m: i for i, m in enumerate(FULL)}


def rank(m):
    return m[0] + m[1] + m[2]


def mfact(m):
    return factorial(m[0]) * factorial(m[1]) * factorial(m[2])


def dfact(n):
    f = 1
    for i in range(n, 1, -2):
        f *= i
    return f


def expand(m):
    """full component m of a traceless tensor as {independent slot: int coef}.
    With c = 2s + t: A_{a,b,c} = (-1)^s sum_i C(s,i) A_{a+2i, b+2(s-i), t}."""
    a, b, c = m
    s, t = divmod(c, 2)
    out = {}
    for i in range(s + 1):
        key = IND_POS[(a + 2 * i, b + 2 * (s - i), t)]
        out[key] = out.get(key, 0) + (-1) ** s * comb(s, i)
    return out


def f_nm(n, m):
    """f_{n,m} = (-1)^|m| (2|n|-2|m|-1)!! n! / (2^|m| m! (n-2m)!)  (Appendix A)"""
    N, M = rank(n), rank(m)
    return Fraction((-1) ** M * dfact(2 * N - 2 * M - 1) * mfact(n),
                    2 ** M * mfact(m) * mfact((n[0] - 2 * m[0], n[1] - 2 * m[1], n[2] - 2 * m[2])))


def detracer_rows():
    """D[A]_n for independent n as {full slot: Fraction} (Eq. Detracer / (2n-1)!!)."""
    rows = []
    for n in IND:
        N = rank(n)
        row = {}
        for m1 in range(n[0] // 2 + 1):
            for m2 in range(n[1] // 2 + 1):
                for m3 in range(n[2] // 2 + 1):
                    m = (m1, m2, m3)
                    M = rank(m)
                    fv = f_nm(n, m)
                    for k1 in range(M + 1):
                        for k2 in range(M - k1 + 1):
                            k = (k1, k2, M - k1 - k2)
                            idx = (n[0] - 2 * m1 + 2 * k[0], n[1] - 2 * m2 + 2 * k[1], n[2] - 2 * m3 + 2 * k[2])
                            w = fv * Fraction(factorial(M), mfact(k)) / dfact(2 * N - 1)
                            key = FULL_POS[idx]
                            row[key] = row.get(key, 0) + w
        rows.append({k: v for k, v in row.items() if v != 0})
    return rows


def p2m_terms():
    """per independent n: [(coef, ex, ey, ez, e_r2)] with
    D[u^n]_n = sum coef * ux^ex uy^ey uz^ez |u|^(2 e_r2)  (Eq. Detracer3)."""
    out = []
    for n in IND:
        N = rank(n)
        terms = []
        for m1 in range(n[0] // 2 + 1):
            for m2 in range(n[1] // 2 + 1):
                for m3 in range(n[2] // 2 + 1):
                    m = (m1, m2, m3)
                    c = f_nm(n, m) / dfact(2 * N - 1)
                    terms.append((c, n[0] - 2 * m1, n[1] - 2 * m2, n[2] - 2 * m3, rank(m)))
        out.append(terms)
    return out


def m2m_matrix(octant):
    """A_o[n][j]: parent M~_n = sum_o sum_j A_o[n][j] child_o M~_j.
    Child centre minus parent centre = (sigma/4) h_parent, sigma_d = 2 o_d - 1.
    M'_n/h_P^|n| = sum_{k<=n} C(n,k) (-sigma/4)^(n-k) 2^-|k| M~_k (full k),
    then the detracer (Eq. M2M, M2M part 2)."""
    sig = [2 * ((octant >> d) & 1) - 1 for d in range(3)]
    D = DET
    # shift: full n <- full k
    A = [dict() for _ in IND]
    for ni, n in enumerate(IND):
        for f, w in D[ni].items():
            nn = FULL[f]  # component of M' needed by the detracer
            for k1 in range(nn[0] + 1):
                for k2 in range(nn[1] + 1):
                    for k3 in range(nn[2] + 1):
                        k = (k1, k2, k3)
                        coef = Fraction(comb(nn[0], k1) * comb(nn[1], k2) * comb(nn[2], k3))
                        for d in range(3):
                            coef *= Fraction(-sig[d], 4) ** (nn[d] - k[d])
                        coef *= Fraction(1, 2 ** rank(k))
                        for j, e in expand(k).items():
                            A[ni][j] = A[ni].get(j, 0) + w * coef * e
    return [{j: v for j, v in row.items() if v != 0} for row in A]


def l2l_matrix(octant):
    """B_o[n][j]: child L~_n = sum_j B_o[n][j] parent L~_j (only rank(j) <= p
    is kept at order p).  delta = (sigma/4) h_P:
    L~c_n = 2^-(|n|+1) sum_k (sigma/4)^k / k! L~P_{n+k}  (Eq. L2L)."""
    sig = [2 * ((octant >> d) & 1) - 1 for d in range(3)]
    B = []
    for n in IND:
        row = {}
        N = rank(n)
        for K in range(PMAX - N + 1):
            for k1 in range(K + 1):
                for k2 in range(K - k1 + 1):
                    k = (k1, k2, K - k1 - k2)
                    coef = Fraction(1, mfact(k) * 2 ** (N + 1))
                    for d in range(3):
                        coef *= Fraction(sig[d], 4) ** k[d]
                    for j, e in expand((n[0] + k[0], n[1] + k[1], n[2] + k[2])).items():
                        row[j] = row.get(j, 0) + coef * e
        B.append({j: v for j, v in row.items() if v != 0})
    return B


def m2l_contraction():
    """c[(n, j)] = {i: coef} with K_v[n][j] = sum_i coef * D_i(v):
    sum over full m with |m| = |j| of E[m][j] E[n+m][i] / m!  (Eq. M2L)."""
    out = {}
    for ni, n in enumerate(IND):
        for ji, jm in enumerate(IND):
            if rank(n) + rank(jm) > PMAX:
                continue
            J = rank(jm)
            acc = {}
            for m1 in range(J + 1):
                for m2 in range(J - m1 + 1):
                    m = (m1, m2, J - m1 - m2)
                    e = expand(m).get(ji, 0)
                    if e == 0:
                        continue
                    for i, e2 in expand((n[0] + m[0], n[1] + m[1], n[2] + m[2])).items():
                        acc[i] = acc.get(i, 0) + Fraction(e * e2, mfact(m))
            acc = {i: v for i, v in acc.items() if v != 0}
            out[(ni, ji)] = acc
    return out


def m2l_pair_code(p, c):
    """Straight-line M2L for one pair at order p (Eq. M2L with the contraction
    c of m2l_contraction), for the outputs of ranks R0..R1 (template
    parameters): L[n - R0^2] += sum_j (sum_i c[n,j,i] D[i]) * Ms[j] * rp[|j|].
    Sources are taken rank by rank (j outer), so each multipole component is
    read once; with AP the rank-1 sources (the dipole) are left out."""
    out = []
    nterms = 0
    for ji, jm in enumerate(IND):
        J = rank(jm)
        if J > p:
            break
        body = []
        for ni, n in enumerate(IND):
            R = rank(n)
            if R + J > p:
                break
            terms = c.get((ni, ji), {})
            if not terms:
                continue
            expr = " + ".join(f"({float(v)!r}) * D[{i}]" for i, v in sorted(terms.items()))
            body.append(f"  if constexpr (R0 <= {R} && {R} <= R1) L[{ni} - R0 * R0] += ({expr}) * m;")
            nterms += len(terms)
        if not body:
            continue
        guard = f"R0 <= {p - J}" + (" && !AP" if J == 1 else "")
        out.append(f"if constexpr ({guard}) {{ const double m = Ms[{ji}] * rp[{J}];")
        out.extend(body)
        out.append("}")
    return out, nterms


DET = None


# ---------------------------------------------------------- straight-line D

def dtensor_code(p):
    """CSE'd straight-line FP64 code for the independent components of the
    traceless gradient of 1/r up to rank p.  Returns (code lines, flops opt,
    flops noopt)."""
    import sympy as sp
    x, y, z, u = sp.symbols("x y z u", real=True)  # u = 1/|r|
    h = x * x + y * y + z * z
    exprs = []
    for n in IND:
        N = rank(n)
        if N > p:
            break
        t = 0
        for m1 in range(n[0] // 2 + 1):
            for m2 in range(n[1] // 2 + 1):
                for m3 in range(n[2] // 2 + 1):
                    m = (m1, m2, m3)
                    fv = f_nm(n, m)
                    t += sp.Rational(fv.numerator, fv.denominator) * h ** rank(m) * \
                        x ** (n[0] - 2 * m1) * y ** (n[1] - 2 * m2) * z ** (n[2] - 2 * m3)
        exprs.append(sp.expand((-1) ** N * u ** (2 * N + 1) * t))
    noopt = sum(_count_ops(e) for e in exprs)
    # stage 2: CSE over all components together, iterated until no gain
    repl, red = sp.cse(exprs, symbols=sp.numbered_symbols("t"), optimizations="basic")
    best = _count_ops_cse(repl, red)
    for _ in range(6):
        allx = [e for _, e in repl] + list(red)
        repl2, red2 = sp.cse(allx, symbols=sp.numbered_symbols("s"), optimizations="basic")
        if not repl2:
            break
        # substitute back into a flat assignment list
        nrep = len(repl)
        tmp = [(s, v) for s, v in repl2]
        new_repl = tmp + [(repl[i][0], red2[i]) for i in range(nrep)]
        new_red = red2[nrep:]
        cost = _count_ops_cse(new_repl, new_red)
        if cost >= best:
            break
        repl, red, best = _toposort(new_repl), new_red, cost
    lines = []
    for s, v in repl:
        lines.append(f"const double {s} = {_c(v)};")
    for i, e in enumerate(red):
        lines.append(f"D[{i}] = {_c(e)};")
    return lines, best, noopt


def _toposort(assigns):
    """order (symbol, expr) assignments so every symbol is defined before use"""
    defined = {sym for sym, _ in assigns}
    deps = {sym: {f for f in expr.free_symbols if f in defined} for sym, expr in assigns}
    expr_of = dict(assigns)
    out, done = [], set()

    def visit(sym):
        stack = [(sym, iter(sorted(deps[sym], key=str)))]
        while stack:
            cur, it = stack[-1]
            nxt = next((d for d in it if d not in done), None)
            if nxt is None:
                stack.pop()
                if cur not in done:
                    done.add(cur)
                    out.append((cur, expr_of[cur]))
            else:
                stack.append((nxt, iter(sorted(deps[nxt], key=str))))
    for sym, _ in assigns:
        if sym not in done:
            visit(sym)
    return out


def _count_ops(e):
    import sympy as sp
    return int(sp.count_ops(e, visual=False))


def _count_ops_cse(repl, red):
    return sum(_count_ops(v) for _, v in repl) + sum(_count_ops(e) for e in red)


def _c(e):
    """C expression: powers expanded into products, rationals as FP64 literals."""
    import sympy as sp

    def rec(e):
        if e.is_Symbol:
            return str(e)
        if e.is_Integer:
            return f"{float(int(e))!r}"
        if e.is_Rational:
            return f"({float(e)!r})"
        if e.is_Add:
            return "(" + " + ".join(rec(a) for a in e.args) + ")"
        if e.is_Mul:
            return "(" + " * ".join(rec(a) for a in e.args) + ")"
        if e.is_Pow:
            b, ex = e.args
            if ex.is_Integer and int(ex) > 0:
                s = rec(b)
                return "(" + " * ".join([s] * int(ex)) + ")"
            if ex.is_Integer and int(ex) < 0:
                s = rec(b)
                return "(1.0 / (" + " * ".join([s] * (-int(ex))) + "))"
        raise ValueError(f"unexpected term {e!r}")
    return rec(sp.sympify(e))


# ---------------------------------------------------------- straight-line L2P

def l2p_code(p):
    """Straight-line L2P (Eq. L2P) for order p: with r = (x - z)/h and the
    independent scaled local coefficients Lt[j],
        f  = sum_{|n|<=p}   r^n/n! L_n,        g_i = sum_{|n|<=p-1} r^n/n! L_{n+e_i},
    where each full component L_n is expanded into independent ones.  The
    monomials are built incrementally (z outer, y middle, x inner), so every
    product is computed once; coefficients are exact rationals rounded once."""
    lines = []
    for v in "xyz":
        lines.append(f"double {v}0 = 1.0;")
        for k in range(1, p + 1):
            lines.append(f"const double {v}{k} = {v}{k - 1} * {v};")
    acc = {"f": [], "gx": [], "gy": [], "gz": []}

    def combo(m, mult):
        e = expand(m)
        terms = []
        for j, cj in sorted(e.items()):
            c = Fraction(cj * mult, mfact(m) if False else 1)
            terms.append((j, c))
        return terms

    nterms = 0
    out = []
    for c in range(p + 1):
        for b in range(p + 1 - c):
            out.append(f"{{ const double* Lg = gen_launder(L); const double yz = y{b} * z{c};")
            for a in range(p + 1 - b - c):
                n = (a, b, c)
                inv = Fraction(1, mfact(n))
                out.append(f"  {{ const double m = x{a} * yz;")
                # potential coefficient: L_n / n!
                t = [(j, inv * cj) for j, cj in sorted(expand(n).items())]
                out.append("    f += m * (" + " + ".join(f"({float(cf)!r}) * LD({j})" for j, cf in t) + ");")
                nterms += len(t)
                if a + b + c < p:
                    for nm, e in (("gx", (1, 0, 0)), ("gy", (0, 1, 0)), ("gz", (0, 0, 1))):
                        n2 = (a + e[0], b + e[1], c + e[2])
                        t = [(j, inv * cj) for j, cj in sorted(expand(n2).items())]
                        out.append(f"    {nm} += m * (" + " + ".join(f"({float(cf)!r}) * LD({j})" for j, cf in t) + ");")
                        nterms += len(t)
                out.append("  }")
            out.append("__builtin_amdgcn_sched_barrier(0); }")
    return lines + out, nterms


# ------------------------------------------------------ nested-Horner L2P

def l2p_horner_layout(p):
    """The full components (a, b, c), |n| <= p, in the order the nested Horner
    scheme reads them: a descending, then b descending, then c descending."""
    return [(a, b, c) for a in range(p, -1, -1) for b in range(p - a, -1, -1) for c in range(p - a - b, -1, -1)]


def l2p_full_table(p):
    """For each slot of l2p_horner_layout(p): the polynomial coefficient
    L_n / n! of the local expansion (Eq. L2P) as {independent slot: weight},
    the full component L_n written through the independent ones (expand)."""
    rows = []
    for m in l2p_horner_layout(p):
        inv = Fraction(1, mfact(m))
        rows.append({j: inv * cj for j, cj in sorted(expand(m).items())})
    return rows


def l2p_build_tables(p):
    """How the kernels build the full coefficients C_n = L_n / n! in Horner
    order: the independent components (c <= 1) are scaled into their slots,
    (slot, 1/n!) per independent index; every other component follows from the
    trace condition L_{a,b,c} = -(L_{a+2,b,c-2} + L_{a,b+2,c-2}), i.e.
        C_{a,b,c} = alpha C_{a+2,b,c-2} + beta C_{a,b+2,c-2},
        alpha = -(a+1)(a+2) / (c(c-1)),  beta = -(b+1)(b+2) / (c(c-1)),
    in passes over c = (2,3), (4,5), ...: each pass reads only slots written
    before it.  Returns (ind, passes), ind[j] = (slot, weight) and passes a list
    of [(dst, src1, src2, alpha, beta)]."""
    lay = l2p_horner_layout(p)
    pos = {m: i for i, m in enumerate(lay)}
    ind = [(pos[m], Fraction(1, mfact(m))) for m in IND if rank(m) <= p]
    passes = []
    for c0 in range(2, p + 1, 2):
        ent = []
        for c in (c0, c0 + 1):
            for m in lay:
                if m[2] == c:
                    a, b, _ = m
                    ent.append((pos[m], pos[(a + 2, b, c - 2)], pos[(a, b + 2, c - 2)],
                                Fraction(-(a + 1) * (a + 2), c * (c - 1)), Fraction(-(b + 1) * (b + 2), c * (c - 1))))
        passes.append(ent)
    return ind, passes


def l2p_horner_ops(p):
    """Potential and gradient of the degree-p polynomial f(r) = sum_n C_n r^n
    (C in l2p_horner_layout order) by nested Horner with derivatives:
        f = sum_a x^a Q_a(y, z),  Q_a = sum_b y^b S_ab(z),  S_ab = sum_c z^c C_abc,
    each level carrying its value and the derivatives it needs (Horner's rule
    for a polynomial and its derivative).  Returned as straight-line
    operations (dst, acc, var, add): dst = acc * var + add, where acc or add
    None means zero and add may be ("C", k), the k-th coefficient; the
    results are the names in the final ("out", ...) entry."""
    ops = []
    cnt = [0]

    def fma(acc, var, add):
        if acc is None and add is None:
            return None
        if acc is None and isinstance(add, str):
            return add
        dst = f"t{cnt[0]}"
        cnt[0] += 1
        ops.append((dst, acc, var, add))
        return dst

    k = 0
    f = gx = gy = gz = None
    for a in range(p, -1, -1):
        q = qy = qz = None
        for b in range(p - a, -1, -1):
            s = sz = None
            for c in range(p - a - b, -1, -1):
                sz = fma(sz, "z", s)
                s = fma(s, "z", ("C", k))
                k += 1
            qy = fma(qy, "y", q)
            q = fma(q, "y", s)
            qz = fma(qz, "y", sz)
        gx = fma(gx, "x", f)
        f = fma(f, "x", q)
        gy = fma(gy, "x", qy)
        gz = fma(gz, "x", qz)
    ops.append(("out", f, gx, gy, gz))
    return ops


def l2p_horner_code(p, chunk=32):
    """C text of l2p_horner_ops(p), the coefficient slot k read as C[k].  The
    reads are software-pipelined in chunks of `chunk` slots: the reads of chunk
    i + 1 are issued before the operations that use chunk i, with a scheduling
    barrier between chunks, so at most two chunks of coefficients are live."""
    ops = l2p_horner_ops(p)
    nf = len(l2p_horner_layout(p))
    chunks = [list(range(k, min(nf, k + chunk))) for k in range(0, nf, chunk)]
    lines = []

    def loads(i):
        if i < len(chunks):
            lines.extend(f"const double c{k} = C[{k}];" for k in chunks[i])

    loads(0)
    ci = 0
    lines.append("__builtin_amdgcn_sched_barrier(0);")
    loads(1)
    for op in ops[:-1]:
        dst, acc, var, add = op
        if isinstance(add, tuple) and add[1] // chunk > ci:
            ci = add[1] // chunk
            lines.append("__builtin_amdgcn_sched_barrier(0);")
            loads(ci + 1)
        addt = f"c{add[1]}" if isinstance(add, tuple) else add
        if acc is None:
            lines.append(f"const double {dst} = {addt};")
        elif add is None:
            lines.append(f"const double {dst} = {acc} * {var};")
        else:
            lines.append(f"const double {dst} = __builtin_fma({acc}, {var}, {addt});")
    _, f, gx, gy, gz = ops[-1]
    for nm, v in (("f", f), ("gx", gx), ("gy", gy), ("gz", gz)):
        lines.append(f"{nm} = {v if v is not None else '0.0'};")
    return lines, sum(1 for op in ops[:-1] if op[1] is not None)


def l2p_horner_global_code(p, chunk=24):
    """Nested-Horner L2P reading the independent coefficients Lt[j] directly
    (one thread per particle, no staging): each full coefficient of chunk i is
    formed from its independent components (l2p_full_table) just before the
    Horner operations that use chunk i - 1 run, through a laundered copy of the
    pointer per chunk (the reads of one chunk are shared, the chunks' are
    not kept live)."""
    ops = l2p_horner_ops(p)
    table = l2p_full_table(p)
    nf = len(table)
    chunks = [list(range(k, min(nf, k + chunk))) for k in range(0, nf, chunk)]
    lines = []

    def coefs(i):
        if i < len(chunks):
            lines.append(f"{{ const double* Lg = gen_launder(L);")
            for k in chunks[i]:
                terms = " + ".join(f"({float(w)!r}) * Lg[{j}]" for j, w in sorted(table[k].items()))
                lines.append(f"  c{k} = {terms};")
            lines.append("}")

    lines.append("double " + ", ".join(f"c{k}" for k in range(nf)) + ";")
    coefs(0)
    ci = 0
    lines.append("__builtin_amdgcn_sched_barrier(0);")
    coefs(1)
    for op in ops[:-1]:
        dst, acc, var, add = op
        if isinstance(add, tuple) and add[1] // chunk > ci:
            ci = add[1] // chunk
            lines.append("__builtin_amdgcn_sched_barrier(0);")
            coefs(ci + 1)
        addt = f"c{add[1]}" if isinstance(add, tuple) else add
        if acc is None:
            lines.append(f"const double {dst} = {addt};")
        elif add is None:
            lines.append(f"const double {dst} = {acc} * {var};")
        else:
            lines.append(f"const double {dst} = __builtin_fma({acc}, {var}, {addt});")
    _, f, gx, gy, gz = ops[-1]
    for nm, v in (("f", f), ("gx", gx), ("gy", gy), ("gz", gz)):
        lines.append(f"{nm} = {v if v is not None else '0.0'};")
    return lines


# ------------------------------------------------------------------ emit

def _hexf(v):
    return float(v).hex() if v != 0 else "0.0"


def emit(outdir):
    global DET
    DET = detracer_rows()
    os.makedirs(outdir, exist_ok=True)
    L = []
    w = L.append
    w("// Generated by paper_1811_06332_amd/gen/gen_operators.py -- do not edit.")
    w("// Cartesian traceless FMM operators (Coles & Bieri, arXiv 1811.06332),")
    w("// reduced to the independent traceless components in exact rational")
    w("// arithmetic; rationals are rounded once to FP64.")
    w("#pragma once")
    w(f"#define GEN_PMAX {PMAX}")
    w(f"#define GEN_NIND {len(IND)}")
    w(f"#define GEN_NFULL {len(FULL)}")
    w("")
    w("// independent slot -> (nx, ny, nz); ordered by rank, then nz, then nx descending")
    w("static const signed char GEN_IND[GEN_NIND][3] = {" + ",".join("{%d,%d,%d}" % m for m in IND) + "};")
    w("// full slot -> (nx, ny, nz); ordered by rank, nx descending, ny descending")
    w("static const signed char GEN_FULL[GEN_NFULL][3] = {" + ",".join("{%d,%d,%d}" % m for m in FULL) + "};")
    # expansion table
    starts, slots, coefs = [0], [], []
    for m in FULL:
        e = expand(m)
        for j in sorted(e):
            slots.append(j); coefs.append(e[j])
        starts.append(len(slots))
    w("// full component f of a traceless polytensor = sum_{t in [EXP_START[f], EXP_START[f+1])} EXP_COEF[t] * ind[EXP_SLOT[t]]")
    w(f"static const short GEN_EXP_START[{len(starts)}] = {{" + ",".join(map(str, starts)) + "};")
    w(f"static const unsigned char GEN_EXP_SLOT[{len(slots)}] = {{" + ",".join(map(str, slots)) + "};")
    w(f"static const int GEN_EXP_COEF[{len(coefs)}] = {{" + ",".join(map(str, coefs)) + "};")
    # P2M terms
    pt = p2m_terms()
    starts, cs, ex = [0], [], []
    for terms in pt:
        for (c, a, b, d, e2) in terms:
            cs.append(_hexf(c)); ex.append("{%d,%d,%d,%d}" % (a, b, d, e2))
        starts.append(len(cs))
    w("// P2M: M~_n += q * sum_t P2M_COEF[t] * ux^e0 uy^e1 uz^e2 (|u|^2)^e3, u = (z - x)/h  (Eq. Detracer3)")
    w(f"static const short GEN_P2M_START[{len(starts)}] = {{" + ",".join(map(str, starts)) + "};")
    w(f"static const double GEN_P2M_COEF[{len(cs)}] = {{" + ",".join(cs) + "};")
    w(f"static const signed char GEN_P2M_EXP[{len(ex)}][4] = {{" + ",".join(ex) + "};")
    # M2M / L2L octant matrices, dense [8][NIND][NIND]
    for name, fn, doc in (("M2M", m2m_matrix, "parent M~_n += sum_j GEN_M2M[o][n][j] * child_o M~_j (exact: rank(j) <= rank(n))"),
                          ("L2L", l2l_matrix, "child_o L~_n += sum_j GEN_L2L[o][n][j] * parent L~_j (order p keeps rank(j) <= p)")):
        w(f"// {doc}")
        rows = []
        for o in range(8):
            Mx = fn(o)
            for n in range(len(IND)):
                rows.append(",".join(_hexf(Mx[n].get(j, 0)) for j in range(len(IND))))
        w(f"static const double GEN_{name}[8][GEN_NIND][GEN_NIND] = {{" + ",\n".join(rows) + "};")
    # M2L contraction
    c = m2l_contraction()
    keys = sorted(c)
    starts, ii, cc = [], [], []
    w("// M2L: K_v[n][j] = sum_{t in [C_START[n][j], C_START[n][j]+C_COUNT[n][j])} C_COEF[t] * D_{C_SLOT[t]}(v)  (Eq. M2L)")
    cstart = [[0] * len(IND) for _ in IND]
    ccount = [[0] * len(IND) for _ in IND]
    for (n, j) in keys:
        cstart[n][j] = len(ii); ccount[n][j] = len(c[(n, j)])
        for i in sorted(c[(n, j)]):
            ii.append(i); cc.append(_hexf(c[(n, j)][i]))
    w("static const int GEN_C_START[GEN_NIND][GEN_NIND] = {" + ",".join("{" + ",".join(map(str, r)) + "}" for r in cstart) + "};")
    w("static const unsigned char GEN_C_COUNT[GEN_NIND][GEN_NIND] = {" + ",".join("{" + ",".join(map(str, r)) + "}" for r in ccount) + "};")
    w(f"static const unsigned char GEN_C_SLOT[{len(ii)}] = {{" + ",".join(map(str, ii)) + "};")
    w(f"static const double GEN_C_COEF[{len(cc)}] = {{" + ",".join(cc) + "};")
    # detracer rows: independent n <- full f (P2M from monomial moments)
    starts, fs, cs = [0], [], []
    for row in DET:
        for f in sorted(row):
            fs.append(f); cs.append(_hexf(row[f]))
        starts.append(len(fs))
    w("// P2M: M~_n = sum_{t in [DET_START[n], DET_START[n+1])} DET_COEF[t] * S_{DET_FULL[t]},")
    w("// S_f = sum_a q_a u_a^f the full monomial moments (Eq. P2M, Eq. Detracer / (2n-1)!!)")
    w(f"static const short GEN_DET_START[{len(starts)}] = {{" + ",".join(map(str, starts)) + "};")
    w(f"static const short GEN_DET_FULL[{len(fs)}] = {{" + ",".join(map(str, fs)) + "};")
    w(f"static const double GEN_DET_COEF[{len(cs)}] = {{" + ",".join(cs) + "};")
    # the same rows as straight-line code per rank (a thread per cell)
    w("// P2M detracer rows of one rank N: out[i] = M~ of the i-th independent component of")
    w("// rank N from S[k], the full monomial moments of rank N in full-slot order")
    w("template <int N> __device__ __forceinline__ void gen_det_rank(const double* __restrict__ S, double* __restrict__ out);")
    for N in range(PMAX + 1):
        f0 = N * (N + 1) * (N + 2) // 6
        w(f"template <> __device__ __forceinline__ void gen_det_rank<{N}>(const double* __restrict__ S, "
          f"double* __restrict__ out) {{")
        for i in range(2 * N + 1):
            row = DET[N * N + i]
            assert all(f0 <= f < f0 + (N + 1) * (N + 2) // 2 for f in row)
            terms = " + ".join(f"{_hexf(row[f])} * S[{f - f0}]" for f in sorted(row))
            w(f"  out[{i}] = {terms if terms else '0.0'};")
        w("}")
    # inverse factorials of full components (L2P)
    w("// 1/n! for full slots (L2P weights)")
    w("static const double GEN_INV_MFACT[GEN_NFULL] = {" + ",".join(_hexf(Fraction(1, mfact(m))) for m in FULL) + "};")
    # straight-line D code per p
    stats = []
    for p in range(PMAX + 1):
        lines, opt, noopt = dtensor_code(p)
        stats.append((p, opt, noopt))
        w(f"// traceless gradient of 1/r, independent components of ranks <= {p}; "
          f"{opt} operations after CSE ({noopt} before)")
        w(f"__host__ __device__ static inline void gen_dtensor_p{p}(double x, double y, double z, double* __restrict__ D) {{")
        w("  const double u = 1.0 / sqrt(x * x + y * y + z * z);")
        for ln in lines:
            w("  " + ln)
        w("}")
    w("// Each (y, z) group of the generated L2P reads the coefficients through a")
    w("// laundered copy of the pointer, so the compiler reloads them per group")
    w("// (L1 hits) instead of keeping every coefficient live across the function.")
    w("__device__ __forceinline__ const double* gen_launder(const double* p) {")
    w("  unsigned long long a = (unsigned long long)p;")
    w('  __asm__ volatile("" : "+v"(a));')
    w("  return (const double*)a;")
    w("}")
    w("#define LD(j) (Lg[(j)])")
    for p in range(PMAX + 1):
        lines, nt = l2p_code(p)
        w(f"// L2P at order {p}: potential and gradient polynomials in r = (x - z)/h, {nt} coefficient terms")
        w(f"__device__ static inline void gen_l2p_p{p}(double x, double y, double z, const double* __restrict__ L,")
        w("                                          double& f, double& gx, double& gy, double& gz) {")
        for ln in lines:
            w("  " + ln)
        w("}")
    w("#undef LD")
    # the same L2P reading the coefficients from LDS
    w("typedef __attribute__((address_space(3))) const double lds_cdouble;")
    w("__device__ __forceinline__ lds_cdouble* gen_launder_lds(lds_cdouble* p) {")
    w("  unsigned a = (unsigned)(unsigned long long)p;")
    w('  __asm__ volatile("" : "+v"(a));')
    w("  return (lds_cdouble*)(unsigned long long)a;")
    w("}")
    w("#define LD(j) (Lg[(j)])")
    for p in range(PMAX + 1):
        lines, nt = l2p_code(p)
        lines = [ln.replace("const double* Lg = gen_launder(L);", "lds_cdouble* Lg = gen_launder_lds(L);") for ln in lines]
        w(f"// L2P at order {p} with the coefficients in LDS")
        w(f"__device__ static inline void gen_l2p_lds_p{p}(double x, double y, double z, lds_cdouble* __restrict__ L,")
        w("                                              double& f, double& gx, double& gy, double& gz) {")
        for ln in lines:
            w("  " + ln)
        w("}")
    w("#undef LD")
    w("template <int P> __device__ inline void gen_l2p_lds(double x, double y, double z, lds_cdouble* L, double& f,")
    w("                                                double& gx, double& gy, double& gz);")
    for p in range(PMAX + 1):
        w(f"template <> __device__ inline void gen_l2p_lds<{p}>(double x, double y, double z, lds_cdouble* L, double& f, "
          f"double& gx, double& gy, double& gz) {{ gen_l2p_lds_p{p}(x, y, z, L, f, gx, gy, gz); }}")
    # nested-Horner L2P: the tables that build the full coefficients, and the evaluation
    w("template <int P> struct GenL2PFull;")
    w("// Nested-Horner L2P.  The full coefficient array C (Horner order: a, b, c")
    w("// descending) holds C_n = L_n / n!: independent index j goes to slot IS[j]")
    w("// times IW[j]; the other slots follow from the trace condition in passes,")
    w("// entry e: C[dst] = DA[e] C[src1] + DB[e] C[src2], DD[e] = dst | src1 << 10 |")
    w("// src2 << 20, pass k holding the entries dep_off(k) .. dep_off(k + 1) - 1.")
    for p in range(PMAX + 1):
        ind, passes = l2p_build_tables(p)
        ent = [e for ps in passes for e in ps]
        offs = [0]
        for ps in passes:
            offs.append(offs[-1] + len(ps))
        w(f"static __device__ const unsigned short gen_l2p_is_p{p}[{len(ind)}] = {{{', '.join(str(s) for s, _ in ind)}}};")
        w(f"static __device__ const double gen_l2p_iw_p{p}[{len(ind)}] = {{{', '.join(repr(float(v)) for _, v in ind)}}};")
        nd = max(1, len(ent))
        dd = [str(d | (s1 << 10) | (s2 << 20)) for d, s1, s2, _, _ in ent] or ["0"]
        da = [repr(float(a)) for _, _, _, a, _ in ent] or ["0.0"]
        db = [repr(float(b)) for _, _, _, _, b in ent] or ["0.0"]
        w(f"static __device__ const unsigned int gen_l2p_dd_p{p}[{nd}] = {{{', '.join(dd)}}};")
        w(f"static __device__ const double gen_l2p_da_p{p}[{nd}] = {{{', '.join(da)}}};")
        w(f"static __device__ const double gen_l2p_db_p{p}[{nd}] = {{{', '.join(db)}}};")
        lines, nf = l2p_horner_code(p)
        w(f"// L2P at order {p} by nested Horner over the {len(l2p_horner_layout(p))} full coefficients in LDS: {nf} FMAs")
        w(f"__device__ static inline void gen_l2p_horner_p{p}(double x, double y, double z, lds_cdouble* __restrict__ C,")
        w("                                                 double& f, double& gx, double& gy, double& gz) {")
        for ln in lines:
            w("  " + ln)
        w("}")
        w(f"template <> struct GenL2PFull<{p}> {{")
        w(f"  static constexpr int NF = {len(l2p_horner_layout(p))}, NI = {len(ind)}, NPASS = {len(passes)};")
        chain = " : ".join(f"k == {k} ? {o}" for k, o in enumerate(offs)) + " : 0"
        w(f"  __host__ __device__ static constexpr int dep_off(int k) {{ return {chain}; }}")
        for nm, arr in (("is", "is"), ("iw", "iw"), ("dd", "dd"), ("da", "da"), ("db", "db")):
            ty = {"is": "unsigned short", "iw": "double", "dd": "unsigned int", "da": "double", "db": "double"}[nm]
            w(f"  __device__ static const {ty}* {nm}() {{ return gen_l2p_{arr}_p{p}; }}")
        w(f"  __device__ static void eval(double x, double y, double z, lds_cdouble* C, double& f, double& gx, double& gy,")
        w(f"                              double& gz) {{ gen_l2p_horner_p{p}(x, y, z, C, f, gx, gy, gz); }}")
        w("};")
    for p in range(PMAX + 1):
        w(f"// L2P at order {p} by nested Horner, the full coefficients formed from Lt in global memory")
        w(f"__device__ static inline void gen_l2p_hg_p{p}(double x, double y, double z, const double* __restrict__ L,")
        w("                                             double& f, double& gx, double& gy, double& gz) {")
        for ln in l2p_horner_global_code(p):
            w("  " + ln)
        w("}")
    w("template <int P> __device__ inline void gen_l2p_hg(double x, double y, double z, const double* L, double& f,")
    w("                                               double& gx, double& gy, double& gz);")
    for p in range(PMAX + 1):
        w(f"template <> __device__ inline void gen_l2p_hg<{p}>(double x, double y, double z, const double* L, double& f, "
          f"double& gx, double& gy, double& gz) {{ gen_l2p_hg_p{p}(x, y, z, L, f, gx, gy, gz); }}")
    w("template <int P> __device__ inline void gen_l2p(double x, double y, double z, const double* L, double& f,")
    w("                                            double& gx, double& gy, double& gz);")
    for p in range(PMAX + 1):
        w(f"template <> __device__ inline void gen_l2p<{p}>(double x, double y, double z, const double* L, double& f, "
          f"double& gx, double& gy, double& gz) {{ gen_l2p_p{p}(x, y, z, L, f, gx, gy, gz); }}")
    for p in range(PMAX + 1):
        lines, nt = m2l_pair_code(p, c)
        w(f"// M2L of one pair at order {p} for the outputs of ranks R0..R1: {nt} contraction terms in all")
        w(f"template <int R0, int R1, bool AP> __device__ __forceinline__ void gen_m2l_pair_p{p}(")
        w("    const double* __restrict__ D, const double* __restrict__ Ms, const double* rp, double* L) {")
        for ln in lines:
            w("  " + ln)
        w("}")
    w("template <int P, int R0, int R1, bool AP> __device__ __forceinline__ void gen_m2l_pair(const double* D, const double* Ms,")
    w("                                                                                   const double* rp, double* L) {")
    for p in range(PMAX + 1):
        kw = "if" if p == 0 else "else if"
        w(f"  {kw} constexpr (P == {p}) gen_m2l_pair_p{p}<R0, R1, AP>(D, Ms, rp, L);")
    w("}")
    w("template <int P> __host__ __device__ inline void gen_dtensor(double x, double y, double z, double* D);")
    for p in range(PMAX + 1):
        w(f"template <> __host__ __device__ inline void gen_dtensor<{p}>(double x, double y, double z, double* D) {{ gen_dtensor_p{p}(x, y, z, D); }}")
    with open(os.path.join(outdir, "ctfmm_gen.h"), "w") as fh:
        fh.write("\n".join(L) + "\n")
    with open(os.path.join(outdir, "dtensor_opcounts.txt"), "w") as fh:
        fh.write("# p  ops_after_cse  ops_before (sympy count_ops; +,-,*,/ and sqrt count 1)\n")
        for p, o, n in stats:
            fh.write(f"{p} {o} {n}\n")


if __name__ == "__main__":
    emit(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "csrc", "generated"))
