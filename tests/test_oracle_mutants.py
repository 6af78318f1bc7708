"""Planted-mistake check of the oracle's pins (CPU only).

Each mutant is a copy of ``oracle/ctfmm_oracle.c`` with one plausible mistake
(a dropped term, a wrong sign, index or operand) patched in, compiled into a
temporary library.  The pins of ``oracle_pins.py`` must reject every mutant.
"""
from __future__ import annotations

import importlib.util
import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle_pins  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ctfmm_oracle.c")

# (name, old text, new text, which occurrence (0-based) or None for all)
MUTANTS = [
    ("f_nm_sign", "double s = (m & 1) ? -1.0 : 1.0;", "double s = 1.0;", None),
    ("f_nm_double_factorial", "dfact(2 * n - 2 * m - 1)", "dfact(2 * n - 2 * m + 1)", None),
    ("detracer_inner_weight_uses_m", "inner += fact(m) / mfact(k1, k2, k3)",
     "inner += fact(m) / mfact(m1, m2, m3)", None),
    ("detracer_f_uses_wrong_factorial",
     "/ (ipow(2.0, m) * mfact(m1, m2, m3) * mfact(n1 - 2 * m1, n2 - 2 * m2, n3 - 2 * m3));",
     "/ (ipow(2.0, m) * mfact(m1, m2, m3) * mfact(n1 - m1, n2 - m2, n3 - m3));", None),
    ("detracer_D_normalisation", "/ dfact(2 * n - 1);", ";", None),
    ("dtensor_power", "ipow(rn, 2 * k + 1)", "ipow(rn, 2 * k)", None),
    ("dtensor_sign", "double sgn = (k & 1) ? -1.0 : 1.0;", "double sgn = 1.0;", None),
    ("p2m_sign", "double rx = -(xyz[3 * a + 0] - z[0]);", "double rx = (xyz[3 * a + 0] - z[0]);", None),
    ("m2m_shift_sign", "ipow(-d[0], n1 - k1)", "ipow(d[0], n1 - k1)", None),
    ("m2m_binomial_dropped",
     "double w = mfact(n1, n2, n3) / (mfact(k1, k2, k3) * mfact(n1 - k1, n2 - k2, n3 - k3));",
     "double w = 1.0;", None),
    ("m2l_weight_dropped", "* D[g_idx[n1 + m1][n2 + m2][n3 + m3]] / mfact(m1, m2, m3);",
     "* D[g_idx[n1 + m1][n2 + m2][n3 + m3]];", None),
    ("m2l_truncation_short", "for (int e = 0; e < g_nfull[p - n]; ++e) {\n            int m1",
     "for (int e = 0; e < (p - n > 0 ? g_nfull[p - n - 1] : 1); ++e) {\n            int m1", None),
    ("l2l_shift_sign", "s += ipow(d[0], k1) * ipow(d[1], k2)", "s += ipow(-d[0], k1) * ipow(d[1], k2)", None),
    ("l2l_truncation_short", "for (int e = 0; e < g_nfull[p - n]; ++e) {\n            int k1",
     "for (int e = 0; e < (p - n > 0 ? g_nfull[p - n - 1] : 1); ++e) {\n            int k1", None),
    ("l2p_gradient_operand", "gx += w * L[g_idx[n1 + 1][n2][n3]];", "gx += w * L[g_idx[n1][n2 + 1][n3]];", None),
    ("p2p_gradient_sign", "grad[0] -= ir3 * dx;", "grad[0] += ir3 * dx;", None),
    ("cell_centre_offset", "z[0] = T->lo[0] + ((double)i + 0.5) * h;", "z[0] = T->lo[0] + ((double)i + 0.25) * h;", None),
    ("m2m_child_offset_reversed",
     "dd[0] = zc[0] - zp[0]; dd[1] = zc[1] - zp[1]; dd[2] = zc[2] - zp[2];",
     "dd[0] = zp[0] - zc[0]; dd[1] = zp[1] - zc[1]; dd[2] = zp[2] - zc[2];", 0),
    ("l2l_child_offset_reversed",
     "dd[0] = zc[0] - zp[0]; dd[1] = zc[1] - zp[1]; dd[2] = zc[2] - zp[2];",
     "dd[0] = zp[0] - zc[0]; dd[1] = zp[1] - zc[1]; dd[2] = zp[2] - zc[2];", 1),
    ("m2l_direction_reversed", "r[0] = zb[0] - za[0]; r[1] = zb[1] - za[1]; r[2] = zb[2] - za[2];",
     "r[0] = za[0] - zb[0]; r[1] = za[1] - zb[1]; r[2] = za[2] - zb[2];", None),
    ("interaction_list_includes_neighbours", "<= 1) continue;\n                double za[3]",
     "<= 0) continue;\n                double za[3]", None),
    ("interaction_list_parent_range", "for (int64_t a = 2 * (I - 1); a <= 2 * (I + 1) + 1; ++a)",
     "for (int64_t a = 2 * (I - 1); a <= 2 * (I + 1); ++a)", None),
    ("near_field_misses_neighbours", "for (int64_t a1 = i - 1; a1 <= i + 1; ++a1)",
     "for (int64_t a1 = i; a1 <= i + 1; ++a1)", None),
    ("adaptive_w_list_dropped", "oracle_l2p(p, zero, Lp, &f, g);", "(void)zero;", None),
    ("adaptive_x_list_dropped", "oracle_m2l(p, r, Mq, T.L[i]);", "(void)Mq;", None),
    ("adaptive_adjacency_strict", "if (alo > bhi || blo > ahi) return 0;", "if (alo >= bhi || blo >= ahi) return 0;", None),
    ("adaptive_v_includes_adjacent", "if (C >= 0 && !oa_adjacent(&T->nd[C], b)) ivec_push(&T->V[B], C);",
     "if (C >= 0) ivec_push(&T->V[B], C);", None),
    ("adaptive_l2l_dropped", "oracle_l2l(p, dd, T.L[par], T.L[i]);", "(void)dd;", None),
    ("adaptive_split_threshold", "if (nd.e - nd.b <= T->leaf_max || nd.level >= OA_DMAX) return;",
     "if (nd.e - nd.b < T->leaf_max / 2 || nd.level >= OA_DMAX) return;", None),
    ("order_table_ignored", "order = order_r2[dx * dx + dy * dy + dz * dz];", "order = p;", None),
    ("order_table_wrong_offset", "order = order_r2[dx * dx + dy * dy + dz * dz];",
     "order = order_r2[dx * dx + dy * dy + dz * dz >= 9 ? 27 : 4];", None),
    ("pair_orders_shifted", "if (vorder) order = vorder[voff[i] + k];",
     "if (vorder) order = vorder[voff[i] + (k + 1) % T.V[i].n];", None),
    ("dipole_p2m_sign", "Md[g_idx[1][0][0]] = -dip[3 * a + 0];", "Md[g_idx[1][0][0]] = dip[3 * a + 0];", None),
    ("dipole_p2m_shift_reversed", "double d[3] = {xyz[3 * a] - z[0], xyz[3 * a + 1] - z[1], xyz[3 * a + 2] - z[2]};",
     "double d[3] = {z[0] - xyz[3 * a], z[1] - xyz[3 * a + 1], z[2] - xyz[3 * a + 2]};", None),
    ("dipole_field_gradient_term", "grad[0] += pa[0] * ir3 - 3.0 * pr * dx * ir5;",
     "grad[0] += pa[0] * ir3 - pr * dx * ir5;", None),
    ("dipole_near_field_dropped",
     "if (T->dip) pair_kernel_dipole(&T->xyz[3 * b], &T->xyz[3 * a], &T->dip[3 * a], &f, g);", "(void)0;", None),
    ("dual_mac_reversed", "if (D->theta * dist > D->zr[a][3] + D->zr[b][3]) {",
     "if (D->theta * dist < D->zr[a][3] + D->zr[b][3]) {", None),
    ("dual_one_way_m2l", "oracle_m2l(p, rm, T.M[b], T.L[a]);  /* B -> A */", "(void)rm;", None),
    ("dual_open_smaller", "(B->leaf || D->zr[a][3] >= D->zr[b][3])", "(B->leaf || D->zr[a][3] <= D->zr[b][3])",
     None),
    ("dual_children_not_self_paired", "for (int j = i; j < 8; ++j) {\n                int cj = A->child[j];",
     "for (int j = i + 1; j < 8; ++j) {\n                int cj = A->child[j];", None),
    ("dual_unweighted_centre", "for (int d = 0; d < 3; ++d) s[d] += q[a] * xyz[3 * a + d];",
     "for (int d = 0; d < 3; ++d) s[d] += q[a] * q[a] * xyz[3 * a + d];", None),
    ("dual_radius_last_particle", "double d = sqrt(dx * dx + dy * dy + dz * dz);\n            if (d > r) r = d;",
     "double d = sqrt(dx * dx + dy * dy + dz * dz);\n            r = d;", None),
    ("dual_ap_drops_monopole", "T.M[i][g_idx[1][0][0]] = 0.0;", "T.M[i][g_idx[0][0][0]] = 0.0;", None),
    ("dual_m2m_offset_reversed",
     "double dd[3] = {D.zr[c][0] - D.zr[i][0], D.zr[c][1] - D.zr[i][1], D.zr[c][2] - D.zr[i][2]};",
     "double dd[3] = {D.zr[i][0] - D.zr[c][0], D.zr[i][1] - D.zr[c][1], D.zr[i][2] - D.zr[c][2]};", None),
    ("dual_l2l_offset_reversed",
     "double dd[3] = {D.zr[i][0] - D.zr[par][0], D.zr[i][1] - D.zr[par][1], D.zr[i][2] - D.zr[par][2]};",
     "double dd[3] = {D.zr[par][0] - D.zr[i][0], D.zr[par][1] - D.zr[i][1], D.zr[par][2] - D.zr[i][2]};", None),
]


# pins that take seconds go last
_SLOW = ("pin_order_table", "pin_dual_vs_direct_decay", "pin_dtensor_sympy", "pin_detracer_vs_gradient")
PINS_BY_COST = sorted(oracle_pins.ALL_PINS, key=lambda f: _SLOW.index(f.__name__) + 1 if f.__name__ in _SLOW else 0)


def _patch(src, old, new, which):
    assert old in src, old
    if which is None:
        return src.replace(old, new)
    parts = src.split(old)
    assert len(parts) > which + 1
    return old.join(parts[: which + 1]) + new + old.join(parts[which + 1:])


def _load(libpath, tag):
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{tag}", os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB = libpath
    mod._lib_handle = None
    return mod


@pytest.mark.parametrize("name,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, which):
    src = open(SRC).read()
    mutated = _patch(src, old, new, which)
    assert mutated != src
    cfile = tmp_path / f"{name}.c"
    cfile.write_text(mutated)
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", str(lib), str(cfile), "-lm"],
                   check=True)
    mod = _load(str(lib), name)
    # the first pin that rejects the mutant settles it (cheap pins first)
    caught = None
    for pin in PINS_BY_COST:
        try:
            pin(mod)
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError, RuntimeError):
            caught = pin.__name__
            break
    assert caught, f"no pin rejects mutant {name}"
