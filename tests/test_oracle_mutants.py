"""Plant plausible mistakes in a copy of the oracle (on the CPU) and require
the pins to catch every one: evidence that the pins constrain each part of
the oracle, not just that the oracle agrees with itself."""
import os
import warnings

import pytest

import oracle as O
import pins

SRC = os.path.join(os.path.dirname(O.__file__), "oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("transposed_operand", "double br = re_(b, k, j), bi = im_(b, k, j);",
     "double br = re_(b, j, k), bi = im_(b, j, k);"),
    ("wrong_sign", "re += (ar * br) - (ai * bi);", "re += (ar * br) + (ai * bi);"),
    ("dropped_term", "im += (ar * bi) + (ai * br);", "im += (ar * bi);"),
    ("mul3_order", "mat_mul(t1, c + 18 * s, zs);", "mat_mul(c + 18 * s, t1, zs);"),
    ("muladd_order", "mat_mul(c + 18 * s, d + 18 * s, t2);",
     "mat_mul(d + 18 * s, c + 18 * s, t2);"),
    ("add_sign", "c[t] = a[t] + b[t];", "c[t] = a[t] - b[t];"),
    ("apb_ab_sum", "mat_add(as, bs, t1);", "mat_mul(as, bs, t1);"),
    ("rebuild_no_conj", "ms[2 * (6 + k) + 1] = -xi;", "ms[2 * (6 + k) + 1] = xi;"),
    ("half_round_up", "if (rem > halfway || (rem == halfway && (q & 1u)))",
     "if (rem >= halfway)"),
    ("half_subnormal_shift", "shift = -e - 1;", "shift = -e;"),
    ("pack_reim_swap", "double v = s < V ? canon[18 * s + 2 * e + c] : 0.0;",
     "double v = s < V ? canon[18 * s + 2 * e + (1 - c)] : 0.0;"),
    ("soa_no_pad", "*Vpad = (V + 63) / 64 * 64;", "*Vpad = V;"),
    ("metrics_no_delta", "if (i == j)\n                    re -= 1.0;", ""),
    ("cshift_sign", "n[mu] = ((c[mu] + shift) % dims[mu] + dims[mu]) % dims[mu];",
     "n[mu] = ((c[mu] - shift) % dims[mu] + dims[mu]) % dims[mu];"),
    ("cshift_no_wrap", "n[mu] = ((c[mu] + shift) % dims[mu] + dims[mu]) % dims[mu];",
     "n[mu] = (c[mu] + shift < dims[mu] && c[mu] + shift >= 0) ? c[mu] + shift : c[mu];"),
    ("dslash_sign_swap", "hop_term(u[mu] + 18 * s, 0, in + 24 * sf, mu, -1.0, acc);",
     "hop_term(u[mu] + 18 * s, 0, in + 24 * sf, mu, +1.0, acc);"),
    ("dslash_no_dagger", "double mi = dagger ? -im_(m, b, a) : im_(m, a, b);",
     "double mi = dagger ? im_(m, b, a) : im_(m, a, b);"),
    ("dslash_backward_link_local", "hop_term(u[mu] + 18 * sb, 1, in + 24 * sb, mu, +1.0, acc);",
     "hop_term(u[mu] + 18 * s, 1, in + 24 * sb, mu, +1.0, acc);"),
    ("dslash_gamma_entry", "     {{0, 0}, {1, 0}, {0, 0}, {0, 0}},\n     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},\n    /* gamma_3 */",
     "     {{0, 0}, {-1, 0}, {0, 0}, {0, 0}},\n     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},\n    /* gamma_3 */"),
    ("vnode_node_outer_swap", "site += (nm * r[mu] + om) * stride;",
     "site += (om * simd[mu] + nm) * stride;"),
    ("vnode_lane_order", "            for (int64_t n = 0; n < nsub; ++n) {\n                const int64_t site = vnode_site(dims, r, simd, o, n);\n                for (int c = 0; c < 2; ++c, ++w) {\n                    const double v",
     "            for (int64_t n = 0; n < nsub; ++n) {\n                const int64_t site = vnode_site(dims, r, simd, o, (n % 2) * (nsub / 2) + n / 2);\n                for (int c = 0; c < 2; ++c, ++w) {\n                    const double v"),
    ("expr_scalar_on_all_entries",
     "const double av = a.mat ? a.m[t] : (i == j ? a.m[c] : 0.0);",
     "const double av = a.mat ? a.m[t] : a.m[c];"),
    ("expr_adj_no_conj", "x->fn == EF_ADJ ? -a.m[2 * (3 * j + i) + 1] : a.m[2 * (3 * j + i) + 1];",
     "a.m[2 * (3 * j + i) + 1];"),
    ("expr_trace_index", "v.m[0] = (a.m[0] + a.m[8]) + a.m[16];",
     "v.m[0] = (a.m[0] + a.m[8]) + a.m[12];"),
    ("expr_product_order", "const double br = b.m[2 * (3 * q + j)], bi = b.m[2 * (3 * q + j) + 1];",
     "const double br = b.m[2 * (3 * j + q)], bi = b.m[2 * (3 * j + q) + 1];"),
    ("expr_sub_sign", "const double sg = x->kind == EN_ADD ? 1.0 : -1.0;",
     "const double sg = 1.0;"),
    ("det_sign", "r += re_(m, 0, j) * cr - im_(m, 0, j) * ci;",
     "r += re_(m, 0, j) * cr + im_(m, 0, j) * ci;"),
]


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, mut):
    text = open(SRC).read()
    assert text.count(orig) == 1, name
    src = tmp_path / f"oracle_{name}.c"
    src.write_text(text.replace(orig, mut))
    lib = O.build(str(src), str(tmp_path / f"liboracle_{name}.so"))
    orc = O.Oracle(lib)
    caught = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        for pin in pins.ALL_PINS:
            try:
                pin(orc)
            except AssertionError:
                caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
