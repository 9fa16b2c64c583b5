"""Plant plausible mistakes in copies of the oracle (CPU only) and check that
the pins in oracle_pins.py reject every one of them."""
import pathlib
import re

import pytest

import oracle
import oracle_pins

SRC = pathlib.Path(oracle.__file__).resolve().parent / "oracle.c"

# (id, function whose body is edited, text to find, replacement)
MUTATIONS = [
    ("gs_plus_x_reads_minus_x", "oracle_gs_f64",
     "s = s + u[IDX(k, j, i + 1)];", "s = s + u[IDX(k, j, i - 1)];"),
    ("jacobi_sign_error", "oracle_jacobi_f64",
     "v = (a * src[IDX(k, j, i)]) + (b * s);", "v = (a * src[IDX(k, j, i)]) - (b * s);"),
    ("jacobi_dropped_zp", "oracle_jacobi_f64",
     "s = s + src[IDX(k + 1, j, i)];", ""),
    ("jacobi_operand_order", "oracle_jacobi_f64",
     "s = s + src[IDX(k, j - 1, i)];\n                    s = s + src[IDX(k, j + 1, i)];\n"
     "                    s = s + src[IDX(k - 1, j, i)];",
     "s = s + src[IDX(k - 1, j, i)];\n                    s = s + src[IDX(k, j + 1, i)];\n"
     "                    s = s + src[IDX(k, j - 1, i)];"),
    # (swapping the j and k loops is NOT a mistake: with a 7-point stencil the
    # result only depends on which axis neighbours are fresh, so every loop
    # permutation with increasing indices is the same program)
    ("gs_reversed_z", "oracle_gs_f64",
     "for (int64_t k = h; k < h + nz; k++)", "for (int64_t k = h + nz - 1; k >= h; k--)"),
    ("jacobi_rhs_weight", "oracle_jacobi_f64",
     "if (f) v = v + (g * f[FIDX(k, j, i)]);", "if (f) v = v + (b * f[FIDX(k, j, i)]);"),
    ("gs_uses_old_values", "oracle_gs_f64",
     "double s = u[IDX(k, j, i - 1)];", "double s = (i > h) ? u[IDX(k, j, i + 1)] : u[IDX(k, j, i - 1)];"),
    ("residual_sign", "oracle_residual_f64",
     "double rv = fv - ((6.0 * c) - s);", "double rv = fv + ((6.0 * c) - s);"),
    ("jacobi_f32_transposed_y", "oracle_jacobi_f32",
     "s = s + src[IDX(k, j + 1, i)];", "s = s + src[IDX(k + 1, j, i)];"),
    ("gs_f32_center_weight_dropped", "oracle_gs_f32",
     "v = (a * u[IDX(k, j, i)]) + (b * s);", "v = (b * s);"),
    ("rb_colour_ignores_k", "oracle_rbgs_f64",
     "if ((((i - h) + (j - h) + (k - h)) & 1) != color) continue;",
     "if ((((i - h) + (j - h)) & 1) != color) continue;"),
    ("rb_black_first", "oracle_rbgs_f64",
     "for (int color = 0; color < 2; color++)", "for (int color = 1; color >= 0; color--)"),
    ("rb_f32_dropped_ym", "oracle_rbgs_f32", "s = s + u[IDX(k, j - 1, i)];", ""),
    ("refine_f32_no_correction", "oracle_refine",
     "u[IDX(k, j, i)] = u[IDX(k, j, i)] + (double)e32[IDX(k, j, i)];",
     "u[IDX(k, j, i)] = u[IDX(k, j, i)] + 0.5 * (double)e32[IDX(k, j, i)];"),
    ("jacobi_f32_operand_order", "oracle_jacobi_f32",
     "s = s + src[IDX(k, j - 1, i)];\n                    s = s + src[IDX(k, j + 1, i)];\n"
     "                    s = s + src[IDX(k - 1, j, i)];",
     "s = s + src[IDX(k - 1, j, i)];\n                    s = s + src[IDX(k, j + 1, i)];\n"
     "                    s = s + src[IDX(k, j - 1, i)];"),
    ("gs_f32_operand_order", "oracle_gs_f32",
     "s = s + u[IDX(k, j + 1, i)];\n                    s = s + u[IDX(k - 1, j, i)];",
     "s = s + u[IDX(k - 1, j, i)];\n                    s = s + u[IDX(k, j + 1, i)];"),
    ("gs_f32_sum_in_double", "oracle_gs_f32",
     "float s = u[IDX(k, j, i - 1)];", "double s = u[IDX(k, j, i - 1)];"),
    ("rbgs_f32_operand_order", "oracle_rbgs_f32",
     "s = s + u[IDX(k - 1, j, i)];\n                        s = s + u[IDX(k + 1, j, i)];",
     "s = s + u[IDX(k + 1, j, i)];\n                        s = s + u[IDX(k - 1, j, i)];"),
    ("jacobi_f32_update_in_double", "oracle_jacobi_f32",
     "v = (a * src[IDX(k, j, i)]) + (b * s);",
     "v = (float)(((double)a * src[IDX(k, j, i)]) + ((double)b * s));"),
    # multigrid
    ("mg_restrict_no_scale", "oracle_mg_restrict_f64",
     "= zs * scale;", "= zs;"),
    ("mg_prolong_swapped_weights", "oracle_mg_prolong_add_f64",
     "vx[b] = (wmx * row[I0]) + (wqx * row[I0 + 1]);",
     "vx[b] = (wqx * row[I0]) + (wmx * row[I0 + 1]);"),
    ("mg_restrict_y_weights_of_x", "oracle_mg_restrict_f64",
     "ys = ys + (mg_w64(j, J, fny, cny) * xs);", "ys = ys + (mg_w64(j, J, fnx, cnx) * xs);"),
    ("mg_restrict_f32_centre_weight", "oracle_mg_restrict_f32",
     "zs = zs + (mg_w32(k, K, fnz, cnz) * ys);", "zs = zs + ys;"),
    ("mg_prolong_f32_z_lo_only", "oracle_mg_prolong_add_f32",
     "const float v = (wmz * vy[0]) + (wqz * vy[1]);", "const float v = vy[0];"),
    ("mg_residual_f32_sign", "oracle_mg_residual_f32",
     "res[FIDX(k, j, i)] = fp[FIDX(k, j, i)] - ((6.0f * c) - s);",
     "res[FIDX(k, j, i)] = fp[FIDX(k, j, i)] + ((6.0f * c) - s);"),
    ("mg_coarse_support_short", "mg_support",
     "*hi = ((I + 1) * (n + 1) - 1) / (nc + 1);", "*hi = (I * (n + 1)) / (nc + 1);"),
]


def _mutate(text, func, old, new):
    m = re.search(r"\n[^\n]*\b%s\(" % re.escape(func), text)
    assert m, func
    start = m.start()
    nxt = text.find("\n}\n", start)
    body = text[start:nxt]
    assert old in body, (func, old)
    return text[:start] + body.replace(old, new, 1) + text[nxt:]


@pytest.mark.parametrize("mid,func,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_reject_mutation(tmp_path, mid, func, old, new):
    src = tmp_path / "oracle_mut.c"
    src.write_text(_mutate(SRC.read_text(), func, old, new))
    lib = oracle.load(oracle.build(force=True, out=tmp_path / "liboracle_mut.so", src=src))
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, "no pin caught mutation %s" % mid
