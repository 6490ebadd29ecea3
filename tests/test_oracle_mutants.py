"""Planted mistakes in the oracle must fail at least one pin.

Each case copies oracle/fno_oracle.c, plants one plausible mistake (a flipped
sign, a dropped term, a wrong index or weight, a transposed operand), builds
the copy into a temporary shared object on the CPU, points the oracle front
end at it and runs the pins of test_oracle_pins.py.  A mutant that passes
every pin would mean the pins cannot see that kind of mistake.
"""
import os
import subprocess

import pytest

import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "fno_oracle.c")

MUTANTS = {
    "t_stage_sign": ("im -= row[t] * et[(kt * Nt + t) * 2 + 1];", "im += row[t] * et[(kt * Nt + t) * 2 + 1];"),
    "z_stage_cross_term": ("re += c * ar + sn * ai;", "re += c * ar - sn * ai;"),
    "y_stage_dropped_term": ("im += c * bi - sn * br;", "im += c * bi;"),
    "x_stage_conj": ("im += c * p[1] - sn * p[0];", "im += c * p[1] + sn * p[0];"),
    "negative_freq_map": ("return j < s->m[a] ? j : s->N[a] - 2 * s->m[a] + j;",
                          "return j < s->m[a] ? j : s->N[a] - s->m[a] + j;"),
    "real_output_weight": ("    return 2.0;\n}", "    return 1.0;\n}"),
    "inverse_no_1_over_N": ("oracle_ct(kt, s->N[3]) / (double)s->ncell", "oracle_ct(kt, s->N[3])"),
    "synth_t_sign": ("acc += w * (vr * c - vi * sn);", "acc += w * (vr * c + vi * sn);"),
    "synth_y_sign": ("re += c * pr - sn * pi;\n                        im += c * pi + sn * pr;\n                    }\n                    U1",
                     "re += c * pr + sn * pi;\n                        im += c * pi - sn * pr;\n                    }\n                    U1"),
    "mix_conjugated": ("re += a[0] * q[0] - a[1] * q[1];", "re += a[0] * q[0] + a[1] * q[1];"),
    "mix_bwd_no_conj": ("re += g[0] * q[0] + g[1] * q[1];", "re += g[0] * q[0] - g[1] * q[1];"),
    "gw_no_conj": ("im += a[0] * g[1] - a[1] * g[0];", "im += a[0] * g[1] + a[1] * g[0];"),
    "pointwise_transposed": ("acc += wpw[o * s->Ci + i] * x[", "acc += wpw[(i % s->Co) * s->Ci + (o % s->Ci)] * x["),
    "gelu_grad_dropped_term": ("return 0.5 * (1.0 + erf(u / sqrt(2.0))) + u * exp(-0.5 * u * u) / sqrt(2.0 * PI_D);",
                               "return 0.5 * (1.0 + erf(u / sqrt(2.0)));"),
    "bias_dropped": ("double acc = bpw ? bpw[o] : 0.0;", "double acc = 0.0;"),
    "gx_pointwise_not_transposed": ("acc += wpw[o * s.Ci + i] * z[", "acc += wpw[(i % s.Co) * s.Ci + (o % s.Ci)] * z["),
    "dft_modes_axes_swapped": ("k[a] = freq_of(&s, a, kidx[i * 4 + a]);", "k[a] = freq_of(&s, a, kidx[i * 4 + (a ^ 1)]);"),
    "dft_modes_sign": ("th += angle(k[a], nn[a], s.N[a]);\n                double v = in[(size_t)bc * s.ncell + n];\n                re += v * cos(th);\n                im -= v * sin(th);\n            }\n            out[((size_t)bc * nk",
                       "th += angle(k[a], nn[a], s.N[a]);\n                double v = in[(size_t)bc * s.ncell + n];\n                re += v * cos(th);\n                im += v * sin(th);\n            }\n            out[((size_t)bc * nk"),
    "lift_gx_sign": ("acc += we[o * Ci + i] * gz[", "acc -= we[o * Ci + i] * gz["),
}

PIN_CALLS = [
    lambda o: pins.test_p1_separable_equals_bruteforce(o, pins.TINY[1]),
    lambda o: pins.test_p2_numpy_fft_special_case(o, pins.TINY[2]),
    lambda o: pins.test_p2_numpy_spectral_layer(o),
    lambda o: pins.test_p3_impulse(o),
    lambda o: pins.test_p4_single_mode(o, (1, 2, 0, 1), 0.3),
    lambda o: pins.test_p5_parseval_bessel(o, 8),
    lambda o: pins.test_p7_adjoint_dot_products(o, pins.TINY[1]),
    lambda o: pins.test_p8_identity_round_trip(o, (4, 6, 4, 8)),
    lambda o: pins.test_p10_gelu(o),
    lambda o: pins.test_p11_finite_differences(o, (2, 3, 2, (6, 5, 4, 6), (2, 2, 1, 3))),
    lambda o: pins.test_p12_torch_autograd_gradient(o, (2, 3, 2, (6, 5, 4, 6), (2, 2, 1, 3))),
    lambda o: pins.test_dft_modes_at_listed_modes(o, pins.TINY[2]),
    lambda o: pins.test_dft_modes_impulse_closed_form(o),
    lambda o: pins.test_lift_bwd_all_gradients_vs_torch(o),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle, tmp_path, monkeypatch, name):
    find, repl = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(find) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(find, repl, 1)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", str(c), "-o", str(so), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load(str(so)))
    failed = 0
    for call in PIN_CALLS:
        try:
            call(oracle)
        except AssertionError:
            failed += 1
    assert failed >= 1, f"planted mistake {name} passed every pin"
