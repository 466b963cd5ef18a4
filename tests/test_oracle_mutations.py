"""The oracle pins must catch plausible mistakes.

Each case plants one slip into a copy of the oracle's C source (on the CPU,
never in the GPU library), builds it into a temporary library and checks that
at least one pin of ``test_oracle_pins`` fails against it.
"""
import os
import subprocess

import pytest

import oracle
import tests.test_oracle_pins as pins

_SRC = os.path.join(os.path.dirname(oracle.__file__), "fsr_oracle.c")

MUTANTS = {
    "conjugated_twiddles": ("ti[q] = -sin(", "ti[q] = sin("),
    "transposed_dft_input": ("sr += x[m * S + n] * tr[q];", "sr += x[n * S + m] * tr[q];"),
    "residual_update_sign": ("Ri[k * S + l] -= cr * ai + ci * ar;", "Ri[k * S + l] -= cr * ai - ci * ar;"),
    "shift_index_wrong_direction": ("int i = (k - u >= 0) ? k - u : S + k - u;",
                                    "int i = (k + u < S) ? k + u : k + u - S;"),
    "model_update_scale": ("Gr[best] += gamma * p_re * (double)n2;", "Gr[best] += gamma * p_re * (double)S;"),
    "no_relaxation_in_residual": ("const double cr = gamma * p_re, ci = gamma * p_im;",
                                  "const double cr = p_re, ci = p_im;"),
    "weight_centre_off_by_half": ("const double c = 0.5 * (double)(S - 1);", "const double c = 0.5 * (double)S;"),
    "freq_weight_transposed": ("double lt = h - fabs((double)l - h);", "double lt = h - fabs((double)k - h);"),
    "argmax_prefers_larger_index": ("if (tie_larger ? (obj >= best_obj) : (obj > best_obj))",
                                    "if (tie_larger ? (obj > best_obj) : (obj >= best_obj))"),
    "inverse_dft_sign": ("acc += Gr[k * S + l] * tr[q] + Gi[k * S + l] * ti[q];",
                         "acc += Gr[k * S + l] * tr[q] - Gi[k * S + l] * ti[q];"),
    "compose_swapped": ("out_target[i * B + j] = known[m * S + n] ? ft[m * S + n]",
                        "out_target[i * B + j] = !known[m * S + n] ? ft[m * S + n]"),
    "projection_not_normalised": ("const double p_re = Rr[best] / w00, p_im = Ri[best] / w00;",
                                  "const double p_re = Rr[best] / (2.0 * w00), p_im = Ri[best] / (2.0 * w00);"),
    "objective_without_freq_weight": ("double obj = wf[b] * (Rr[b] * Rr[b] + Ri[b] * Ri[b]);",
                                      "double obj = (Rr[b] * Rr[b] + Ri[b] * Ri[b]);"),
    "separation_keeps_tied_conjugate": ("if (b == conj && ob == best_obj) continue;", ""),
    "separation_from_the_smallest": ("if (ob > next) next = ob;", "if (ob < next || next == 0.0) next = ob;"),
    "objective_rounded_to_float32": ("double obj = wf[b] * (Rr[b] * Rr[b] + Ri[b] * Ri[b]);",
                                     "double obj = (float)(wf[b] * (Rr[b] * Rr[b] + Ri[b] * Ri[b]));"),
}

PIN_CALLS = [
    lambda o: pins.test_dft_matches_numpy_fft2(o, 8),
    lambda o: pins.test_dft_matches_numpy_fft2(o, 32),
    lambda o: pins.test_dft_matches_numpy_fft2(o, 24),
    pins.test_twiddle_table_exact_symmetry,
    pins.test_weights_closed_form,
    lambda o: pins.test_spectra_bitwise_hermitian(o, 32),
    lambda o: pins.test_spectra_bitwise_hermitian(o, 24),
    pins.test_orthogonal_case_recovers_fft,
    lambda o: pins.test_energy_descent_closed_form(o, 0.5, 32),
    lambda o: pins.test_energy_descent_closed_form(o, 0.5, 24),
    lambda o: pins.test_residual_matches_definition(o, 32),
    lambda o: pins.test_residual_matches_definition(o, 24),
    lambda o: pins.test_first_step_matches_bruteforce_least_squares(o, 1),
    lambda o: pins.test_grid_sinusoid_recovered(o, 1, 2, 0.9),
    pins.test_fully_known_image_unchanged,
    pins.test_known_pixels_copied_bitwise,
    pins.test_zero_iterations_gives_zero_model,
    pins.test_fp64_decision_resolves_sub_float32_differences,
    pins.test_separation_of_the_first_pick_closed_form,
    lambda o: pins.test_separation_log_matches_the_residual(o, 16),
]


@pytest.fixture
def mutant_oracle(tmp_path):
    saved = (oracle._LIB, oracle._lib)

    def make(name):
        before, after = MUTANTS[name]
        src = open(_SRC).read()
        assert src.count(before) == 1, name
        path = tmp_path / f"{name}.c"
        path.write_text(src.replace(before, after))
        lib = tmp_path / f"lib{name}.so"
        subprocess.check_call(["gcc", *oracle.CFLAGS, "-w", str(path), "-o", str(lib), "-lm"])
        oracle._LIB, oracle._lib = str(lib), None
        return oracle

    yield make
    oracle._LIB, oracle._lib = saved


def test_unmutated_source_passes_every_pin(oracle_lib):
    for call in PIN_CALLS:
        call(oracle_lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(mutant_oracle, name):
    o = mutant_oracle(name)
    caught = []
    for call in PIN_CALLS:
        try:
            call(o)
        except AssertionError:
            caught.append(call)
    assert caught, f"no pin caught mutant {name}"
