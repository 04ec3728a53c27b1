"""Mutation check of the oracle's pins (CPU only).

Each case compiles a copy of the oracle with one plausible mistake planted
(a sign, a dropped conjugate, an index off by one, a wrong threshold, the CP
left in, ...) and runs the pin suites against it; at least one pin must fail.
The mistakes are planted in the oracle source on the CPU; nothing here runs
on a GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rx_oracle.c")

MUTANTS = {
    "fft_sign": ("-2.0 * ORACLE_PI * (double)j", "2.0 * ORACLE_PI * (double)j"),
    "fft_butterfly": ("x[i + j + half] = u - v;", "x[i + j + half] = v - u;"),
    "fft_bitrev_skipped": ("if (i < j) {", "if (0) {"),
    "subcarrier_off_by_one": (": d - u / 2 + 1;", ": d - u / 2;"),
    "subcarrier_order_swapped": ("(d < u / 2) ? d - u / 2 : d - u / 2 + 1", "(d < u / 2) ? d + 1 : d - u"),
    "cp_not_removed": ("* len + p->cp_len + n) * 2;\n  return (double)iq",
                       "* len + n) * 2;\n  return (double)iq"),
    "ls_no_conjugate": ("* conj(xp) / mag2", "* xp / mag2"),
    "ls_no_normalisation": ("* conj(xp) / mag2", "* conj(xp)"),
    "mrc_no_conjugate": ("z += conj(Hs[(size_t)a * U + d]) * Y", "z += Hs[(size_t)a * U + d] * Y"),
    "mrc_not_normalised": ("x = z / gs[d];", "x = z;"),
    "g_not_squared": ("s += creal(h) * creal(h) + cimag(h) * cimag(h);", "s += creal(h) + cimag(h);"),
    "g_drops_imag": ("s += creal(h) * creal(h) + cimag(h) * cimag(h);", "s += creal(h) * creal(h);"),
    "zf_no_conjugate": ("double complex w = conj(Hs[(size_t)a * U + d]) / gs[d];",
                        "double complex w = Hs[(size_t)a * U + d] / gs[d];"),
    "pilot_wrong_index": ("double complex xp = p->pilot[2 * d] + I * p->pilot[2 * d + 1];",
                          "double complex xp = p->pilot[2 * ((d + 1) % U)] + I * p->pilot[2 * ((d + 1) % U) + 1];"),
    "demap_sign_bit": ("out[0] = (uint8_t)(c < 0.0);", "out[0] = (uint8_t)(signbit(c) != 0);"),
    "demap_16qam_threshold": ("sqrt(10.0) > 2.0", "sqrt(10.0) > 3.0"),
    "demap_64qam_third_bit": ("fabs(u - 4.0) > 2.0", "fabs(u - 4.0) < 2.0"),
    "demap_axes_swapped": ("bitvals[i * bits_per_sym + 2 * j] = re[j];", "bitvals[i * bits_per_sym + 2 * j] = im[j];"),
    "fft_symbols_slot_stride": ("size_t slot_elems = (size_t)T * A * (N + p->cp_len) * 2;",
                                "size_t slot_elems = (size_t)T * A * N * 2;"),
    "fft_symbols_output_order": ("double* o = out + ((((size_t)s * T + t) * A + a) * N) * 2;",
                                 "double* o = out + ((((size_t)s * A + a) * T + t) * N) * 2;"),
    "pack_lsb_first": ("v = (uint8_t)((v << 1) | (bitvals[8 * i + j] & 1));",
                       "v = (uint8_t)(v | ((bitvals[8 * i + j] & 1) << j));"),
}


# Mistakes in the comb estimate and the training-channel generator; their pins
# live in their own suites.
COMB_GEN_MUTANTS = {
    "comb_interp_by_index": ("(double)(signed_freq(d, U) - signed_freq(d0, U)) /\n"
                             "                       (double)(signed_freq(d1, U) - signed_freq(d0, U));",
                             "(double)(d - d0) / (double)(d1 - d0);"),
    "comb_holds_first_pilot": ("h[2 * d] = h[2 * last];", "h[2 * d] = h[0];"),
    "comb_interp_wrong_end": ("h[2 * d] = h[2 * d0] + t * (h[2 * d1] - h[2 * d0]);",
                              "h[2 * d] = h[2 * d1] + t * (h[2 * d1] - h[2 * d0]);"),
    "philox_nine_rounds": ("for (int round = 0; round < 10; round++)", "for (int round = 0; round < 9; round++)"),
    "philox_no_key_bump": ("k0 += 0x9E3779B97F4A7C15ull;", "k0 += 0;"),
    "gen_delay_truncated": ("(l * span + (L - 1) / 2) / (L - 1)", "(l * span) / (L - 1)"),
    "gen_phase_sign": ("+ I * sin(-2.0 * ORACLE_PI * m / N)", "+ I * sin(2.0 * ORACLE_PI * m / N)"),
    "gen_power_not_normalised": ("/ psum / 2.0) * z;", "/ 2.0) * z;"),
    "gen_noise_too_strong": ("sqrt(pow(10.0, -snr_db / 10.0) / 2.0)", "sqrt(pow(10.0, -snr_db / 10.0))"),
    "gen_noise_block_shared": ("block_words(seed, row, noise_block + j / 2, b);",
                               "block_words(seed, row, 1 + j / 2, b);"),
    "gen_wrong_uniform": ("(double)(2 * (w >> 41) + 1) * 0x1p-24", "(double)((w >> 40) + 1) * 0x1p-24"),
    "sync_last_maximum": ("if (best < 0 || acc > best_v) {", "if (best < 0 || acc >= best_v) {"),
    "sync_drops_quadrature": ("acc += (uint64_t)(re * re) + (uint64_t)(im * im);", "acc += (uint64_t)(re * re);"),
    "sync_chip_order_reversed": ("re += (int64_t)pn[m] * s[0];\n        im += (int64_t)pn[m] * s[1];",
                                 "re += (int64_t)pn[L - 1 - m] * s[0];\n        im += (int64_t)pn[L - 1 - m] * s[1];"),
    "sync_off_by_one": ("const int64_t i = n + m;", "const int64_t i = n + m + 1;"),
}


def _compile_mutant(tmp_path, old, new, name):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "rx_oracle_mut.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(lib), str(mutated), "-lm", "-lpthread"])
    return lib


@pytest.mark.parametrize("name", sorted(COMB_GEN_MUTANTS))
def test_comb_and_generator_pins_catch_planted_mistake(name, tmp_path):
    old, new = COMB_GEN_MUTANTS[name]
    lib = _compile_mutant(tmp_path, old, new, name)
    env = dict(os.environ, RX_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_comb.py"),
                        os.path.join(ROOT, "tests", "test_oracle_gen.py"),
                        os.path.join(ROOT, "tests", "test_oracle_sync.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


# Mistakes in the FP64 denoiser (numpy); the pins are the functions of
# test_oracle_denoiser run against the mutated module.
DN_SRC = os.path.join(ROOT, "oracle", "denoiser.py")
DN_MUTANTS = {
    "transposed_conv_index": ("dp[:, :, 2 * HALF - k:2 * HALF - k + U]", "dp[:, :, k:k + U]"),
    "relu_mask_dropped": ("delta = rnd(gx * (xin > 0))", "delta = rnd(gx)"),
    "bias_grad_missing_rows": ("gb = delta.sum(axis=(0, 2))", "gb = delta[0].sum(axis=1)"),
    "loss_not_normalised": ("n = R * U", "n = U"),
    "conv_flipped_taps": ("W[:, :, k], xp[:, :, k:k + U])\n    return y",
                          "W[:, :, TAPS - 1 - k], xp[:, :, k:k + U])\n    return y"),
    "no_relu_forward": ("x = rnd(np.maximum(a, 0.0))", "x = rnd(a)"),
    "residual_missing": ("out = h + s[:, None] * (a4[:, 0] + 1j * a4[:, 1])",
                         "out = s[:, None] * (a4[:, 0] + 1j * a4[:, 1])"),
    "scale_is_mean_abs": ("np.sqrt(np.mean(np.abs(h) ** 2, axis=-1))", "np.mean(np.abs(h), axis=-1)"),
    "adam_no_bias_correction": ("mh = m / (1 - beta1 ** step)", "mh = m"),
    "adam_sqrt_missing": ("(np.sqrt(vh) + eps)", "(vh + eps)"),
    "fallback_inverted": ("fell = ~np.isfinite(e) | ~(e <= max_corr", "fell = ~np.isfinite(e) | (e <= max_corr"),
    "fallback_limit_not_squared": ("~(e <= max_corr ** 2 * np.sum", "~(e <= max_corr * np.sum"),
    "fallback_ignores_non_finite": ("fell = ~np.isfinite(e) | ~(e", "fell = ~(e"),
    "bf16_truncates": ("(u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u & 0xFFFF0000"),
    "bf16_input_not_rounded": ("x = rnd(_input(h, s))", "x = _input(h, s)"),
    "bf16_weights_not_rounded": ("a = conv(x, rnd(W), b)", "a = conv(x, W, b)"),
    "bf16_activation_not_rounded": ("x = rnd(np.maximum(a, 0.0))", "x = np.maximum(a, 0.0)"),
    "bf16_delta_not_rounded": ("delta = rnd(2.0 * e / n)", "delta = 2.0 * e / n"),
    "term_rss_not_squared": ("np.einsum(\"rou,rcu->oc\", delta ** 2, xp[:, :, k:k + U] ** 2)",
                             "np.einsum(\"rou,rcu->oc\", delta ** 2, xp[:, :, k:k + U])"),
    "term_rss_tap_shifted": ("delta ** 2, xp[:, :, k:k + U] ** 2", "delta ** 2, xp[:, :, 2 * HALF - k:2 * HALF - k + U] ** 2"),
    "term_rss_bias_unsquared": ("np.sqrt((delta ** 2).sum(axis=(0, 2)))", "np.sqrt(np.abs(delta.sum(axis=(0, 2))))"),
}


@pytest.mark.parametrize("name", sorted(DN_MUTANTS))
def test_denoiser_pins_catch_planted_mistake(name, tmp_path):
    import importlib.util

    from tests import test_oracle_denoiser as suite
    old, new = DN_MUTANTS[name]
    src = open(DN_SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    path = tmp_path / "denoiser_mut.py"
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location("denoiser_mut", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    saved = suite.dn
    suite.dn = mod
    failed = []
    try:
        for fname in sorted(dir(suite)):
            fn = getattr(suite, fname)
            if not fname.startswith("test_") or not callable(fn):
                continue
            args = [0] if fname == "test_training_reduces_loss" else []
            try:
                fn(*args)
            except Exception as e:  # a pin failed (or the mutant crashed)
                failed.append((fname, type(e).__name__))
                break
    finally:
        suite.dn = saved
    assert failed, f"mutant {name} survived the pins"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "rx_oracle_mut.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(lib), str(mutated), "-lm", "-lpthread"])
    env = dict(os.environ, RX_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_fft.py"),
                        os.path.join(ROOT, "tests", "test_oracle_path.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
