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
    "pack_lsb_first": ("v = (uint8_t)((v << 1) | (bitvals[8 * i + j] & 1));",
                       "v = (uint8_t)(v | ((bitvals[8 * i + j] & 1) << j));"),
}


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
