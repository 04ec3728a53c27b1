"""Pins of the oracle's comb-pilot estimate (LS on every s-th used subcarrier,
linear interpolation in signed frequency across the DC gap, last pilot held)
and of its combining with a caller-supplied channel estimate.

The paper's LS (Sec. II-C, LS paragraph) is a block estimate; the comb form is
the standard LS-with-interpolation baseline the learned denoiser refines.
Pins use closed forms (a channel linear in frequency is reproduced exactly),
special cases (s = 1 is the block estimate; a flat channel is recovered
exactly) and the transmitter's ground truth.
"""
import numpy as np
import pytest

import oracle
from rxgen import C1, C5, make_frames


def _signed(U):
    return np.concatenate([np.arange(-U // 2, 0), np.arange(1, U // 2 + 1)])


@pytest.mark.parametrize("U,s", [(52, 4), (1200, 4), (600, 3), (72, 5), (8, 2), (10, 10)])
def test_line_in_frequency_is_reproduced(U, s):
    rng = np.random.default_rng(U * 10 + s)
    alpha, beta = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    f = _signed(U)
    line = alpha + beta * f
    rows = np.where(np.arange(U) % s == 0, line, 1e6 + 0j)[None, :]   # junk off the comb
    out = oracle.comb_interp(rows, s)[0]
    last = ((U - 1) // s) * s
    np.testing.assert_allclose(out[:last + 1], line[:last + 1], rtol=0, atol=1e-9 * np.abs(line).max())
    # beyond the last pilot its value is held
    np.testing.assert_array_equal(out[last:], np.full(U - last, line[last]))


def test_dc_gap_weights_by_frequency_not_index():
    # U = 8, s = 2: pilots at d = 0, 2, 4, 6 with frequencies -4, -2, +1, +3.
    # d = 3 (f = -1) lies between f = -2 and f = +1: weight 1/3 toward the upper pilot.
    U, s = 8, 2
    rows = np.zeros((1, U), dtype=complex)
    rows[0, 2], rows[0, 4] = 3.0, 6.0
    out = oracle.comb_interp(rows, s)[0]
    assert abs(out[3] - 4.0) < 1e-12
    assert abs(out[1] - 1.5) < 1e-12      # midway between d = 0 (0) and d = 2 (3)
    assert out[7] == out[6]               # held past the last pilot


def test_spacing_one_is_block_ls():
    f = make_frames(C1, 1, seed=3)
    kw = dict(n_ant=C1.n_ant, fft_len=C1.fft_len, cp_len=C1.cp_len, n_used=C1.n_used, n_sym=C1.n_sym,
              bits_per_sym=C1.bits_per_sym)
    a = oracle.process_frame(f.iq, f.pilot, pilot_spacing=1, **kw)
    b = oracle.process_frame(f.iq, f.pilot, pilot_spacing=0, **kw)
    np.testing.assert_array_equal(a.H, b.H)
    np.testing.assert_array_equal(a.bits, b.bits)


SMALL_COMB = C1.replace(name="comb_tiny", n_ant=4, pilot_spacing=4, n_taps=1, unit_spaced_taps=True)


def _run(fr, **over):
    c = fr.cfg
    kw = dict(n_ant=c.n_ant, fft_len=c.fft_len, cp_len=c.cp_len, n_used=c.n_used, n_sym=c.n_sym,
              bits_per_sym=c.bits_per_sym, pilot_spacing=c.pilot_spacing)
    kw.update(over)
    return oracle.process_frame(fr.iq if "f64" not in over else fr.y, fr.pilot, **kw)


def test_comb_pilot_zero_off_the_comb():
    fr = make_frames(C5.replace(n_ant=2, n_slots=1), 1, seed=1)
    nz = np.nonzero(fr.pilot)[0]
    np.testing.assert_array_equal(nz, np.arange(0, C5.n_used, 4))
    assert set(np.abs(fr.pilot[nz]).tolist()) == {1.0}


def test_flat_channel_recovered_exactly_and_error_free():
    # One tap at delay 0: H is the same on every subcarrier, so interpolation is exact.
    fr = make_frames(SMALL_COMB, 2, seed=5, channel="flat", noise=False, keep_float=True)
    r = _run(fr, f64=True)
    np.testing.assert_allclose(r.H, fr.H_true, rtol=1e-9, atol=1e-9 * np.abs(fr.H_true).max())
    np.testing.assert_array_equal(r.bits, fr.packed_bits())


def test_comb_pilots_equal_block_ls_on_the_comb():
    # On the comb the estimate is the LS value of that subcarrier: the same as a
    # block-pilot run with the pilot's values placed on the comb.
    fr = make_frames(SMALL_COMB.replace(n_taps=4), 1, seed=6)
    comb = _run(fr)
    pilot_full = fr.pilot.copy()
    pilot_full[pilot_full == 0] = 1.0        # any non-zero value off the comb
    blk = _run(fr.__class__(**{**fr.__dict__, "pilot": pilot_full}), pilot_spacing=1)
    on = np.arange(SMALL_COMB.n_used) % 4 == 0
    np.testing.assert_array_equal(comb.H[:, :, on], blk.H[:, :, on])


def test_given_estimate_reproduces_ls_run():
    fr = make_frames(C1, 2, seed=8)
    base = _run(fr)
    again = _run(fr, H_in=base.H)
    np.testing.assert_array_equal(again.xhat, base.xhat)
    np.testing.assert_array_equal(again.bits, base.bits)
    np.testing.assert_array_equal(again.g, base.g)


def test_given_estimate_true_channel_noiseless_is_error_free():
    fr = make_frames(C5.replace(n_ant=4, n_slots=1), 1, seed=9, noise=False)
    r = _run(fr, H_in=fr.H_true)
    np.testing.assert_array_equal(r.bits, fr.packed_bits())


def test_comb_rejects_zero_pilot_on_the_comb():
    fr = make_frames(SMALL_COMB, 1, seed=2)
    bad = fr.pilot.copy()
    bad[4] = 0.0
    with pytest.raises(ValueError):
        _run(fr.__class__(**{**fr.__dict__, "pilot": bad}))
