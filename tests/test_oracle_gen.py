"""Pins of the oracle's training-channel generator.

Philox4x64-10 is checked against numpy's independent implementation; the
frequency response against the oracle FFT of the drawn impulse response
(itself pinned to the brute-force DFT); the draws against their stated
ranges and statistics (unit mean channel power, exponential profile, noise
variance from the SNR), and the noisy estimate against the comb interpolation.
"""
import numpy as np
import pytest

import oracle

GP = oracle.GenParams()


@pytest.mark.parametrize("ctr,key", [([0, 0, 0, 0], [0, 0]), ([5, 7, 0, 0], [123, 0]),
                                     ([2**63, 1, 2, 3], [2**64 - 1, 17]), ([99, 2**40, 0, 5], [1, 2])])
def test_philox_matches_numpy(ctr, key):
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    raw = bg.random_raw(8)
    # numpy increments the counter's first word before each block
    c1 = [ctr[0] + 1, ctr[1], ctr[2], ctr[3]]
    c2 = [ctr[0] + 2, ctr[1], ctr[2], ctr[3]]
    np.testing.assert_array_equal(raw[:4], oracle.philox4x64(c1, key))
    np.testing.assert_array_equal(raw[4:], oracle.philox4x64(c2, key))


def test_deterministic_and_row_addressable():
    a = oracle.gen_channels(GP, 5, 0, 20)
    b = oracle.gen_channels(GP, 5, 12, 8)
    np.testing.assert_array_equal(a[0][12:], b[0])
    np.testing.assert_array_equal(a[1][12:], b[1])
    c = oracle.gen_channels(GP, 6, 0, 20)
    assert not np.array_equal(a[0], c[0])


def test_frequency_response_is_fft_of_impulse_response():
    N, U = GP.fft_len, GP.n_used
    ht, _, dr = oracle.gen_channels(GP, 9, 100, 6, draws=True)
    bins = oracle.subcarrier_map(N, U)
    for r in range(6):
        L = dr["n_taps"][r]
        imp = np.zeros(N, dtype=complex)
        for l in range(L):
            imp[dr["delays"][r, l]] += dr["taps"][r, l]
        np.testing.assert_allclose(ht[r], oracle.fft(imp)[bins], rtol=0, atol=1e-12)


def test_draw_ranges_and_delay_rule():
    gp = oracle.GenParams(taps=(8, 24), tau_samples=(15, 154), cp_len=144)
    _, _, dr = oracle.gen_channels(gp, 1, 0, 3000, draws=True)
    L = dr["n_taps"]
    assert L.min() == 8 and L.max() == 24
    assert np.all((dr["snr_db"] >= 0) & (dr["snr_db"] <= 30))
    for r in range(200):
        d = dr["delays"][r, :L[r]]
        assert d[0] == 0 and np.all(np.diff(d) >= 0) and d.max() <= 144
        assert np.all(dr["delays"][r, L[r]:] == 0)
    # two-tap rows put the second tap at the drawn span exactly
    gp2 = oracle.GenParams(taps=(2, 2), tau_samples=(30, 30))
    _, _, dr2 = oracle.gen_channels(gp2, 1, 0, 5, draws=True)
    assert np.all(dr2["delays"][:, :2] == [0, 30])
    # delays round l * span / (L - 1) to the nearest sample, halves up: 5 / 2 -> 3
    gp3 = oracle.GenParams(taps=(3, 3), tau_samples=(5, 5))
    _, _, dr3 = oracle.gen_channels(gp3, 1, 0, 2, draws=True)
    assert np.all(dr3["delays"][:, :3] == [0, 3, 5])
    # and never past the cyclic prefix
    gp4 = oracle.GenParams(taps=(2, 2), tau_samples=(200, 200), cp_len=144)
    _, _, dr4 = oracle.gen_channels(gp4, 1, 0, 2, draws=True)
    assert np.all(dr4["delays"][:, :2] == [0, 144])


def test_channel_power_and_profile():
    gp = oracle.GenParams(taps=(10, 10))
    ht, _, dr = oracle.gen_channels(gp, 2, 0, 4000, draws=True)
    assert abs(np.mean(np.abs(ht) ** 2) - 1.0) < 0.05
    p = np.mean(np.abs(dr["taps"][:, :10]) ** 2, axis=0)
    want = 10 ** (-0.3 * np.arange(10))
    want /= want.sum()
    np.testing.assert_allclose(p, want, rtol=0.1)


def test_noise_variance_follows_snr():
    gp = oracle.GenParams(snr_db=(10.0, 10.0), pilot_spacing=1)
    ht, hl = oracle.gen_channels(gp, 3, 0, 500)
    assert abs(np.mean(np.abs(hl - ht) ** 2) / 0.1 - 1.0) < 0.03
    # the noise has no mean and is circular
    n = (hl - ht).reshape(-1)
    assert abs(np.mean(n)) < 0.01 and abs(np.mean(n * n)) < 0.01


def test_noise_independent_of_taps():
    # noise and tap gains come from different Philox blocks: no correlation
    gp = oracle.GenParams(snr_db=(0.0, 0.0), taps=(2, 2), tau_samples=(0, 0), pilot_spacing=1)
    ht, hl, dr = oracle.gen_channels(gp, 8, 0, 4000, draws=True)
    n = hl - ht
    for j in (0, 1):
        for l in (0, 1):
            h = dr["taps"][:, l]
            c = np.mean(n[:, j] * np.conj(h)) / np.sqrt(np.mean(np.abs(n[:, j]) ** 2) * np.mean(np.abs(h) ** 2))
            assert abs(c) < 0.1


def test_uniforms_are_odd_multiples_of_2_pow_minus_24():
    # u = (2k + 1) 2^-24: strictly inside (0, 1); seen through snr = 30 u
    _, _, dr = oracle.gen_channels(GP, 12, 0, 500, draws=True)
    k2 = dr["snr_db"] / 30.0 * 2.0 ** 24
    assert np.allclose(k2, np.rint(k2), atol=1e-6)
    assert np.all(np.rint(k2).astype(np.int64) % 2 == 1)


def test_noisy_estimate_is_comb_interpolation_of_noisy_pilots():
    ht, hl = oracle.gen_channels(GP, 4, 0, 3)
    on = np.arange(GP.n_used) % GP.pilot_spacing == 0
    again = oracle.comb_interp(np.where(on, hl, 0), GP.pilot_spacing)
    np.testing.assert_array_equal(again, hl)
    # noiseless (very high SNR) estimates approach the truth on the comb
    hi = oracle.GenParams(snr_db=(200.0, 200.0))
    t2, l2 = oracle.gen_channels(hi, 4, 0, 3)
    np.testing.assert_allclose(l2[:, on], t2[:, on], atol=1e-9)


def test_rejects_bad_parameters():
    for bad in (dict(fft_len=1000), dict(n_used=7), dict(pilot_spacing=0), dict(taps=(0, 3)),
                dict(taps=(5, 4)), dict(tau_samples=(10, 5)), dict(taps=(1, 65))):
        with pytest.raises(ValueError):
            oracle.gen_channels(oracle.GenParams(**bad), 0, 0, 1)
