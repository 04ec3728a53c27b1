"""Pins of the oracle's receive path against what the paper and mathematics fix.

Paper Section II-B: the CP is removed and an FFT taken on every antenna; the
first symbol drives block LS; later symbols are demodulated.  Section II-C: LS
divides each received subcarrier by the pilot; MRC sums per subcarrier over
antennas; subcarriers are in fftshift order.  None of these pins re-types the
oracle's own formulas: they use the transmitter's ground truth, closed forms,
invariants and special cases that reduce to numpy routines.
"""
import math

import numpy as np
import pytest

import oracle
from rxgen import C1, C2, C2_20DB, make_frames, qam_symbols, used_subcarrier_bins


def _kw(cfg, **over):
    d = dict(n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len, n_used=cfg.n_used,
             n_sym=cfg.n_sym, bits_per_sym=cfg.bits_per_sym)
    d.update(over)
    return d


def _signed_freqs(U):
    return np.concatenate([np.arange(-U // 2, 0), np.arange(1, U // 2 + 1)])


# ----------------------------------------------------------------- subcarrier map
def test_subcarrier_map_tiny_workload_by_hand():
    # 52 used bins of a 64-point FFT: signed frequencies -26..-1 then +1..+26,
    # i.e. FFT bins 38..63 then 1..26 (DC = bin 0 and bins 27..37 unused).
    want = list(range(38, 64)) + list(range(1, 27))
    assert oracle.subcarrier_map(64, 52).tolist() == want


@pytest.mark.parametrize("n,u", [(64, 52), (1024, 600), (2048, 1200), (128, 72), (256, 2), (64, 62)])
def test_subcarrier_map_properties(n, u):
    k = oracle.subcarrier_map(n, u)
    assert len(set(k.tolist())) == u          # distinct
    assert 0 not in k                          # DC never used
    assert n // 2 not in k                     # Nyquist never used
    f = np.where(k > n // 2, k - n, k)         # back to signed frequency
    assert np.all(np.diff(f) > 0)              # ascending frequency (fftshift order)
    assert f[0] == -u // 2 and f[-1] == u // 2


def test_tone_lands_on_its_subcarrier_only():
    cfg = C1.replace(n_ant=2, n_sym=2)
    N, CP, U = cfg.fft_len, cfg.cp_len, cfg.n_used
    n = np.arange(-CP, N)
    for f in (-26, -1, 1, 13, 26):
        y = np.exp(2j * np.pi * f * n / N)
        buf = np.broadcast_to(y, (1, cfg.n_sym, cfg.n_ant, N + CP)).copy()
        r = oracle.process_frame(buf, np.ones(U), f64=True, **_kw(cfg))
        mag = np.abs(r.H[0, 0])
        d = int(np.nonzero(_signed_freqs(U) == f)[0][0])
        assert abs(mag[d] - N) < 1e-9
        assert np.max(np.delete(mag, d)) < 1e-9
    # a DC tone is on no used subcarrier
    buf = np.ones((1, cfg.n_sym, cfg.n_ant, N + CP), complex)
    r = oracle.process_frame(buf, np.ones(U), f64=True, **_kw(cfg))
    assert np.max(np.abs(r.H)) < 1e-9


# ----------------------------------------------------------------- CP removal + LS
@pytest.mark.parametrize("cfg", [C1, C2.replace(n_ant=4, n_sym=3)])
def test_pure_delay_channel_gives_linear_phase(cfg):
    N, U = cfg.fft_len, cfg.n_used
    for dly in (0, 1, cfg.cp_len // 2, cfg.cp_len):
        fr = make_frames(cfg, n_slots=1, channel="delay", delay=dly, noise=False, keep_float=True, scale=1.0)
        r = oracle.process_frame(fr.y, fr.pilot, f64=True, **_kw(cfg))
        want = math.sqrt(N) * np.exp(-2j * np.pi * _signed_freqs(U) * dly / N)
        assert np.max(np.abs(r.H[0] - want[None, :])) <= 1e-12 * math.sqrt(N)


def test_delay_beyond_cp_breaks_the_estimate():
    # One sample more than the CP: the FFT window now sees the previous
    # (here: empty) symbol, so the estimate is no longer a pure phase ramp.
    cfg = C1
    N, U = cfg.fft_len, cfg.n_used
    dly = cfg.cp_len + 1
    fr = make_frames(cfg.replace(cp_len=cfg.cp_len), n_slots=1, channel="delay", delay=dly,
                     noise=False, keep_float=True, scale=1.0)
    # the generator clamps delays to the CP only for Rayleigh taps; a pure delay is exact
    r = oracle.process_frame(fr.y, fr.pilot, f64=True, **_kw(cfg))
    want = math.sqrt(N) * np.exp(-2j * np.pi * _signed_freqs(U) * dly / N)
    assert np.max(np.abs(r.H[0] - want[None, :])) > 1e-2 * math.sqrt(N)


@pytest.mark.parametrize("cfg", [C1, C2.replace(n_ant=8, n_sym=3)])
def test_exact_channel_recovery_noiseless(cfg):
    fr = make_frames(cfg, n_slots=2, noise=False, keep_float=True)
    r = oracle.process_frame(fr.y, fr.pilot, f64=True, **_kw(cfg))
    scale = np.max(np.abs(fr.H_true))
    assert np.max(np.abs(r.H - fr.H_true)) <= 1e-12 * scale


def test_exact_channel_recovery_complex_non_unit_pilot():
    # LS divides by the pilot; with complex pilots of varying magnitude this
    # exercises both the conjugate and the 1/|X|^2 normalisation.
    cfg = C2.replace(n_ant=4, n_sym=3)
    rng = np.random.default_rng(5)
    pil = (rng.uniform(0.3, 2.0, cfg.n_used) * np.exp(2j * np.pi * rng.uniform(size=cfg.n_used)))
    fr = make_frames(cfg, n_slots=2, noise=False, keep_float=True, pilot=pil)
    r = oracle.process_frame(fr.y, fr.pilot, f64=True, **_kw(cfg))
    assert np.max(np.abs(r.H - fr.H_true)) <= 1e-12 * np.max(np.abs(fr.H_true))
    # and the data symbols come back exactly
    assert np.max(np.abs(r.xhat - fr.X)) <= 1e-12


def test_int16_channel_recovery_within_quantisation_bound():
    cfg = C2.replace(n_ant=8, n_sym=3)
    fr = make_frames(cfg, n_slots=2, noise=False)
    r = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    # each int16 component is off by at most 1/2 LSB; after an N-point FFT the
    # per-bin error is at most N * sqrt(2)/2 and its RMS is sqrt(N/6)
    err = np.abs(r.H - fr.H_true)
    N = cfg.fft_len
    assert np.max(err) <= N * math.sqrt(2) / 2
    assert np.sqrt(np.mean(err ** 2)) <= 1.2 * math.sqrt(N / 6)


def test_ls_error_variance_equals_noise_variance():
    cfg = C2_20DB.replace(n_sym=2)
    fr = make_frames(cfg, n_slots=3)
    r = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    N = cfg.fft_len
    # unit-modulus pilot: the LS error of every estimate is the FFT of the noise,
    # variance N * sigma^2 in time-domain units, times the int16 gain squared
    for s in range(3):
        want = N * 10 ** (-fr.snr_db[s] / 10) * fr.scale[s] ** 2
        got = np.mean(np.abs(r.H[s] - fr.H_true[s]) ** 2)
        assert abs(got / want - 1) < 0.02          # 38 400 estimates per slot
    nmse_db = 10 * np.log10(np.mean(np.abs(r.H - fr.H_true) ** 2 / (N * fr.scale[:, None, None] ** 2)))
    assert abs(nmse_db + 20.0) < 0.05              # -SNR in dB per unit channel power


# ----------------------------------------------------------------- combining
@pytest.mark.parametrize("cfg", [C1, C2.replace(n_ant=16, n_sym=3)])
def test_pilot_self_equalisation_any_noise(cfg):
    fr = make_frames(cfg.replace(snr_db=(0.0, 0.0)), n_slots=2)
    iq = fr.iq.copy()
    iq[:, 1] = iq[:, 0]             # data symbol 1 := the received pilot symbol itself
    r = oracle.process_frame(iq, fr.pilot, **_kw(cfg))
    assert np.max(np.abs(r.xhat[:, 0] - fr.pilot[None, :])) <= 1e-12


@pytest.mark.parametrize("cfg", [C1, C2.replace(n_ant=16, n_sym=4)])
def test_mrc_equals_zf_single_user(cfg):
    fr = make_frames(cfg, n_slots=2)
    a = oracle.process_frame(fr.iq, fr.pilot, combiner=oracle.MRC, **_kw(cfg))
    b = oracle.process_frame(fr.iq, fr.pilot, combiner=oracle.ZF, **_kw(cfg))
    assert np.max(np.abs(a.xhat - b.xhat)) <= 1e-12 * max(1.0, np.max(np.abs(a.xhat)))


def test_single_antenna_reduces_to_ratio_of_numpy_ffts():
    cfg = C2.replace(n_ant=1, n_sym=4)
    fr = make_frames(cfg, n_slots=1)
    r = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    N, CP = cfg.fft_len, cfg.cp_len
    y = fr.iq[0, :, 0, CP:, 0].astype(float) + 1j * fr.iq[0, :, 0, CP:, 1]
    Y = np.fft.fft(y, axis=-1)[:, used_subcarrier_bins(N, cfg.n_used)]
    want = Y[1:] / Y[0][None, :] * fr.pilot[None, :]
    assert np.max(np.abs(r.xhat[0] - want)) <= 1e-10 * max(1.0, np.max(np.abs(want)))


def test_scale_invariance():
    cfg = C1
    fr = make_frames(cfg, n_slots=1)
    small = (fr.iq // 2).astype(np.int16)        # any int16 input will do; halved so doubling cannot wrap
    a = oracle.process_frame(small, fr.pilot, **_kw(cfg))
    b = oracle.process_frame((small.astype(np.int32) * 2).astype(np.int16), fr.pilot, **_kw(cfg))
    assert np.max(np.abs(b.H - 2 * a.H)) <= 1e-12 * np.max(np.abs(a.H))
    assert np.max(np.abs(b.xhat - a.xhat)) <= 1e-12
    assert np.array_equal(a.bits, b.bits)


def test_xhat_recovers_transmitted_symbols_statistically():
    cfg = C2_20DB.replace(n_sym=4)
    fr = make_frames(cfg, n_slots=2)
    r = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    evm = np.sqrt(np.mean(np.abs(r.xhat - fr.X) ** 2))
    # 64 antennas at 20 dB: post-combining SNR ~ 38 dB, LS error adds about the same
    assert evm < 0.03


# ----------------------------------------------------------------- demap + packing
@pytest.mark.parametrize("b", [2, 4, 6])
def test_demap_inverts_the_transmit_map_and_gray(b):
    allbits = ((np.arange(2 ** b)[:, None] >> np.arange(b)[::-1][None, :]) & 1).astype(np.uint8)
    pts = qam_symbols(allbits, b)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-12        # unit average energy
    assert len(set(np.round(pts, 9).tolist())) == 2 ** b        # distinct points
    assert np.array_equal(oracle.demap(pts, b), allbits)        # exact round trip
    # Gray: nearest neighbours along an axis differ in exactly one bit
    step = {2: math.sqrt(2) * 2 / 2, 4: 2 / math.sqrt(10), 6: 2 / math.sqrt(42)}[b]
    for i, p in enumerate(pts):
        for q, j in ((p + step, None), (p + 1j * step, None)):
            near = np.nonzero(np.abs(pts - q) < 1e-9)[0]
            for j in near:
                assert np.sum(allbits[i] != allbits[j]) == 1


def test_demap_ties_and_negative_zero_give_zero_bits():
    z = np.array([0.0 + 0.0j, complex(-0.0, -0.0)])
    assert oracle.demap(z, 2).tolist() == [[0, 0], [0, 0]]
    assert oracle.demap(z, 4).tolist() == [[0, 0, 0, 0], [0, 0, 0, 0]]
    # 64-QAM at the origin: |u| - 4 = -4, so the third bit of each axis is 1
    assert oracle.demap(z, 6).tolist() == [[0, 0, 0, 0, 1, 1], [0, 0, 0, 0, 1, 1]]


def test_all_zero_slot_gives_zero_symbols():
    cfg = C1
    iq = np.zeros((1, cfg.n_sym, cfg.n_ant, cfg.fft_len + cfg.cp_len, 2), np.int16)
    pilot = make_frames(cfg, n_slots=1).pilot
    r = oracle.process_frame(iq, pilot, **_kw(cfg))
    assert np.all(r.g == 0) and np.all(r.xhat == 0)
    assert np.all(r.bits == 0)          # QPSK: 00 per symbol


def test_bit_packing_fixed_pattern():
    # QPSK points with known bit pairs (b0 b1): (0,0) (0,1) (1,0) (1,1) -> bits
    # 00 01 10 11 -> one byte 0b00011011 = 0x1B, MSB first; then 11 10 01 00 = 0xE4.
    cfg = C1.replace(n_ant=1, n_used=8, n_sym=2)
    N, CP = cfg.fft_len, cfg.cp_len
    seq = [(0, 0), (0, 1), (1, 0), (1, 1), (1, 1), (1, 0), (0, 1), (0, 0)]
    X = qam_symbols(np.array(seq, np.uint8), 2)
    bins = used_subcarrier_bins(N, 8)
    grid = np.zeros((2, N), complex)
    grid[0, bins] = 1.0
    grid[1, bins] = X
    x = np.fft.ifft(grid, axis=1) * N
    y = np.concatenate([x[:, N - CP:], x], axis=1)[None, :, None, :]
    r = oracle.process_frame(y, np.ones(8), f64=True, **_kw(cfg))
    assert r.bits[0, 0].tolist() == [0x1B, 0xE4]


@pytest.mark.parametrize("b", [2, 4, 6])
@pytest.mark.parametrize("A", [1, 8, 64])
def test_zero_bit_errors_noiseless_flat_channel(b, A):
    base = {2: C1, 4: C2, 6: C2}[b]
    cfg = base.replace(n_ant=A, n_sym=4, bits_per_sym=b, n_used=base.n_used)
    fr = make_frames(cfg, n_slots=2, channel="flat", noise=False)
    r = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    assert np.array_equal(r.bits, fr.packed_bits())
