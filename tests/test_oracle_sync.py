"""Pins of the oracle's PN frame synchronisation and slot extraction.

The paper correlates the received stream with the maximum-length PN sequence
(length 255, Table I) that opens each frame and takes the correlation peak as
the offset of the first OFDM frame (Sec. II-B).  Pins: the m-sequence's
defining properties; the metric against numpy's correlate (a library routine)
and closed forms; shift equivariance; the first-maximum rule; and extraction
against the transmitter's own slot buffer.
"""
import numpy as np
import pytest

import oracle
from rxgen import C1, C2, make_stream, pn_sequence


def test_pn_is_a_maximum_length_sequence():
    p = pn_sequence()
    assert p.size == 255 and set(np.unique(p)) == {-1.0, 1.0}
    assert (p < 0).sum() == 128 and (p > 0).sum() == 127       # 2^(n-1) ones
    # two-valued periodic autocorrelation: 255 at lag 0, -1 elsewhere
    ac = np.array([np.dot(p, np.roll(p, k)) for k in range(255)])
    assert ac[0] == 255 and np.all(ac[1:] == -1)
    # period exactly 255
    q = pn_sequence(length=510)
    assert np.array_equal(q[:255], q[255:])
    for per in (3, 5, 15, 17, 51, 85):          # the proper divisors of 255 are not periods
        assert not np.array_equal(q[:255 - per], q[per:255])


def _rand_stream(A, n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-3000, 3000, size=(A, n, 2)).astype(np.int16)


def test_metric_matches_numpy_correlate():
    raw = _rand_stream(3, 700, 1)
    p = pn_sequence()
    n_search = 700 - 255 + 1
    M, off = oracle.sync_metric(raw, p, n_search)
    want = np.zeros(n_search)
    for a in range(3):
        y = raw[a, :, 0].astype(np.float64) + 1j * raw[a, :, 1]
        c = np.correlate(y, p, mode="valid")
        want += np.abs(c) ** 2
    np.testing.assert_array_equal(M.astype(np.float64), np.rint(want))
    assert off == int(np.argmax(want))


def test_closed_form_peak_and_zero_tail():
    p = pn_sequence()
    A, n, o, c = 2, 1000, 333, 7
    raw = np.zeros((A, n, 2), dtype=np.int16)
    raw[0, o:o + 255, 0] = (c * p).astype(np.int16)
    raw[1, o:o + 255, 1] = (-c * p).astype(np.int16)
    M, off = oracle.sync_metric(raw, p, n)            # candidates past n - 255 see zeros
    assert off == o and int(M[o]) == 2 * (255 * c) ** 2
    assert np.all(M[np.arange(n) != o] < M[o])
    assert int(M[n - 1]) == 0


def test_shift_equivariance_and_antenna_sum():
    raw = _rand_stream(2, 900, 3)
    p = pn_sequence()
    M, _ = oracle.sync_metric(raw, p, 500)
    Ms, _ = oracle.sync_metric(raw[:, 40:], p, 460)
    np.testing.assert_array_equal(Ms, M[40:])
    M0, _ = oracle.sync_metric(raw[:1], p, 500)
    M1, _ = oracle.sync_metric(raw[1:], p, 500)
    np.testing.assert_array_equal(M, M0 + M1)


def test_first_maximum_wins_ties():
    p = pn_sequence()
    raw = np.zeros((1, 1200, 2), dtype=np.int16)
    raw[0, 100:355, 0] = p.astype(np.int16)
    raw[0, 700:955, 0] = p.astype(np.int16)
    M, off = oracle.sync_metric(raw, p, 900)
    assert M[100] == M[700] and off == 100


def test_sync_finds_the_preamble_on_a_flat_channel():
    st = make_stream(C2.replace(n_ant=8, n_sym=3), 1, 517, seed=11, channel="flat", snr_db=0.0)
    M, off = oracle.sync_metric(st.raw, st.pn, 2000)
    assert off == st.lead


def test_sync_peak_at_a_tap_delay_with_multipath():
    st = make_stream(C2.replace(n_ant=16, n_sym=3), 1, 300, seed=12, snr_db=10.0)
    _, off = oracle.sync_metric(st.raw, st.pn, 1500)
    assert off - st.lead in set(st.delays.tolist())


@pytest.mark.parametrize("lead", [0, 1, 250])
def test_extraction_gives_the_transmitted_slot_buffer(lead):
    st = make_stream(C1, 3, lead, seed=13)
    cfg = st.frames.cfg
    out = oracle.extract_slots(st.raw, lead + 255, 3, cfg.n_sym, cfg.fft_len + cfg.cp_len)
    np.testing.assert_array_equal(out, st.frames.iq)


def test_extraction_past_the_stream_reads_zeros():
    raw = _rand_stream(2, 100, 5)
    out = oracle.extract_slots(raw, 90, 1, 2, 8)
    np.testing.assert_array_equal(out[0, 0, :, :8], raw[:, 90:98])
    np.testing.assert_array_equal(out[0, 1, :, :2], raw[:, 98:100])
    assert not out[0, 1, :, 2:].any()
    neg = oracle.extract_slots(raw, -3, 1, 1, 8)
    assert not neg[0, 0, :, :3].any()
    np.testing.assert_array_equal(neg[0, 0, :, 3:], raw[:, :5])


def test_end_to_end_sync_then_receive_is_error_free_at_high_snr():
    st = make_stream(C2.replace(n_ant=16), 1, 400, seed=14, channel="flat", snr_db=30.0)
    cfg = st.frames.cfg
    _, off = oracle.sync_metric(st.raw, st.pn, 1000)
    iq = oracle.extract_slots(st.raw, off + 255, 1, cfg.n_sym, cfg.fft_len + cfg.cp_len)
    r = oracle.process_frame(iq, st.frames.pilot, n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len,
                             n_used=cfg.n_used, n_sym=cfg.n_sym, bits_per_sym=cfg.bits_per_sym)
    np.testing.assert_array_equal(r.bits, st.frames.packed_bits())
