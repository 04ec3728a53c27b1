"""GPU parity of PN frame synchronisation and slot extraction against the
oracle, through the C ABI.  The metric is integer arithmetic on both sides,
so the metric, the peak and the offset must be bit-exact, and so must the
extracted samples."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from rxgen import C1, C2, make_stream, pn_sequence  # noqa: E402
from tests.parity import as_complex, check_bits, check_xhat  # noqa: E402


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _check_find(rx, raw, pn, n_search, n_samples=None):
    off, peak, M = rx.sync_find(torch.from_numpy(raw).cuda(), pn, n_search, n_samples=n_samples, want_metric=True)
    torch.cuda.synchronize()
    rM, roff = oracle.sync_metric(raw, pn, n_search, n_samples=n_samples)
    np.testing.assert_array_equal(_u64(M), rM)
    assert off.item() == roff and _u64(peak)[0] == rM[roff]
    return roff


@pytest.mark.parametrize("A,n,stride,n_search,L", [(5, 3000, 3100, 2500, 255), (1, 600, 600, 600, 255),
                                                   (7, 1000, 1024, 300, 31), (3, 5000, 5000, 4900, 1023),
                                                   (2, 200, 256, 1, 1)])
def test_metric_matches_oracle_on_random_streams(rx, A, n, stride, n_search, L):
    _say("sync metric", A, n, stride, n_search, L)
    rng = np.random.default_rng(A * 1000 + L)
    raw = rng.integers(-32768, 32768, size=(A, stride, 2)).astype(np.int16)
    pn = rng.choice([-1, 0, 1], size=L) if L != 255 else pn_sequence()
    _check_find(rx, raw, pn, n_search, n_samples=n)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13, 16, 18, 20, 23, 24, 29, 44, 1021, 1024])
def test_metric_every_chip_count_path(rx, L):
    # chip lengths covering each way the correlation loop ends: whole groups of
    # twelve chips, one or two further steps of four, and a tail of 0..3 chips
    _say("sync metric chips", L)
    rng = np.random.default_rng(7000 + L)
    raw = rng.integers(-32768, 32768, size=(3, 1200 + L, 2)).astype(np.int16)
    pn = rng.choice([-1, 0, 1], size=L)
    _check_find(rx, raw, pn, 1100, n_samples=1180 + L)


def test_full_scale_extremes_stay_exact(rx):
    pn = pn_sequence()
    raw = np.full((8, 800, 2), -32768, dtype=np.int16)
    raw[:, ::2] = 32767
    _check_find(rx, raw, pn, 600)
    raw2 = np.zeros((4, 700, 2), dtype=np.int16)
    raw2[:, 100:355, 0] = np.where(pn > 0, 32767, -32768)
    raw2[:, 100:355, 1] = np.where(pn > 0, -32768, 32767)
    assert _check_find(rx, raw2, pn, 700) == 100


def test_ties_resolve_to_the_first_offset(rx):
    pn = pn_sequence()
    raw = np.zeros((2, 3000, 2), dtype=np.int16)
    for o in (1500, 129, 2000):
        raw[:, o:o + 255, 0] = (pn * 9).astype(np.int16)
    assert _check_find(rx, raw, pn, 3000) == 129


@pytest.mark.parametrize("channel,snr", [("flat", 0.0), ("rayleigh", 10.0)])
def test_preamble_offset_matches_oracle(rx, channel, snr):
    st = make_stream(C2.replace(n_ant=16, n_sym=3), 2, 777, seed=21, channel=channel, snr_db=snr)
    _say("sync stream", channel, snr)
    off = _check_find(rx, st.raw, st.pn, 3000)
    if channel == "flat":
        assert off == st.lead
    else:
        assert off - st.lead in set(st.delays.tolist())


@pytest.mark.parametrize("lead", [0, 3, 1000])
def test_extraction_is_exact(rx, lead):
    st = make_stream(C1, 3, lead, seed=22)
    cfg = st.frames.cfg
    raw = torch.from_numpy(st.raw).cuda()
    start = torch.tensor([lead], dtype=torch.int64, device="cuda")
    iq = rx.sync_extract(raw, start, 255, cfg.fft_len + cfg.cp_len, cfg.n_sym, 3)
    iq0 = rx.sync_extract(raw, None, lead + 255, cfg.fft_len + cfg.cp_len, cfg.n_sym, 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(iq.cpu().numpy(), st.frames.iq)
    np.testing.assert_array_equal(iq0.cpu().numpy(), st.frames.iq)


def test_extraction_outside_the_stream_is_zero(rx):
    rng = np.random.default_rng(5)
    raw = rng.integers(-100, 100, size=(3, 120, 2)).astype(np.int16)
    t = torch.from_numpy(raw).cuda()
    for start in (-7, 100, 400):
        out = rx.sync_extract(t, None, start, 9, 2, 2, n_samples=110)
        torch.cuda.synchronize()
        want = oracle.extract_slots(raw, start, 2, 2, 9, n_samples=110)
        np.testing.assert_array_equal(out.cpu().numpy(), want)


def test_sync_extract_receive_end_to_end(rx):
    st = make_stream(C2.replace(n_ant=32), 2, 611, seed=23, snr_db=20.0)
    cfg = st.frames.cfg
    _say("sync end to end", cfg.seed)
    raw = torch.from_numpy(st.raw).cuda()
    off, _, _ = rx.sync_find(raw, st.pn, 4000)
    iq = rx.sync_extract(raw, off, 255, cfg.fft_len + cfg.cp_len, cfg.n_sym, 2)
    plan = rx.Plan.from_config(cfg, st.frames.pilot)
    _, xhat, bits = plan.process(iq)
    torch.cuda.synchronize()
    roff = oracle.sync_metric(st.raw, st.pn, 4000)[1]
    assert off.item() == roff
    riq = oracle.extract_slots(st.raw, roff + 255, 2, cfg.n_sym, cfg.fft_len + cfg.cp_len)
    np.testing.assert_array_equal(iq.cpu().numpy(), riq)
    ref = oracle.process_frame(riq, st.frames.pilot, n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len,
                               n_used=cfg.n_used, n_sym=cfg.n_sym, bits_per_sym=cfg.bits_per_sym)
    check_xhat(as_complex(xhat), ref.xhat)
    check_bits(bits.cpu().numpy(), ref.bits, ref.xhat, cfg.bits_per_sym)


def test_argument_errors(rx):
    raw = torch.zeros((2, 100, 2), dtype=torch.int16, device="cuda")
    off = torch.zeros((1,), dtype=torch.int64, device="cuda")
    ws = torch.empty((4096,), dtype=torch.uint8, device="cuda")
    chips, cp = rx._chips(np.array([1, 2, -1]))
    assert rx.rx_sync_find(raw.data_ptr(), 2, 100, 100, cp, 3, 50, None, off.data_ptr(), None, ws.data_ptr(),
                           None) == rx.RX_E_INVALID_ARG          # chip 2
    chips, cp = rx._chips(np.array([1, -1]))
    assert rx.rx_sync_find(raw.data_ptr(), 0, 100, 100, cp, 2, 50, None, off.data_ptr(), None, ws.data_ptr(),
                           None) == rx.RX_E_INVALID_ARG          # no antenna
    assert rx.rx_sync_find(raw.data_ptr(), 2, 100, 90, cp, 2, 50, None, off.data_ptr(), None, ws.data_ptr(),
                           None) == rx.RX_E_INVALID_ARG          # stride < n_samples
    assert rx.rx_sync_find(raw.data_ptr(), 2, 100, 100, cp, 2, 0, None, off.data_ptr(), None, ws.data_ptr(),
                           None) == rx.RX_E_INVALID_ARG          # empty search
    assert rx.rx_sync_find(raw.data_ptr(), 2, 100, 100, cp, 2, 50, None, None, None, ws.data_ptr(),
                           None) == rx.RX_E_INVALID_ARG          # no offset output
    assert rx.rx_sync_extract(raw.data_ptr(), 2, 100, 100, None, 0, 8, 2, 0, None, None) == rx.RX_OK
    assert rx.rx_sync_extract(raw.data_ptr(), 2, 100, 100, None, 0, 0, 2, 1, raw.data_ptr(), None) == \
        rx.RX_E_INVALID_ARG
