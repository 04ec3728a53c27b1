"""rx_process_frame_noalloc (the entry point for callers that cannot
allocate) against rx_process_frame on the same inputs, through the C ABI:
two calls in a row, the second with fewer slots, and a workload larger than
the library's fixed scratch (several chunks).  Results must be identical."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from rxgen import C2, make_frames  # noqa: E402


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _noalloc(rx, plan, iq, S, cfg):
    x = torch.full((S, cfg.n_sym - 1, cfg.n_used, 2), float("nan"), device="cuda")
    b = torch.full((S, cfg.n_sym - 1, plan.row_bytes), 0xAA, dtype=torch.uint8, device="cuda")
    st = rx.rx_process_frame_noalloc(plan._plan, iq.data_ptr(), S, x.data_ptr(), b.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == rx.RX_OK, st
    return x, b


@pytest.mark.parametrize("combiner", [0, 1])
def test_noalloc_equals_process_frame_two_calls(rx, combiner):
    # 64 antennas x 600 subcarriers: 307 200 B of estimate per slot, so 218 slots
    # per 64 MiB chunk; 240 slots take two chunks, then 5 slots one
    cfg = C2.replace(n_slots=240, n_sym=4)
    uniq = make_frames(cfg, n_slots=6)
    src = np.arange(cfg.n_slots) % 6
    iq = torch.from_numpy(uniq.iq).cuda()[torch.from_numpy(src).cuda()].contiguous()
    plan = rx.Plan.from_config(cfg, uniq.pilot, combiner)
    for S in (cfg.n_slots, 5):
        _say("noalloc", "combiner", combiner, "S", S)
        sub = iq[:S]
        _, xr, br = plan.process(sub)
        xn, bn = _noalloc(rx, plan, sub, S, cfg)
        torch.cuda.synchronize()
        assert torch.equal(xn, xr) and torch.equal(bn, br)


def test_noalloc_argument_errors(rx):
    cfg = C2.replace(n_slots=1, n_sym=2)
    fr = make_frames(cfg, n_slots=1)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    x = torch.zeros((1, 1, cfg.n_used, 2), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert rx.rx_process_frame_noalloc(plan._plan, iq.data_ptr(), 1, None, None, s) == rx.RX_E_INVALID_ARG
    assert rx.rx_process_frame_noalloc(None, iq.data_ptr(), 1, x.data_ptr(), None, s) == rx.RX_E_INVALID_ARG
    assert rx.rx_process_frame_noalloc(plan._plan, iq.data_ptr(), 0, None, None, s) == rx.RX_OK
    # one slot's estimate larger than the scratch: 8192 antennas x 1200 subcarriers x 8 B
    big = C2.replace(n_ant=8192, fft_len=2048, cp_len=144, n_used=1200, n_sym=2, bits_per_sym=2)
    pbig = rx.Plan.from_config(big, np.ones(1200))
    assert 8192 * 1200 * 8 > rx.RX_NOALLOC_SCRATCH_BYTES
    assert rx.rx_process_frame_noalloc(pbig._plan, iq.data_ptr(), 1, x.data_ptr(), None, s) == rx.RX_E_SCRATCH
