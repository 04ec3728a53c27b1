"""GPU parity of batched mixed-shape frames (one graph launch) against the FP64 oracle per frame."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from rxgen import make_batch  # noqa: E402
from tests.parity import check_bits, check_H, check_xhat  # noqa: E402


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _check_frames(batch, bt, H, x, b, refs=None):
    Hc = H.cpu().numpy().astype(np.float64)
    xc = x.cpu().numpy().astype(np.float64)
    bc = b.cpu().numpy()
    for i, fr in enumerate(bt.frames):
        c = fr.cfg
        ref = refs[i] if refs is not None else oracle.run_config(fr)
        Hi = Hc[batch.h_off[i]:batch.h_off[i + 1]].reshape(1, c.n_ant, c.n_used, 2)
        xi = xc[batch.x_off[i]:batch.x_off[i + 1]].reshape(1, c.n_sym - 1, c.n_used, 2)
        bi = bc[batch.b_off[i]:batch.b_off[i + 1]].reshape(1, c.n_sym - 1, -1)
        check_H(Hi[..., 0] + 1j * Hi[..., 1], ref.H)
        check_xhat(xi[..., 0] + 1j * xi[..., 1], ref.xhat)
        check_bits(bi, ref.bits, ref.xhat, c.bits_per_sym)


def _make(rx, n, seed, **kw):
    bt = make_batch(n, seed, **kw)
    batch = rx.Batch(bt.configs, [f.pilot for f in bt.frames])
    iq = torch.from_numpy(bt.iq).cuda()
    return bt, batch, iq


def test_batch_every_fft_length_matches_oracle(rx):
    _say("batch mixed", 14, 31)
    bt, batch, iq = _make(rx, 14, 31, antennas=(3, 8, 17), fft_lens=(64, 128, 256, 512, 1024, 2048))
    assert len({c.fft_len for c in bt.configs}) >= 4
    out = batch.outputs(iq.device)
    batch.process(iq, out)
    torch.cuda.synchronize()
    _check_frames(batch, bt, *out[:3])
    lat = batch.frame_latency_ms()
    assert np.all(np.isfinite(lat)) and np.all(lat > 0) and np.all(lat < 1e4)


def test_batch_autotune_then_graph_replays(rx):
    _say("batch autotune", 9, 32)
    bt, batch, iq = _make(rx, 9, 32, antennas=(4, 16), fft_lens=(128, 1024, 2048))
    out = batch.outputs(iq.device)
    batch.autotune(iq, out, reps=1)
    for n in sorted({c.fft_len for c in bt.configs}):
        w, j = batch.config(n)
        assert w in (2, 4, 8) and j in (2, 4, 8)
        sd, se = batch.schedules(n)
        assert rx.fft_radices(n, sd) is not None and rx.fft_radices(n, se) is not None
    x_prev = None
    for rep in range(3):                      # replays of the same graph, eager work between them
        out[1].fill_(float("nan"))
        batch.process(iq, out)
        torch.cuda.synchronize()
        _check_frames(batch, bt, *out[:3])
        if x_prev is not None:
            assert torch.equal(out[1], x_prev)
        x_prev = out[1].clone()


@pytest.mark.parametrize("sched", [(1, 1), (1, 0), (0, 1)])
def test_batch_forced_radix_schedules_match_oracle(rx, sched):
    # each radix schedule of each kernel, on every length that has two, and
    # the demod at every workgroup size; lengths with one schedule keep it
    sd, se = sched
    _say("batch schedules", sched, 12, 34)
    bt, batch, iq = _make(rx, 12, 34, antennas=(3, 17, 40), fft_lens=(256, 512, 1024, 2048))
    lens = sorted({c.fft_len for c in bt.configs})
    assert {512, 1024, 2048} <= set(lens)
    out = batch.outputs(iq.device)
    refs = [oracle.run_config(fr) for fr in bt.frames]
    for w, j in ((2, 8), (4, 2), (8, 4)):
        for n in lens:
            two = rx.fft_radices(n, 1) is not None
            batch.set_config(n, w, j, sd if two else 0, se if two else 0)
            assert batch.config(n) == (w, j)
            assert batch.schedules(n) == ((sd, se) if two else (0, 0))
        out[1].fill_(float("nan"))
        batch.process(iq, out)
        torch.cuda.synchronize()
        _check_frames(batch, bt, *out[:3], refs=refs)
    with pytest.raises(rx.RxError):
        batch.set_config(256, 4, 4, 1, 0)            # 256 has one schedule
    with pytest.raises(rx.RxError):
        batch.set_config(1024, 3, 4, 0, 0)
    assert batch.schedules(256) == (0, 0) and batch.config(1024) == (8, 4)


def test_batch_new_buffers_and_workspace(rx):
    _say("batch buffers", 5, 33)
    bt, batch, iq = _make(rx, 5, 33, antennas=(8,), fft_lens=(256, 512))
    out1 = batch.outputs(iq.device, want_H=True)
    out2 = batch.outputs(iq.device, want_H=False)   # estimates in the workspace
    batch.process(iq, out1)
    batch.process(iq, out2)
    torch.cuda.synchronize()
    assert torch.equal(out1[1], out2[1]) and torch.equal(out1[2], out2[2])


def test_batch_rejects_bad_frames(rx):
    from rxgen import batch_frame_config
    c = batch_frame_config(1, 0)
    bad = c.replace(bits_per_sym=3)
    with pytest.raises(rx.RxError):
        rx.Batch([c, bad], [np.ones(c.n_used), np.ones(bad.n_used)])
