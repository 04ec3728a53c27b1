"""GPU parity: librx.so through its C ABI against the FP64 oracle, on the same seeded inputs.

Every case prints its name, shape and seed before touching the GPU so that a
failure can be traced from the log alone.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from rxgen import C1, C2, C4, make_frames  # noqa: E402
from tests.parity import as_complex, check_bits, check_H, check_xhat  # noqa: E402


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod   # raises if librx.so is missing
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _kw(cfg):
    return dict(n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len, n_used=cfg.n_used,
                n_sym=cfg.n_sym, bits_per_sym=cfg.bits_per_sym)


def _run_both(rx, cfg, fr, combiner=0):
    plan = rx.Plan.from_config(cfg, fr.pilot, combiner)
    iq = torch.from_numpy(fr.iq).cuda()
    H, xhat, bits = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, combiner=combiner, **_kw(cfg))
    return plan, iq, (as_complex(H), as_complex(xhat), bits.cpu().numpy()), ref


# ---------------------------------------------------------------- FFT stage
@pytest.mark.parametrize("N,cp,U", [(64, 16, 52), (128, 9, 72), (256, 18, 180), (512, 37, 300),
                                    (1024, 72, 600), (2048, 144, 1200)])
def test_fft_stage_matches_oracle(rx, N, cp, U):
    cfg = C2.replace(n_ant=5, fft_len=N, cp_len=cp, n_used=U, n_sym=3, bits_per_sym=4)
    _say("fft", N, cfg.seed)
    fr = make_frames(cfg, n_slots=2)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    Y = as_complex(plan.debug_fft(torch.from_numpy(fr.iq).cuda()))
    ref = oracle.fft_symbols(fr.iq, fr.pilot, **_kw(cfg))
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=-1, keepdims=True))
    assert np.max(np.abs(Y - ref) / rms) < 1e-5


def test_fft_stage_random_full_scale_input(rx):
    # arbitrary int16 (not OFDM-shaped), including the extreme values
    rng = np.random.default_rng(11)
    cfg = C2.replace(n_ant=3, n_sym=2)
    iq = rng.integers(-32768, 32768, size=(1, 2, 3, cfg.fft_len + cfg.cp_len, 2), dtype=np.int16)
    iq[0, 0, 0, cfg.cp_len:cfg.cp_len + 8] = -32768
    _say("fft-random", cfg.fft_len)
    pilot = np.ones(cfg.n_used)
    plan = rx.Plan.from_config(cfg, pilot)
    Y = as_complex(plan.debug_fft(torch.from_numpy(iq).cuda()))
    ref = oracle.fft_symbols(iq, pilot, **_kw(cfg))
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=-1, keepdims=True))
    assert np.max(np.abs(Y - ref) / rms) < 1e-5


# ---------------------------------------------------------------- whole path
CASES = {
    "c1_tiny": C1,
    "c2_shape_3slots": C2.replace(n_slots=3),
    "A37_ragged": C2.replace(n_ant=37, n_slots=2, n_sym=5),
    "N64_A5_qpsk": C1.replace(n_ant=5, n_slots=3),
    "N128_A16_64qam": C2.replace(n_ant=16, fft_len=128, cp_len=9, n_used=72, bits_per_sym=6, n_slots=2),
    "N256_A32_qpsk": C2.replace(n_ant=32, fft_len=256, cp_len=18, n_used=180, bits_per_sym=2, n_slots=2),
    "N512_A7_16qam": C2.replace(n_ant=7, fft_len=512, cp_len=37, n_used=300, bits_per_sym=4, n_slots=2),
    "N2048_A9_64qam": C4.replace(n_ant=9, n_slots=2, n_sym=4),
    "N2048_A1": C4.replace(n_ant=1, n_slots=2, n_sym=3),
    # more pilot symbols (3700) than a MI355X holds estimate transforms at once (3072): the
    # resident-grid estimate walks its job list more than once, stepping (slot, antenna)
    "A37_S100_estimate_grid_wraps": C2.replace(n_ant=37, n_sym=2, n_slots=100),
    "N2048_A2_qpsk": C4.replace(n_ant=2, bits_per_sym=2, n_slots=3, n_sym=3),
    "A1": C2.replace(n_ant=1, n_slots=2, n_sym=4),
    "U2_minimal": C2.replace(n_ant=4, n_used=2, n_slots=1, n_sym=3),
    "U_max": C2.replace(n_ant=4, fft_len=256, cp_len=18, n_used=254, bits_per_sym=4, n_slots=1, n_sym=3),
    "CP0_T2": C2.replace(n_ant=6, cp_len=0, n_sym=2, n_slots=2, n_taps=1),
    "U_not_mult_4": C2.replace(n_ant=3, n_used=598, n_slots=1, n_sym=3),
    # 1000 of 1024 bins used: the widest spectrum window of the demod (8 + 8 registers per lane)
    "N1024_U1000_wide": C2.replace(n_ant=6, n_used=1000, n_slots=2, n_sym=3),
    # 1600 of 2048 bins: the 2048-point demod's 8 + 8 register window
    "N2048_U1600_wide": C4.replace(n_ant=3, n_used=1600, n_slots=2, n_sym=3),
    # 128-point transforms (8 lanes each) with a CP that keeps the records 16-byte aligned: the
    # staged 16-byte sample loads (the CP 9 cases above take the direct loads)
    "N128_CP8_staged": C2.replace(n_ant=6, fft_len=128, cp_len=8, n_used=72, bits_per_sym=4, n_slots=5, n_sym=7),
    # two and three antennas at N = 1024: two wavefronts per item, several items per workgroup
    "A2_two_waves_per_item": C2.replace(n_ant=2, n_slots=3, n_sym=5),
    "A3_two_waves_per_item": C2.replace(n_ant=3, n_slots=2, n_sym=6),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("combiner", [0, 1])
def test_process_frame_matches_oracle(rx, name, combiner):
    cfg = CASES[name]
    _say(name, "combiner", combiner, "A", cfg.n_ant, "N", cfg.fft_len, "U", cfg.n_used, "S", cfg.n_slots)
    fr = make_frames(cfg)
    plan, iq, (H, xhat, bits), ref = _run_both(rx, cfg, fr, combiner)
    check_H(H, ref.H)
    check_xhat(xhat, ref.xhat)
    check_bits(bits, ref.bits, ref.xhat, cfg.bits_per_sym)


def test_split_calls_equal_fused_call(rx):
    cfg = C2.replace(n_slots=2, n_ant=24)
    _say("split", cfg.seed)
    fr = make_frames(cfg)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    H1, g = plan.estimate(iq, with_g=True)
    x1, b1 = plan.demod(iq, H1)
    H2, x2, b2 = plan.process(iq, want_H=True)
    _, x3, b3 = plan.process(iq)                # estimate kept in the workspace
    torch.cuda.synchronize()
    assert torch.equal(H1, H2) and torch.equal(x1, x2) and torch.equal(b1, b2)
    assert torch.equal(x1, x3) and torch.equal(b1, b3)
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    gg = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gg - ref.g) / np.max(ref.g)) < 1e-5


def test_mrc_and_zf_agree_on_gpu(rx):
    cfg = C2.replace(n_slots=2)
    _say("mrc-vs-zf", cfg.seed)
    fr = make_frames(cfg)
    iq = torch.from_numpy(fr.iq).cuda()
    a = rx.Plan.from_config(cfg, fr.pilot, 0).process(iq)[1]
    b = rx.Plan.from_config(cfg, fr.pilot, 1).process(iq)[1]
    xa, xb = as_complex(a), as_complex(b)
    assert np.max(np.abs(xa - xb) / np.maximum(1, np.abs(xa))) < 1e-5


def test_deterministic_and_poisoned_outputs_overwritten(rx):
    cfg = C2.replace(n_slots=2, n_ant=20)
    _say("determinism", cfg.seed)
    fr = make_frames(cfg)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    S, Td, U = 2, cfg.n_sym - 1, cfg.n_used
    H = torch.full((S, cfg.n_ant, U, 2), float("nan"), device="cuda")
    x = torch.full((S, Td, U, 2), float("nan"), device="cuda")
    b = torch.full((S, Td, plan.row_bytes), 0xAA, dtype=torch.uint8, device="cuda")
    plan.process(iq, out=(H, x, b))
    H2, x2, b2 = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    assert not torch.isnan(H).any() and not torch.isnan(x).any()
    assert torch.equal(H, H2) and torch.equal(x, x2) and torch.equal(b, b2)


def test_zero_and_saturated_slots(rx):
    cfg = C2.replace(n_slots=3, n_ant=8, n_sym=4)
    _say("zero-saturated", cfg.seed)
    fr = make_frames(cfg)
    iq = fr.iq.copy()
    iq[0] = 0                                                     # g = 0 -> x-hat = 0
    iq[1] = np.where(iq[1] >= 0, 32767, -32768).astype(np.int16)  # clipped everywhere
    plan = rx.Plan.from_config(cfg, fr.pilot)
    H, xhat, bits = plan.process(torch.from_numpy(iq).cuda(), want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(iq, fr.pilot, **_kw(cfg))
    x = as_complex(xhat)
    assert np.all(x[0] == 0)
    check_xhat(x, ref.xhat)
    check_bits(bits.cpu().numpy(), ref.bits, ref.xhat, cfg.bits_per_sym)
    assert np.all(bits.cpu().numpy()[0] == 0)                     # 16-QAM at the origin: 0000


def test_empty_batch_is_a_no_op(rx):
    cfg = C1
    fr = make_frames(cfg)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.empty((0,) + fr.iq.shape[1:], dtype=torch.int16, device="cuda")
    H, xhat, bits = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    assert H.numel() == 0 and xhat.numel() == 0 and bits.numel() == 0


def test_invalid_calls_write_nothing(rx):
    cfg = C1
    fr = make_frames(cfg)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    x = torch.full((1, cfg.n_sym - 1, cfg.n_used, 2), 7.0, device="cuda")
    # misaligned input pointer -> rejected before launch
    st = rx.rx_process_frame(plan._plan, iq.data_ptr() + 2, 1, None, x.data_ptr(), None,
                             torch.empty(4096, dtype=torch.uint8, device="cuda").data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    assert st == rx.RX_E_INVALID_ARG
    # no workspace and no H
    st = rx.rx_process_frame(plan._plan, iq.data_ptr(), 1, None, x.data_ptr(), None, None,
                             torch.cuda.current_stream().cuda_stream)
    assert st == rx.RX_E_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(x == 7.0)


# ---------------------------------------------------------------- full-size launch
def test_full_size_c2_launch_all_slots_checked(rx):
    """The benchmarked shape (64 antennas, N=1024, 200 slots, one launch pair).

    Eight distinct generated slots are tiled over the 200 slots, so every output
    slot is checked against the oracle of its source slot.
    """
    cfg = C2
    _say("full-size", cfg.name, "S", cfg.n_slots)
    uniq = make_frames(cfg, n_slots=8)
    src = np.arange(cfg.n_slots) % 8
    iq = uniq.iq[src]
    ref = oracle.process_frame(uniq.iq, uniq.pilot, n_threads=8, **_kw(cfg))
    plan = rx.Plan.from_config(cfg, uniq.pilot)
    H, xhat, bits = plan.process(torch.from_numpy(iq).cuda(), want_H=True)
    torch.cuda.synchronize()
    check_H(as_complex(H), ref.H[src])
    check_xhat(as_complex(xhat), ref.xhat[src])
    check_bits(bits.cpu().numpy(), ref.bits[src], ref.xhat[src], cfg.bits_per_sym)


@pytest.mark.parametrize("fft_mode", [0, 3])
def test_full_size_c4_launch_all_slots_checked(rx, fft_mode):
    """The largest configured shape (128 antennas, N=2048, 64-QAM, 500 slots,
    7.86 GB of input: offsets past 4 GiB), with the FP32 radix FFT and with the
    fp16 hi+lo DFT-GEMM FFT.  Eight distinct generated slots are tiled over the
    500 on the device; every output element is checked against the oracle of
    its source slot."""
    cfg = C4
    _say("full-size", cfg.name, "S", cfg.n_slots, "fft_mode", fft_mode)
    uniq = make_frames(cfg, n_slots=8)
    ref = oracle.process_frame(uniq.iq, uniq.pilot, n_threads=8, **_kw(cfg))
    S = cfg.n_slots
    src = np.arange(S) % 8
    iq = torch.from_numpy(uniq.iq).cuda()[torch.from_numpy(src).cuda()].contiguous()
    assert iq.numel() * 2 > 4 * 2 ** 30
    plan = rx.Plan.from_config(cfg, uniq.pilot, fft_mode=fft_mode)
    H, xhat, bits = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    del iq
    for c0 in range(0, S, 50):
        sl = slice(c0, min(S, c0 + 50))
        check_H(as_complex(H[sl]), ref.H[src[sl]])
    check_xhat(as_complex(xhat), ref.xhat[src])
    check_bits(bits.cpu().numpy(), ref.bits[src], ref.xhat[src], cfg.bits_per_sym)


# Antenna-count x FFT-length sweep points at their full size (about 1 GiB of
# input each): launches with several (slot, symbol) items per workgroup and
# one to four wavefronts per item, and the resident-grid estimate over short
# transforms.  Eight distinct slots are tiled over the buffer; bits are checked
# for every slot, H and x-hat for every slot of the first and last 64 and a
# stride through the rest (the tail of the grid and its partial workgroup).
@pytest.mark.parametrize("N,A", [(64, 1), (64, 2), (64, 3), (64, 16), (64, 128),
                                 (1024, 1), (1024, 2), (1024, 8), (1024, 16), (1024, 32)])
def test_sweep_point_full_size(rx, N, A, combiner=0):
    from rxgen import sweep_config
    if A in (1, 2, 8, 16, 32, 128):
        cfg = sweep_config(N, A)
    else:  # an antenna count off the sweep's powers of two, same input size
        cfg = sweep_config(N, 2).replace(n_ant=A)
        cfg = cfg.replace(n_slots=-(-(1 << 30) // cfg.slot_bytes))
    S = cfg.n_slots
    _say("sweep-point", cfg.name, "N", N, "A", A, "S", S, "seed", cfg.seed)
    uniq = make_frames(cfg, n_slots=8)
    ref = oracle.process_frame(uniq.iq, uniq.pilot, n_threads=8, combiner=combiner, **_kw(cfg))
    plan = rx.Plan.from_config(cfg, uniq.pilot, combiner)
    u = torch.from_numpy(uniq.iq).cuda()
    iq = u[torch.arange(S, device="cuda") % 8].contiguous()
    H, xhat, bits = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    src = np.arange(S) % 8
    check_bits(bits.cpu().numpy(), ref.bits[src], ref.xhat[src], cfg.bits_per_sym)
    pick = np.unique(np.concatenate([np.arange(min(64, S)), np.arange(max(0, S - 64), S),
                                     np.arange(0, S, 97)]))
    pk = torch.from_numpy(pick).cuda()
    check_H(as_complex(H[pk]), ref.H[src[pick]])
    check_xhat(as_complex(xhat[pk]), ref.xhat[src[pick]])


# ZF on sweep-sized launches: one wavefront per item holding eight antennas (N = 1024, A = 8) and
# the 16-transform wavefronts at N = 64 with two wavefronts per item (A = 16)
@pytest.mark.parametrize("N,A", [(1024, 8), (64, 16)])
def test_sweep_point_full_size_zf(rx, N, A):
    test_sweep_point_full_size(rx, N, A, combiner=1)
