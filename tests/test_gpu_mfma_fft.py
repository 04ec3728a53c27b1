"""GPU checks of the 2048-point FFT recast as DFT-stage GEMMs on the fp16 /
bf16 matrix cores (fft_mode 1..4) against the FP64 oracle, through the C ABI.

Error model (from the arithmetic): each GEMM operand is rounded to the
format's precision u (fp16: 2^-11, bf16: 2^-8, relative); with two GEMM
stages the spectrum's RMS relative error is about u.  The hi+lo split leaves
about u^2 plus FP32 accumulation.  Bounds on the RMS error relative to the
oracle spectrum's RMS: fp16 2e-3, bf16 1.5e-2, fp16 split 5e-6, bf16 split
1e-4 (measured values are printed); every element within 6 times that."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from rxgen import C4, make_frames  # noqa: E402
from tests.parity import as_complex, check_bits, check_H, check_xhat  # noqa: E402

MODES = {"f16": (1, 2e-3), "bf16": (2, 1.5e-2), "f16_split": (3, 5e-6), "bf16_split": (4, 1e-4)}
ELEM_FACTOR = 6.0


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod
    return mod


def _kw(cfg):
    return dict(n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len, n_used=cfg.n_used, n_sym=cfg.n_sym,
                bits_per_sym=cfg.bits_per_sym)


SMALL = C4.replace(n_ant=6, n_sym=3, n_slots=2)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("kind", ["ofdm", "full_scale"])
def test_fft_error_within_the_format_bound(rx, mode, kind):
    code, bound = MODES[mode]
    fr = make_frames(SMALL, n_slots=2)
    iq = fr.iq
    if kind == "full_scale":
        rng = np.random.default_rng(3)
        iq = rng.integers(-32768, 32768, size=iq.shape).astype(np.int16)
        iq[0, 0, 0] = -32768          # one symbol at the extreme of the range
    print(f"[case] mfma fft {mode} {kind}", flush=True)
    plan = rx.Plan.from_config(SMALL, fr.pilot, fft_mode=code)
    Y = as_complex(plan.debug_fft(torch.from_numpy(iq).cuda()))
    torch.cuda.synchronize()
    ref = oracle.fft_symbols(iq, fr.pilot, **_kw(SMALL))
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=-1))
    err = np.sqrt(np.mean(np.abs(Y - ref) ** 2, axis=-1)) / rms
    elem = np.abs(Y - ref) / rms[..., None]
    print(f"[mfma] {mode} {kind}: RMS relative error max {err.max():.3e}, mean {err.mean():.3e}; "
          f"element max {elem.max():.3e}", flush=True)
    assert err.max() <= bound
    # per element: the error of one bin is a sum of many independent operand
    # roundings (near Gaussian), so over 2048 bins its maximum stays within
    # about 4.5 standard deviations of the RMS
    assert elem.max() <= ELEM_FACTOR * bound


def test_split_f16_path_meets_the_fp32_parity_bar(rx):
    cfg = C4.replace(n_ant=32, n_slots=2)
    fr = make_frames(cfg, n_slots=2)
    print("[case] mfma path f16_split", flush=True)
    plan = rx.Plan.from_config(cfg, fr.pilot, fft_mode=3)
    H, xhat, bits = plan.process(torch.from_numpy(fr.iq).cuda(), want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    check_H(as_complex(H), ref.H)
    check_xhat(as_complex(xhat), ref.xhat)
    check_bits(bits.cpu().numpy(), ref.bits, ref.xhat, cfg.bits_per_sym)


@pytest.mark.parametrize("A,S", [(5, 3), (1, 1), (130, 1)])
def test_split_f16_path_ragged_antenna_counts(rx, A, S):
    # antenna counts that leave wavefronts idle in the estimate and demod loops
    cfg = C4.replace(n_ant=A, n_slots=S, n_sym=4)
    fr = make_frames(cfg, n_slots=S)
    print(f"[case] mfma path f16_split A={A} S={S}", flush=True)
    plan = rx.Plan.from_config(cfg, fr.pilot, fft_mode=3)
    H, xhat, bits = plan.process(torch.from_numpy(fr.iq).cuda(), want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    check_H(as_complex(H), ref.H)
    check_xhat(as_complex(xhat), ref.xhat)
    check_bits(bits.cpu().numpy(), ref.bits, ref.xhat, cfg.bits_per_sym)


@pytest.mark.parametrize("mode", ["f16", "bf16", "bf16_split"])
def test_path_error_follows_the_fft_error(rx, mode):
    code, bound = MODES[mode]
    cfg = C4.replace(n_ant=32, n_slots=2)
    fr = make_frames(cfg, n_slots=2)
    print(f"[case] mfma path {mode}", flush=True)
    plan = rx.Plan.from_config(cfg, fr.pilot, fft_mode=code)
    H, xhat, bits = plan.process(torch.from_numpy(fr.iq).cuda(), want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    # equalised symbols: both H and Y carry the FFT error (about 2 x bound relative)
    x = as_complex(xhat)
    rel = np.sqrt(np.mean(np.abs(x - ref.xhat) ** 2)) / np.sqrt(np.mean(np.abs(ref.xhat) ** 2))
    elem = np.abs(x - ref.xhat) / np.maximum(1.0, np.abs(ref.xhat))
    print(f"[mfma] {mode}: x-hat RMS relative error {rel:.3e}, element max {elem.max():.3e}", flush=True)
    assert rel <= 4 * bound
    assert elem.max() <= ELEM_FACTOR * 4 * bound
    hrel = np.sqrt(np.mean(np.abs(as_complex(H) - ref.H) ** 2) / np.mean(np.abs(ref.H) ** 2))
    assert hrel <= 2 * bound


def test_mfma_modes_reject_unsupported_shapes(rx):
    fr = make_frames(C4.replace(n_ant=2, n_slots=1), n_slots=1)
    base = dict(n_ant=2, fft_len=2048, cp_len=144, n_used=1200, n_sym=14, bits_per_sym=6)
    ok = rx.make_params(pilot=fr.pilot, fft_mode=1, **base)
    assert rx.rx_params_check(ok[0]) == rx.RX_OK
    for over, pil in ((dict(fft_len=1024, cp_len=72, n_used=600), fr.pilot[:600]),
                      (dict(n_used=1600), np.ones(1600))):
        b = dict(base)
        b.update(over)
        p = rx.make_params(pilot=pil, fft_mode=1, **b)
        assert rx.rx_params_check(p[0]) == rx.RX_E_UNSUPPORTED
    zf = rx.make_params(pilot=fr.pilot, fft_mode=2, combiner=rx.RX_COMB_ZF, **base)
    assert rx.rx_params_check(zf[0]) == rx.RX_E_UNSUPPORTED
    comb = rx.make_params(pilot=fr.pilot, fft_mode=3, pilot_spacing=4, **base)
    assert rx.rx_params_check(comb[0]) == rx.RX_E_UNSUPPORTED
    bad = rx.make_params(pilot=fr.pilot, fft_mode=5, **base)
    assert rx.rx_params_check(bad[0]) == rx.RX_E_UNSUPPORTED
    arr = (rx.rx_params * 1)(ok[0])
    st, b = rx.rx_batch_create(arr, 1)
    assert st == rx.RX_E_UNSUPPORTED and b is None
