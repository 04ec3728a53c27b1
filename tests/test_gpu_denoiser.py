"""GPU parity of the comb-pilot estimate, the training-channel generator and
the learned estimate refinement (forward, gradient, Adam) against the FP64
oracle, all through the C ABI.

Tolerances (from the arithmetic):
* comb estimate: the LS values are the block estimate's (1e-5 of the slot
  RMS); interpolation adds two FP32 operations.
* generator: FP32 sincos/log/exp of Philox uniforms that both sides derive
  exactly; |H| ~ 1, sums of at most 24 taps: 2e-5 absolute.
* forward: products take bf16 operands on both sides, but the kernel sums in
  FP32 and computes h / s in FP32, so an operand near a bf16 rounding boundary
  can round the other way (one bf16 step, 2^-8 relative) and move nearby
  outputs.  Bounds, relative to the RMS of the refinement out - h: RMS error
  2e-4, 99.9th percentile 2e-3, maximum 2e-2 (an FP32 emulation of the kernel
  order gives 4e-5, 4e-4 and 3e-3).
* gradient: the same effects through the backward pass, bounded per
  parameter from the root-sum-square of the entry's terms (see
  _check_grad); loss 1e-4.
* LS fallback: the decision is compared on rows whose correction energy
  ratio lies more than 2 % from the limit; rows that keep LS are bit-exact.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import denoiser as odn  # noqa: E402
from rxgen import C5, init_denoiser_params, make_frames  # noqa: E402
from tests.parity import as_complex, check_bits, check_H, check_xhat  # noqa: E402


@pytest.fixture(scope="module")
def rx():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1901_07499_amd import rx as mod
    return mod


def _say(*a):
    print("[case]", *a, flush=True)


def _kw(cfg):
    return dict(n_ant=cfg.n_ant, fft_len=cfg.fft_len, cp_len=cfg.cp_len, n_used=cfg.n_used, n_sym=cfg.n_sym,
                bits_per_sym=cfg.bits_per_sym, pilot_spacing=cfg.pilot_spacing)


def _cuda(z):
    """complex numpy [..] -> float32 CUDA tensor [.., 2]"""
    a = np.stack([z.real, z.imag], axis=-1).astype(np.float32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------- comb estimate
@pytest.mark.parametrize("N,cp,U,s,A", [(64, 16, 52, 4, 8), (256, 18, 180, 4, 5), (1024, 72, 600, 3, 7),
                                        (2048, 144, 1200, 4, 16), (512, 37, 300, 6, 3)])
def test_comb_estimate_matches_oracle(rx, N, cp, U, s, A):
    cfg = C5.replace(n_ant=A, fft_len=N, cp_len=cp, n_used=U, pilot_spacing=s, n_sym=3, bits_per_sym=4,
                     tau_max_us=(0.5, 2.0))
    _say("comb estimate", N, U, s, A, cfg.seed)
    fr = make_frames(cfg, n_slots=2)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    H = as_complex(plan.estimate(iq))
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    check_H(H, ref.H)


def test_comb_estimate_when_the_estimate_grid_wraps(rx):
    # 37 antennas x 100 slots = 3700 pilot symbols, more than a MI355X holds estimate transforms
    # at once (3072): the N = 1024 estimate walks its job list more than once
    cfg = C5.replace(n_ant=37, fft_len=1024, cp_len=72, n_used=600, pilot_spacing=3, n_sym=2, bits_per_sym=4,
                     tau_max_us=(0.5, 2.0))
    _say("comb estimate, grid wraps", cfg.seed)
    fr = make_frames(cfg, n_slots=100)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    H = as_complex(plan.estimate(torch.from_numpy(fr.iq).cuda()))
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    check_H(H, ref.H)


def test_comb_path_end_to_end_c5_shape(rx):
    cfg = C5.replace(n_slots=2)
    _say("comb path c5 shape", cfg.seed)
    fr = make_frames(cfg, n_slots=2)
    plan = rx.Plan.from_config(cfg, fr.pilot)
    iq = torch.from_numpy(fr.iq).cuda()
    H, xhat, bits = plan.process(iq, want_H=True)
    torch.cuda.synchronize()
    ref = oracle.process_frame(fr.iq, fr.pilot, **_kw(cfg))
    check_H(as_complex(H), ref.H)
    check_xhat(as_complex(xhat), ref.xhat)
    check_bits(bits.cpu().numpy(), ref.bits, ref.xhat, cfg.bits_per_sym)


def test_comb_rejected_by_batches(rx):
    fr = make_frames(C5.replace(n_ant=2, fft_len=256, cp_len=18, n_used=180), n_slots=1)
    p, keep = rx.make_params(2, 256, 18, 180, 14, 6, fr.pilot, pilot_spacing=4)
    arr = (rx.rx_params * 1)(p)
    st, b = rx.rx_batch_create(arr, 1)
    assert st == rx.RX_E_UNSUPPORTED and b is None


# ---------------------------------------------------------------- generator
@pytest.mark.parametrize("recipe", [dict(), dict(pilot_spacing=1, snr_db=(10.0, 10.0)),
                                    dict(fft_len=256, n_used=180, cp_len=18, taps=(1, 3), tau_samples=(0, 20))])
def test_generator_matches_oracle(rx, recipe):
    gp = oracle.GenParams(**recipe)
    g = rx.chan_gen(fft_len=gp.fft_len, n_used=gp.n_used, cp_len=gp.cp_len, pilot_spacing=gp.pilot_spacing,
                    taps=gp.taps, tau_samples=gp.tau_samples, snr_db=gp.snr_db, tap_decay_db=gp.tap_decay_db)
    _say("generator", recipe)
    ht, hl = rx.generate(g, 77, 1000, 48, "cuda")
    torch.cuda.synchronize()
    rt, rl = oracle.gen_channels(gp, 77, 1000, 48)
    assert np.abs(as_complex(ht) - rt).max() < 2e-5
    assert np.abs(as_complex(hl) - rl).max() < 2e-5


def test_generator_partial_outputs_and_errors(rx):
    g = rx.chan_gen()
    ht, _ = rx.generate(g, 5, 0, 8, "cuda", want_ls=False)
    _, hl = rx.generate(g, 5, 0, 8, "cuda", want_true=False)
    ht2, hl2 = rx.generate(g, 5, 0, 8, "cuda")
    torch.cuda.synchronize()
    assert torch.equal(ht, ht2) and torch.equal(hl, hl2)
    bad = rx.chan_gen(taps=(5, 4))
    assert rx.rx_dn_generate(bad, 0, 0, 1, ht.data_ptr(), None, None) == rx.RX_E_INVALID_ARG
    assert rx.rx_dn_generate(g, 0, 0, 0, None, None, None) == rx.RX_OK


# ---------------------------------------------------------------- network
def _params(seed, last_scale=1.0):
    rng = np.random.default_rng(seed)
    th = init_denoiser_params(seed, last_scale=last_scale).astype(np.float64)
    th += 0.02 * rng.standard_normal(th.size)          # non-zero biases
    return th


def _arith_denoiser(rx, U, th):
    """A denoiser with parameters th and the LS fallback limited to non-finite
    rows: the forward checks use random parameters, whose corrections are
    larger than the rows themselves."""
    dn = rx.Denoiser(U)
    dn.load(torch.from_numpy(th.astype(np.float32)).cuda())
    dn.set_fallback(float("inf"))
    return dn


def _rows(n, seed, **recipe):
    gp = oracle.GenParams(**recipe)
    return oracle.gen_channels(gp, seed, 0, n)


def _check_forward(out, ref, h):
    err = np.abs(out - ref)
    scale = np.sqrt(np.mean(np.abs(ref - h) ** 2))
    assert np.sqrt(np.mean(err ** 2)) <= 2e-4 * scale, (np.sqrt(np.mean(err ** 2)) / scale)
    assert np.quantile(err, 0.999) <= 2e-3 * scale
    assert err.max() <= 2e-2 * scale, err.max() / scale


@pytest.mark.parametrize("U,rows,seed", [(1200, 40, 1), (600, 9, 2), (180, 3, 3), (52, 5, 4), (250, 2, 5),
                                         (2046, 2, 6)])
def test_forward_matches_oracle(rx, U, rows, seed):
    _say("dn forward", U, rows, seed)
    recipe = dict(n_used=U, fft_len=max(64, 1 << int(np.ceil(np.log2(U + 2)))), cp_len=16)
    recipe["pilot_spacing"] = 4 if U >= 8 else 1
    ht, hl = _rows(rows, seed, **recipe)
    th = _params(seed)
    dn = _arith_denoiser(rx, U, th)
    out = as_complex(dn.apply(_cuda(hl)))
    torch.cuda.synchronize()
    ref = odn.forward(th.astype(np.float32).astype(np.float64), hl.astype(np.complex64).astype(np.complex128),
                      bf16_ops=True)
    _check_forward(out, ref, hl)


@pytest.mark.parametrize("U,rows", [(3, 4), (7, 1), (241, 3), (481, 2)])
def test_forward_odd_lengths_and_tile_edges(rx, U, rows):
    # arbitrary row lengths: one position past a 240-output tile, odd U, a single row
    rng = np.random.default_rng(U)
    h = rng.standard_normal((rows, U)) + 1j * rng.standard_normal((rows, U))
    th = _params(U)
    dn = _arith_denoiser(rx, U, th)
    out = as_complex(dn.apply(_cuda(h)))
    torch.cuda.synchronize()
    ref = odn.forward(th.astype(np.float32).astype(np.float64), h.astype(np.complex64).astype(np.complex128),
                      bf16_ops=True)
    _check_forward(out, ref, h)


def test_gradient_single_row_odd_length(rx):
    rng = np.random.default_rng(8)
    U = 243
    ht = rng.standard_normal((1, U)) + 1j * rng.standard_normal((1, U))
    hl = ht + 0.3 * (rng.standard_normal((1, U)) + 1j * rng.standard_normal((1, U)))
    th = _params(8, last_scale=0.3).astype(np.float32).astype(np.float64)
    dn = rx.Denoiser(U)
    dn.load(torch.from_numpy(th.astype(np.float32)).cuda())
    loss, g = dn.grad(_cuda(hl), _cuda(ht))
    torch.cuda.synchronize()
    rl, rg, rss = odn.loss_grad(th, hl.astype(np.complex64).astype(np.complex128),
                                ht.astype(np.complex64).astype(np.complex128), bf16_ops=True, term_rss=True)
    assert abs(loss.item() - rl) <= 1e-4 * rl
    _check_grad(g.cpu().numpy().astype(np.float64), rg, rss, U)


def test_forward_in_place_zero_rows_and_identity(rx):
    U = 300
    _, hl = _rows(6, 9, n_used=U, fft_len=512, cp_len=37)
    hl[2] = 0
    th = _params(9)
    dn = _arith_denoiser(rx, U, th)
    H = _cuda(hl)
    out = dn.apply(H)
    H2 = H.clone()
    dn.apply(H2, out=H2)           # in place
    torch.cuda.synchronize()
    assert torch.equal(out, H2)
    assert torch.equal(out[2], H[2])   # a zero row passes through
    # zero last layer: the output is the input, exactly
    layers = odn.unpack(th.copy())
    layers[3][0][...] = 0
    layers[3][1][...] = 0
    dn.load(torch.from_numpy(odn.pack(layers).astype(np.float32)).cuda())
    ident = dn.apply(H)
    torch.cuda.synchronize()
    assert torch.equal(ident, H)


def test_apply_argument_errors(rx):
    dn = rx.Denoiser(100)
    H = torch.zeros((4, 100, 2), dtype=torch.float32, device="cuda")
    assert rx.rx_dn_set_fallback(dn._dn, 0.0) == rx.RX_E_INVALID_ARG
    assert rx.rx_dn_set_fallback(dn._dn, float("nan")) == rx.RX_E_INVALID_ARG
    assert rx.rx_dn_set_fallback(None, 1.0) == rx.RX_E_INVALID_ARG
    fl = torch.empty(4, dtype=torch.uint8, device="cuda")
    assert rx.rx_dn_apply_judged(dn._dn, H.data_ptr(), 4, H.data_ptr(), H.data_ptr() + 8, None) == \
        rx.RX_E_INVALID_ARG  # flags inside the rows
    assert rx.rx_dn_apply_judged(dn._dn, H.data_ptr(), 4, H.data_ptr(), fl.data_ptr(), None) == rx.RX_OK
    dn.load(torch.zeros(rx.RX_DN_PARAMS, dtype=torch.float32, device="cuda"))
    assert rx.rx_dn_apply(dn._dn, H.data_ptr(), -1, H.data_ptr(), None) == rx.RX_E_INVALID_ARG
    assert rx.rx_dn_apply(dn._dn, H.data_ptr(), 4, H.data_ptr() + 8, None) == rx.RX_E_INVALID_ARG  # overlap
    assert rx.rx_dn_apply(dn._dn, H.data_ptr(), 0, H.data_ptr(), None) == rx.RX_OK
    st, _ = rx.rx_dn_create(1)
    assert st == rx.RX_E_INVALID_ARG


def test_unloaded_denoiser_keeps_ls(rx):
    # no parameters: LS is the fallback, every row passes through and is flagged
    _, hl = _rows(5, 3, n_used=180, fft_len=256, cp_len=18)
    dn = rx.Denoiser(180)
    H = _cuda(hl)
    out, fell = dn.apply(H, flags=True)
    H2 = H.clone()
    dn.apply(H2, out=H2)
    torch.cuda.synchronize()
    assert torch.equal(out, H) and torch.equal(H2, H)
    assert fell.cpu().tolist() == [1] * 5


@pytest.mark.parametrize("in_place", [False, True])
def test_ls_fallback_matches_oracle_rule(rx, in_place):
    # Parameters scaled so that rows' correction energy ratios straddle the
    # limit; the limit is set between them, away from every row's ratio.  One
    # row carries a NaN (its correction is not finite) and one is zero.
    _say("dn LS fallback", in_place)
    U, R = 600, 24
    _, hl = _rows(R, 51, n_used=U, fft_len=1024, cp_len=72)
    hl[5, 17] = np.nan
    hl[9] = 0
    th = _params(51) * 0.6
    ref = odn.forward(th.astype(np.float32).astype(np.float64), hl.astype(np.complex64).astype(np.complex128),
                      bf16_ops=True)
    h64 = hl.astype(np.complex64).astype(np.complex128)
    with np.errstate(invalid="ignore"):
        ratio = np.sum(np.abs(ref - h64) ** 2, axis=-1) / np.sum(np.abs(h64) ** 2, axis=-1)
    live = np.isfinite(ratio)
    lim = float(np.median(ratio[live]))
    near = live & (np.abs(ratio / lim - 1) < 0.02)
    lim = float(np.sqrt(lim))
    want, want_fell = odn.ls_fallback(h64, ref, max_corr=lim)
    assert want_fell[5] and not want_fell[9] and 3 <= want_fell.sum() <= R - 3
    dn = rx.Denoiser(U)
    dn.load(torch.from_numpy(th.astype(np.float32)).cuda())
    dn.set_fallback(lim)
    H = _cuda(hl)
    if in_place:
        out = H.clone()
        out, fell = dn.apply(out, out=out, flags=True)
    else:
        out, fell = dn.apply(H, flags=True)
    torch.cuda.synchronize()
    fell = fell.cpu().numpy().astype(bool)
    assert np.array_equal(fell[~near], want_fell[~near]), (np.flatnonzero(fell != want_fell), ratio / lim ** 2)
    bits_out = out.cpu().numpy().view(np.uint32)
    bits_in = H.cpu().numpy().view(np.uint32)
    got = as_complex(out)
    for r in range(R):
        if fell[r]:
            assert np.array_equal(bits_out[r], bits_in[r]), r      # the LS row, bit for bit
        else:
            # the scaled-down parameters give corrections much smaller than
            # the row, so the bound is taken relative to the row itself
            rms = np.sqrt(np.mean(np.abs(h64[r]) ** 2))
            err = np.abs(got[r] - ref[r])
            assert np.sqrt(np.mean(err ** 2)) <= 2e-4 * rms and err.max() <= 2e-3 * rms, (r, err.max() / rms)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


# Parameter segments: W1 b1 W2 b2 W3 b3 W4 b4.
GRAD_SEGMENTS = (0, 448, 480, 7648, 7680, 14848, 14880, 15328, 15330)


def _check_grad(g, rg, rss, n_terms):
    """Per parameter, with rss the root of the sum of the squares of the
    entry's n_terms terms (oracle) and m its segment's median rss:
        |g - g_ref| <= (2^-5 + 2^-24 n_terms) rss + 2^-6 m.
    * bf16 operands: where the kernel's FP32 value and the oracle's FP64 one
      straddle a rounding boundary the two round one bf16 step (2^-7
      relative) apart; such terms are rare and their signs random, far below
      2^-5 rss (4 x 2^-7 of every term at once).
    * FP32 accumulation: terms of one sign summed one by one drift by about
      2^-24 n_terms rss.
    * A ReLU mask decided the other way at an activation within FP32
      rounding of zero adds or drops a whole term; a term is about
      m / sqrt(n_terms), so 2^-6 m covers several.
    An entry computed from wrong terms misses by about its rss."""
    err = np.abs(g - rg)
    med = np.empty_like(rss)
    for a, b in zip(GRAD_SEGMENTS[:-1], GRAD_SEGMENTS[1:]):
        med[a:b] = np.median(rss[a:b])
    bound = (2.0 ** -5 + 2.0 ** -24 * n_terms) * rss + 2.0 ** -6 * med
    worst = float((err / bound).max())
    print(f"[dn] gradient: max |g - g_ref| / bound = {worst:.3f}; max |g - g_ref| / rss = "
          f"{float((err / np.maximum(rss, 1e-300)).max()):.2e}", flush=True)
    assert worst <= 1.0, (int(np.argmax(err / bound)), worst)


@pytest.mark.parametrize("U,rows,seed", [(1200, 12, 11), (180, 7, 12), (600, 600, 13)])
def test_gradient_matches_oracle(rx, U, rows, seed):
    _say("dn gradient", U, rows, seed)
    fft = max(64, 1 << int(np.ceil(np.log2(U + 2))))
    ht, hl = _rows(rows, seed, n_used=U, fft_len=fft, cp_len=16, snr_db=(10.0, 20.0))
    th = _params(seed, last_scale=0.3).astype(np.float32).astype(np.float64)
    dn = rx.Denoiser(U)
    dn.load(torch.from_numpy(th.astype(np.float32)).cuda())
    loss, g = dn.grad(_cuda(hl), _cuda(ht))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    rl, rg, rss = odn.loss_grad(th, hl.astype(np.complex64).astype(np.complex128),
                                ht.astype(np.complex64).astype(np.complex128), bf16_ops=True, term_rss=True)
    assert abs(loss.item() - rl) <= 1e-4 * rl
    _check_grad(g, rg, rss, rows * U)


def test_gradient_deterministic(rx):
    ht, hl = _rows(64, 21)
    dn = rx.Denoiser(1200)
    dn.load(torch.from_numpy(_params(21).astype(np.float32)).cuda())
    a = dn.grad(_cuda(hl), _cuda(ht))
    b = dn.grad(_cuda(hl), _cuda(ht))
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_adam_step_matches_oracle(rx):
    ht, hl = _rows(16, 31)
    th = _params(31, last_scale=0.3).astype(np.float32)
    dn = rx.Denoiser(1200)
    p = torch.from_numpy(th).cuda()
    dn.load(p)
    H, T = _cuda(hl), _cuda(ht)
    _, g = dn.grad(H, T)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    lr = 1e-3
    # the kernel receives the hyperparameters as float32: give the oracle the same values
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    b1, b2 = f32(0.9), f32(0.999)
    for step in (1, 2):
        gg = dn.grad(H, T)[1].cpu().numpy().astype(np.float64)
        m0, v0 = m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        want, wm, wv = odn.adam(p.cpu().numpy().astype(np.float64), m0, v0, gg, step, f32(lr), b1, b2, f32(1e-8))
        dn.train_step(p, m, v, step, H, T, lr=lr)
        torch.cuda.synchronize()
        # FP32: each moment is two rounded products and a rounded sum
        ulp = 2.0 ** -23
        bm = 3 * ulp * (b1 * np.abs(m0) + (1 - b1) * np.abs(gg))
        bv = 4 * ulp * (b2 * v0 + (1 - b2) * gg * gg)
        assert np.all(np.abs(m.cpu().numpy() - wm) <= bm + 1e-30)
        assert np.all(np.abs(v.cpu().numpy() - wv) <= bv + 1e-30)
        # the step is lr * m_hat / (sqrt(v_hat) + eps), at most about lr
        np.testing.assert_allclose(p.cpu().numpy(), want, rtol=0, atol=1e-5 * lr + 1e-7)
    # the updated parameters are loaded: apply equals a fresh load of them
    out1 = dn.apply(H)
    dn2 = rx.Denoiser(1200)
    dn2.load(p.clone())
    out2 = dn2.apply(H)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)


def test_training_gains_over_plain_interpolation(rx):
    # Train on GPU-generated channels; on held-out rows at 20 dB the refined
    # estimate must beat comb LS + linear interpolation by a clear margin.
    _say("dn training")
    g_train = rx.chan_gen()
    dn = rx.Denoiser(1200)
    p = torch.from_numpy(init_denoiser_params(1)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    dn.load(p)
    rows = 256
    for step in range(1, 301):
        ht, hl = rx.generate(g_train, 1234, (step - 1) * rows, rows, "cuda")
        dn.train_step(p, m, v, step, hl, ht, lr=2e-3)
    g_eval = rx.chan_gen(snr_db=(20.0, 20.0))
    ht, hl = rx.generate(g_eval, 999, 0, 512, "cuda")
    ref = dn.apply(hl)
    torch.cuda.synchronize()
    t, l, r = as_complex(ht), as_complex(hl), as_complex(ref)
    gain = odn.nmse_db(l, t) - odn.nmse_db(r, t)
    print(f"[dn] NMSE at 20 dB: interpolation {odn.nmse_db(l, t):.2f} dB, refined {odn.nmse_db(r, t):.2f} dB",
          flush=True)
    assert gain > 1.0
