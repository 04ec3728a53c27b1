"""Pins of the FP64 denoiser oracle (oracle/denoiser.py).

The analytic gradient is checked against central finite differences of the
loss in FP64; the convolution against numpy's correlate; the residual form,
the row scale and Adam's first step against closed forms; the bfloat16
rounding against torch's conversion and against its error bound.
"""
import numpy as np
import pytest
import torch

from oracle import denoiser as dn
from rxgen import denoiser_param_count, init_denoiser_params


def _rows(R, U, seed, smooth=True):
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((R, U)) + 1j * rng.standard_normal((R, U))
    if smooth:
        k = np.ones(9) / 9
        h = np.stack([np.convolve(r, k, mode="same") for r in h])
    return h


def test_param_count_and_layout():
    assert dn.param_count() == denoiser_param_count() == 15330
    th = np.arange(dn.param_count(), dtype=np.float64)
    layers = dn.unpack(th)
    assert [W.shape for W, _ in layers] == [(32, 2, 7), (32, 32, 7), (32, 32, 7), (2, 32, 7)]
    np.testing.assert_array_equal(dn.pack(layers), th)
    assert layers[0][1][0] == 448 and layers[1][0][0, 0, 0] == 480


def test_conv_matches_numpy_correlate():
    rng = np.random.default_rng(1)
    U = 37
    x = rng.standard_normal((1, 1, U))
    W = rng.standard_normal((1, 1, 7))
    b = np.array([0.25])
    want = np.correlate(x[0, 0], W[0, 0], mode="same") + 0.25
    np.testing.assert_allclose(dn.conv(x, W, b)[0, 0], want, rtol=1e-13, atol=1e-13)


def test_conv_sums_over_input_channels():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 20))
    W = rng.standard_normal((4, 3, 7))
    b = rng.standard_normal(4)
    y = dn.conv(x, W, b)
    for r in range(2):
        for o in range(4):
            want = b[o] + sum(np.correlate(x[r, c], W[o, c], mode="same") for c in range(3))
            np.testing.assert_allclose(y[r, o], want, rtol=1e-12, atol=1e-12)


def test_zero_last_layer_is_identity_and_loss_closed_form():
    th = init_denoiser_params(3).astype(np.float64)
    layers = dn.unpack(th)
    layers[3][0][...] = 0.0
    layers[3][1][...] = 0.0
    th = dn.pack(layers)
    h = _rows(3, 40, 4)
    ht = _rows(3, 40, 5)
    np.testing.assert_allclose(dn.forward(th, h), h, rtol=1e-15, atol=0)
    s = np.sqrt(np.mean(np.abs(h) ** 2, axis=1))
    want = np.mean(np.abs(h / s[:, None] - ht / s[:, None]) ** 2)
    loss, _ = dn.loss_grad(th, h, ht)
    assert abs(loss - want) < 1e-13 * want


def test_last_layer_bias_shifts_output_by_row_scale():
    th = init_denoiser_params(3).astype(np.float64)
    layers = dn.unpack(th)
    layers[3][0][...] = 0.0
    layers[3][1][...] = (0.5, -0.25)
    h = _rows(2, 16, 6)
    s = np.sqrt(np.mean(np.abs(h) ** 2, axis=1))
    np.testing.assert_allclose(dn.forward(dn.pack(layers), h), h + s[:, None] * (0.5 - 0.25j), rtol=1e-14)


def test_scale_equivariance():
    th = init_denoiser_params(7).astype(np.float64)
    h = _rows(2, 30, 8)
    for c in (0.5, 3.0, 1e3):
        np.testing.assert_allclose(dn.forward(th, c * h), c * dn.forward(th, h), rtol=1e-12,
                                   atol=1e-12 * c * np.abs(h).max())


def test_zero_row_passes_through():
    th = init_denoiser_params(7).astype(np.float64)
    h = _rows(2, 30, 8)
    h[1] = 0
    out = dn.forward(th, h)
    np.testing.assert_array_equal(out[1], 0)
    loss, g = dn.loss_grad(th, h, _rows(2, 30, 9))
    assert np.all(np.isfinite(g)) and np.isfinite(loss)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(11)
    th = init_denoiser_params(11, last_scale=1.0).astype(np.float64)
    th += 0.05 * rng.standard_normal(th.size)       # non-zero biases too
    h = _rows(2, 24, 12)
    ht = h + 0.3 * _rows(2, 24, 13)
    loss, g = dn.loss_grad(th, h, ht)
    idx = np.concatenate([rng.choice(th.size, 150, replace=False),
                          [0, 447, 448, 479, 480, 15330 - 3, 15330 - 1]])   # layer edges, biases
    eps = 1e-6
    fd = np.empty(idx.size)
    for n, i in enumerate(idx):
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        fd[n] = (dn.loss_grad(tp, h, ht)[0] - dn.loss_grad(tm, h, ht)[0]) / (2 * eps)
    scale = np.abs(g).max()
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=1e-7 * scale)


def test_gradient_term_rss_from_single_row_gradients():
    # One position per row (U = 1): every gradient entry is a sum over rows of
    # one term each, and row r's term is the gradient of row r alone divided
    # by the row count (the loss is a mean; 8 rows keep the scaling exact).
    rng = np.random.default_rng(41)
    th = init_denoiser_params(41, last_scale=1.0).astype(np.float64) + 0.05 * rng.standard_normal(15330)
    R = 8
    h = rng.standard_normal((R, 1)) + 1j * rng.standard_normal((R, 1))
    ht = h + 0.3 * (rng.standard_normal((R, 1)) + 1j * rng.standard_normal((R, 1)))
    _, g, rss = dn.loss_grad(th, h, ht, term_rss=True)
    singles = np.stack([dn.loss_grad(th, h[r:r + 1], ht[r:r + 1])[1] / R for r in range(R)])
    np.testing.assert_allclose(g, singles.sum(axis=0), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(rss, np.sqrt((singles ** 2).sum(axis=0)), rtol=1e-10, atol=1e-14)


def test_gradient_term_rss_last_layer_brute_force():
    # Last layer, several positions: the terms are delta4[co][p] x3[ci][p+k-3]
    # with delta4 = 2 (x0 + a4 - h_true / s) / (R U), summed by explicit loops.
    rng = np.random.default_rng(43)
    th = init_denoiser_params(43, last_scale=1.0).astype(np.float64) + 0.05 * rng.standard_normal(15330)
    R, U = 2, 5
    h = _rows(R, U, 44, smooth=False)
    ht = h + 0.3 * _rows(R, U, 45, smooth=False)
    _, _, rss = dn.loss_grad(th, h, ht, term_rss=True)
    _, acts, s = dn.forward(th, h, cache=True)
    x3, a4 = acts[3], acts[4]
    d4 = np.empty((R, 2, U))
    for r in range(R):
        t = ht[r] / s[r]
        x0 = h[r] / s[r]
        d4[r, 0] = 2 * (x0.real + a4[r, 0] - t.real) / (R * U)
        d4[r, 1] = 2 * (x0.imag + a4[r, 1] - t.imag) / (R * U)
    want_w = np.zeros((2, 32, 7))
    for co in range(2):
        for ci in range(32):
            for k in range(7):
                for r in range(R):
                    for p in range(U):
                        if 0 <= p + k - 3 < U:
                            want_w[co, ci, k] += (d4[r, co, p] * x3[r, ci, p + k - 3]) ** 2
    got_w = rss[15330 - 2 - 2 * 32 * 7:15330 - 2].reshape(2, 32, 7)
    np.testing.assert_allclose(got_w, np.sqrt(want_w), rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(rss[-2:], np.sqrt((d4 ** 2).sum(axis=(0, 2))), rtol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, -0.0, 65504.0]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(dn.bf16(x), want)
    assert dn.bf16(np.array([1 + 2 ** -8]))[0] == 1.0               # tie to even
    assert dn.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def _tbf16(x):
    """bf16 rounding by torch's conversion (an implementation other than the oracle's)."""
    f = torch.from_numpy(np.asarray(x, dtype=np.float64).astype(np.float32))
    return f.to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_rounding_points_closed_form():
    # A sparse network whose weights and inputs lie off the bf16 grid, so that
    # each rounding point of the bf16 mode -- the normalised input, every
    # weight, every ReLU output and the output deltas -- changes the result.
    # The forward output and the last layer's bias gradient must equal a
    # hand-built evaluation exactly (products of bf16 values and sums of a few
    # of them are exact in FP64, so no summation order enters).
    U = 8
    layers = [(np.zeros((co, ci, dn.TAPS)), np.zeros(co)) for ci, co in dn.LAYERS]
    w1, w2, w3 = 1 + 3 * 2.0 ** -9, 1.5 + 3 * 2.0 ** -10, 0.75 + 5 * 2.0 ** -12
    w4, w5 = 0.5 + 3 * 2.0 ** -11, -0.25 - 5 * 2.0 ** -13
    layers[0][0][0, 0, 2:5] = w1  # a1[0][p] = w1 (x[p-1] + x[p] + x[p+1]) over the real input channel
    layers[1][0][0, 0, 3] = w2
    layers[2][0][0, 0, 3] = w3
    layers[3][0][0, 0, 3] = w4    # real output
    layers[3][0][1, 0, 3] = w5    # imaginary output
    theta = dn.pack(layers)
    rng = np.random.default_rng(5)
    sign = np.array([[1, 1, -1, 1, 1, -1, -1, 1]], dtype=np.float64)
    h = sign * (1 + rng.integers(1, 200, size=(1, U)) * 2.0 ** -11) + 1j * rng.standard_normal((1, U))
    ht = h + 0.25 * (rng.standard_normal((1, U)) + 1j * rng.standard_normal((1, U)))

    s = np.sqrt(np.mean(np.abs(h) ** 2))
    x = _tbf16(h.real[0] / s)
    xp = np.concatenate([[0.0], x, [0.0]])
    a1 = _tbf16(w1) * (xp[:-2] + xp[1:-1] + xp[2:])
    x1 = _tbf16(np.maximum(a1, 0.0))
    x2 = _tbf16(np.maximum(_tbf16(w2) * x1, 0.0))
    x3 = _tbf16(np.maximum(_tbf16(w3) * x2, 0.0))
    a4r, a4i = _tbf16(w4) * x3, _tbf16(w5) * x3
    assert (a1 > 0).any() and (a1 < 0).any()  # the ReLU both passes and blocks
    want = h + s * (a4r + 1j * a4i)
    got = dn.forward(theta, h, bf16_ops=True)
    assert np.array_equal(got, want)
    assert not np.allclose(dn.forward(theta, h), want, rtol=1e-9, atol=0)  # the roundings matter

    n = U
    er = h.real[0] / s + a4r - ht.real[0] / s
    ei = h.imag[0] / s + a4i - ht.imag[0] / s
    gb4 = np.array([_tbf16(2 * er / n).sum(), _tbf16(2 * ei / n).sum()])
    _, g = dn.loss_grad(theta, h, ht, bf16_ops=True)
    assert np.array_equal(g[-2:], gb4)


def test_bf16_operands_stay_within_their_error_bound():
    # Each rounding is within 2^-9 relative; over 4 layers the refined part of
    # the output must stay within a few percent of the exact one, and the
    # gradient direction must be essentially unchanged.
    th = init_denoiser_params(21, last_scale=1.0).astype(np.float64)
    h = _rows(4, 64, 22)
    ht = h + 0.2 * _rows(4, 64, 23)
    exact = dn.forward(th, h) - h
    rounded = dn.forward(th, h, bf16_ops=True) - h
    rel = np.linalg.norm(rounded - exact) / np.linalg.norm(exact)
    assert 1e-5 < rel < 2e-2
    _, g0 = dn.loss_grad(th, h, ht)
    _, g1 = dn.loss_grad(th, h, ht, bf16_ops=True)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 3e-2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    new, m, v = dn.adam(th, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    # bias correction makes m_hat = g and v_hat = g^2 on step 1
    np.testing.assert_allclose(new, th - lr * g / (np.abs(g) + eps), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_lr_per_step():
    th = np.zeros(3)
    m = v = np.zeros(3)
    g = np.array([2.0, -0.5, 1e-3])
    for t in range(1, 6):
        th, m, v = dn.adam(th, m, v, g, t, 0.01, eps=0.0)
    # with a constant gradient m_hat = g and v_hat = g^2 exactly at every step
    np.testing.assert_allclose(th, -0.05 * np.sign(g), rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_training_reduces_loss(seed):
    # A few Adam steps on a fixed batch must lower the loss (plain gradient descent sanity).
    th = init_denoiser_params(seed).astype(np.float64)
    h_true = _rows(4, 48, 100 + seed)
    h = h_true + 0.3 * _rows(4, 48, 200 + seed, smooth=False)
    m = v = np.zeros_like(th)
    first = None
    for t in range(1, 16):
        loss, g = dn.loss_grad(th, h, h_true)
        first = loss if first is None else first
        th, m, v = dn.adam(th, m, v, g, t, 3e-3)
    assert dn.loss_grad(th, h, h_true)[0] < 0.8 * first


def _bias_only(b0, b1=0.0):
    th = init_denoiser_params(3).astype(np.float64)
    layers = dn.unpack(th)
    layers[3][0][...] = 0.0
    layers[3][1][...] = (b0, b1)
    return dn.pack(layers)


def test_ls_fallback_threshold_closed_form():
    # a last layer of bias (b, 0) alone corrects every subcarrier by s*b, so the
    # correction's energy is b^2 times the row's: kept below max_corr, LS above
    h = _rows(3, 50, 12)
    for b, mc, want in ((0.9, 1.0, False), (1.1, 1.0, True), (1.5, 2.0, False), (1.5, 1.4, True),
                        (-0.99, 1.0, False)):
        out = dn.forward(_bias_only(b), h)
        got, fell = dn.ls_fallback(h, out, max_corr=mc)
        assert np.all(fell == want), (b, mc)
        np.testing.assert_array_equal(got, h if want else out)


def test_ls_fallback_per_row_and_non_finite():
    h = _rows(4, 20, 13)
    out = h + 0.5 * h                       # correction energy 0.25 of the row's: kept
    out[1] = h[1] + 2.0 * h[1]              # 4x: LS
    out[2, 7] = np.nan                      # non-finite refinement: LS
    got, fell = dn.ls_fallback(h, out)
    np.testing.assert_array_equal(fell, [False, True, True, False])
    np.testing.assert_array_equal(got[[1, 2]], h[[1, 2]])
    np.testing.assert_array_equal(got[[0, 3]], out[[0, 3]])
    # with no energy limit an infinite output still falls back
    out2 = h.copy()
    out2[3, 0] = np.inf
    _, fell2 = dn.ls_fallback(h, out2, max_corr=np.inf)
    np.testing.assert_array_equal(fell2, [False, False, False, True])
    # a zero row that passes through keeps its (zero) estimate, not a fallback
    hz = h.copy()
    hz[0] = 0
    _, fell3 = dn.ls_fallback(hz, dn.forward(_bias_only(0.5), hz))
    assert not fell3[0]
