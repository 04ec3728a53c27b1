"""FP64 reference of the learned channel-estimate denoiser -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library.

The network (a refinement of the least-squares estimate; the paper computes
LS only, Sec. II-C, LS paragraph, and cites LS estimation for OFDM, whose
comb-pilot form with interpolation is the input here):

  per row (one antenna of one slot) with estimate h[d], d = 0..U-1:
    s      = sqrt(mean_d |h[d]|^2)                    (row scale; no gradient)
    x0     = (Re h / s, Im h / s)                     2 channels x U
    a_l    = b_l + sum_ci sum_k W_l[co][ci][k] x_{l-1}[ci][d + k - 3]
             (x zero outside 0..U-1), l = 1..4, 7 taps
    x_l    = max(a_l, 0) for l = 1, 2, 3;  channels 2 -> 32 -> 32 -> 32 -> 2
    out    = h + s (a_4[0] + i a_4[1])                (residual)
  a row with s == 0 passes through unchanged.
  loss (training) = mean over rows and d of |x0 + a_4 - h_true / s|^2.

``bf16=True`` rounds, as the GPU kernels do, the weights, x0..x3 and the
backward deltas to bfloat16 (round to nearest even, through float32) before
they enter a product; sums stay exact (FP64) here.

Parameter vector layout: for l = 1..4, W_l[co][ci][k] then b_l[co].
"""
from __future__ import annotations

import numpy as np

LAYERS = ((2, 32), (32, 32), (32, 32), (32, 2))
TAPS = 7
HALF = TAPS // 2


def param_count() -> int:
    return sum(co * ci * TAPS + co for ci, co in LAYERS)


def unpack(theta: np.ndarray):
    """[(W [co][ci][k], b [co]) per layer] as float64 views/copies."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ci, co in LAYERS:
        W = theta[o:o + co * ci * TAPS].reshape(co, ci, TAPS)
        o += co * ci * TAPS
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) through float32; returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """'Same' 1-D correlation with zero padding: x [R][ci][U] -> [R][co][U]."""
    R, ci, U = x.shape
    xp = np.zeros((R, ci, U + 2 * HALF))
    xp[:, :, HALF:HALF + U] = x
    y = np.broadcast_to(b[None, :, None], (R, W.shape[0], U)).copy()
    for k in range(TAPS):
        y += np.einsum("oc,rcu->rou", W[:, :, k], xp[:, :, k:k + U])
    return y


def _scale(h: np.ndarray) -> np.ndarray:
    return np.sqrt(np.mean(np.abs(h) ** 2, axis=-1))


def _input(h: np.ndarray, s: np.ndarray) -> np.ndarray:
    safe = np.where(s > 0, s, 1.0)
    return np.stack([h.real / safe[:, None], h.imag / safe[:, None]], axis=1)


def forward(theta: np.ndarray, h: np.ndarray, *, bf16_ops: bool = False, cache: bool = False):
    """Refined estimate for rows h (complex [R][U]); with ``cache`` also the
    activations (x0, x1, x2, x3, a4) and the row scales."""
    h = np.asarray(h, dtype=np.complex128)
    rnd = bf16 if bf16_ops else (lambda v: v)
    s = _scale(h)
    x = rnd(_input(h, s))
    acts = [x]
    layers = unpack(theta)
    for li, (W, b) in enumerate(layers):
        a = conv(x, rnd(W), b)
        if li < len(layers) - 1:
            x = rnd(np.maximum(a, 0.0))
            acts.append(x)
        else:
            acts.append(a)
    a4 = acts[-1]
    out = h + s[:, None] * (a4[:, 0] + 1j * a4[:, 1])
    out = np.where(s[:, None] > 0, out, h)
    if cache:
        return out, acts, s
    return out


def ls_fallback(h: np.ndarray, out: np.ndarray, max_corr: float = 1.0):
    """Plain LS as the refinement's fallback and judge: row r keeps its LS
    estimate h[r] when the correction c = out[r] - h[r] has a non-finite entry
    or carries more energy than max_corr^2 times the row's own,
    sum_d |c[d]|^2 > max_corr^2 sum_d |h[d]|^2.  (An ideal denoiser removes
    noise, and the noise's energy never exceeds the noisy estimate's.)
    Returns (the rows kept or refined, boolean mask of rows that fell back)."""
    h = np.asarray(h, dtype=np.complex128)
    out = np.asarray(out, dtype=np.complex128)
    with np.errstate(invalid="ignore", over="ignore"):
        e = np.sum(np.abs(out - h) ** 2, axis=-1)
        fell = ~np.isfinite(e) | ~(e <= max_corr ** 2 * np.sum(np.abs(h) ** 2, axis=-1))
    return np.where(fell[:, None], h, out), fell


def loss_grad(theta: np.ndarray, h: np.ndarray, h_true: np.ndarray, *, bf16_ops: bool = False,
              term_rss: bool = False):
    """Training loss and its gradient with respect to theta (analytic backward).

    Each gradient entry is a sum over rows and positions of products
    delta * x (weights) or of deltas (biases).  With ``term_rss`` a third
    result gives, per entry, the root of the sum of those terms' squares: the
    scale of the difference a second implementation makes when it rounds a
    few of the terms' operands to the other neighbouring bf16 value
    (independent errors of relative size u on the terms add up to about
    u * rss)."""
    h = np.asarray(h, dtype=np.complex128)
    h_true = np.asarray(h_true, dtype=np.complex128)
    rnd = bf16 if bf16_ops else (lambda v: v)
    _, acts, s = forward(theta, h, bf16_ops=bf16_ops, cache=True)
    R, U = h.shape
    safe = np.where(s > 0, s, 1.0)
    t = np.stack([h_true.real / safe[:, None], h_true.imag / safe[:, None]], axis=1)
    x0 = acts[0]
    # the residual adds the unrounded normalised input; x0 is its bf16 image
    # only as the first layer's operand
    x0_exact = _input(h, s)
    e = x0_exact + acts[-1] - t
    live = (s > 0)[:, None, None]
    e = np.where(live, e, 0.0)
    n = R * U
    loss = float(np.sum(e ** 2) / n)
    delta = rnd(2.0 * e / n)  # dL/da4
    layers = unpack(theta)
    grads = [None] * len(layers)
    rss = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        Wr = rnd(W)
        xin = acts[li]
        xp = np.zeros(xin.shape[:2] + (U + 2 * HALF,))
        xp[:, :, HALF:HALF + U] = xin
        gW = np.empty_like(W)
        for k in range(TAPS):
            gW[:, :, k] = np.einsum("rou,rcu->oc", delta, xp[:, :, k:k + U])
        gb = delta.sum(axis=(0, 2))
        grads[li] = (gW, gb)
        if term_rss:
            qW = np.empty_like(W)
            for k in range(TAPS):
                qW[:, :, k] = np.einsum("rou,rcu->oc", delta ** 2, xp[:, :, k:k + U] ** 2)
            rss[li] = (np.sqrt(qW), np.sqrt((delta ** 2).sum(axis=(0, 2))))
        if li == 0:
            break
        # dL/dx_{li} = transposed correlation of delta with W, then the ReLU mask
        dp = np.zeros(delta.shape[:2] + (U + 2 * HALF,))
        dp[:, :, HALF:HALF + U] = delta
        gx = np.zeros(xin.shape)
        for k in range(TAPS):
            # x[d + k - 3] fed a[d]: so dx[u] += W[:, :, k]^T delta[u - k + 3]
            gx += np.einsum("oc,rou->rcu", Wr[:, :, k], dp[:, :, 2 * HALF - k:2 * HALF - k + U])
        delta = rnd(gx * (xin > 0))
    if term_rss:
        return loss, pack(grads), pack(rss)
    return loss, pack(grads)


def adam(theta, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015, Algorithm 1); returns new (theta, m, v)."""
    theta = np.asarray(theta, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def nmse_db(h_est: np.ndarray, h_true: np.ndarray) -> float:
    """10 log10(sum |h_est - h_true|^2 / sum |h_true|^2)."""
    return float(10 * np.log10(np.sum(np.abs(h_est - h_true) ** 2) / np.sum(np.abs(h_true) ** 2)))
