"""Comparison rules between the GPU library and the FP64 oracle.

x-hat: per element |x_gpu - x_ref| <= 1e-4 * max(1, |x_ref|) (FP32 path; the
constellation has unit RMS, so this is a relative bound for typical points
and does not blow up near 0).

bits: identical, except a bit whose oracle coordinate lies within 1e-3 of one
of that bit's decision thresholds (normalised units), where either value is
accepted.  Thresholds: first bit of an axis {0}; 16-QAM second {2/sqrt(10)};
64-QAM second {4/sqrt(42)}, third {2/sqrt(42), 6/sqrt(42)}.

H: the LS estimate is one FFT bin times a pilot factor; FP32 FFT rounding
gives an error near eps * log2(N) times the RMS of the spectrum, so H is
compared against 1e-5 of the RMS of the oracle's estimates of that slot.
"""
import math

import numpy as np

XHAT_RTOL = 1e-4
BAND = 1e-3
H_RTOL = 1e-5


def as_complex(t):
    """float32 [..., 2] tensor/array -> complex128 numpy."""
    a = t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def check_xhat(x_gpu, x_ref):
    err = np.abs(x_gpu - x_ref)
    bound = XHAT_RTOL * np.maximum(1.0, np.abs(x_ref))
    bad = err > bound
    assert not bad.any(), (f"{bad.sum()} x-hat elements out of tolerance; worst err {err.max():.3e}, "
                           f"first at {np.argwhere(bad)[0].tolist()}")
    return float(err.max())


def exempt_mask(x_ref, b):
    """Bit-level mask [..., U, b] of bits inside the 1e-3 decision band."""
    axes = [x_ref.real, x_ref.imag]
    thr = {2: [[0.0]],
           4: [[0.0], [2 / math.sqrt(10)]],
           6: [[0.0], [4 / math.sqrt(42)], [2 / math.sqrt(42), 6 / math.sqrt(42)]]}[b]
    m = np.zeros(x_ref.shape + (b,), dtype=bool)
    for j, ts in enumerate(thr):
        for ax in (0, 1):
            c = np.abs(axes[ax])
            near = np.zeros_like(c, dtype=bool)
            for t in ts:
                near |= np.abs(c - t) < BAND
            m[..., 2 * j + ax] = near
    return m


def check_bits(bits_gpu, bits_ref, x_ref, b):
    """Packed bits [S][Td][U*b/8]; x_ref complex [S][Td][U] from the oracle."""
    g = np.unpackbits(np.asarray(bits_gpu), axis=-1).reshape(x_ref.shape + (b,))
    r = np.unpackbits(np.asarray(bits_ref), axis=-1).reshape(x_ref.shape + (b,))
    ex = exempt_mask(x_ref, b)
    diff = (g != r) & ~ex
    assert not diff.any(), f"{diff.sum()} bits differ outside the decision band, first at {np.argwhere(diff)[0].tolist()}"
    return int(((g != r) & ex).sum()), int(ex.sum())


def check_H(H_gpu, H_ref):
    scale = np.sqrt(np.mean(np.abs(H_ref) ** 2, axis=(1, 2), keepdims=True))
    scale = np.maximum(scale, 1e-30)
    rel = np.abs(H_gpu - H_ref) / scale
    assert rel.max() <= H_RTOL, f"H error {rel.max():.3e} of the slot RMS"
    return float(rel.max())
