"""Pins of the oracle's FFT against mathematics that does not depend on it.

The oracle FFT is the forward, unnormalised DFT Y[k] = sum_n y[n] e^{-2 pi i k n/N}
(the transform taken after CP removal, paper Section II-B; sign and scale are a
stated reading).  It is pinned by brute force on tiny N, by closed forms, by
numpy's FFT (a library special case), by Parseval and by a round trip.
"""
import numpy as np
import pytest

import oracle


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64])
def test_fft_equals_bruteforce_dft(n):
    x = _rand(n, n)
    # O(N^2) sum written as nested Python loops: the definition itself.
    ref = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        acc = 0j
        for m in range(n):
            acc += x[m] * complex(np.cos(-2 * np.pi * k * m / n), np.sin(-2 * np.pi * k * m / n))
        ref[k] = acc
    got = oracle.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048])
def test_fft_matches_numpy(n):
    x = _rand(n, 100 + n) * 1000
    ref = np.fft.fft(x)
    got = oracle.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [8, 64, 1024])
def test_fft_closed_forms(n):
    k = np.arange(n)
    delta = np.zeros(n, complex)
    delta[0] = 1
    assert np.allclose(oracle.fft(delta), np.ones(n), atol=1e-13, rtol=0)
    # delayed impulse -> linear phase e^{-2 pi i k m / N}
    m = 3
    dm = np.zeros(n, complex)
    dm[m] = 1
    assert np.allclose(oracle.fft(dm), np.exp(-2j * np.pi * k * m / n), atol=1e-13, rtol=0)
    # constant -> N at DC only
    c = oracle.fft(np.ones(n, complex))
    want = np.zeros(n, complex)
    want[0] = n
    assert np.max(np.abs(c - want)) <= 1e-12 * n
    # complex tone at bin k0 -> N at k0 only (so the sign convention is forward)
    k0 = 5
    tone = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    want = np.zeros(n, complex)
    want[k0] = n
    assert np.max(np.abs(oracle.fft(tone) - want)) <= 1e-12 * n


@pytest.mark.parametrize("n", [64, 1024, 2048])
def test_fft_parseval_roundtrip_linearity(n):
    x = _rand(n, 7 * n)
    y = _rand(n, 7 * n + 1)
    X = oracle.fft(x)
    # Parseval: sum |x|^2 = sum |X|^2 / N
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / n) <= 1e-12 * np.sum(np.abs(x) ** 2)
    # inverse through conjugation, then forward again: the identity
    xinv = np.conj(oracle.fft(np.conj(X))) / n
    assert np.max(np.abs(xinv - x)) <= 1e-12 * np.max(np.abs(x))
    # linearity
    a, b = 0.3 - 1.1j, 2.5 + 0.25j
    lhs = oracle.fft(a * x + b * y)
    rhs = a * X + b * oracle.fft(y)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12, complex))


@pytest.mark.parametrize("S,T,A,N,CP", [(2, 3, 3, 64, 16), (3, 4, 5, 128, 9), (2, 3, 4, 64, 0)])
def test_fft_symbols_is_cp_strip_then_numpy_fft(S, T, A, N, CP):
    """CP removal + FFT of every antenna's symbol (paper Sec. II-B): each
    [S][T][A] record of the int16 buffer loses its first CP samples and the
    remaining N go through the forward DFT, output in [s][t][a][k] order.
    Every record holds different random samples (CP included), so a wrong slot
    stride, symbol/antenna order or CP offset shows as a mismatch."""
    rng = np.random.default_rng(1000 * S + 100 * T + 10 * A + CP)
    iq = rng.integers(-32768, 32768, size=(S, T, A, CP + N, 2), dtype=np.int16)
    pilot = np.ones(N // 2, dtype=np.complex128)
    got = oracle.fft_symbols(iq, pilot, n_ant=A, fft_len=N, cp_len=CP, n_used=N // 2, n_sym=T, bits_per_sym=2)
    assert got.shape == (S, T, A, N)
    y = iq[..., CP:, 0].astype(np.float64) + 1j * iq[..., CP:, 1].astype(np.float64)
    ref = np.fft.fft(y, axis=-1)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale
