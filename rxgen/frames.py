"""Seeded synthetic uplink frames for the single-user massive-MIMO OFDM receiver.

This module produces *inputs* only: the int16 IQ buffer a receiver consumes,
the pilot it is configured with, and the ground truth that produced them
(transmitted bits and symbols, the true channel, the SNR).  It implements the
transmit side and the radio channel, never the receive side: there is no FFT
of received samples, no channel estimate, no combining and no demapping here.
Both the FP64 oracle and the GPU library read the very same buffers.

Frame structure follows the paper's Section II-B: one channel-estimation
(pilot) OFDM symbol followed by QAM data symbols, a cyclic prefix on every
symbol, the same frame received on every antenna.  Table I fixes the FFT
lengths (64, 1024) and CP lengths (16, 72).  Everything the paper leaves open
(subcarrier placement, constellation, channel model, SNR definition, int16
scaling) follows the readings listed in the design notes: used subcarriers are
the signed frequencies -U/2..-1, +1..+U/2; QAM is per-axis Gray PAM with unit
average energy; the channel is a tapped-delay Rayleigh channel with an
exponential power-delay profile, constant over a slot; AWGN is set so that the
per-antenna, per-subcarrier Es/N0 equals the SNR; samples are scaled per slot
so that the largest |I| or |Q| is half of int16 full scale.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

INT16_FS = 32767.0

# Seeds of the named workloads (base + configuration index).
SEED_BASE = 190107499


@dataclasses.dataclass(frozen=True)
class FrameConfig:
    """Shape and channel recipe of one synthetic workload."""
    name: str
    n_ant: int            # A receive antennas
    fft_len: int          # N
    cp_len: int           # CP samples per symbol
    n_sym: int            # T symbols per slot: 1 pilot + T-1 data
    n_used: int           # U used subcarriers
    bits_per_sym: int     # b: 2 (QPSK), 4 (16-QAM), 6 (64-QAM)
    n_slots: int          # S slots per run
    n_taps: int           # L channel taps
    tau_max_us: Tuple[float, float]  # maximum excess delay, uniform in [lo, hi] microseconds
    fs_hz: float          # sample rate
    snr_db: Tuple[float, float]      # per-slot SNR, uniform in [lo, hi] dB
    seed: int
    tap_decay_db: float = 3.0        # power drop per tap index
    unit_spaced_taps: bool = False   # taps at delays 0..L-1 samples (tiny workload)
    pilot_spacing: int = 1           # 1: every used subcarrier of symbol 0 is a pilot; s > 1: only d % s == 0 (comb)
    n_taps_range: Optional[Tuple[int, int]] = None  # if set, L is drawn per slot uniformly in [lo, hi]

    @property
    def slot_samples(self) -> int:
        return self.n_sym * self.n_ant * (self.fft_len + self.cp_len)

    @property
    def slot_bytes(self) -> int:
        return 4 * self.slot_samples

    def replace(self, **kw) -> "FrameConfig":
        return dataclasses.replace(self, **kw)


# Tiny workload: 8 antennas, N=64, CP 16, 1 BPSK pilot + 10 QPSK data, 52 used
# subcarriers, 4-tap Rayleigh at 3 dB/tap, 20 dB, one slot.
C1 = FrameConfig("c1_tiny_A8_N64", n_ant=8, fft_len=64, cp_len=16, n_sym=11, n_used=52,
                 bits_per_sym=2, n_slots=1, n_taps=4, tau_max_us=(0.0, 0.0), fs_hz=20e6,
                 snr_db=(20.0, 20.0), seed=SEED_BASE + 1, unit_spaced_taps=True)

# Workload at scale: 64 antennas, N=1024, CP 72, 1 pilot + 13 16-QAM, 600 used,
# 10-tap exponential-PDP Rayleigh, max delay U[0.5, 3] us at 15.36 MS/s,
# SNR U[5, 30] dB, 200 slots (785.6 MB of int16 IQ).
C2 = FrameConfig("c2_A64_N1024_S200", n_ant=64, fft_len=1024, cp_len=72, n_sym=14, n_used=600,
                 bits_per_sym=4, n_slots=200, n_taps=10, tau_max_us=(0.5, 3.0), fs_hz=15.36e6,
                 snr_db=(5.0, 30.0), seed=SEED_BASE + 2)

# Same as C2 with the SNR fixed at 20 dB (quality figures at 20 dB).
C2_20DB = C2.replace(name="c2_A64_N1024_S200_20dB", snr_db=(20.0, 20.0), seed=SEED_BASE + 12)

# Largest shape: 128 antennas, N=2048, CP 144, 1 pilot + 13 64-QAM, 1200 used,
# 500 slots (7.86 GB of int16 IQ).  Delays are clamped to the CP.
C4 = FrameConfig("c4_A128_N2048_S500", n_ant=128, fft_len=2048, cp_len=144, n_sym=14, n_used=1200,
                 bits_per_sym=6, n_slots=500, n_taps=10, tau_max_us=(0.5, 3.0), fs_hz=30.72e6,
                 snr_db=(10.0, 30.0), seed=SEED_BASE + 4)

# Learned-denoiser workload: the C4 shape with a comb pilot on every 4th used
# subcarrier (300 of 1200; the pilot symbol carries nothing elsewhere), 8-24
# taps per slot, maximum delay U[0.5, 5] us (clamped to the CP), SNR U[0, 30] dB.
C5 = FrameConfig("c5_A128_N2048_comb4", n_ant=128, fft_len=2048, cp_len=144, n_sym=14, n_used=1200,
                 bits_per_sym=6, n_slots=32, n_taps=24, tau_max_us=(0.5, 5.0), fs_hz=30.72e6,
                 snr_db=(0.0, 30.0), seed=SEED_BASE + 5, pilot_spacing=4, n_taps_range=(8, 24))

# The same at a fixed 20 dB (quality figures).
C5_20DB = C5.replace(name="c5_A128_N2048_comb4_20dB", snr_db=(20.0, 20.0), seed=SEED_BASE + 15)

CONFIGS = {c.name: c for c in (C1, C2, C2_20DB, C4, C5, C5_20DB)}

# Antenna-count x FFT-length sweep: Table I's two FFT lengths (64 with a
# 16-sample CP, 1024 with 72) at 1..16 receive antennas, extended to 128;
# 14 symbols per slot (1 pilot + 13 data).  N = 64 carries 52 used
# subcarriers of QPSK at the paper's 10 MHz; N = 1024 the C2 shape (600 used,
# 16-QAM, 15.36 MS/s).  Channel and SNR as C2 (delays clamped to the CP).
SWEEP_ANTENNAS = (1, 2, 4, 8, 16, 32, 64, 128)
SWEEP_FFT_LENS = (64, 1024)


def sweep_config(fft_len: int, n_ant: int, target_bytes: int = 1 << 30) -> FrameConfig:
    """One sweep point, with enough slots that the int16 input fills
    ``target_bytes`` (rounded up to a whole slot)."""
    if fft_len == 64:
        cp, used, b, fs = 16, 52, 2, 10e6
    elif fft_len == 1024:
        cp, used, b, fs = 72, 600, 4, 15.36e6
    else:
        raise ValueError("the sweep covers FFT lengths 64 and 1024")
    i = SWEEP_FFT_LENS.index(fft_len) * len(SWEEP_ANTENNAS) + SWEEP_ANTENNAS.index(n_ant)
    cfg = C2.replace(name=f"sweep_N{fft_len}_A{n_ant}", n_ant=n_ant, fft_len=fft_len, cp_len=cp, n_used=used,
                     bits_per_sym=b, fs_hz=fs, seed=SEED_BASE + 100 + i)
    return cfg.replace(n_slots=-(-target_bytes // cfg.slot_bytes))


def used_subcarrier_bins(fft_len: int, n_used: int) -> np.ndarray:
    """FFT bin of each used subcarrier, in ascending signed frequency.

    Transmit-side placement: subcarrier d carries signed frequency
    -U/2..-1 for the first half and +1..+U/2 for the second (DC unused),
    i.e. the centred order an fftshift produces (Section II-C).
    """
    half = n_used // 2
    freqs = np.concatenate([np.arange(-half, 0), np.arange(1, half + 1)])
    return np.mod(freqs, fft_len).astype(np.int64)


def qam_symbols(bits: np.ndarray, bits_per_sym: int) -> np.ndarray:
    """Gray-mapped square QAM with unit average energy (transmit side).

    ``bits`` has a trailing axis of length ``bits_per_sym`` holding
    b0, b1, ..., b_{b-1}; even-indexed bits drive the in-phase axis and
    odd-indexed bits the quadrature axis.  Per axis the amplitude is the
    3GPP-style nested Gray PAM: 2 bits/symbol -> +-1, 4 -> +-(1, 3),
    6 -> +-(1, 3, 5, 7), scaled by 1/sqrt(2), 1/sqrt(10), 1/sqrt(42).
    """
    b = np.asarray(bits, dtype=np.int64)
    if bits_per_sym == 2:
        scale = 1.0 / math.sqrt(2.0)
        re = 1 - 2 * b[..., 0]
        im = 1 - 2 * b[..., 1]
    elif bits_per_sym == 4:
        scale = 1.0 / math.sqrt(10.0)
        re = (1 - 2 * b[..., 0]) * (2 - (1 - 2 * b[..., 2]))
        im = (1 - 2 * b[..., 1]) * (2 - (1 - 2 * b[..., 3]))
    elif bits_per_sym == 6:
        scale = 1.0 / math.sqrt(42.0)
        re = (1 - 2 * b[..., 0]) * (4 - (1 - 2 * b[..., 2]) * (2 - (1 - 2 * b[..., 4])))
        im = (1 - 2 * b[..., 1]) * (4 - (1 - 2 * b[..., 3]) * (2 - (1 - 2 * b[..., 5])))
    else:
        raise ValueError("bits_per_sym must be 2, 4 or 6")
    return (re + 1j * im) * scale


def tap_delays_powers(cfg: FrameConfig, tau_max_s: float, n_taps: Optional[int] = None
                      ) -> Tuple[np.ndarray, np.ndarray]:
    """Delays (samples) and normalised powers of the L taps of one slot."""
    L = cfg.n_taps if n_taps is None else int(n_taps)
    if cfg.unit_spaced_taps or L == 1:
        delays = np.arange(L, dtype=np.int64)
    else:
        span = tau_max_s * cfg.fs_hz
        delays = np.rint(np.arange(L) * span / (L - 1)).astype(np.int64)
    delays = np.minimum(delays, cfg.cp_len)  # never beyond the cyclic prefix
    p = 10.0 ** (-cfg.tap_decay_db / 10.0 * np.arange(L))
    return delays, p / p.sum()


@dataclasses.dataclass
class Frames:
    """One run of synthetic slots plus everything needed to evaluate a receiver."""
    cfg: FrameConfig
    iq: np.ndarray          # int16 [S][T][A][CP+N][2]
    pilot: np.ndarray       # complex128 [U], the known pilot symbol X_p[d]
    bits: np.ndarray        # uint8 {0,1} [S][T-1][U][b], transmitted data bits
    X: np.ndarray           # complex128 [S][T-1][U], transmitted data symbols
    H_true: np.ndarray      # complex128 [S][A][U], true channel in receiver units
    snr_db: np.ndarray      # float64 [S]
    scale: np.ndarray       # float64 [S], int16 gain applied to the slot
    y: Optional[np.ndarray] = None  # complex128 [S][T][A][CP+N] before quantisation (if kept)

    def packed_bits(self) -> np.ndarray:
        """Transmitted bits packed MSB-first, rows of U*b/8 bytes per data symbol."""
        S, Td = self.bits.shape[:2]
        flat = self.bits.reshape(S, Td, -1)
        return np.packbits(flat, axis=-1, bitorder="big")


def _slot(cfg: FrameConfig, rng: np.random.Generator, pilot: np.ndarray, bins: np.ndarray,
          channel: str, delay: int, noise: bool, scale_override: Optional[float]):
    N, CP, T, A, U, b = cfg.fft_len, cfg.cp_len, cfg.n_sym, cfg.n_ant, cfg.n_used, cfg.bits_per_sym
    bits = rng.integers(0, 2, size=(T - 1, U, b), dtype=np.uint8)
    X = qam_symbols(bits, b)
    grid = np.zeros((T, N), dtype=np.complex128)
    grid[0, bins] = pilot
    grid[1:, bins] = X
    # x[n] = (1/sqrt(N)) sum_k X[k] e^{+j 2 pi k n / N}, with the CP prepended.
    x = np.fft.ifft(grid, axis=1) * math.sqrt(N)
    x = np.concatenate([x[:, N - CP:], x], axis=1).reshape(-1)

    lo, hi = cfg.tau_max_us
    tau = rng.uniform(lo, hi) * 1e-6
    n_taps = None
    if cfg.n_taps_range is not None:
        n_taps = int(rng.integers(cfg.n_taps_range[0], cfg.n_taps_range[1] + 1))
    if channel == "rayleigh":
        delays, p = tap_delays_powers(cfg, tau, n_taps)
        h = (rng.standard_normal((A, len(p))) + 1j * rng.standard_normal((A, len(p)))) * np.sqrt(p / 2.0)
    elif channel == "flat":
        delays = np.zeros(1, dtype=np.int64)
        h = (rng.standard_normal((A, 1)) + 1j * rng.standard_normal((A, 1))) / math.sqrt(2.0)
    elif channel == "delay":
        delays = np.array([delay], dtype=np.int64)
        h = np.ones((A, 1), dtype=np.complex128)
    else:
        raise ValueError(channel)

    # Linear convolution from zero state at the start of the slot.
    y = np.zeros((A, x.size), dtype=np.complex128)
    for l, dl in enumerate(delays):
        y[:, dl:] += h[:, l:l + 1] * x[None, :x.size - dl]

    snr = rng.uniform(*cfg.snr_db)
    if noise:
        sigma2 = 10.0 ** (-snr / 10.0)
        amp = np.float32(math.sqrt(sigma2 / 2.0))
        y.real += rng.standard_normal(y.shape, dtype=np.float32) * amp
        y.imag += rng.standard_normal(y.shape, dtype=np.float32) * amp

    peak = max(np.abs(y.real).max(), np.abs(y.imag).max())
    scale = scale_override if scale_override is not None else (0.5 * INT16_FS / peak if peak > 0 else 1.0)

    # True channel per used subcarrier, in the units a receiver sees after an
    # unnormalised FFT of the int16 samples: sqrt(N) * scale * sum_l h_l e^{-j2pi k d_l/N}.
    ph = np.exp(-2j * np.pi * np.outer(bins, delays) / N)          # [U][L]
    H = (h @ ph.T) * (math.sqrt(N) * scale)                          # [A][U]

    y = y.reshape(A, T, N + CP).transpose(1, 0, 2)                   # [T][A][N+CP]
    return bits, X, H, snr, scale, y


def _slot_job(job):
    cfg, child, pilot, bins, channel, delay, noise, scale, keep_float = job
    rng = np.random.Generator(np.random.PCG64(child))
    bi, Xs, Hs, sn, sc, y = _slot(cfg, rng, pilot, bins, channel, delay, noise, scale)
    q = np.rint(y * sc)
    iq = np.empty(y.shape + (2,), dtype=np.int16)
    iq[..., 0] = np.clip(q.real, -32768, 32767)
    iq[..., 1] = np.clip(q.imag, -32768, 32767)
    return iq, bi, Xs, Hs, sn, sc, (y * sc if keep_float else None)


def make_frames(cfg: FrameConfig, n_slots: Optional[int] = None, seed: Optional[int] = None, *,
                channel: str = "rayleigh", delay: int = 0, noise: bool = True,
                keep_float: bool = False, scale: Optional[float] = None,
                first_slot: int = 0, workers: int = 1,
                pilot: Optional[np.ndarray] = None) -> Frames:
    """Generate ``n_slots`` slots (default ``cfg.n_slots``) deterministically from ``seed``.

    channel: "rayleigh" (tapped-delay, per the config), "flat" (one Rayleigh tap)
    or "delay" (a pure delay of ``delay`` samples, unit gain).  ``noise=False``
    gives noiseless frames; ``keep_float`` keeps the complex samples before
    int16 quantisation; ``scale`` fixes the int16 gain instead of normalising
    each slot's peak.  Slot ``s`` always draws from the same child stream, so a
    run of ``n_slots`` starting at ``first_slot`` is a window of the full run,
    and the result does not depend on ``workers`` (processes used to generate
    slots in parallel; start them before the process touches a GPU).
    ``pilot`` replaces the seeded BPSK pilot by any U non-zero complex values.
    With ``cfg.pilot_spacing`` s > 1 the pilot symbol is a comb: the seeded
    BPSK values sit on subcarriers d % s == 0 and the others carry zero.
    """
    S = cfg.n_slots if n_slots is None else int(n_slots)
    seed = cfg.seed if seed is None else int(seed)
    N, CP, T, A, U, b = cfg.fft_len, cfg.cp_len, cfg.n_sym, cfg.n_ant, cfg.n_used, cfg.bits_per_sym
    if U % 2 or not (2 <= U <= N - 2):
        raise ValueError("n_used must be even and in [2, N-2]")
    children = np.random.SeedSequence(seed).spawn(first_slot + S + 1)
    prng = np.random.Generator(np.random.PCG64(children[0]))
    seeded_pilot = (1 - 2 * prng.integers(0, 2, size=U)).astype(np.complex128)   # BPSK +-1
    if cfg.pilot_spacing > 1:
        seeded_pilot[np.arange(U) % cfg.pilot_spacing != 0] = 0.0
    pilot = seeded_pilot if pilot is None else np.asarray(pilot, dtype=np.complex128).reshape(U)
    bins = used_subcarrier_bins(N, U)

    iq = np.empty((S, T, A, N + CP, 2), dtype=np.int16)
    bits = np.empty((S, T - 1, U, b), dtype=np.uint8)
    X = np.empty((S, T - 1, U), dtype=np.complex128)
    H = np.empty((S, A, U), dtype=np.complex128)
    snr = np.empty(S)
    scl = np.empty(S)
    yk = np.empty((S, T, A, N + CP), dtype=np.complex128) if keep_float else None
    jobs = [(cfg, children[first_slot + s + 1], pilot, bins, channel, delay, noise, scale, keep_float)
            for s in range(S)]
    if workers > 1 and S > 1:
        import multiprocessing as mp
        # close() + join() rather than the context manager, whose exit
        # terminates the workers with SIGTERM (a profiler's signal handler in
        # them reports that as an abort)
        pool = mp.get_context("fork").Pool(min(workers, S))
        try:
            for s, r in enumerate(pool.imap(_slot_job, jobs, chunksize=1)):
                iq[s], bits[s], X[s], H[s], snr[s], scl[s], y = r
                if keep_float:
                    yk[s] = y
            pool.close()
        except BaseException:
            pool.terminate()
            raise
        finally:
            pool.join()
    else:
        for s, job in enumerate(jobs):
            iq[s], bits[s], X[s], H[s], snr[s], scl[s], y = _slot_job(job)
            if keep_float:
                yk[s] = y
    return Frames(cfg, iq, pilot, bits, X, H, snr, scl, yk)


# ---------------------------------------------------------------------------
# Batches of frames with mixed shapes: one slot per frame; antennas from
# {16, 32, 64, 128}, FFT length from {128, ..., 2048} with CP = round(N/14)
# and the used-subcarrier count of that length, QPSK/16-QAM/64-QAM, sample
# rate 15 kHz x N, 1 pilot + 13 data symbols.
USED_BY_FFT = {64: 52, 128: 72, 256: 180, 512: 300, 1024: 600, 2048: 1200}


def batch_frame_config(seed: int, index: int, antennas=(16, 32, 64, 128),
                       fft_lens=(128, 256, 512, 1024, 2048), bits=(2, 4, 6)) -> FrameConfig:
    """Shape of frame ``index`` of a mixed batch, drawn from its own seed stream."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, index, 7])))
    N = int(rng.choice(fft_lens))
    return FrameConfig(f"batch{seed}_f{index}", n_ant=int(rng.choice(antennas)), fft_len=N,
                       cp_len=int(round(N / 14)), n_sym=14, n_used=USED_BY_FFT[N],
                       bits_per_sym=int(rng.choice(bits)), n_slots=1, n_taps=10, tau_max_us=(0.5, 3.0),
                       fs_hz=15e3 * N, snr_db=(5.0, 30.0), seed=seed * 1000 + index)


def _batch_job(job):
    cfg = job
    return make_frames(cfg, n_slots=1)


@dataclasses.dataclass
class Batch:
    """A packed batch: frames[i] is the Frames of frame i (one slot), iq the
    concatenation of their int16 samples in batch order."""
    frames: list
    iq: np.ndarray  # int16, flat

    @property
    def configs(self):
        return [f.cfg for f in self.frames]


def make_batch(n_frames: int, seed: int, workers: int = 1, **shape_choices) -> Batch:
    cfgs = [batch_frame_config(seed, i, **shape_choices) for i in range(n_frames)]
    if workers > 1 and n_frames > 1:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(min(workers, n_frames))
        try:
            frames = list(pool.imap(_batch_job, cfgs, chunksize=1))
            pool.close()
        except BaseException:
            pool.terminate()
            raise
        finally:
            pool.join()
    else:
        frames = [_batch_job(c) for c in cfgs]
    iq = np.concatenate([f.iq.reshape(-1) for f in frames])
    return Batch(frames, iq)


# ---------------------------------------------------------------------------
# Initial weights of the learned channel-estimate denoiser (random numbers
# only; the network itself is defined by the receiver).  Layers 2->32->32->32->2
# channels, 7 taps; per layer the weights W[co][ci][k] then the biases b[co].
DENOISER_LAYERS = ((2, 32), (32, 32), (32, 32), (32, 2))
DENOISER_TAPS = 7


def denoiser_param_count() -> int:
    return sum(co * ci * DENOISER_TAPS + co for ci, co in DENOISER_LAYERS)


def init_denoiser_params(seed: int, last_scale: float = 0.1) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases; the last
    layer's weights are scaled by ``last_scale`` so an untrained network is
    close to the identity on its residual path.  float32 [P]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1901])))
    out = []
    for li, (ci, co) in enumerate(DENOISER_LAYERS):
        bound = math.sqrt(6.0 / (ci * DENOISER_TAPS))
        w = rng.uniform(-bound, bound, size=(co, ci, DENOISER_TAPS))
        if li == len(DENOISER_LAYERS) - 1:
            w *= last_scale
        out += [w.reshape(-1), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)
# Raw per-antenna streams with a PN preamble (frame synchronisation inputs).
def pn_sequence(taps=(8, 6, 5, 4), length: int = 255, seed_state: int = 1) -> np.ndarray:
    """Maximum-length sequence of a Fibonacci LFSR, chips mapped 0 -> +1, 1 -> -1.

    Default feedback polynomial x^8 + x^6 + x^5 + x^4 + 1 (primitive), period 255.
    """
    n = max(taps)
    state = [(seed_state >> i) & 1 for i in range(n)]  # state[0] is the output stage
    out = np.empty(length, dtype=np.float64)
    for i in range(length):
        bit = state[0]
        out[i] = 1.0 - 2.0 * bit
        fb = 0
        for t in taps:
            fb ^= state[n - t]
        state = state[1:] + [fb]
    return out


@dataclasses.dataclass
class Stream:
    """Received streams of every antenna: `raw` int16 [A][n_samples][2] holding
    `lead` samples of noise, the PN preamble, then `frames.iq`'s slots back to
    back.  `frames.iq` is exactly what cutting the aligned slots out of `raw`
    must give."""
    raw: np.ndarray
    pn: np.ndarray     # complex128 [L], the preamble chips
    lead: int          # samples before the preamble
    frames: Frames
    delays: np.ndarray  # channel tap delays (samples)


def make_stream(cfg: FrameConfig, n_slots: int, lead: int, seed: int, tail: int = 64,
                pn: Optional[np.ndarray] = None, snr_db: float = 10.0, channel: str = "rayleigh") -> Stream:
    """One transmission: `lead` noise samples, the PN preamble (BPSK chips at the
    OFDM signal's RMS), then `n_slots` OFDM slots, through one channel per
    antenna constant over the stream ("rayleigh": the config's tapped-delay
    profile; "flat": one Rayleigh tap at delay 0), AWGN with the per-subcarrier
    SNR `snr_db` (as in make_frames), and one int16 gain for the whole stream."""
    pn = pn_sequence() if pn is None else np.asarray(pn, dtype=np.complex128)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    N, CP, T, A, U, b = cfg.fft_len, cfg.cp_len, cfg.n_sym, cfg.n_ant, cfg.n_used, cfg.bits_per_sym
    bins = used_subcarrier_bins(N, U)
    pilot = (1 - 2 * rng.integers(0, 2, size=U)).astype(np.complex128)
    sym = []
    bits_all, X_all = [], []
    for _ in range(n_slots):
        bits = rng.integers(0, 2, size=(T - 1, U, b), dtype=np.uint8)
        X = qam_symbols(bits, b)
        grid = np.zeros((T, N), dtype=np.complex128)
        grid[0, bins] = pilot
        grid[1:, bins] = X
        x = np.fft.ifft(grid, axis=1) * math.sqrt(N)
        sym.append(np.concatenate([x[:, N - CP:], x], axis=1).reshape(-1))
        bits_all.append(bits)
        X_all.append(X)
    ofdm = np.concatenate(sym)
    rms = math.sqrt(U / N)
    x = np.concatenate([np.zeros(lead), pn * rms, ofdm, np.zeros(tail)])
    if channel == "rayleigh":
        delays, p = tap_delays_powers(cfg, rng.uniform(*cfg.tau_max_us) * 1e-6)
    elif channel == "flat":
        delays, p = np.zeros(1, dtype=np.int64), np.ones(1)
    else:
        raise ValueError(channel)
    h = (rng.standard_normal((A, len(p))) + 1j * rng.standard_normal((A, len(p)))) * np.sqrt(p / 2.0)
    y = np.zeros((A, x.size), dtype=np.complex128)
    for l, dl in enumerate(delays):
        y[:, dl:] += h[:, l:l + 1] * x[None, :x.size - dl]
    sigma2 = 10.0 ** (-snr_db / 10.0)
    y += (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)) * math.sqrt(sigma2 / 2.0)
    peak = max(np.abs(y.real).max(), np.abs(y.imag).max())
    scale = 0.5 * INT16_FS / peak
    q = np.rint(y * scale)
    raw = np.empty((A, x.size, 2), dtype=np.int16)
    raw[..., 0] = np.clip(q.real, -32768, 32767)
    raw[..., 1] = np.clip(q.imag, -32768, 32767)
    start = lead + len(pn)
    sl = raw[:, start:start + n_slots * T * (N + CP)].reshape(A, n_slots, T, N + CP, 2)
    iq = np.ascontiguousarray(sl.transpose(1, 2, 0, 3, 4))
    ph = np.exp(-2j * np.pi * np.outer(bins, delays) / N)
    H = np.broadcast_to((h @ ph.T) * (math.sqrt(N) * scale), (n_slots, A, U)).copy()
    fr = Frames(cfg.replace(n_slots=n_slots), iq, pilot, np.stack(bits_all), np.stack(X_all), H,
                np.full(n_slots, snr_db), np.full(n_slots, scale))
    return Stream(raw, pn.astype(np.complex128), lead, fr, delays)
