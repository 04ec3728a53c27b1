"""Seeded synthetic input generator shared by the oracle tests, the GPU tests and the benchmark.

Holds the transmit side and the channel only (see ``rxgen.frames``); none of
the receiver's arithmetic lives here.
"""
from .frames import (C1, C2, C2_20DB, C4, C5, C5_20DB, CONFIGS, DENOISER_LAYERS,
                     SWEEP_ANTENNAS, SWEEP_FFT_LENS, sweep_config, DENOISER_TAPS,
                     USED_BY_FFT, Batch, FrameConfig, Frames, Stream, batch_frame_config, denoiser_param_count,
                     init_denoiser_params, make_batch, make_frames, make_stream, pn_sequence, qam_symbols,
                     tap_delays_powers, used_subcarrier_bins)

__all__ = ["C1", "C2", "C2_20DB", "C4", "C5", "C5_20DB", "CONFIGS", "DENOISER_LAYERS", "DENOISER_TAPS",
           "SWEEP_ANTENNAS", "SWEEP_FFT_LENS", "sweep_config",
           "USED_BY_FFT", "Batch", "FrameConfig", "Frames", "Stream", "batch_frame_config", "denoiser_param_count",
           "init_denoiser_params", "make_batch", "make_frames", "make_stream", "pn_sequence", "qam_symbols",
           "tap_delays_powers", "used_subcarrier_bins"]
