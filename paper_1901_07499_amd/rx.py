"""Thin Python binding of ``librx.so`` (the C ABI in ``include/rx.h``).

Argument marshalling only: every step of the receive path runs in the HIP
kernels behind the C calls.  PyTorch provides device memory and the stream.
The module-level functions carry the C names and take raw integer pointers;
``Plan`` wraps them for torch tensors.  If ``librx.so`` has not been built the
import fails with an explicit error -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librx.so")

RX_OK, RX_E_INVALID_ARG, RX_E_UNSUPPORTED, RX_E_HIP, RX_E_NOMEM, RX_E_SCRATCH = 0, -1, -2, -3, -4, -5
RX_NOALLOC_SCRATCH_BYTES = 64 << 20
RX_COMB_MRC, RX_COMB_ZF = 0, 1
RX_FFT_RADIX_F32, RX_FFT_MFMA_F16, RX_FFT_MFMA_BF16, RX_FFT_MFMA_F16_SPLIT, RX_FFT_MFMA_BF16_SPLIT = 0, 1, 2, 3, 4
FFT_MODES = {"f32": 0, "f16": 1, "bf16": 2, "f16_split": 3, "bf16_split": 4}

# Every symbol the header declares; the CPU test checks they are all exported.
EXPORTS = ("rx_params_check", "rx_plan_create", "rx_plan_destroy", "rx_workspace_bytes", "rx_estimate",
           "rx_demod", "rx_process_frame", "rx_process_frame_noalloc", "rx_debug_fft", "rx_status_string",
           "rx_batch_create", "rx_batch_destroy", "rx_batch_layout", "rx_batch_workspace_bytes",
           "rx_batch_process", "rx_batch_autotune", "rx_batch_config", "rx_batch_schedules", "rx_batch_set_config",
           "rx_fft_radices", "rx_batch_frame_latency",
           "rx_dn_create", "rx_dn_destroy", "rx_dn_load", "rx_dn_apply", "rx_dn_apply_judged", "rx_dn_set_fallback",
           "rx_dn_workspace_bytes", "rx_dn_grad",
           "rx_dn_train_step", "rx_dn_generate", "rx_sync_workspace_bytes", "rx_sync_find", "rx_sync_extract")
RX_DN_PARAMS = 15330


class rx_chan_gen(ctypes.Structure):
    _fields_ = [("fft_len", ctypes.c_int32), ("n_used", ctypes.c_int32), ("cp_len", ctypes.c_int32),
                ("pilot_spacing", ctypes.c_int32), ("taps_min", ctypes.c_int32), ("taps_max", ctypes.c_int32),
                ("tau_min", ctypes.c_int32), ("tau_max", ctypes.c_int32), ("snr_min_db", ctypes.c_float),
                ("snr_max_db", ctypes.c_float), ("tap_decay_db", ctypes.c_float)]


class RxError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {rx_status_string(status)} ({status})")
        self.status = status


class rx_params(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("fft_len", ctypes.c_int32), ("cp_len", ctypes.c_int32),
                ("n_used", ctypes.c_int32), ("n_sym", ctypes.c_int32), ("bits_per_sym", ctypes.c_int32),
                ("combiner", ctypes.c_int32), ("n_users", ctypes.c_int32),
                ("pilot", ctypes.POINTER(ctypes.c_float)), ("pilot_spacing", ctypes.c_int32),
                ("fft_mode", ctypes.c_int32)]


def _load() -> ctypes.CDLL:
    # torch bundles its own HIP runtime under the same SONAME as the system
    # one; loading torch first makes librx.so bind to that single runtime, so
    # device pointers and streams handed over by torch are valid in our calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1901_07499_amd.build` "
                          "(the receive path has no non-HIP implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.rx_params_check.argtypes = [ctypes.POINTER(rx_params)]
    lib.rx_plan_create.argtypes = [ctypes.POINTER(rx_params), ctypes.POINTER(vp)]
    lib.rx_plan_destroy.argtypes = [vp]
    lib.rx_workspace_bytes.argtypes = [vp, i64]
    lib.rx_workspace_bytes.restype = sz
    lib.rx_estimate.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.rx_demod.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    lib.rx_process_frame.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.rx_process_frame_noalloc.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.rx_debug_fft.argtypes = [vp, vp, i64, vp, vp]
    lib.rx_status_string.argtypes = [ctypes.c_int]
    lib.rx_status_string.restype = ctypes.c_char_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.rx_batch_create.argtypes = [ctypes.POINTER(rx_params), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.rx_batch_destroy.argtypes = [vp]
    lib.rx_batch_layout.argtypes = [vp, i64p, i64p, i64p, i64p]
    lib.rx_batch_workspace_bytes.argtypes = [vp]
    lib.rx_batch_workspace_bytes.restype = sz
    lib.rx_batch_process.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.rx_batch_autotune.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp]
    lib.rx_batch_config.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.rx_batch_schedules.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.rx_batch_set_config.argtypes = [vp] + [ctypes.c_int32] * 5
    lib.rx_fft_radices.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.rx_batch_frame_latency.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    f32 = ctypes.c_float
    lib.rx_dn_create.argtypes = [ctypes.c_int32, ctypes.POINTER(vp)]
    lib.rx_dn_destroy.argtypes = [vp]
    lib.rx_dn_load.argtypes = [vp, vp, vp]
    lib.rx_dn_apply.argtypes = [vp, vp, i64, vp, vp]
    lib.rx_dn_apply_judged.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.rx_dn_set_fallback.argtypes = [vp, f32]
    lib.rx_dn_workspace_bytes.argtypes = [vp, i64]
    lib.rx_dn_workspace_bytes.restype = sz
    lib.rx_dn_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    lib.rx_dn_train_step.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, vp, vp, i64, vp, vp, vp]
    lib.rx_dn_generate.argtypes = [ctypes.POINTER(rx_chan_gen), ctypes.c_uint64, i64, i64, vp, vp, vp]
    lib.rx_sync_workspace_bytes.argtypes = [ctypes.c_int32, i64]
    lib.rx_sync_workspace_bytes.restype = sz
    lib.rx_sync_find.argtypes = [vp, ctypes.c_int32, i64, i64, ctypes.POINTER(ctypes.c_int8), ctypes.c_int32, i64,
                                 vp, vp, vp, vp, vp]
    lib.rx_sync_extract.argtypes = [vp, ctypes.c_int32, i64, i64, vp, i64, ctypes.c_int32, ctypes.c_int32, i64, vp,
                                    vp]
    for name in EXPORTS:
        if name not in ("rx_workspace_bytes", "rx_status_string", "rx_batch_workspace_bytes",
                        "rx_dn_workspace_bytes", "rx_sync_workspace_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


# ---------------------------------------------------------------- C names, raw pointers
def rx_params_check(p: rx_params) -> int:
    return _lib.rx_params_check(ctypes.byref(p))


def rx_plan_create(p: rx_params) -> Tuple[int, Optional[int]]:
    out = ctypes.c_void_p()
    st = _lib.rx_plan_create(ctypes.byref(p), ctypes.byref(out))
    return st, (out.value if st == RX_OK else None)


def rx_plan_destroy(plan: Optional[int]) -> int:
    return _lib.rx_plan_destroy(plan)


def rx_workspace_bytes(plan: Optional[int], n_slots: int) -> int:
    return _lib.rx_workspace_bytes(plan, n_slots)


def rx_estimate(plan, iq, n_slots, H, g, workspace, stream) -> int:
    return _lib.rx_estimate(plan, iq, n_slots, H, g, workspace, stream)


def rx_demod(plan, iq, H, n_slots, xhat, bits, workspace, stream) -> int:
    return _lib.rx_demod(plan, iq, H, n_slots, xhat, bits, workspace, stream)


def rx_process_frame(plan, iq, n_slots, H, xhat, bits, workspace, stream) -> int:
    return _lib.rx_process_frame(plan, iq, n_slots, H, xhat, bits, workspace, stream)


def rx_process_frame_noalloc(plan, iq, n_slots, xhat, bits, stream) -> int:
    return _lib.rx_process_frame_noalloc(plan, iq, n_slots, xhat, bits, stream)


def rx_debug_fft(plan, iq, n_slots, Y, stream) -> int:
    return _lib.rx_debug_fft(plan, iq, n_slots, Y, stream)


def rx_status_string(status: int) -> str:
    return _lib.rx_status_string(status).decode()


def rx_batch_create(params_array, n_frames: int) -> Tuple[int, Optional[int]]:
    out = ctypes.c_void_p()
    st = _lib.rx_batch_create(params_array, n_frames, ctypes.byref(out))
    return st, (out.value if st == RX_OK else None)


def rx_batch_destroy(batch) -> int:
    return _lib.rx_batch_destroy(batch)


def rx_batch_layout(batch, iq_off, h_off, x_off, b_off) -> int:
    return _lib.rx_batch_layout(batch, iq_off, h_off, x_off, b_off)


def rx_batch_workspace_bytes(batch) -> int:
    return _lib.rx_batch_workspace_bytes(batch)


def rx_batch_process(batch, iq, H, xhat, bits, workspace, stream) -> int:
    return _lib.rx_batch_process(batch, iq, H, xhat, bits, workspace, stream)


def rx_batch_autotune(batch, iq, H, xhat, bits, workspace, reps, stream) -> int:
    return _lib.rx_batch_autotune(batch, iq, H, xhat, bits, workspace, reps, stream)


def rx_batch_config(batch, fft_len, demod_waves, est_jobs) -> int:
    return _lib.rx_batch_config(batch, fft_len, demod_waves, est_jobs)


def rx_batch_schedules(batch, fft_len, dem_sched, est_sched) -> int:
    return _lib.rx_batch_schedules(batch, fft_len, dem_sched, est_sched)


def rx_batch_set_config(batch, fft_len, demod_waves, est_jobs, dem_sched, est_sched) -> int:
    return _lib.rx_batch_set_config(batch, fft_len, demod_waves, est_jobs, dem_sched, est_sched)


def rx_fft_radices(fft_len, sched, radices) -> int:
    return _lib.rx_fft_radices(fft_len, sched, radices)


def fft_radices(fft_len: int, sched: int) -> Optional[Tuple[int, ...]]:
    """Radices of schedule ``sched`` of the fft_len-point transform, first pass first; None if there is none."""
    r = (ctypes.c_int32 * 3)()
    if rx_fft_radices(fft_len, sched, r) != RX_OK:
        return None
    return tuple(v for v in r[:] if v)


def rx_batch_frame_latency(batch, ms, stream) -> int:
    return _lib.rx_batch_frame_latency(batch, ms, stream)


def rx_dn_create(n_used: int) -> Tuple[int, Optional[int]]:
    out = ctypes.c_void_p()
    st = _lib.rx_dn_create(n_used, ctypes.byref(out))
    return st, (out.value if st == RX_OK else None)


def rx_dn_destroy(dn) -> int:
    return _lib.rx_dn_destroy(dn)


def rx_dn_load(dn, params, stream) -> int:
    return _lib.rx_dn_load(dn, params, stream)


def rx_dn_apply(dn, H_in, rows, H_out, stream) -> int:
    return _lib.rx_dn_apply(dn, H_in, rows, H_out, stream)


def rx_dn_apply_judged(dn, H_in, rows, H_out, fell, stream) -> int:
    return _lib.rx_dn_apply_judged(dn, H_in, rows, H_out, fell, stream)


def rx_dn_set_fallback(dn, max_corr) -> int:
    return _lib.rx_dn_set_fallback(dn, max_corr)


def rx_dn_workspace_bytes(dn, rows) -> int:
    return _lib.rx_dn_workspace_bytes(dn, rows)


def rx_dn_grad(dn, H_in, H_true, rows, grad, loss, workspace, stream) -> int:
    return _lib.rx_dn_grad(dn, H_in, H_true, rows, grad, loss, workspace, stream)


def rx_dn_train_step(dn, params, m, v, step, lr, beta1, beta2, eps, H_in, H_true, rows, loss, workspace,
                     stream) -> int:
    return _lib.rx_dn_train_step(dn, params, m, v, step, lr, beta1, beta2, eps, H_in, H_true, rows, loss,
                                 workspace, stream)


def rx_dn_generate(gen: rx_chan_gen, seed: int, first_row: int, rows: int, H_true, H_ls, stream) -> int:
    return _lib.rx_dn_generate(ctypes.byref(gen), seed, first_row, rows, H_true, H_ls, stream)


def rx_sync_workspace_bytes(n_ant: int, n_search: int) -> int:
    return _lib.rx_sync_workspace_bytes(n_ant, n_search)


def rx_sync_find(raw, n_ant, n_samples, stride, pn, pn_len, n_search, metric, offset, peak, workspace,
                 stream) -> int:
    return _lib.rx_sync_find(raw, n_ant, n_samples, stride, pn, pn_len, n_search, metric, offset, peak, workspace,
                             stream)


def rx_sync_extract(raw, n_ant, n_samples, stride, start, start_add, sym_len, n_sym, n_slots, iq, stream) -> int:
    return _lib.rx_sync_extract(raw, n_ant, n_samples, stride, start, start_add, sym_len, n_sym, n_slots, iq,
                                stream)


def make_params(n_ant: int, fft_len: int, cp_len: int, n_used: int, n_sym: int, bits_per_sym: int,
                pilot: Sequence[complex], combiner: int = RX_COMB_MRC, n_users: int = 1, pilot_spacing: int = 1,
                fft_mode: int = RX_FFT_RADIX_F32):
    """Build an ``rx_params`` plus the float buffer its pilot pointer refers to (keep both alive)."""
    pil = np.ascontiguousarray(np.asarray(pilot, dtype=np.complex64)).view(np.float32)
    p = rx_params(n_ant, fft_len, cp_len, n_used, n_sym, bits_per_sym, combiner, n_users,
                  pil.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), pilot_spacing, fft_mode)
    return p, pil


# ---------------------------------------------------------------- torch-level wrapper
def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Plan:
    """A receive plan on the current CUDA (HIP) device.

    ``iq`` tensors are int16 [S][T][A][CP+N][2] on that device.  Outputs are
    float32 tensors with a trailing (re, im) axis and uint8 packed bits, laid
    out as in ``include/rx.h``.  Calls are queued on torch's current stream.
    """

    def __init__(self, n_ant: int, fft_len: int, cp_len: int, n_used: int, n_sym: int, bits_per_sym: int,
                 pilot: Sequence[complex], combiner: int = RX_COMB_MRC, n_users: int = 1,
                 pilot_spacing: int = 1, fft_mode: int = RX_FFT_RADIX_F32):
        self.n_ant, self.fft_len, self.cp_len, self.n_used = n_ant, fft_len, cp_len, n_used
        self.n_sym, self.bits_per_sym, self.combiner = n_sym, bits_per_sym, combiner
        self.pilot_spacing, self.fft_mode = pilot_spacing, fft_mode
        self._params, self._pilot = make_params(n_ant, fft_len, cp_len, n_used, n_sym, bits_per_sym, pilot,
                                                combiner, n_users, pilot_spacing, fft_mode)
        st, self._plan = rx_plan_create(self._params)
        if st != RX_OK:
            raise RxError(st, "rx_plan_create")

    @classmethod
    def from_config(cls, cfg, pilot, combiner: int = RX_COMB_MRC, fft_mode: int = RX_FFT_RADIX_F32) -> "Plan":
        return cls(cfg.n_ant, cfg.fft_len, cfg.cp_len, cfg.n_used, cfg.n_sym, cfg.bits_per_sym, pilot, combiner,
                   pilot_spacing=getattr(cfg, "pilot_spacing", 1), fft_mode=fft_mode)

    def close(self):
        if getattr(self, "_plan", None):
            rx_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    def _slots(self, iq) -> int:
        import torch
        want = (self.n_sym, self.n_ant, self.fft_len + self.cp_len, 2)
        if iq.dtype != torch.int16 or tuple(iq.shape[1:]) != want or not iq.is_contiguous() or not iq.is_cuda:
            raise ValueError(f"iq must be a contiguous int16 CUDA tensor of shape [S, {', '.join(map(str, want))}]")
        return iq.shape[0]

    def _empty(self, shape, dtype, like):
        import torch
        return torch.empty(shape, dtype=dtype, device=like.device)

    def _stream(self) -> int:
        import torch
        return torch.cuda.current_stream().cuda_stream

    @property
    def row_bytes(self) -> int:
        return self.n_used * self.bits_per_sym // 8

    def workspace_bytes(self, n_slots: int) -> int:
        return rx_workspace_bytes(self._plan, n_slots)

    def estimate(self, iq, H=None, with_g: bool = False):
        import torch
        S = self._slots(iq)
        H = self._empty((S, self.n_ant, self.n_used, 2), torch.float32, iq) if H is None else H
        g = self._empty((S, self.n_used), torch.float32, iq) if with_g else None
        st = rx_estimate(self._plan, iq.data_ptr(), S, H.data_ptr(), _ptr(g), None, self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_estimate")
        return (H, g) if with_g else H

    def demod(self, iq, H, want_xhat: bool = True, want_bits: bool = True):
        import torch
        S = self._slots(iq)
        Td = self.n_sym - 1
        xhat = self._empty((S, Td, self.n_used, 2), torch.float32, iq) if want_xhat else None
        bits = self._empty((S, Td, self.row_bytes), torch.uint8, iq) if want_bits else None
        st = rx_demod(self._plan, iq.data_ptr(), H.data_ptr(), S, _ptr(xhat), _ptr(bits), None, self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_demod")
        return xhat, bits

    def process(self, iq, want_H: bool = False, want_xhat: bool = True, want_bits: bool = True, out=None,
                workspace=None):
        """Whole path.  ``out`` = (H or None, xhat or None, bits or None) preallocated buffers."""
        import torch
        S = self._slots(iq)
        Td = self.n_sym - 1
        if out is not None:
            H, xhat, bits = out
        else:
            H = self._empty((S, self.n_ant, self.n_used, 2), torch.float32, iq) if want_H else None
            xhat = self._empty((S, Td, self.n_used, 2), torch.float32, iq) if want_xhat else None
            bits = self._empty((S, Td, self.row_bytes), torch.uint8, iq) if want_bits else None
        ws = None
        if H is None:
            ws = workspace if workspace is not None else self._empty((max(1, self.workspace_bytes(S)),),
                                                                     torch.uint8, iq)
        st = rx_process_frame(self._plan, iq.data_ptr(), S, _ptr(H), _ptr(xhat), _ptr(bits), _ptr(ws),
                              self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_process_frame")
        return H, xhat, bits

    def debug_fft(self, iq):
        import torch
        S = self._slots(iq)
        Y = self._empty((S, self.n_sym, self.n_ant, self.fft_len, 2), torch.float32, iq)
        st = rx_debug_fft(self._plan, iq.data_ptr(), S, Y.data_ptr(), self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_debug_fft")
        return Y


class Batch:
    """A batch of frames with mixed shapes (one slot each), processed by one graph launch.

    ``frames``: sequence of (n_ant, fft_len, cp_len, n_used, n_sym, bits_per_sym, pilot)
    tuples or objects with those attributes plus a pilot passed separately via
    ``pilots``.  Buffers are flat and packed in batch order; ``layout`` gives the offsets.
    """

    def __init__(self, configs, pilots):
        self.n = len(configs)
        arr = (rx_params * self.n)()
        self._keep = []
        for i, (c, pil) in enumerate(zip(configs, pilots)):
            p, buf = make_params(c.n_ant, c.fft_len, c.cp_len, c.n_used, c.n_sym, c.bits_per_sym, pil)
            arr[i] = p
            self._keep.append(buf)
        st, self._b = rx_batch_create(arr, self.n)
        if st != RX_OK:
            raise RxError(st, "rx_batch_create")
        offs = [(ctypes.c_int64 * (self.n + 1))() for _ in range(4)]
        st = rx_batch_layout(self._b, *offs)
        if st != RX_OK:
            raise RxError(st, "rx_batch_layout")
        self.iq_off, self.h_off, self.x_off, self.b_off = (np.array(o[:], dtype=np.int64) for o in offs)

    def close(self):
        if getattr(self, "_b", None):
            rx_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self, device, want_H=True):
        import torch
        H = torch.empty((int(self.h_off[-1]), 2), dtype=torch.float32, device=device) if want_H else None
        x = torch.empty((int(self.x_off[-1]), 2), dtype=torch.float32, device=device)
        b = torch.empty((int(self.b_off[-1]),), dtype=torch.uint8, device=device)
        ws = None if want_H else torch.empty((max(1, rx_batch_workspace_bytes(self._b)),), dtype=torch.uint8,
                                             device=device)
        return H, x, b, ws

    def _check(self, iq):
        import torch
        if iq.dtype != torch.int16 or iq.numel() != int(self.iq_off[-1]) or not iq.is_contiguous() or not iq.is_cuda:
            raise ValueError(f"iq must be a contiguous int16 CUDA tensor of {int(self.iq_off[-1])} elements")

    def process(self, iq, out):
        import torch
        self._check(iq)
        H, x, b, ws = out
        st = rx_batch_process(self._b, iq.data_ptr(), _ptr(H), _ptr(x), _ptr(b), _ptr(ws),
                              torch.cuda.current_stream().cuda_stream)
        if st != RX_OK:
            raise RxError(st, "rx_batch_process")

    def autotune(self, iq, out, reps: int = 3):
        import torch
        self._check(iq)
        H, x, b, ws = out
        st = rx_batch_autotune(self._b, iq.data_ptr(), _ptr(H), _ptr(x), _ptr(b), _ptr(ws), reps,
                               torch.cuda.current_stream().cuda_stream)
        if st != RX_OK:
            raise RxError(st, "rx_batch_autotune")

    def config(self, fft_len: int):
        w, j = ctypes.c_int32(), ctypes.c_int32()
        st = rx_batch_config(self._b, fft_len, ctypes.byref(w), ctypes.byref(j))
        if st != RX_OK:
            raise RxError(st, "rx_batch_config")
        return w.value, j.value

    def schedules(self, fft_len: int):
        """(demod, estimate) radix schedule indices of the class of length fft_len."""
        d, e = ctypes.c_int32(), ctypes.c_int32()
        st = rx_batch_schedules(self._b, fft_len, ctypes.byref(d), ctypes.byref(e))
        if st != RX_OK:
            raise RxError(st, "rx_batch_schedules")
        return d.value, e.value

    def set_config(self, fft_len: int, demod_waves: int, est_jobs: int, dem_sched: int = 0, est_sched: int = 0):
        st = rx_batch_set_config(self._b, fft_len, demod_waves, est_jobs, dem_sched, est_sched)
        if st != RX_OK:
            raise RxError(st, "rx_batch_set_config")

    def frame_latency_ms(self):
        import torch
        ms = (ctypes.c_double * self.n)()
        st = rx_batch_frame_latency(self._b, ms, torch.cuda.current_stream().cuda_stream)
        if st != RX_OK:
            raise RxError(st, "rx_batch_frame_latency")
        return np.array(ms[:])


# ---------------------------------------------------------------- learned estimate refinement
def chan_gen(fft_len=2048, n_used=1200, cp_len=144, pilot_spacing=4, taps=(8, 24), tau_samples=(15, 154),
             snr_db=(0.0, 30.0), tap_decay_db=3.0) -> rx_chan_gen:
    """Training-channel recipe (see ``rx_dn_generate`` in include/rx.h)."""
    return rx_chan_gen(fft_len, n_used, cp_len, pilot_spacing, taps[0], taps[1], tau_samples[0], tau_samples[1],
                       snr_db[0], snr_db[1], tap_decay_db)


def generate(gen: rx_chan_gen, seed: int, first_row: int, rows: int, device, want_true=True, want_ls=True):
    """(H_true, H_ls) float32 [rows][U][2] tensors on ``device`` (either may be None)."""
    import torch
    ht = torch.empty((rows, gen.n_used, 2), dtype=torch.float32, device=device) if want_true else None
    hl = torch.empty((rows, gen.n_used, 2), dtype=torch.float32, device=device) if want_ls else None
    st = rx_dn_generate(gen, seed, first_row, rows, _ptr(ht), _ptr(hl), torch.cuda.current_stream().cuda_stream)
    if st != RX_OK:
        raise RxError(st, "rx_dn_generate")
    return ht, hl


class Denoiser:
    """The learned refinement of comb-pilot LS estimates for rows of ``n_used``
    subcarriers (float32 [rows][U][2] CUDA tensors), on torch's current stream."""

    def __init__(self, n_used: int):
        self.n_used = n_used
        st, self._dn = rx_dn_create(n_used)
        if st != RX_OK:
            raise RxError(st, "rx_dn_create")
        self._ws = None

    def close(self):
        if getattr(self, "_dn", None):
            rx_dn_destroy(self._dn)
            self._dn = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def load(self, params):
        self._check(params, (RX_DN_PARAMS,))
        st = rx_dn_load(self._dn, params.data_ptr(), self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_dn_load")

    def _check(self, t, shape):
        import torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a contiguous float32 CUDA tensor of shape {shape}")

    def apply(self, H, out=None, flags: bool = False):
        """Refined rows (LS kept where the refinement is not trusted); with
        ``flags`` also a uint8 tensor [rows], 1 where a row kept LS."""
        import torch
        rows = H.shape[0]
        self._check(H, (rows, self.n_used, 2))
        out = torch.empty_like(H) if out is None else out
        fell = torch.empty((max(rows, 1),), dtype=torch.uint8, device=H.device) if flags else None
        st = rx_dn_apply_judged(self._dn, H.data_ptr(), rows, out.data_ptr(),
                                None if fell is None else fell.data_ptr(), self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_dn_apply_judged")
        return (out, fell[:rows]) if flags else out

    def set_fallback(self, max_corr: float):
        st = rx_dn_set_fallback(self._dn, max_corr)
        if st != RX_OK:
            raise RxError(st, "rx_dn_set_fallback")

    def workspace(self, rows: int):
        import torch
        need = rx_dn_workspace_bytes(self._dn, rows)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty((need,), dtype=torch.uint8, device="cuda")
        return self._ws

    def grad(self, H, H_true):
        import torch
        rows = H.shape[0]
        self._check(H, (rows, self.n_used, 2))
        self._check(H_true, (rows, self.n_used, 2))
        g = torch.empty((RX_DN_PARAMS,), dtype=torch.float32, device=H.device)
        loss = torch.empty((1,), dtype=torch.float32, device=H.device)
        ws = self.workspace(rows)
        st = rx_dn_grad(self._dn, H.data_ptr(), H_true.data_ptr(), rows, g.data_ptr(), loss.data_ptr(),
                        ws.data_ptr(), self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_dn_grad")
        return loss, g

    def train_step(self, params, m, v, step: int, H, H_true, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   loss=None):
        rows = H.shape[0]
        for t in (params, m, v):
            self._check(t, (RX_DN_PARAMS,))
        self._check(H, (rows, self.n_used, 2))
        self._check(H_true, (rows, self.n_used, 2))
        ws = self.workspace(rows)
        st = rx_dn_train_step(self._dn, params.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, beta1, beta2, eps,
                              H.data_ptr(), H_true.data_ptr(), rows, _ptr(loss), ws.data_ptr(), self._stream())
        if st != RX_OK:
            raise RxError(st, "rx_dn_train_step")


# ---------------------------------------------------------------- frame synchronisation
def _chips(pn):
    c = np.ascontiguousarray(np.rint(np.asarray(pn).real), dtype=np.int8)
    return c, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def sync_find(raw, pn, n_search: int, n_samples: Optional[int] = None, want_metric: bool = False):
    """PN correlation over int16 CUDA streams ``raw`` [A][stride][2]: returns
    (offset [1], peak [1], metric [n_search] or None) as int64 CUDA tensors;
    peak and metric hold the library's uint64 values bit for bit."""
    import torch
    if raw.dtype != torch.int16 or raw.dim() != 3 or raw.shape[2] != 2 or not raw.is_contiguous() or not raw.is_cuda:
        raise ValueError("raw must be a contiguous int16 CUDA tensor [A][stride][2]")
    A, stride = raw.shape[0], raw.shape[1]
    ns = stride if n_samples is None else int(n_samples)
    chips, cp = _chips(pn)
    dev = raw.device
    off = torch.empty((1,), dtype=torch.int64, device=dev)
    # uint64 values held in int64 tensors (view them as uint64 on the host)
    peak = torch.empty((1,), dtype=torch.int64, device=dev)
    M = torch.empty((n_search,), dtype=torch.int64, device=dev) if want_metric else None
    ws = torch.empty((max(256, rx_sync_workspace_bytes(A, n_search)),), dtype=torch.uint8, device=dev)
    st = rx_sync_find(raw.data_ptr(), A, ns, stride, cp, chips.size, n_search, _ptr(M), off.data_ptr(),
                      peak.data_ptr(), ws.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if st != RX_OK:
        raise RxError(st, "rx_sync_find")
    return off, peak, M


def sync_extract(raw, start, start_add: int, sym_len: int, n_sym: int, n_slots: int,
                 n_samples: Optional[int] = None, out=None):
    """Slots cut from the streams at (*start + start_add): int16 CUDA tensor
    [n_slots][n_sym][A][sym_len][2] (``start``: int64 CUDA tensor [1] or None)."""
    import torch
    A, stride = raw.shape[0], raw.shape[1]
    ns = stride if n_samples is None else int(n_samples)
    if out is None:
        out = torch.empty((n_slots, n_sym, A, sym_len, 2), dtype=torch.int16, device=raw.device)
    st = rx_sync_extract(raw.data_ptr(), A, ns, stride, _ptr(start), start_add, sym_len, n_sym, n_slots,
                         out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if st != RX_OK:
        raise RxError(st, "rx_sync_extract")
    return out
