"""C-ABI contract of librx.so, checked without a GPU.

The library must load, export every function ``include/rx.h`` declares, and
reject bad arguments with the documented status codes before touching the GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rx.h")

rx = pytest.importorskip("paper_1901_07499_amd.rx", reason="librx.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rx_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(rx.LIB_PATH)
    declared = _declared()
    assert declared, "no declarations parsed"
    assert sorted(rx.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_library_is_built_for_gfx950():
    blob = open(rx.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def _p(**over):
    base = dict(n_ant=8, fft_len=64, cp_len=16, n_used=52, n_sym=11, bits_per_sym=2, pilot=np.ones(52))
    base.update(over)
    comb = base.pop("combiner", rx.RX_COMB_MRC)
    users = base.pop("n_users", 1)
    return rx.make_params(combiner=comb, n_users=users, **base)


@pytest.mark.parametrize("over,status", [
    ({}, rx.RX_OK),
    (dict(fft_len=1024, cp_len=72, n_used=600, bits_per_sym=4, pilot=np.ones(600)), rx.RX_OK),
    (dict(fft_len=2048, cp_len=144, n_used=1200, bits_per_sym=6, pilot=np.ones(1200)), rx.RX_OK),
    (dict(combiner=rx.RX_COMB_ZF), rx.RX_OK),
    (dict(n_ant=0), rx.RX_E_INVALID_ARG),
    (dict(fft_len=0), rx.RX_E_INVALID_ARG),
    (dict(fft_len=96), rx.RX_E_UNSUPPORTED),          # not a power of two
    (dict(fft_len=32, cp_len=8, n_used=20, pilot=np.ones(20)), rx.RX_E_UNSUPPORTED),
    (dict(fft_len=4096, n_used=52), rx.RX_E_UNSUPPORTED),
    (dict(cp_len=64), rx.RX_E_INVALID_ARG),           # CP >= N
    (dict(cp_len=-1), rx.RX_E_INVALID_ARG),
    (dict(n_used=51, pilot=np.ones(51)), rx.RX_E_INVALID_ARG),   # odd
    (dict(n_used=64, pilot=np.ones(64)), rx.RX_E_INVALID_ARG),   # > N-2
    (dict(n_used=0, pilot=np.ones(1)), rx.RX_E_INVALID_ARG),
    (dict(n_used=50, pilot=np.ones(50)), rx.RX_E_INVALID_ARG),   # 50*2 bits not whole bytes
    (dict(n_sym=1), rx.RX_E_INVALID_ARG),
    (dict(bits_per_sym=3), rx.RX_E_UNSUPPORTED),
    (dict(bits_per_sym=8), rx.RX_E_UNSUPPORTED),
    (dict(combiner=7), rx.RX_E_UNSUPPORTED),
    (dict(n_users=2), rx.RX_E_UNSUPPORTED),
    (dict(n_users=0), rx.RX_E_INVALID_ARG),
    (dict(pilot=np.r_[np.ones(51), 0.0]), rx.RX_E_INVALID_ARG),   # a zero pilot
    (dict(pilot=np.r_[np.ones(51), np.nan]), rx.RX_E_INVALID_ARG),
])
def test_params_check_status(over, status):
    p, keep = _p(**over)
    assert rx.rx_params_check(p) == status
    if status != rx.RX_OK:
        st, plan = rx.rx_plan_create(p)       # fails in validation, before any HIP call
        assert st == status and plan is None


def test_null_pilot_and_null_params():
    p, keep = _p()
    p.pilot = None
    assert rx.rx_params_check(p) == rx.RX_E_INVALID_ARG
    assert rx._lib.rx_params_check(None) == rx.RX_E_INVALID_ARG
    assert rx._lib.rx_plan_create(None, None) == rx.RX_E_INVALID_ARG


def test_calls_without_plan_are_rejected():
    assert rx.rx_plan_destroy(None) == rx.RX_OK
    assert rx.rx_workspace_bytes(None, 10) == 0
    assert rx.rx_estimate(None, 16, 1, 16, None, None, None) == rx.RX_E_INVALID_ARG
    assert rx.rx_demod(None, 16, 16, 1, 16, 16, None, None) == rx.RX_E_INVALID_ARG
    assert rx.rx_process_frame(None, 16, 1, None, 16, 16, 256, None) == rx.RX_E_INVALID_ARG
    assert rx.rx_debug_fft(None, 16, 1, 16, None) == rx.RX_E_INVALID_ARG


def test_status_strings():
    for st in (rx.RX_OK, rx.RX_E_INVALID_ARG, rx.RX_E_UNSUPPORTED, rx.RX_E_HIP, rx.RX_E_NOMEM):
        assert rx.rx_status_string(st) and rx.rx_status_string(st) != "unknown status"
    assert rx.rx_status_string(12345) == "unknown status"


def test_plan_creation_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p, keep = _p()
    st, plan = rx.rx_plan_create(p)
    assert st == rx.RX_E_HIP and plan is None


def test_single_hip_runtime_in_process():
    # torch and librx.so must share one libamdhip64 (same SONAME, two files on
    # disk); two copies would give two device contexts and invalid pointers.
    paths = set()
    for line in open("/proc/self/maps"):
        if "libamdhip64" in line:
            paths.add(line.split()[-1])
    assert len(paths) == 1, paths


def test_batch_create_validates_before_touching_the_gpu():
    arr = (rx.rx_params * 2)()
    p0, k0 = _p()
    p1, k1 = _p(bits_per_sym=3)
    arr[0], arr[1] = p0, p1
    st, b = rx.rx_batch_create(arr, 2)
    assert st == rx.RX_E_UNSUPPORTED and b is None
    p2, k2 = _p(combiner=rx.RX_COMB_ZF)
    arr[1] = p2
    st, b = rx.rx_batch_create(arr, 2)
    assert st == rx.RX_E_UNSUPPORTED                 # batches combine by MRC only
    st, b = rx.rx_batch_create(arr, 0)
    assert st == rx.RX_E_INVALID_ARG
    assert rx.rx_batch_destroy(None) == rx.RX_OK
    assert rx.rx_batch_workspace_bytes(None) == 0
    assert rx.rx_batch_process(None, 16, 16, 16, 16, None, None) == rx.RX_E_INVALID_ARG


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048])
def test_fft_radix_schedules_factor_the_length(n):
    # every schedule is a Stockham plan of the n-point DFT: radix 16 first,
    # the radices multiply to n; the three-pass lengths have a second
    # schedule with the last two radices swapped
    scheds = []
    for s in range(4):
        r = rx.fft_radices(n, s)
        if r is None:
            break
        scheds.append(r)
    assert rx.fft_radices(n, len(scheds)) is None and rx.fft_radices(n, -1) is None
    assert len(scheds) == (2 if n >= 512 else 1)
    for r in scheds:
        assert r[0] == 16 and int(np.prod(r)) == n and all(v in (2, 4, 8, 16) for v in r)
    if len(scheds) == 2:
        assert scheds[1] == (scheds[0][0], scheds[0][2], scheds[0][1]) and scheds[0] != scheds[1]


def test_fft_radices_and_batch_config_reject_bad_arguments():
    r = (ctypes.c_int32 * 3)()
    assert rx.rx_fft_radices(1000, 0, r) == rx.RX_E_UNSUPPORTED
    assert rx.rx_fft_radices(1024, 0, None) == rx.RX_E_INVALID_ARG
    d, e = ctypes.c_int32(), ctypes.c_int32()
    assert rx.rx_batch_schedules(None, 1024, ctypes.byref(d), ctypes.byref(e)) == rx.RX_E_INVALID_ARG
    assert rx.rx_batch_set_config(None, 1024, 4, 4, 0, 0) == rx.RX_E_INVALID_ARG
