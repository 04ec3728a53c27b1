"""Every kernel of the library, compiled as the build compiles it, has no
workgroup barrier inside a loop that lanes can leave one by one (see
tests/barrier_scan.py).  Compiles the HIP sources to gfx950 assembly with
hipcc; runs on the CPU."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.barrier_scan import scan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_07499_amd", "csrc")
SOURCES = ("rx_kernels.hip", "rx_denoise.hip", "rx_mfma_fft.hip", "rx_sync.hip", "rx_noalloc.hip")

# A loop (header BB0_2) whose lanes leave one by one, with a barrier inside,
# then the same loop with the barrier after it.
_BAD = """_Zbad:
.LBB0_2:                                ; =>This Inner Loop Header: Depth=1
\ts_barrier
\tv_add_u32_e32 v1, 1, v1
\tv_cmp_le_i32_e32 vcc, s4, v1
\ts_or_b64 s[6:7], vcc, s[6:7]
\ts_andn2_b64 exec, exec, s[6:7]
\ts_cbranch_execnz .LBB0_2
; %bb.3:
\ts_endpgm
"""
_GOOD = _BAD.replace("\ts_barrier\n", "").replace("\ts_endpgm", "\ts_barrier\n\ts_endpgm")


def test_scan_flags_a_barrier_in_a_lanewise_loop():
    assert scan(_BAD) == {"_Zbad": ["BB0_2"]}
    assert scan(_GOOD) == {}


def _asm(src, tmp):
    from paper_1901_07499_amd import build
    out = os.path.join(tmp, src + ".s")
    cmd = [build.hipcc(), *build.COMMON, f"--offload-arch={build.ARCH}", *build.DEVICE_FLAGS, "-x", "hip",
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is needed to compile the kernels")
def test_no_barrier_inside_a_lanewise_loop(tmp_path):
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        texts = list(ex.map(lambda s: _asm(s, str(tmp_path)), SOURCES))
    found = {}
    for src, text in zip(SOURCES, texts):
        assert src == "rx_noalloc.hip" or "s_endpgm" in text, src  # rx_noalloc.hip holds no kernels
        for k, v in scan(text).items():
            found[f"{src}:{k}"] = v
    assert not found, found
