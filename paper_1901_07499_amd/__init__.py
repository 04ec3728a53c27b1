"""MI355X (gfx950) uplink OFDM receive path: CP removal, batched FFT, LS channel
estimation, MRC/ZF combining and hard QAM demapping, as HIP kernels behind a
C ABI (``include/rx.h``, ``librx.so``).  ``paper_1901_07499_amd.rx`` is the
Python binding; build the library with ``python -m paper_1901_07499_amd.build``.
"""
