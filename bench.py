#!/usr/bin/env python3
"""Throughput of the uplink receive path (CP removal + FFT + LS + MRC + demap) on one MI355X.

One step = ``rx_process_frame`` over every slot of the workload (the estimate
and demod kernels), with the int16 input already resident in HBM.  Prints one
JSON line.  Defaults: the 64-antenna, N=1024, 200-slot workload, 1 GPU.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c4|sweep|batch|denoiser|sync|precision]
                    [--no-cpu] [--workers P]

Timing: W untimed steps, then untimed steps until the clocks have settled
(windows of 20 steps, at least 200 ms, two windows within 2 %; reported as
warmup_ms / warmup_settle_steps), a synchronisation, about 15 ms of untimed
steps enqueued behind it (lead_in_steps: the GPU idles at the
synchronisation and its clocks need that long to come back), then exactly K
timed steps with an event before each and one after the last (ms_per_step
over all K, step_ms_median and step_ms_min).

Besides the headline it reports, for the dominant kernel (demod), algorithmic
bytes per launch (payload samples without CP, x-hat and bits; the channel
estimate's read is listed apart) over its average HIP-event-timed duration,
against the 8 TB/s HBM peak and a device copy measured in the same run; the
FP64 oracle timed on every usable host CPU and on one thread, with the CPU
model; and LS NMSE, BER and EVM at 20 dB SNR.  ``--workload sweep`` runs the
antenna-count x FFT-length sweep (N = 64, 1024; 1..128 antennas).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X, published (with packed FP32)
CSRC = os.path.join(ROOT, "paper_1901_07499_amd", "csrc")
KERNEL_SOURCES = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                        if f.endswith((".hip", ".hpp", ".cpp", ".h")))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_demod_c2.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Library sources each workload's kernels are built from (the launchers and
# API files included); "all" is the whole library.
WORKLOAD_SOURCES = {
    "path": ("rx_kernels.hip", "rx_fft.hpp", "rx_comb.hpp", "rx_launch.h", "rx_api.cpp"),
    "batch": ("rx_kernels.hip", "rx_fft.hpp", "rx_comb.hpp", "rx_launch.h", "rx_batch.cpp"),
    "denoiser": ("rx_denoise.hip", "rx_dn_api.cpp", "rx_comb.hpp", "rx_launch.h", "rx_kernels.hip", "rx_fft.hpp",
                 "rx_api.cpp"),
    "mfma": ("rx_mfma_fft.hip", "rx_kernels.hip", "rx_fft.hpp", "rx_launch.h", "rx_api.cpp"),
    "sync": ("rx_sync.hip", "rx_sync_api.cpp", "rx_kernels.hip", "rx_fft.hpp", "rx_launch.h", "rx_api.cpp"),
}


def kernel_hash(part: str = "all") -> str:
    """sha256 prefix of the library sources behind a workload's kernels
    (every source for "all"): ties a profile or counter file to the code it
    measured."""
    h = hashlib.sha256()
    files = KERNEL_SOURCES if part == "all" else [os.path.join(CSRC, f) for f in sorted(WORKLOAD_SOURCES[part])]
    for p in files:
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(cfg, S: int, part: str) -> int:
    """Bytes the method must move: payload samples (no CP) of the symbols a
    call reads and the outputs it writes.  Excludes CP samples, re-reads and
    the channel estimate, which the method need not move through HBM (the
    estimate's own output and the demod's read of it are the "h" part,
    reported beside the roofline)."""
    A, N, U, T, b = cfg.n_ant, cfg.fft_len, cfg.n_used, cfg.n_sym, cfg.bits_per_sym
    Td = T - 1
    out = Td * U * 8 + Td * U * b // 8       # x-hat (complex64) + packed bits
    if part == "path":                        # whole path
        return S * (T * A * N * 4 + out)
    if part == "demod":                       # data symbols in, outputs
        return S * (Td * A * N * 4 + out)
    if part == "estimate":                    # pilot symbol in
        return S * (A * N * 4)
    if part == "h":                           # one pass of the estimate over HBM
        return S * (A * U * 8)
    raise ValueError(part)


def host_cpus():
    """CPUs this process may run on (affinity), capped by a cgroup CPU quota
    when one is set, and the CPU model name."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    quota = None
    try:
        q, p = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(p)
    except (OSError, ValueError):
        pass
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = n if quota is None else max(1, min(n, int(quota)))
    return usable, {"affinity_cpus": n, "cgroup_cpu_quota": quota, "model": model}


def time_oracle(fr, cfg, threads: int, budget_s: float):
    """The FP64 oracle over a bounded prefix of the workload's slots on
    `threads` threads: the slot count is grown until one pass takes about
    budget_s / 3, then passes repeat until budget_s.  Returns
    (antenna-samples/s, slots per pass, seconds per pass)."""
    import oracle
    S = fr.iq.shape[0]
    n = max(1, min(S, threads))
    while True:
        t0 = time.perf_counter()
        oracle.run_config(fr, n_threads=threads, slots=slice(0, n))
        dt = time.perf_counter() - t0
        if dt >= budget_s / 3 or n == S:
            break
        n = min(S, max(n + 1, int(n * min(8.0, budget_s / 3 / max(dt, 1e-4)))))
    reps, total = 1, dt
    while total < budget_s and reps < 100:
        t0 = time.perf_counter()
        oracle.run_config(fr, n_threads=threads, slots=slice(0, n))
        total += time.perf_counter() - t0
        reps += 1
    per_pass = total / reps
    return n * cfg.n_sym * cfg.n_ant * (cfg.fft_len + cfg.cp_len) / per_pass, n, per_pass


def cpu_baseline(fr, cfg, budget_s: float = 8.0):
    """The oracle on every usable host CPU and on one thread (the paper's
    CPU baseline is one core), same int16 slots as the GPU run."""
    threads, info = host_cpus()
    v_all, n_all, dt_all = time_oracle(fr, cfg, threads, budget_s)
    v_one, n_one, dt_one = time_oracle(fr, cfg, 1, budget_s)
    log(f"cpu baseline {v_all:.4e} antenna-samples/s on {threads} threads, {v_one:.4e} on 1 ({info['model']})")
    return {"value": v_all, "unit": "antenna-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_all} of {fr.iq.shape[0]} slots of {cfg.name}, FP64 C oracle, {threads} threads, "
                      f"{dt_all:.3f} s per pass, passes repeated for ~{budget_s:g} s",
            "cpu_model": info["model"], "affinity_cpus": info["affinity_cpus"],
            "cgroup_cpu_quota": info["cgroup_cpu_quota"],
            "single_thread": {"value": v_one, "unit": "antenna-samples/s", "cores": 1,
                              "sample": f"first {n_one} slots, {dt_one:.3f} s per pass"}}


def settle(step, min_ms: float = 200.0, max_ms: float = 3000.0, window: int = 20):
    """Untimed steps after the fixed warm-up until the clocks have settled:
    windows of `window` steps are timed with events until at least min_ms
    have passed and two consecutive windows agree within 2 %.  Returns
    (ms spent, steps run, last window's ms per step)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    spent, steps, prev = 0.0, 0, None
    while True:
        e0.record()
        for _ in range(window):
            step()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        spent += ms
        steps += window
        cur = ms / window
        if (spent >= min_ms and prev is not None and abs(cur - prev) <= 0.02 * prev) or spent >= max_ms:
            return spent, steps, cur
        prev = cur


def lead_in(step, ms_per_step: float, target_ms: float = 15.0, min_steps: int = 8) -> int:
    """Untimed steps enqueued after the synchronisation that opens the timed
    region and before its first event, about target_ms of work at the settled
    step time.  The GPU idles at that synchronisation; without these steps the
    first ~40 timed steps ran up to 14 % slower in some runs while its clocks
    came back.  Returns the number of steps enqueued."""
    n = max(min_steps, int(target_ms / max(ms_per_step, 1e-3) + 0.5))
    for _ in range(n):
        step()
    return n


def copy_peak_gbps(nbytes: int = 1 << 30, reps: int = 10):
    """Device-to-device copy rate (bytes read + written per second), the
    measured second denominator of the HBM fraction."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


COPY_BYTES = 1 << 30


def copy_calibration():
    """A plain device-to-device copy of COPY_BYTES: reads and writes COPY_BYTES each."""
    import torch
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copied {COPY_BYTES} B x 3")


def _counter_per_dispatch(path, kernel_substr, counter):
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} for {kernel_substr} in {path}")
    return sum(vals) / len(vals)


def write_traffic(demod_fetch, demod_write, copy_fetch, copy_write):
    """HBM bytes per demod launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    each scaled by COPY_BYTES / (what the counter reads for the reference copy)."""
    from rxgen import C2
    cf = _counter_per_dispatch(copy_fetch, "copyBuffer", "FETCH_SIZE") * 1024
    cw = _counter_per_dispatch(copy_write, "copyBuffer", "WRITE_SIZE") * 1024
    kf = COPY_BYTES / cf
    kw = COPY_BYTES / cw
    df = _counter_per_dispatch(demod_fetch, "demod_kernel", "FETCH_SIZE") * 1024 * kf
    dw = _counter_per_dispatch(demod_write, "demod_kernel", "WRITE_SIZE") * 1024 * kw
    rec = {"workload": C2.name, "kernel": "demod_kernel", "kernel_hash": kernel_hash("path"),
           "fetch_bytes": df, "write_bytes": dw, "bytes_per_launch": df + dw,
           "fetch_scale": kf, "write_scale": kw,
           "algorithmic_bytes_per_launch": algorithmic_bytes(C2, C2.n_slots, "demod")}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


BATCH_SEED = 190107499 + 3


def bench_batch(args):
    """Mixed batch: frames with antennas in {16,32,64,128}, FFT length in
    {128..2048} (CP = N/14), QPSK/16-QAM/64-QAM, 1 pilot + 13 data symbols;
    one graph launch per step after autotuning; per-frame latency percentiles."""
    import numpy as np
    from rxgen import make_batch
    t0 = time.time()
    workers = args.workers if args.workers > 0 else min(16, os.cpu_count() or 1)
    bt = make_batch(args.frames, BATCH_SEED, workers=workers)
    log(f"generated batch of {args.frames} frames: {bt.iq.nbytes / 1e6:.1f} MB in {time.time() - t0:.1f} s")
    import torch
    from paper_1901_07499_amd import rx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    batch = rx.Batch(bt.configs, [f.pilot for f in bt.frames])
    iq = torch.from_numpy(bt.iq).to(dev)
    out = batch.outputs(dev, want_H=False)
    t0 = time.time()
    batch.autotune(iq, out, reps=8)
    classes = sorted({c.fft_len for c in bt.configs})
    chosen = {n: batch.config(n) + batch.schedules(n) for n in classes}
    log(f"autotuned in {time.time() - t0:.1f} s: {chosen}")
    for _ in range(args.warmup):
        batch.process(iq, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        batch.process(iq, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    samples = sum(c.n_sym * c.n_ant * (c.fft_len + c.cp_len) for c in bt.configs)
    lat = []
    for _ in range(max(5, min(args.steps, 20))):
        batch.process(iq, out)
        lat.append(batch.frame_latency_ms())
    lat = np.concatenate(lat)
    alg = sum(c.n_sym * c.n_ant * c.fft_len * 4 + (c.n_sym - 1) * c.n_used * (8 + c.bits_per_sym / 8)
              for c in bt.configs)
    rec = {"metric": "antenna-samples/s through FFT+LS+demod, batched mixed sizes in one graph launch",
           "value": samples / (ms * 1e-3), "unit": "antenna-samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"batch_{args.frames}_mixed", "frames": args.frames,
                      "antennas": [16, 32, 64, 128], "fft_len": [128, 256, 512, 1024, 2048],
                      "input_MB": round(bt.iq.nbytes / 1e6, 1), "combiner": "mrc"},
           "algorithmic_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
           "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "frame_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                "max": float(lat.max()), "samples": int(lat.size)},
           "autotuned": {str(n): {"demod_waves": w, "est_jobs": j,
                                  "demod_radices": list(rx.fft_radices(n, sd)),
                                  "est_radices": list(rx.fft_radices(n, se))}
                         for n, (w, j, sd, se) in chosen.items()},
           "kernel_hash": kernel_hash("batch"), "library_hash": kernel_hash()}
    print(json.dumps(rec), flush=True)


DN_SEED = 190107499 + 5
# MACs of one refinement row of 1200 subcarriers: 1200 * (2*32 + 32*32 + 32*32 + 32*2) * 7
DN_ROW_MACS = 1200 * (2 * 32 + 32 * 32 * 2 + 32 * 2) * 7
MFMA_BF16_PEAK_TFLOPS = 2500.0


def bench_denoiser(args):
    """Learned refinement of the comb-pilot LS estimate on the 128-antenna,
    N=2048, 1200-subcarrier shape (pilot on every 4th subcarrier, 64-QAM):
    train on channels generated on the GPU, then time comb estimate +
    refinement + demod over resident slots, and report NMSE (against the true
    channel) and BER of plain interpolation and of the refined estimate."""
    import numpy as np
    from rxgen import C5, C5_20DB, init_denoiser_params, make_frames
    workers = args.workers if args.workers > 0 else min(16, os.cpu_count() or 1)
    t0 = time.time()
    S = args.slots
    fr = make_frames(C5, n_slots=S, workers=workers)
    qual = {snr: make_frames(C5_20DB.replace(snr_db=(snr, snr)), n_slots=args.quality_slots, workers=workers)
            for snr in (20.0, 5.0)}
    log(f"generated {S} slots of {C5.name} ({fr.iq.nbytes / 1e6:.1f} MB) and quality sets in {time.time() - t0:.1f} s")
    import torch
    from paper_1901_07499_amd import rx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    A, U, T, N, CP = C5.n_ant, C5.n_used, C5.n_sym, C5.fft_len, C5.cp_len
    dn = rx.Denoiser(U)
    p = torch.from_numpy(init_denoiser_params(DN_SEED)).to(dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    dn.load(p)

    # ---- training on generated channels (8-24 taps, delay 0.5-5 us at 30.72 MS/s, SNR 0-30 dB)
    gen = rx.chan_gen(fft_len=N, n_used=U, cp_len=CP, pilot_spacing=C5.pilot_spacing, taps=(8, 24),
                      tau_samples=(15, 154), snr_db=(0.0, 30.0))
    R = args.dn_rows
    losses = torch.zeros(args.dn_steps, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for step in range(1, args.dn_steps + 1):
        ht, hl = rx.generate(gen, DN_SEED, (step - 1) * R, R, dev)
        dn.train_step(p, m, v, step, hl, ht, lr=args.dn_lr, loss=losses[step - 1:step])
        if step % 500 == 0:
            log(f"training step {step}: loss {losses[step - 1].item():.5f}")
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    rows_trained = args.dn_steps * R
    lc = losses.cpu().numpy()
    log(f"trained {args.dn_steps} steps x {R} rows in {train_ms:.0f} ms")

    # ---- inference: comb estimate -> refinement (in place) -> demod, slots resident in HBM
    plan = rx.Plan.from_config(C5, fr.pilot)
    iq = torch.from_numpy(fr.iq).to(dev)
    H = torch.empty((S, A, U, 2), dtype=torch.float32, device=dev)
    rows = H.view(S * A, U, 2)

    def step_once():
        plan.estimate(iq, H=H)
        dn.apply(rows, out=rows)
        return plan.demod(iq, H)

    for _ in range(args.warmup):
        step_once()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step_once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    plan.estimate(iq, H=H)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        dn.apply(rows, out=rows)
    e1.record()
    torch.cuda.synchronize()
    dn_ms = e0.elapsed_time(e1) / args.steps
    tflops = 2.0 * DN_ROW_MACS * S * A / (dn_ms * 1e-3) / 1e12
    samples = S * T * A * (N + CP)

    # ---- quality: NMSE and BER of plain interpolation vs refined, same frames
    quality = {}
    for snr, q in qual.items():
        qp = rx.Plan.from_config(q.cfg, q.pilot)
        qiq = torch.from_numpy(q.iq).to(dev)
        h_ls = qp.estimate(qiq)
        h_dn = dn.apply(h_ls.view(-1, U, 2)).view_as(h_ls)
        res = {}
        truth = q.H_true
        sent = np.unpackbits(q.packed_bits(), axis=-1)
        for name, h in (("interp", h_ls), ("refined", h_dn)):
            _, bits = qp.demod(qiq, h)
            hc = h.cpu().numpy()
            hc = hc[..., 0] + 1j * hc[..., 1]
            nmse = 10 * np.log10(np.sum(np.abs(hc - truth) ** 2) / np.sum(np.abs(truth) ** 2))
            errs = int(np.count_nonzero(np.unpackbits(bits.cpu().numpy(), axis=-1) != sent))
            res[name] = {"nmse_db": round(float(nmse), 3), "ber": errs / sent.size, "bit_errors": errs}
        res["nmse_gain_db"] = round(res["interp"]["nmse_db"] - res["refined"]["nmse_db"], 3)
        res["bits"] = int(sent.size)
        quality[f"{snr:g}dB"] = res
    log(f"quality: {quality}")
    rec = {"metric": "antenna-samples/s through comb LS + learned refinement + demod; NMSE/BER at 20 dB vs plain",
           "value": samples / (ms * 1e-3), "unit": "antenna-samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 path, bf16 MFMA refinement", "data": "synthetic",
           "config": {"workload": C5.name, "n_ant": A, "fft_len": N, "cp_len": CP, "n_used": U, "n_sym": T,
                      "bits_per_sym": C5.bits_per_sym, "pilot_spacing": C5.pilot_spacing, "n_slots": S},
           "roofline": {"bound": "mfma", "kernel": "dn_forward_kernel", "achieved": round(tflops, 1),
                        "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                        "algorithmic_flop_per_launch": 2 * DN_ROW_MACS * S * A, "avg_launch_ms": round(dn_ms, 5)},
           "refinement_ms": round(dn_ms, 5), "refinement_rows_per_s": S * A / (dn_ms * 1e-3),
           "training": {"steps": args.dn_steps, "rows_per_step": R, "rows": rows_trained,
                        "slots_equivalent": rows_trained / A, "ms": round(train_ms, 1),
                        "rows_per_s": rows_trained / (train_ms * 1e-3), "lr": args.dn_lr,
                        "loss_first_100": float(lc[:100].mean()), "loss_last_100": float(lc[-100:].mean())},
           "quality": quality, "kernel_hash": kernel_hash("denoiser"), "library_hash": kernel_hash()}
    print(json.dumps(rec), flush=True)


# Integer multiply-adds per second of the vector ALU for the correlation's
# 2-way 16-bit dot products (v_dot2c_i32_i16: two multiply-adds per lane per
# instruction at one wave64 instruction per CU per clock, as the other 32-bit
# vector operations), 256 CUs at 2.4 GHz.
VALU_INT_MAC_PEAK = 2 * 256 * 64 * 2.4e9


def bench_sync(args):
    """PN synchronisation on a stream of the 64-antenna, N=1024 shape: a
    255-chip preamble at a random offset, then `--slots` slots; time the
    correlation metric over one slot's worth of candidate offsets, the slot
    extraction, and sync + extraction + receive."""
    import numpy as np
    from rxgen import C2, make_stream
    S = args.slots
    t0 = time.time()
    lead = 5000
    st = make_stream(C2.replace(name="c2_stream"), S, lead, seed=190107499 + 7, snr_db=20.0)
    cfg = st.frames.cfg
    log(f"generated a {cfg.n_ant}-antenna stream of {st.raw.shape[1]} samples with {S} slots in {time.time() - t0:.1f} s")
    import torch
    from paper_1901_07499_amd import rx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    raw = torch.from_numpy(st.raw).to(dev)
    A, L, T = cfg.n_ant, st.pn.size, cfg.n_sym
    sym_len = cfg.fft_len + cfg.cp_len
    n_search = T * sym_len
    plan = rx.Plan.from_config(cfg, st.frames.pilot)
    iq = torch.empty((S, T, A, sym_len, 2), dtype=torch.int16, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # Buffers allocated once and the C ABI called directly, so the timed loops
    # measure the GPU rather than per-call allocation in the Python wrappers.
    stream = torch.cuda.current_stream().cuda_stream
    chips = np.ascontiguousarray(np.rint(st.pn), dtype=np.int8)
    chips_p = chips.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    n_samp, stride = raw.shape[1], raw.shape[1]
    off = torch.empty((1,), dtype=torch.int64, device=dev)
    peak = torch.empty((1,), dtype=torch.int64, device=dev)
    ws = torch.empty((max(256, rx.rx_sync_workspace_bytes(A, n_search)),), dtype=torch.uint8, device=dev)
    xhat = torch.empty((S, T - 1, cfg.n_used, 2), dtype=torch.float32, device=dev)
    bits = torch.empty((S, T - 1, plan.row_bytes), dtype=torch.uint8, device=dev)
    pws = torch.empty((plan.workspace_bytes(S),), dtype=torch.uint8, device=dev)

    def find():
        assert rx.rx_sync_find(raw.data_ptr(), A, n_samp, stride, chips_p, chips.size, n_search, None,
                               off.data_ptr(), peak.data_ptr(), ws.data_ptr(), stream) == rx.RX_OK

    def extract():
        assert rx.rx_sync_extract(raw.data_ptr(), A, n_samp, stride, off.data_ptr(), L, sym_len, T, S,
                                  iq.data_ptr(), stream) == rx.RX_OK

    def chain():
        find()
        extract()
        assert rx.rx_process_frame(plan._plan, iq.data_ptr(), S, None, xhat.data_ptr(), bits.data_ptr(),
                                   pws.data_ptr(), stream) == rx.RX_OK

    find_ms = timed(find, args.steps)
    ext_ms = timed(extract, args.steps)
    chain_ms = timed(chain, args.steps)
    chain()
    torch.cuda.synchronize()
    sent = np.unpackbits(st.frames.packed_bits(), axis=-1)
    errs = int(np.count_nonzero(np.unpackbits(bits.cpu().numpy(), axis=-1) != sent))
    macs = 2.0 * A * n_search * L
    ext_bytes = 2 * S * T * A * sym_len * 4
    samples = S * T * A * sym_len
    rec = {"metric": "antenna-samples/s through PN sync + slot extraction + FFT+LS+demod", "value": samples / (chain_ms * 1e-3),
           "unit": "antenna-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": chain_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32 metric, f32 path", "data": "synthetic",
           "config": {"workload": "c2_stream_pn255", "n_ant": A, "fft_len": cfg.fft_len, "cp_len": cfg.cp_len,
                      "n_slots": S, "pn_len": int(L), "n_search": n_search, "lead": lead},
           "roofline": {"bound": "alu", "kernel": "rx_sync_find (metric, group sum, argmax)",
                        "achieved": round(macs / (find_ms * 1e-3) / 1e12, 3),
                        "peak": round(VALU_INT_MAC_PEAK / 1e12, 3), "unit": "T int-MAC/s",
                        "frac": round(macs / (find_ms * 1e-3) / VALU_INT_MAC_PEAK, 4), "traffic": None,
                        "algorithmic_macs_per_launch": macs, "avg_launch_ms": round(find_ms, 5)},
           "sync_find_ms": round(find_ms, 5), "extract_ms": round(ext_ms, 5),
           "extract_GBps": round(ext_bytes / (ext_ms * 1e-3) / 1e9, 1),
           "offset": int(off.item()), "lead": lead, "bit_errors": errs, "bits": int(sent.size),
           "kernel_hash": kernel_hash("sync"), "library_hash": kernel_hash()}
    print(json.dumps(rec), flush=True)


def bench_precision(args):
    """The 128-antenna, N=2048, 64-QAM shape with the FFT in each arithmetic:
    FP32 radix (vector units) and the DFT-stage GEMMs on fp16 / bf16 MFMA,
    with and without the hi+lo split.  Per mode: throughput over `--slots`
    resident slots, the FFT's RMS error against an FP64 FFT (numpy) of the same
    int16 symbols, and EVM and BER at 10, 20 and 30 dB."""
    import numpy as np
    from rxgen import C4, make_frames
    workers = args.workers if args.workers > 0 else min(16, os.cpu_count() or 1)
    S = args.slots
    t0 = time.time()
    if args.gen_unique > 0:
        import dataclasses
        k = min(args.gen_unique, S)
        fr = make_frames(C4, n_slots=k)
        fr = dataclasses.replace(fr, iq=np.ascontiguousarray(fr.iq[np.arange(S) % k]))
    else:
        fr = make_frames(C4, n_slots=S, workers=workers)
    qual = {snr: make_frames(C4.replace(name=f"c4_{snr:g}dB", snr_db=(snr, snr), seed=C4.seed + int(snr)),
                             n_slots=args.quality_slots, workers=workers) for snr in (10.0, 20.0, 30.0)}
    log(f"generated {S} slots of {C4.name} ({fr.iq.nbytes / 1e6:.1f} MB) and quality sets in {time.time() - t0:.1f} s")
    import torch
    from paper_1901_07499_amd import rx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    A, N, CP, T, U, B = C4.n_ant, C4.fft_len, C4.cp_len, C4.n_sym, C4.n_used, C4.bits_per_sym
    iq = torch.from_numpy(fr.iq).to(dev)
    # FP64 reference spectrum of the first slot's symbols (numpy, not the receiver's oracle)
    x = fr.iq[0].astype(np.float64)
    ref = np.fft.fft(x[..., CP:, 0] + 1j * x[..., CP:, 1], axis=-1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, code in rx.FFT_MODES.items():
        plan = rx.Plan.from_config(C4, fr.pilot, fft_mode=code)
        bufs = (torch.empty((S, A, U, 2), dtype=torch.float32, device=dev), None,
                torch.empty((S, T - 1, U * B // 8), dtype=torch.uint8, device=dev))
        for _ in range(args.warmup):
            plan.process(iq, out=bufs)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            plan.process(iq, out=bufs)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        Y = plan.debug_fft(iq[:1]).cpu().numpy()
        Y = Y[0, ..., 0].astype(np.float64) + 1j * Y[0, ..., 1]
        fft_err = float(np.sqrt(np.mean(np.abs(Y - ref) ** 2) / np.mean(np.abs(ref) ** 2)))
        q = {}
        for snr, f in qual.items():
            qp = rx.Plan.from_config(f.cfg, f.pilot, fft_mode=code)
            _, xh, bits = qp.process(torch.from_numpy(f.iq).to(dev))
            xh = xh.cpu().numpy()
            xc = xh[..., 0].astype(np.float64) + 1j * xh[..., 1]
            evm = float(np.sqrt(np.mean(np.abs(xc - f.X) ** 2) / np.mean(np.abs(f.X) ** 2)))
            sent = np.unpackbits(f.packed_bits(), axis=-1)
            errs = int(np.count_nonzero(np.unpackbits(bits.cpu().numpy(), axis=-1) != sent))
            q[f"{snr:g}dB"] = {"evm_rms": round(evm, 6), "ber": errs / sent.size, "bit_errors": errs}
        samples = S * T * A * (N + CP)
        out[name] = {"ms_per_step": round(ms, 5), "antenna_samples_per_s": samples / (ms * 1e-3),
                     "fft_rms_rel_error_vs_fp64": fft_err, "quality": q}
        log(f"{name}: {ms:.4f} ms, FFT error {fft_err:.3e}, {q}")
    best = out["f16_split"]
    rec = {"metric": "antenna-samples/s through FFT+LS+demod with the FFT as fp16/bf16 MFMA DFT GEMMs; "
                     "FFT error, EVM, BER per mode", "value": best["antenna_samples_per_s"],
           "unit": "antenna-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f16 MFMA with hi+lo split, f32 accumulate", "data": "synthetic",
           "config": {"workload": C4.name, "n_ant": A, "fft_len": N, "cp_len": CP, "n_used": U, "n_sym": T,
                      "bits_per_sym": B, "n_slots": S, "quality_slots": args.quality_slots,
                      "distinct_slots": min(args.gen_unique, S) if args.gen_unique > 0 else S},
           "modes": out, "kernel_hash": kernel_hash("mfma"), "library_hash": kernel_hash()}
    print(json.dumps(rec), flush=True)


def bench_sweep(args):
    """Antenna-count x FFT-length sweep: N = 64 and 1024 at 1..128 antennas,
    14 symbols per slot, each point ~1 GiB of int16 input resident in HBM
    (distinct generated slots tiled over the buffer).  Per point: the whole
    path's throughput, algorithmic bytes against the HBM peak, time per OFDM
    symbol (every antenna), and the FP64 oracle on one host thread beside it."""
    import math
    import numpy as np
    from rxgen import SWEEP_ANTENNAS, SWEEP_FFT_LENS, make_frames, sweep_config
    workers = args.workers if args.workers > 0 else min(16, os.cpu_count() or 1)
    points = [(n, a) for n in SWEEP_FFT_LENS for a in SWEEP_ANTENNAS]
    if args.sweep_points:
        points = [tuple(int(x) for x in p.split("x")) for p in args.sweep_points.split(",")]
    # Generate every point's distinct slots before the process touches the GPU.
    frames = {}
    t0 = time.time()
    for n, a in points:
        cfg = sweep_config(n, a)
        k = min(cfg.n_slots, max(8, math.ceil(args.sweep_unique_mb * 2 ** 20 / cfg.slot_bytes)))
        frames[(n, a)] = (cfg, make_frames(cfg, n_slots=k, workers=workers))
    log(f"generated {len(points)} sweep points in {time.time() - t0:.1f} s")
    cpu_rates = {}
    if not args.no_cpu:
        for p in points:
            cfg, fr = frames[p]
            cpu_rates[p] = time_oracle(fr, cfg, 1, args.sweep_cpu_s)
    import torch
    from paper_1901_07499_amd import rx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    copy_gbs = copy_peak_gbps()
    rows = []
    for p in points:
        cfg, fr = frames[p]
        S, k = cfg.n_slots, fr.iq.shape[0]
        uniq = torch.from_numpy(fr.iq).to(dev)
        iq = uniq[torch.arange(S, device=dev) % k].contiguous()
        del uniq
        plan = rx.Plan.from_config(cfg, fr.pilot)
        Td = cfg.n_sym - 1
        out = (None, torch.empty((S, Td, cfg.n_used, 2), dtype=torch.float32, device=dev),
               torch.empty((S, Td, plan.row_bytes), dtype=torch.uint8, device=dev))
        ws = torch.empty(max(256, plan.workspace_bytes(S)), dtype=torch.uint8, device=dev)

        def step():
            plan.process(iq, out=out, workspace=ws)

        for _ in range(args.warmup):
            step()
        _, _, settled = settle(step, min_ms=100.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lead_in(step, settled)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        samples = S * cfg.n_sym * cfg.n_ant * (cfg.fft_len + cfg.cp_len)
        alg = algorithmic_bytes(cfg, S, "path")
        gbs = alg / (ms * 1e-3) / 1e9
        row = {"fft_len": cfg.fft_len, "n_ant": cfg.n_ant, "n_slots": S, "distinct_slots": k,
               "input_MB": round(S * cfg.slot_bytes / 1e6, 1), "ms_per_step": round(ms, 5),
               "antenna_samples_per_s": samples / (ms * 1e-3),
               "us_per_ofdm_symbol": round(ms * 1e3 / (S * cfg.n_sym), 6),
               "algorithmic_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
               "copy_frac": round(gbs / copy_gbs, 4)}
        if p in cpu_rates:
            v1, n1, dt1 = cpu_rates[p]
            row["oracle_1thread_antenna_samples_per_s"] = v1
            row["oracle_1thread_sample"] = f"first {n1} slots, {dt1:.3f} s per pass"
            row["gpu_over_oracle_1thread"] = round(row["antenna_samples_per_s"] / v1, 1)
        log(f"N={cfg.fft_len} A={cfg.n_ant} S={S}: {ms:.4f} ms, {row['antenna_samples_per_s']:.3e} "
            f"antenna-samples/s, {row['hbm_frac'] * 100:.1f} % HBM")
        rows.append(row)
        del iq, out, ws, plan
        torch.cuda.empty_cache()
    head = next((r for r in rows if r["fft_len"] == 1024 and r["n_ant"] == 64), rows[-1])
    threads, info = host_cpus()
    rec = {"metric": "antenna-samples/s through FFT+LS+demod, % HBM peak, over antennas x FFT length",
           "value": head["antenna_samples_per_s"], "unit": "antenna-samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sweep", "value_point": f"N={head['fft_len']} A={head['n_ant']}",
                      "fft_len": sorted({r["fft_len"] for r in rows}), "n_ant": sorted({r["n_ant"] for r in rows}),
                      "n_sym": 14, "input_per_point": "~1 GiB int16 IQ resident in HBM"},
           "copy_peak_GBps": round(copy_gbs, 1), "cpu_model": info["model"], "points": rows,
           "kernel_hash": kernel_hash("path"), "library_hash": kernel_hash()}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # about 50 ms of untimed work first: the GPU's clocks settle within ~100 steps
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4", "batch", "denoiser", "sync", "precision", "sweep"])
    ap.add_argument("--frames", type=int, default=256, help="frames of the batch workload")
    ap.add_argument("--slots", type=int, default=None,
                    help="slots of the denoiser (default 32), sync (32) and precision (500, its configuration) workloads")
    ap.add_argument("--quality-slots", type=int, default=8,
                    help="slots per SNR of the denoiser and precision quality figures")
    # 25 000 steps x 1024 rows = 25.6 M antenna rows = 200 k slots of 128 antennas, the configured budget
    ap.add_argument("--dn-steps", type=int, default=25000, help="training steps of the denoiser workload")
    ap.add_argument("--dn-rows", type=int, default=1024, help="rows (antenna estimates) per training step")
    ap.add_argument("--dn-lr", type=float, default=2e-3, help="Adam learning rate")
    ap.add_argument("--workers", type=int, default=0,
                    help="generator processes of every workload (0 = up to 16; 1 under a profiler)")
    ap.add_argument("--sweep-points", default="",
                    help="sweep points as NxA, comma separated (default: N in {64, 1024} x A in {1..128})")
    ap.add_argument("--sweep-unique-mb", type=float, default=16.0,
                    help="MiB of distinct generated slots per sweep point (tiled to ~1 GiB)")
    ap.add_argument("--sweep-cpu-s", type=float, default=1.0, help="seconds of one-thread oracle per sweep point")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-quality", action="store_true", help="skip the 20 dB quality figures")
    ap.add_argument("--gen-unique", type=int, default=0,
                    help="generate only this many distinct slots in this process and tile them over the "
                         "workload (for profiler runs, where no worker processes may be started; c1, c2, c4, precision)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for the traffic counters)")
    ap.add_argument("--write-traffic", nargs=4, metavar=("DEMOD_FETCH", "DEMOD_WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="turn four rocprofv3 --pmc counter_collection.csv files into " + TRAFFIC_FILE)
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this receive path shards by slot with no exchange, "
              "so multi-GPU throughput is N x the one-GPU figure; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.slots is None:
        args.slots = 500 if args.workload == "precision" else 32
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "denoiser":
        bench_denoiser(args)
        return
    if args.workload == "sync":
        bench_sync(args)
        return
    if args.workload == "precision":
        bench_precision(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    from rxgen import C1, C2, C2_20DB, C4, make_frames
    cfg = {"c1": C1, "c2": C2, "c4": C4}[args.workload]
    S = cfg.n_slots
    workers = args.workers if args.workers > 0 else min(16, os.cpu_count() or 1)

    # Generate every input before the process touches the GPU (fork-based pool).
    t0 = time.time()
    if args.gen_unique > 0:
        import dataclasses
        import numpy as np
        k = min(args.gen_unique, S)
        fr = make_frames(cfg, n_slots=k)
        fr = dataclasses.replace(fr, iq=np.ascontiguousarray(fr.iq[np.arange(S) % k]))
    else:
        fr = make_frames(cfg, workers=workers)
    log(f"generated {cfg.name}: {fr.iq.nbytes / 1e6:.1f} MB int16 in {time.time() - t0:.1f} s")
    q20 = None
    if not args.no_quality:
        q_slots = min(S, 24)
        q20 = make_frames(C2_20DB.replace(fft_len=cfg.fft_len, cp_len=cfg.cp_len, n_used=cfg.n_used,
                                          n_ant=cfg.n_ant, bits_per_sym=cfg.bits_per_sym, n_sym=cfg.n_sym,
                                          fs_hz=cfg.fs_hz),
                          n_slots=q_slots, workers=workers)
        log(f"generated {q_slots} slots at 20 dB for quality figures")

    import numpy as np
    import torch
    from paper_1901_07499_amd import rx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = rx.Plan.from_config(cfg, fr.pilot)

    # Host->device copy of the whole input, from pinned memory (context only).
    pinned = torch.empty(fr.iq.shape, dtype=torch.int16, pin_memory=True)
    pinned.numpy()[...] = fr.iq
    iq = torch.empty(fr.iq.shape, dtype=torch.int16, device=dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    iq.copy_(pinned, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    h2d_ms = e0.elapsed_time(e1)
    log(f"H2D {fr.iq.nbytes / 1e6:.1f} MB in {h2d_ms:.2f} ms")

    Td = cfg.n_sym - 1
    xhat = torch.empty((S, Td, cfg.n_used, 2), dtype=torch.float32, device=dev)
    bits = torch.empty((S, Td, plan.row_bytes), dtype=torch.uint8, device=dev)
    H = torch.empty((S, cfg.n_ant, cfg.n_used, 2), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    # One step = the path's two launches through the C ABI, rx_estimate into H
    # then rx_demod from it (the kernels rx_process_frame launches for a batch
    # whose H fits its workspace).  In the timed region each step records two
    # HIP events on the launch stream, before each launch; the next step's
    # first event (or one after the last step) ends the demod, so every
    # kernel's duration is measured inside the timed region.  (Each event
    # record costs the GPU about 2 us; a third event per step measured 2 %
    # slower steps.)
    def step(ev=None):
        if ev is not None:
            ev[0].record()
        assert rx.rx_estimate(plan._plan, iq.data_ptr(), S, H.data_ptr(), None, None, stream) == rx.RX_OK
        if ev is not None:
            ev[1].record()
        assert rx.rx_demod(plan._plan, iq.data_ptr(), H.data_ptr(), S, xhat.data_ptr(), bits.data_ptr(), None,
                           stream) == rx.RX_OK

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # The GPU's clocks take ~100 ms of load to settle: keep stepping (untimed)
    # until the step time is steady.
    settle_ms, settle_steps, settle_last = settle(step)
    log(f"warmup {args.warmup} steps, then {settle_steps} settling steps in {settle_ms:.1f} ms "
        f"(last window {settle_last:.4f} ms/step)")

    # Timed region: exactly K steps, two events each, and one after the last.
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    ev_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    n_lead = lead_in(step, settle_last)
    for k in range(args.steps):
        step(evs[k])
    ev_end.record()
    torch.cuda.synchronize()
    ms_per_step = evs[0][0].elapsed_time(ev_end) / args.steps
    import statistics
    nxt = [evs[k + 1][0] for k in range(args.steps - 1)] + [ev_end]
    step_ms = [evs[k][0].elapsed_time(nxt[k]) for k in range(args.steps)]
    est_each = [e[0].elapsed_time(e[1]) for e in evs]
    dem_each = [evs[k][1].elapsed_time(nxt[k]) for k in range(args.steps)]
    samples_per_step = S * cfg.n_sym * cfg.n_ant * (cfg.fft_len + cfg.cp_len)
    value = samples_per_step / (ms_per_step * 1e-3)
    log(f"timed {args.steps} steps: {ms_per_step:.4f} ms/step (median {statistics.median(step_ms):.4f}, "
        f"min {min(step_ms):.4f}), {value:.4e} antenna-samples/s")
    est_ms = sum(est_each) / len(est_each)
    dem_ms = sum(dem_each) / len(dem_each)
    # the same batch through the boundary's one-call entry point, for comparison
    ws = torch.empty(plan.workspace_bytes(S), dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.process(iq, out=(None, xhat, bits), workspace=ws)
    e1.record()
    e1.synchronize()
    process_ms = e0.elapsed_time(e1) / args.steps
    dem_bytes = algorithmic_bytes(cfg, S, "demod")
    achieved = dem_bytes / (dem_ms * 1e-3) / 1e9
    log(f"estimate {est_ms:.4f} ms, demod {dem_ms:.4f} ms (means over the timed steps) -> demod {achieved:.1f} GB/s "
        f"algorithmic; rx_process_frame {process_ms:.4f} ms per step")
    copy_gbs = copy_peak_gbps()
    log(f"device copy {copy_gbs:.1f} GB/s")

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_hash") == kernel_hash("path") and t.get("workload") == cfg.name:
            traffic = t.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": "demod_kernel", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes_per_launch": dem_bytes,
                "avg_launch_ms": round(dem_ms, 5),
                "h_read_bytes_per_launch": algorithmic_bytes(cfg, S, "h"),
                "copy_peak_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    # The same kernel against the FP32 vector peak: algorithmic flops are 5 N log2 N per transform
    # plus 12 per used subcarrier and antenna for conj(H) Y and |H|^2 (packed FP32 is not used, so
    # the reachable vector rate is half of the published peak).
    import math
    dem_flop = S * (cfg.n_sym - 1) * cfg.n_ant * (5.0 * cfg.fft_len * math.log2(cfg.fft_len) + 12.0 * cfg.n_used)
    dem_tflops = dem_flop / (dem_ms * 1e-3) / 1e12
    alu_view = {"bound": "alu", "kernel": "demod_kernel", "achieved": round(dem_tflops, 2),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(dem_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                "algorithmic_flop_per_launch": dem_flop}
    path_bytes = algorithmic_bytes(cfg, S, "path")
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9

    quality = None
    if q20 is not None:
        qplan = rx.Plan.from_config(q20.cfg, q20.pilot)
        qH, qx, qb = qplan.process(torch.from_numpy(q20.iq).to(dev), want_H=True)
        torch.cuda.synchronize()
        Hg = qH.cpu().numpy().astype(np.float64)
        Hg = Hg[..., 0] + 1j * Hg[..., 1]
        N = q20.cfg.fft_len
        nmse = np.mean(np.abs(Hg - q20.H_true) ** 2 / (N * q20.scale[:, None, None] ** 2))
        xg = qx.cpu().numpy().astype(np.float64)
        xg = xg[..., 0] + 1j * xg[..., 1]
        evm = float(np.sqrt(np.mean(np.abs(xg - q20.X) ** 2)))
        nerr = int(np.unpackbits(qb.cpu().numpy() ^ q20.packed_bits()).sum())
        nbits = int(q20.bits.size)
        quality = {"snr_db": 20.0, "slots": int(q20.iq.shape[0]), "ls_nmse_db": round(10 * np.log10(nmse), 3),
                   "evm_rms": round(evm, 5), "bit_errors": nerr, "bits": nbits,
                   "ber": nerr / nbits, "ber_95_upper": (3.0 / nbits if nerr == 0 else None)}
        log(f"quality at 20 dB: {quality}")

    cpu = None if args.no_cpu else cpu_baseline(fr, cfg)

    rec = {
        "metric": "antenna-samples/s through FFT+LS+demod, % HBM peak; BER/NMSE at 20 dB vs plain",
        "value": value,
        "unit": "antenna-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_ant": cfg.n_ant, "fft_len": cfg.fft_len, "cp_len": cfg.cp_len,
                   "n_sym": cfg.n_sym, "n_used": cfg.n_used, "bits_per_sym": cfg.bits_per_sym,
                   "n_slots": S, "combiner": "mrc", "input": "int16 IQ resident in HBM"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "alu_view": alu_view,
        "path_algorithmic_GBps": round(path_gbs, 1),
        "path_hbm_frac": round(path_gbs / HBM_PEAK_GBS, 4),
        "path_copy_frac": round(path_gbs / copy_gbs, 4),
        "step_ms_median": round(statistics.median(step_ms), 5),
        "step_ms_min": round(min(step_ms), 5),
        "step_ms_p90": round(sorted(step_ms)[int(0.9 * (len(step_ms) - 1))], 5),
        "step_ms_max": round(max(step_ms), 5),
        "events_per_step": 2,
        "warmup_ms": round(settle_ms, 1),
        "warmup_settle_steps": settle_steps,
        "lead_in_steps": n_lead,
        "estimate_ms": round(est_ms, 5),
        "demod_ms": round(dem_ms, 5),
        "demod_ms_median": round(statistics.median(dem_each), 5),
        "process_frame_ms_per_step": round(process_ms, 5),
        "h2d_ms_pinned": round(h2d_ms, 3),
        "h2d_inclusive_antenna_samples_per_s": samples_per_step / ((ms_per_step + h2d_ms) * 1e-3),
        "quality_20db": quality,
        "kernel_hash": kernel_hash("path"), "library_hash": kernel_hash(),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
