#!/usr/bin/env python3
"""Benchmark of the spectrometer hot path on one MI355X.

One step = one whole integration of the paper-shaped workload: reset, accumulate 61 frames of two int8
streams (16 Msps, 2^18-point frames: 0.999424 s of data), then calibrated Stokes.  Inputs are resident in
HBM before timing starts; each step integrates a different second of data from a ring of copies (larger
than the last-level cache) into its own output, and the steps run as a replayed hipGraph of the streaming
loop (--no-graph: eager launches).  Prints one JSON line with the throughput (input Gsamples/s), the
real-time factor, the per-kernel roofline of the dominant kernel (timed live with hipEvents on the plan's
stream), the other forms' sections, and the FP64 CPU oracle timed on the host on a bounded sample of the
same workload.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
  python bench.py --copy-probe BYTES   # plain device copy, for calibrating HBM byte counters
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "input Gsamples/s (×real-time) FFT+Stokes at 2^18 pts; fwd+bwd vs plain"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3
MFMA_16BIT_PEAK_TFLOPS = 2500.0  # dense FP16 / BF16 matrix-core peak, published
SAMPLE_RATE = 16e6             # per stream


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true", help="skip the 16-bit precision-form section")
    ap.add_argument("--no-batching", action="store_true", help="skip the 64-instance batching section")
    ap.add_argument("--ring", type=int, default=24, help="distinct input buffers cycled through by the steps")
    ap.add_argument("--no-graph", action="store_true", help="time the headline with eager launches only")
    ap.add_argument("--depth", type=int, default=2,
                    help="integrations in flight: plans, each on its own stream, taking integrations in turn")
    ap.add_argument("--warmup-ms", type=float, default=150.0,
                    help="sustained untimed integrations before the timed region (after the W warm-up steps)")
    ap.add_argument("--separate", action="store_true",
                    help="headline as ps_accumulate then ps_stokes (default: the one-call ps_accumulate_stokes)")
    ap.add_argument("--main-only", action="store_true",
                    help="only the headline workload (for profiler runs): no other sections, no CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=6.0, help="minimum oracle time (whole integrations)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES")
    ap.add_argument("--only", choices=["short_transforms", "long_transforms", "post_reduction", "table1_modes",
                                       "overlap_form", "fwd_bwd", "precision_form", "batching_form"],
                    help="run one further section alone and print it (for profiler runs)")
    return ap.parse_args()


def copy_probe(nbytes: int, steps: int):
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(json.dumps({"copy_probe_bytes": nbytes, "read_bytes": nbytes, "write_bytes": nbytes,
                      "ms": dt * 1e3, "GBps_read_plus_write": 2 * nbytes / dt / 1e9}), flush=True)


def kernel_bytes(kind: str, inst: dict, frames: int) -> float:
    """Algorithmic HBM bytes of one launch of a kernel kind over `frames` frames."""
    N, S, P, b = inst["fft_len"], inst["n_streams"], len(inst["pairs"]), inst["bits"]
    C = N // 2
    if kind == "colpass":   # packed input once + FP32 complex intermediate written once
        win = 0 if inst["window"] == "rect" else N * 4
        return frames * N * S * b / 8 + frames * P * N * 8 + win
    if kind == "rowpass":   # intermediate read once + FP64 accumulators written (first call: no read)
        return frames * P * N * 8 + P * C * 32
    if kind == "rowpass_stokes":  # the row pass with the Stokes epilogue: also writes FP32 I, Q, U, V
        return frames * P * N * 8 + P * C * 32 + P * C * 16
    if kind == "stokes":    # FP64 accumulators read + FP32 I, Q, U, V written
        return P * C * 32 + P * C * 16
    if kind == "spectra":
        return P * C * 32 * 2
    return float("nan")


# the plain path's device code: the counter record is valid only for these exact sources
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1412_1256_amd", "csrc", f) for f in
                  ("polaris_kernels.hip", "polaris_device.h", "polaris_internal.h")]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_paper_2e18.txt")
KIND_OF = {"k_colpass": "colpass", "k_rowpass": "rowpass", "k_rowpass_stokes": "rowpass", "k_output": "stokes"}


def counter_traffic() -> dict:
    """HBM bytes per launch from the committed counter record, if it was taken on the current kernel source."""
    import hashlib
    if not os.path.exists(TRAFFIC_RECORD):
        return {}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    sha = h.hexdigest()
    out, rec_sha = {}, None
    for line in open(TRAFFIC_RECORD):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "source_sha256":
            rec_sha = f[1]
        elif f[0] == "kernel":
            name = line.split("kernel ", 1)[1].split(" fetch_kib")[0]
            vals = dict(zip(f[-12::2], f[-11::2]))
            out[KIND_OF.get(name.split("<")[0], name)] = float(vals["traffic_bytes"])
    return out if rec_sha == sha else {}


def cpu_baseline(inst: dict, min_seconds: float):
    """The FP64 oracle on the host: the paper-shaped integration (the headline workload) on all threads (up to
    16) and on one, and the other configurations: the tiny case, the differentiation case (forward + analytic
    gradient), and bounded subsets of the precision case (1 s of its 10 s) and of the batching case (frames
    capped at 16 per instance), each extrapolated linearly in frames to the whole configuration."""
    import numpy as np

    import oracle
    import synth
    threads = min(16, os.cpu_count() or 1)

    def run(fn, min_s, max_reps=10 ** 6, warm=True):
        if warm:
            fn()  # untimed: builds/loads the oracle and touches the data
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_s or reps >= max_reps:
                return dt / reps

    def integrate(d, nt, psi=0.25):
        acc, nf, s2, _ = oracle.run_instance(d, nthreads=nt)
        oracle.stokes(acc, nf, s2, psi=psi)

    def entry(samples, seconds_of_data, t, nt, sample):
        return {"Gsamples_per_s": samples / t / 1e9, "x_realtime": seconds_of_data / t, "seconds_per_integration": t,
                "threads": nt, "sample": sample}

    n2 = inst["n_samples"] * inst["n_streams"]
    sec2 = inst["n_samples"] / SAMPLE_RATE
    t_all = run(lambda: integrate(inst, threads), min_seconds)
    t_one = run(lambda: integrate(inst, 1), 0.0, max_reps=1, warm=False)
    out = {"value": n2 / t_all / 1e9, "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
           "sample": f"whole integrations of the paper-shaped workload ({inst['n_frames']} frames of 2 x 2^18 int8 "
                     f"samples), FP64 radix-2 oracle incl. Stokes, repeated for >= {min_seconds:g} s on {threads} "
                     "threads",
           "x_realtime": sec2 / t_all,
           "one_core": entry(n2, sec2, t_one, 1, "one whole integration on one thread")}
    cfg = {}
    tiny = synth.make_tiny()
    nt_ = tiny["n_samples"] * tiny["n_streams"]
    cfg["tiny"] = {"all_threads": entry(nt_, tiny["n_samples"] / SAMPLE_RATE, run(lambda: integrate(tiny, threads), 0.5),
                                        threads, "whole integrations (2 x 2-bit, 1024-pt Hann frames, 64 frames)"),
                   "one_core": entry(nt_, tiny["n_samples"] / SAMPLE_RATE, run(lambda: integrate(tiny, 1), 0.5), 1,
                                     "whole integrations")}
    dif = synth.make_differentiation()
    N5, C5 = dif["fft_len"], dif["fft_len"] // 2
    rng = np.random.default_rng(5)
    g = rng.standard_normal((1, 4, C5))
    gx = dif["init_gain_x"][None].astype(np.complex128)
    gy = dif["init_gain_y"][None].astype(np.complex128)
    taps = np.ones(64)

    def fwd_bwd():
        w, s2 = oracle.window("taps", N5, taps=taps)
        acc, nf = oracle.accumulate(dif["packed"], 8, 2, dif["n_samples"], N5, w, dif["pairs"], nthreads=threads)
        oracle.stokes(acc, nf, s2, gain_x=gx, gain_y=gy, dterms=np.zeros((1, 2)))
        oracle.calibrate_backward(dif["packed"], 8, 2, dif["n_samples"], N5, w, dif["pairs"], acc, nf, s2, g,
                                  gain_x=gx, gain_y=gy, dterms=np.zeros((1, 2)), taps=taps, nthreads=threads)
    n5 = dif["n_samples"] * 2
    cfg["differentiation_fwd_bwd"] = entry(n5, dif["n_samples"] / SAMPLE_RATE, run(fwd_bwd, 1.0), threads,
                                           "forward (64-tap window, integration, calibrated Stokes) + analytic "
                                           "gradient of gains, leakage and taps, 2 x int8, 2^16 pts, 128 frames")
    # the oracle's cost does not depend on the sample values: random codes of each configuration's format
    rb = np.random.default_rng(14121256)
    N3, F3 = 1 << 18, 61
    d3 = dict(packed=rb.integers(0, 256, F3 * N3 * 4, dtype=np.uint8), bits=8, n_streams=4, fft_len=N3, n_frames=F3,
              n_samples=F3 * N3, window="rect", pairs=[(0, 2), (1, 3)])
    t3 = run(lambda: integrate(d3, threads), 1.0)
    e3 = entry(4 * F3 * N3, F3 * N3 / SAMPLE_RATE, t3, threads, "1 s (61 frames) of the precision case's 4 int8 "
               "streams, 2 pairs, FP64 (the oracle has no 16-bit form)")
    e3["extrapolated_seconds_per_10s_integration"] = t3 * 610 / 61
    cfg["precision_1s_subset"] = e3
    e, F, bits, _ = synth.batching_params()
    t4_sub, t4_full, s4_sub, s4_full = 0.0, 0.0, 0, 0
    for ei, Fi, bi in zip(e, F, bits):
        Ni, Fc = 1 << int(ei), min(int(Fi), 16)
        di = dict(packed=rb.integers(0, 256, Fc * Ni * 2 * int(bi) // 8, dtype=np.uint8), bits=int(bi), n_streams=2,
                  fft_len=Ni, n_frames=Fc, n_samples=Fc * Ni, window="rect", pairs=[(0, 1)])
        ti = run(lambda: integrate(di, threads, psi=0.0), 0.0, max_reps=1, warm=False)
        t4_sub += ti
        t4_full += ti * int(Fi) / Fc
        s4_sub += 2 * Fc * Ni
        s4_full += 2 * int(Fi) * Ni
    cfg["batching_F16_subset"] = {"Gsamples_per_s": s4_sub / t4_sub / 1e9, "seconds": t4_sub, "threads": threads,
                                  "extrapolated_seconds_per_integration": t4_full,
                                  "extrapolated_Gsamples_per_s": s4_full / t4_full / 1e9,
                                  "sample": "the 64 instances (2^12 .. 2^20 pts, 2/8-bit) with frames capped at 16, "
                                            "each timed once; whole-set time scaled per instance by F / min(F, 16)"}
    out["configs"] = cfg
    return out


def time_steps(torch, dev, fn, steps, warmup, warmup_s=0.05):
    """seconds per call of fn over `steps` calls, after `warmup` calls and at least warmup_s of them"""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize(dev)
    t_end = time.perf_counter() + warmup_s
    while time.perf_counter() < t_end:
        fn()
        torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize(dev)
    return (time.perf_counter() - t0) / steps


_PIPE = []


def pipe_streams(torch, dev, n=2):
    """The streams that take turns in every two-in-flight measurement, created once per process: streams
    taken afresh from the runtime's pool may share a hardware queue, which runs their kernels one after the
    other and hides the overlap being measured."""
    while len(_PIPE) < n:
        _PIPE.append(torch.cuda.Stream(dev))
    return _PIPE[:n]


def pipelined_time(torch, dev, plans, run_on, steps, warmup_s=0.05):
    """Seconds per integration with len(plans) integrations in flight: integration i is run_on(plans[i % d], i),
    enqueued on that plan's own stream (each plan holds its own workspace, so one integration's column pass
    overlaps the previous one's row pass)."""
    d = len(plans)

    def run(n):
        for i in range(n):
            run_on(plans[i % d], i)

    run(2 * d)
    torch.cuda.synchronize(dev)
    t_end = time.perf_counter() + warmup_s
    while time.perf_counter() < t_end:
        run(2 * d)
        torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize(dev)
    return (time.perf_counter() - t0) / steps


def differentiation_form(pk, torch, dev, steps, warmup):
    """fwd+bwd vs plain on the differentiation workload: 2 int8 pols, 2^16-point frames, 128 frames, learnable
    per-channel gains, leakage terms and a 64-tap window.  The backward takes the column-pass output the
    forward left in the inter-pass buffer (one accumulate call); fwd_bwd_recompute_us accumulates the same
    frames in two calls, so the backward transforms every frame again."""
    import numpy as np
    import synth
    inst = synth.make_differentiation()
    N, F, S = inst["fft_len"], inst["n_frames"], inst["n_streams"]
    samples = F * N * S
    packed = torch.from_numpy(inst["packed"]).to(dev)
    gx = torch.from_numpy(inst["init_gain_x"].astype(np.complex64)[None]).to(dev)
    gy = torch.from_numpy(inst["init_gain_y"].astype(np.complex64)[None]).to(dev)
    dt = torch.zeros((1, 2), dtype=torch.complex64, device=dev)
    taps = torch.ones(64, dtype=torch.float32, device=dev)
    g = torch.randn((1, 4, N // 2), dtype=torch.float32, device=dev, generator=torch.Generator(dev).manual_seed(5))
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    plain = pk.Plan([pk.Instance(fft_len=N, bits=8)], device=dev)
    out = torch.empty((1, 4, N // 2), dtype=torch.float32, device=dev)

    def plain_step():
        plain.reset()
        plain.accumulate(packed)
        plain.stokes(out=out)

    def fwd():
        plan.set_window_taps(taps)
        plan.reset()
        plan.accumulate(packed)
        plan.stokes(gain_x=gx, gain_y=gy, dterms=dt, out=out)

    def fwd_bwd():
        fwd()
        plan.calibrate_backward(packed, g, gain_x=gx, gain_y=gy, dterms=dt)

    cut = (F // 2) * N * S * inst["bits"] // 8

    def fwd_bwd_recompute():
        plan.set_window_taps(taps)
        plan.reset()
        plan.accumulate(packed[:cut])
        plan.accumulate(packed[cut:])
        plan.stokes(gain_x=gx, gain_y=gy, dterms=dt, out=out)
        plan.calibrate_backward(packed, g, gain_x=gx, gain_y=gy, dterms=dt)

    t_plain = time_steps(torch, dev, plain_step, steps, warmup)
    t_fwd = time_steps(torch, dev, fwd, steps, warmup)
    t_fb = time_steps(torch, dev, fwd_bwd, steps, warmup)
    t_fbr = time_steps(torch, dev, fwd_bwd_recompute, steps, warmup)
    # the backward alone (forward + backward less the forward) against its algorithmic bytes: the adjoint row
    # pass reads the inter-pass buffer and writes its adjoint (8 + 8 B per complex point), the adjoint column
    # pass reads that and the packed samples once (8 + S bits/8 B), and the channel adjoint reads the FP64
    # accumulators and the upstream gradient and writes the per-channel terms (32 + 16 + 16 B per channel)
    t_bwd = t_fb - t_fwd
    bwd_bytes = F * N * (8 + 8 + 8) + F * N * S * inst["bits"] / 8 + (N // 2) * (32 + 16 + 16)
    return {"workload": "2 int8 pols, 2^16-pt frames, 128 frames (0.524 s), learnable gains, leakage and 64 taps",
            "plain_us": t_plain * 1e6, "fwd_us": t_fwd * 1e6, "fwd_bwd_us": t_fb * 1e6,
            "bwd_us": t_bwd * 1e6, "bwd_alg_bytes": bwd_bytes, "bwd_GBps": bwd_bytes / t_bwd / 1e9,
            "bwd_frac_hbm": bwd_bytes / t_bwd / 1e9 / HBM_PEAK_GBS,
            "fwd_bwd_recompute_us": t_fbr * 1e6, "fwd_bwd_recompute_vs_fwd": t_fbr / t_fwd,
            "fwd_bwd_vs_plain": t_fb / t_plain, "fwd_bwd_vs_fwd": t_fb / t_fwd,
            "fwd_bwd_Gsamples_per_s": samples / t_fb / 1e9, "fwd_bwd_x_realtime": F * N / SAMPLE_RATE / t_fb}


def kernel_bytes_mx(kind: str, inst: dict, frames: int) -> float:
    """Algorithmic HBM bytes of one launch of a precision-form kernel (16-bit complex intermediate)."""
    N, S, P, b = inst["fft_len"], inst["n_streams"], len(inst["pairs"]), inst["bits"]
    C = N // 2
    if kind == "colpass":   # packed input once + 16-bit complex intermediate written once
        return frames * N * S * b / 8 + frames * P * N * 4
    if kind == "rowpass":   # intermediate read once + FP64 accumulators read and written
        return frames * P * N * 4 + 2 * P * C * 32
    return kernel_bytes(kind, inst, frames)


def precision_form(pk, torch, dev, steps, warmup, with_oracle=True):
    """Plain FP32 path vs the 16-bit matrix-core passes (compensated FP32 integration) on the precision
    workload: 4 int8 streams (X0, X1, Y0, Y1; pairs (0,2), (1,3)), 2^18-point frames, 610 frames (9.99 s).
    Error of each Stokes product against the FP64 oracle: max_k |P - P_ref| / I_ref,k."""
    import numpy as np
    import oracle
    import synth
    inst = synth.make_precision(n_frames=610)
    N, S, F, P = inst["fft_len"], inst["n_streams"], inst["n_frames"], len(inst["pairs"])
    samples = F * N * S
    packed = torch.from_numpy(inst["packed"]).to(dev)
    ref = None
    if with_oracle:
        acc, nf, s2, _ = oracle.run_instance(inst, nthreads=min(16, os.cpu_count() or 1))
        ref = oracle.stokes(acc, nf, s2)
    res = {"workload": "4 int8 streams (2 bands x 2 pols), 2^18-pt rect frames, 610 frames (9.99 s), Stokes of "
                       "pairs (0,2), (1,3)", "samples_per_step": samples}
    out = torch.empty((P, 4, N // 2), dtype=torch.float32, device=dev)
    packed2 = packed.clone()
    for prec, accum in (("fp32", "fp64"), ("fp16", "kahan32"), ("bf16", "kahan32")):
        plan = pk.Plan([pk.Instance.from_synth(inst, precision=prec, accum=accum, chunk_frames=128)], device=dev)

        def step():
            plan.reset()
            plan.accumulate(packed)
            plan.stokes(out=out)

        t = time_steps(torch, dev, step, steps, warmup)
        plan.profile_enable(True)
        for _ in range(2):
            step()
        torch.cuda.synchronize(dev)
        prof = plan.profile_read()
        plan.profile_enable(False)
        kb = kernel_bytes if prec == "fp32" else kernel_bytes_mx
        kern = {}
        for k, (ms, n) in prof.items():
            # algorithmic bytes of the whole step; the passes run once per chunk of 128 frames
            nbytes = kb(k, inst, F)
            if k == "rowpass":
                nbytes = F * P * N * (8 if prec == "fp32" else 4) + (n / 2) * 2 * P * (N // 2) * 32
            kern[k] = {"us_per_step": ms / 2 * 1e3, "launches_per_step": n / 2,
                       "GBps": nbytes / (ms / 2 / 1e3) / 1e9}
        r = {"us_per_step": t * 1e6, "Gsamples_per_s": samples / t / 1e9, "x_realtime": F * N / SAMPLE_RATE / t,
             "path_GBps": (kb("colpass", inst, F) + kb("rowpass", inst, F) + P * (N // 2) * 48) / t / 1e9,
             "kernels": kern}
        if prec != "fp32":
            # matrix-core work actually issued: N / 16 products of 16 x 16 x 32 (hi and lo parts of the DFT
            # matrices both counted) per frame and pair, 2 x 16 x 16 x 32 flops each
            mf = 1024.0 * N * F * P / t / 1e12
            r["mfma_tflops"] = mf
            r["mfma_frac_dense_peak"] = mf / MFMA_16BIT_PEAK_TFLOPS
        if ref is not None:
            got = out.cpu().numpy().astype(np.float64)
            e = np.max(np.abs(got - ref) / ref[:, 0:1, :], axis=2)
            r["err_vs_oracle_IQUV"] = [float(v) for v in e.max(axis=0)]
        res[f"{prec}_{accum}"] = r
        del plan
    # two integrations in flight: two plans, each on its own stream with its own copy of the input and its own
    # output, take the integrations in turn (timed after every single-plan case, each with fresh plans)
    outs2 = [out, torch.empty_like(out)]
    bufs = [packed, packed2]
    for prec, accum in (("fp16", "kahan32"), ("bf16", "kahan32"), ("fp32", "fp64")):
        streams = pipe_streams(torch, dev)
        plans2 = [pk.Plan([pk.Instance.from_synth(inst, precision=prec, accum=accum, chunk_frames=128)],
                          device=dev, stream=st) for st in streams]

        def run_on(pl, i):
            pl.reset()
            pl.accumulate(bufs[i % 2])
            pl.stokes(out=outs2[i % 2])

        t2 = pipelined_time(torch, dev, plans2, run_on, max(4, 2 * steps), warmup_s=0.2)
        kb = kernel_bytes if prec == "fp32" else kernel_bytes_mx
        d2 = {"us_per_step": t2 * 1e6, "Gsamples_per_s": samples / t2 / 1e9, "x_realtime": F * N / SAMPLE_RATE / t2,
              "path_GBps": (kb("colpass", inst, F) + kb("rowpass", inst, F) + P * (N // 2) * 48) / t2 / 1e9}
        if prec != "fp32":
            d2["mfma_tflops"] = 1024.0 * N * F * P / t2 / 1e12
            d2["mfma_frac_dense_peak"] = d2["mfma_tflops"] / MFMA_16BIT_PEAK_TFLOPS
        res[f"{prec}_{accum}"]["depth2"] = d2
        torch.cuda.synchronize(dev)
        del plans2
    return res


def batching_form(pk, torch, dev, reps):
    """Batching workload: 64 uneven instances (N = 2^12 .. 2^20, 8 .. 256 frames, 2- or 8-bit, one X/Y pair
    each).  One integration of all of them as 64 separate plans, as one plan (grouped persistent launches,
    one Stokes launch), and as that plan's captured hipGraph replayed.  The input of each instance is its own
    device buffer, filled by repeating a block of quantised correlated noise of its format (the kernels'
    cost does not depend on the values)."""
    import numpy as np
    import synth
    e, F, bits, rho = synth.batching_params(64)
    pool = {}
    for b in (2, 8):
        d = synth.make_correlated_noise(int(b), 0.25, 1 << 16, 32, seed_extra=int(b))
        pool[int(b)] = torch.from_numpy(d["packed"]).to(dev)
    insts, packed = [], []
    for i in range(64):
        N, Fi, b = 1 << int(e[i]), int(F[i]), int(bits[i])
        nbytes = Fi * N * 2 * b // 8
        src = pool[b]
        buf = src.repeat((nbytes + src.numel() - 1) // src.numel())[:nbytes].clone()
        insts.append(pk.Instance(fft_len=N, bits=b))
        packed.append(buf)
    samples = int(sum(int(F[i]) * (1 << int(e[i])) * 2 for i in range(64)))
    outs = [torch.empty((1, 4, I.channels), dtype=torch.float32, device=dev) for I in insts]
    side, side2 = pipe_streams(torch, dev)
    with torch.cuda.stream(side):
        sep = [pk.Plan([I], device=dev, stream=side) for I in insts]
        grp = pk.Plan(insts, device=dev, stream=side)
    side.synchronize()

    def run_separate():
        for p, buf, o in zip(sep, packed, outs):
            p.reset()
            p.accumulate(buf)
            p.stokes(out=o)

    def run_grouped():
        grp.reset()
        grp.accumulate(packed)
        grp.stokes_all(outs)

    def timed(fn):
        with torch.cuda.stream(side):
            for _ in range(2):
                fn()
            side.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            side.synchronize()
        return (time.perf_counter() - t0) / reps

    t_sep = timed(run_separate)
    t_grp = timed(run_grouped)
    grp.graph_capture(run_grouped)
    t_graph = timed(grp.graph_replay)
    # two integrations in flight: a second grouped plan on its own stream, with its own copies of the inputs
    # and outputs, replays its own graph; the two graphs alternate
    with torch.cuda.stream(side2):
        packed2 = [b.clone() for b in packed]
        outs2 = [torch.empty_like(o) for o in outs]
        grp2 = pk.Plan(insts, device=dev, stream=side2)
    side2.synchronize()

    def run_grouped2():
        grp2.reset()
        grp2.accumulate(packed2)
        grp2.stokes_all(outs2)

    grp2.graph_capture(run_grouped2)
    t_graph2 = pipelined_time(torch, dev, [grp, grp2], lambda pl, i: pl.graph_replay(), 2 * reps)
    del grp, grp2, packed2, outs2
    # the same with every instance on its autotuned schedule (tuned alone, one shape at a time)
    from paper_1412_1256_amd import autotune
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "polaris_bench_batch_tune.json")
    t0 = time.perf_counter()
    scheds = [autotune.tune(I, device=dev, reps=3, cache=cache)[0] for I in insts]
    tune_s = time.perf_counter() - t0
    with torch.cuda.stream(side):
        tuned = pk.Plan(insts, device=dev, stream=side, schedules=scheds)
    side.synchronize()

    def run_tuned():
        tuned.reset()
        tuned.accumulate(packed)
        tuned.stokes_all(outs)

    tuned.graph_capture(run_tuned)
    t_tuned = timed(tuned.graph_replay)
    return {"workload": "64 instances, N = 2^12..2^20, 8..256 frames, 2/8-bit, one X/Y pair each",
            "samples_per_integration": samples, "separate_plans_us": t_sep * 1e6, "grouped_us": t_grp * 1e6,
            "grouped_graph_us": t_graph * 1e6, "grouped_graph_tuned_us": t_tuned * 1e6,
            "Gsamples_per_s_grouped_graph": samples / t_graph / 1e9,
            "grouped_graph_depth2_us": t_graph2 * 1e6,
            "Gsamples_per_s_grouped_graph_depth2": samples / t_graph2 / 1e9,
            "Gsamples_per_s_grouped_graph_tuned": samples / t_tuned / 1e9,
            "x_realtime_tuned": samples / 2 / SAMPLE_RATE / t_tuned,
            "speedup_grouped_vs_separate": t_sep / t_grp, "speedup_graph_vs_separate": t_sep / t_graph,
            "speedup_tuned_vs_separate": t_sep / t_tuned, "tuning_seconds": tune_s,
            "launches_separate": 64 * 3, "n_instances": 64}


def autotune_form(pk, torch, dev, inst, packed, steps):
    """The paper workload with the default schedule and with the autotuner's choice (timed on this device)."""
    from paper_1412_1256_amd import autotune
    I = pk.Instance.from_synth(inst)
    best, timings = autotune.tune(I, device=dev, frames=inst["n_frames"], reps=5, cache=os.path.join(
        os.environ.get("TMPDIR", "/tmp"), "polaris_bench_tune.json"), force=True)
    res = {"candidates": len(timings), "best": best.__dict__}
    for name, sched in (("default", None), ("tuned", best)):
        plan = pk.Plan([I], device=dev, schedules=None if sched is None else [sched])
        out = torch.empty((1, 4, I.channels), dtype=torch.float32, device=dev)

        def step():
            plan.reset()
            plan.accumulate(packed)
            plan.stokes(psi=0.25, out=out)

        res[f"{name}_us"] = time_steps(torch, dev, step, steps, 3) * 1e6
    return res


def power_form(pk, torch, dev, inst, packed, steps):
    """Level histograms counted inside the column pass (total power, the paper's bit-distribution method):
    the paper workload's whole integration and column pass with counting off and on, and the estimates."""
    res = {}
    for on in (False, True):
        plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
        plan.set_histograms(on)
        out = torch.empty((1, 4, inst["fft_len"] // 2), dtype=torch.float32, device=dev)

        def step():
            plan.reset()
            plan.accumulate(packed)
            plan.stokes(out=out)

        t = time_steps(torch, dev, step, steps, 3)
        plan.profile_enable(True)
        for _ in range(steps):
            step()
        prof = plan.profile_read()
        plan.profile_enable(False)
        key = "on" if on else "off"
        res[f"{key}_us"] = t * 1e6
        res[f"colpass_{key}_us"] = prof["colpass"][0] / prof["colpass"][1] * 1e3
        if on:
            counts, power, nf = plan.histograms()
            res["mean_square_level_XY"] = [float(v) for v in power[0, :, 0].cpu()]
            res["frames_counted"] = nf
    res["colpass_overhead"] = res["colpass_on_us"] / res["colpass_off_us"] - 1.0
    return res


def _ring_integrations(pk, torch, dev, inst, ring, steps, warmup=3):
    """Whole integrations (reset, accumulate, Stokes of every pair) of an instance, each from the next
    HBM-resident buffer of a ring; returns the mean time per integration and per-kernel averages."""
    side, st2 = pipe_streams(torch, dev)
    with torch.cuda.stream(side):
        plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev, stream=side)
        out = torch.empty((len(inst["pairs"]), 4, inst["fft_len"] // 2), dtype=torch.float32, device=dev)
    pos = [0]

    def step():
        buf = ring[pos[0] % len(ring)]
        pos[0] += 1
        plan.reset()
        plan.accumulate(buf)
        plan.stokes(psi=0.25, out=out)

    with torch.cuda.stream(side):
        t = time_steps(torch, dev, step, steps, warmup)
        plan.profile_enable(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize(dev)
    prof = plan.profile_read()
    plan.profile_enable(False)
    kern = {k: {"launches": n / steps, "avg_us": ms / n * 1e3} for k, (ms, n) in prof.items()}
    # two integrations in flight (a second plan on its own stream with its own output takes every other one)
    with torch.cuda.stream(st2):
        plan2 = pk.Plan([pk.Instance.from_synth(inst)], device=dev, stream=st2)
        out2 = torch.empty_like(out)
    st2.synchronize()

    def run_on(pl, i):
        pl.reset()
        pl.accumulate(ring[i % len(ring)])
        pl.stokes(psi=0.25, out=out if pl is plan else out2)

    kern["depth2_us"] = pipelined_time(torch, dev, [plan, plan2], run_on, max(4, steps)) * 1e6
    del plan2
    return t, kern, plan


def overlap_form(pk, torch, dev, inst, ring, steps):
    """The paper workload (2 int8 streams, 2^18 points, 0.999 s of data) with 50 % overlapped frames and
    a Hamming window (Sec. 3.1), against contiguous rectangular frames, on the same streamed input."""
    N = inst["fft_len"]
    res = {}
    for name, hop, window in (("contiguous_rect", N, "rect"), ("half_overlap_hamming", N // 2, "hamming")):
        d = dict(inst, hop=hop, window=window)
        t, kern, plan = _ring_integrations(pk, torch, dev, d, ring, steps)
        frames = (inst["n_samples"] - N) // hop + 1
        r = {"frames": frames, "us": t * 1e6, "Gsamples_per_s": inst["n_samples"] * 2 / t / 1e9,
             "frames_per_s": frames / t, "x_realtime": inst["n_samples"] / SAMPLE_RATE / t}
        for k in ("colpass", "rowpass", "stokes"):
            if k in kern:
                r[f"{k}_us"] = kern[k]["avg_us"]
                r[f"{k}_launches"] = kern[k]["launches"]
        r["depth2_us"] = kern["depth2_us"]
        r["depth2_Gsamples_per_s"] = inst["n_samples"] * 2 / (kern["depth2_us"] * 1e-6) / 1e9
        # column pass: each frame's input bytes (overlapped samples are read by both frames) + intermediate
        cp = kernel_bytes("colpass", d, frames)
        r["colpass_GBps_frame_bytes"] = cp / (r["colpass_us"] * 1e-6) / 1e9 if "colpass_us" in r else None
        res[name] = r
    res["time_ratio"] = res["half_overlap_hamming"]["us"] / res["contiguous_rect"]["us"]
    return res


def modes_form(pk, torch, dev, steps, ring_n):
    """Table 1's two sampler modes with all four IFs, one second of data per integration: 8 MHz (16 Msps,
    4-bit, 2^18 points) and 4 MHz (8 Msps, 8-bit, 2^17 points), each from a ring of HBM-resident buffers."""
    import synth
    res = {}
    for mode in ("8MHz", "4MHz"):
        d = synth.make_mode(mode, n_frames=61)
        packed = torch.from_numpy(d["packed"]).to(dev)
        ring = [packed] + [packed.clone() for _ in range(max(1, ring_n) - 1)]
        t, kern, _ = _ring_integrations(pk, torch, dev, d, ring, steps)
        seconds = d["n_samples"] / d["sample_rate_hz"]
        res[mode] = {"bits": d["bits"], "fft_len": d["fft_len"], "n_streams": 4, "frames": d["n_frames"],
                     "data_seconds": seconds, "us": t * 1e6,
                     "Gsamples_per_s": d["n_samples"] * 4 / t / 1e9, "x_realtime": seconds / t,
                     "depth2_us": kern["depth2_us"],
                     "depth2_Gsamples_per_s": d["n_samples"] * 4 / (kern["depth2_us"] * 1e-6) / 1e9,
                     "kernels_us": {k: v["avg_us"] for k, v in kern.items() if k != "depth2_us"}}
        del ring, packed
    return res


def long_form(pk, torch, dev, steps):
    """Long transforms (two streams, 2- and 8-bit, 2^19 and 2^20 points, 2^25 samples per stream per
    integration, streamed from a ring of HBM-resident buffers larger than the last-level cache): whole
    integrations with one and with two integrations in flight, per-kernel times from the one-plan run."""
    import synth
    res = {}
    for m in (19, 20):
        N = 1 << m
        for bits in (2, 8):
            d = synth.make_correlated_noise(bits, 0.3, N, (1 << 25) // N, seed_extra=m + bits)
            packed = torch.from_numpy(d["packed"]).to(dev)
            ring = [packed] + [packed.clone() for _ in range(max(1, (512 << 20) // packed.numel()) - 1)]
            t, kern, plan = _ring_integrations(pk, torch, dev, d, ring, steps)
            samples = d["n_samples"] * 2
            res[f"2^{m}_{bits}bit"] = {
                "frames": d["n_frames"], "us": t * 1e6, "Gsamples_per_s": samples / t / 1e9,
                "depth2_us": kern["depth2_us"], "depth2_Gsamples_per_s": samples / (kern["depth2_us"] * 1e-6) / 1e9,
                "kernels_us": {k: v["avg_us"] for k, v in kern.items() if k != "depth2_us"}}
            del ring, packed, plan
    return res


def short_form(pk, torch, dev, steps):
    """Short transforms (two int8 streams, 2^24 samples per stream per integration, streamed from a ring of
    HBM-resident buffers): the single pass (whole frames in LDS, up to 2^12 points) against the four-step
    passes, whole integrations including Stokes."""
    import synth
    res = {}
    for m in (8, 10, 12, 14):
        N = 1 << m
        d = synth.make_correlated_noise(8, 0.3, N, (1 << 24) // N, seed_extra=m)
        packed = torch.from_numpy(d["packed"]).to(dev)
        ring = [packed] + [packed.clone() for _ in range(23)]
        r = {}
        for name, sched in (("single_pass", pk.Schedule(single_pass=1)), ("four_step", pk.Schedule(single_pass=2))):
            if name == "single_pass" and m > 12:
                continue
            side = torch.cuda.Stream(dev)
            with torch.cuda.stream(side):
                plan = pk.Plan([pk.Instance.from_synth(d)], device=dev, stream=side, schedules=[sched])
                out = torch.empty((1, 4, N // 2), dtype=torch.float32, device=dev)
            pos = [0]

            def step():
                plan.reset()
                plan.accumulate(ring[pos[0] % len(ring)])
                pos[0] += 1
                plan.stokes(out=out)

            with torch.cuda.stream(side):
                t = time_steps(torch, dev, step, steps, 3)
            r[f"{name}_us"] = t * 1e6
            r[f"{name}_Gsamples_per_s"] = d["n_samples"] * 2 / t / 1e9
        if "single_pass_us" in r:
            r["speedup"] = r["four_step_us"] / r["single_pass_us"]
        res[f"2^{m}"] = r
        del ring, packed
    return res


def post_form(pk, torch, dev, reps):
    """The post-integration reductions at the paper's sizes (time per call: events on the current stream around
    back-to-back calls, so a short reduction shows the binding's call rate; the kernels' own durations come
    from a kernel trace): channel averaging of one integration's Stokes spectra 131072 -> 4096 channels with a flagged
    channel (Sec. 4); the bandpass table of 131072 channels (128-channel knots, 6 % edges) and the variation
    of 30 integrations H^_k = H_k / (G_k H), averaged over 256 channels, with mean and SD (Sec. 3.3.2); the
    TAV (Eq. 3) of every channel over 1800 1-s integrations and the SAV (Eq. 4) of 30 spectra, 8 lags each."""
    g = torch.Generator(device=dev)
    g.manual_seed(1412)
    C = 131072
    stokes = 1 + 0.01 * torch.randn((1, 4, C), generator=g, device=dev)
    flags = torch.zeros(C, dtype=torch.uint8, device=dev)
    flags[C // 2] = 1
    hk = 1 + 0.01 * torch.randn((30, C), generator=g, device=dev)
    gain = torch.linspace(1.0, 1.03, 30, device=dev, dtype=torch.float64)
    series = 1 + 0.01 * torch.randn((1800, C), generator=g, device=dev)
    lags = [1, 2, 4, 8, 16, 64, 256, 512]
    smooth = pk.bandpass_fit(hk[0])
    hat = pk.bandpass_correct(hk, smooth, gain)
    binned = pk.channel_average(hat, 256)[0]
    calls = {
        "channel_average_stokes_32": lambda: pk.channel_average(stokes, 32, flags),
        "bandpass_fit_131072": lambda: pk.bandpass_fit(hk[0], 128, 0.06),
        "bandpass_correct_30x131072": lambda: pk.bandpass_correct(hk, smooth, gain),
        "channel_average_30x131072_256": lambda: pk.channel_average(hat, 256),
        "band_stats_30x512": lambda: pk.band_stats(binned),
        "tav_1800x131072_8lags": lambda: pk.allan(series, lags, spacing=1.0, normalize=True, axis=0),
        "sav_30x131072_8lags": lambda: pk.allan(hat, lags, spacing=SAMPLE_RATE / 2 ** 18, axis=1),
    }
    res = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize(dev)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        res[f"{name}_us"] = a.elapsed_time(b) / reps * 1e3
    res["tav_input_GBps"] = series.numel() * 4 / (res["tav_1800x131072_8lags_us"] * 1e-6) / 1e9
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path: "
              "each GPU would run its own pairs/instances independently (see the sharding notes).", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe, args.steps)
        return

    import torch

    import paper_1412_1256_amd as pk
    import synth

    pk.lib()  # fail loudly when the HIP library is missing
    dev = torch.device("cuda:0")
    if args.only in ("short_transforms", "long_transforms", "post_reduction", "table1_modes", "fwd_bwd",
                     "precision_form", "batching_form"):
        fn = {"short_transforms": lambda: short_form(pk, torch, dev, args.steps),
              "long_transforms": lambda: long_form(pk, torch, dev, args.steps),
              "batching_form": lambda: batching_form(pk, torch, dev, args.steps),
              "post_reduction": lambda: post_form(pk, torch, dev, args.steps),
              "table1_modes": lambda: modes_form(pk, torch, dev, args.steps, args.ring),
              "fwd_bwd": lambda: differentiation_form(pk, torch, dev, args.steps, 2),
              "precision_form": lambda: precision_form(pk, torch, dev, args.steps, 1, with_oracle=False)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    inst = synth.make_paper()
    N, S, F = inst["fft_len"], inst["n_streams"], inst["n_frames"]
    samples = F * N * S
    packed = torch.from_numpy(inst["packed"]).to(dev)
    # streaming: each step integrates a different, HBM-resident second of data (a ring of copies larger
    # than the 256 MB last-level cache) into its own output, so no step finds its input in cache.  `depth`
    # integrations are in flight: integration i runs on plan i mod depth, each plan with its own workspace
    # (inter-pass buffer and accumulators) on its own stream, so one integration's column pass overlaps the
    # previous one's row pass and Stokes output.
    depth = max(1, args.depth)
    streams = pipe_streams(torch, dev, depth)
    side = streams[0]
    with torch.cuda.stream(side):
        ring = [packed.clone() for _ in range(max(1, args.ring))]
        outs = [torch.empty((1, 4, N // 2), dtype=torch.float32, device=dev) for _ in ring]
    plans = []
    for st in streams:
        with torch.cuda.stream(st):
            plans.append(pk.Plan([pk.Instance.from_synth(inst)], device=dev, stream=st))
    torch.cuda.synchronize(dev)
    plan = plans[0]
    if args.only == "overlap_form":
        print(json.dumps({"overlap_form": overlap_form(pk, torch, dev, inst, ring, args.steps)}), flush=True)
        return
    pos = {"i": 0}

    def step_on(pl, i):
        pl.reset()
        if args.separate:
            pl.accumulate(ring[i % len(ring)])
            pl.stokes(psi=0.25, out=outs[i % len(ring)])
        else:
            pl.accumulate_stokes(ring[i % len(ring)], psi=0.25, out=outs[i % len(ring)])

    def step():
        i = pos["i"]
        pos["i"] += 1
        with torch.cuda.stream(side):
            step_on(plan, i)

    def run_eager(n, d):
        """n integrations, integration i on plan i mod d (its own stream)"""
        for i in range(n):
            with torch.cuda.stream(streams[i % d]):
                step_on(plans[i % d], i)

    def timed(fn, n):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) / n

    # warm-up: W integrations, then at least --warmup-ms of the same work (clocks, TLBs and caches reach their
    # steady state only after some tens of milliseconds of sustained integrations)
    run_eager(args.warmup, depth)
    torch.cuda.synchronize(dev)
    t_end = time.perf_counter() + args.warmup_ms / 1e3
    while time.perf_counter() < t_end:
        run_eager(len(ring), depth)
        torch.cuda.synchronize(dev)
    dt_eager = timed(lambda: run_eager(args.steps, depth), args.steps)
    dt_eager_single = timed(lambda: run_eager(args.steps, 1), args.steps)
    dt, dt_graph_single, graph = dt_eager, None, None
    if not args.no_graph:
        # each plan captures its share of exactly K integrations (i = j, j + depth, ... < K) as one hipGraph;
        # the timed region launches every plan's graph on its own stream once
        share = [list(range(j, args.steps, depth)) for j in range(depth)]
        used = [j for j in range(depth) if share[j]]
        for j in used:
            plans[j].graph_capture(lambda j=j: [step_on(plans[j], i) for i in share[j]])

        def replay_all():
            for j in used:
                with torch.cuda.stream(streams[j]):
                    plans[j].graph_replay()
        t_end = time.perf_counter() + args.warmup_ms / 2e3
        while True:
            replay_all()
            torch.cuda.synchronize(dev)
            if time.perf_counter() >= t_end:
                break
        dt = timed(replay_all, args.steps)
        graph = {"depth": depth, "integrations_per_graph": [len(share[j]) for j in used]}
        # reference: all K integrations on one plan and stream, one graph
        plan.graph_capture(lambda: [step_on(plan, i) for i in range(args.steps)])
        with torch.cuda.stream(side):
            plan.graph_replay()
            dt_graph_single = timed(plan.graph_replay, args.steps)

    # per-kernel durations, hipEvents around each launch on the plan's stream (eager steps)
    plan.profile_enable(True)
    torch.cuda.synchronize(dev)
    with torch.cuda.stream(side):
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize(dev)
        dt_prof = (time.perf_counter() - t0) / args.steps
    prof = plan.profile_read()
    plan.profile_enable(False)
    kernels = {}
    # one-call integration: the last row-pass launch of a step also writes the Stokes spectra, and no
    # Stokes pass runs (its accumulator read is not part of the path)
    fused = "stokes" not in prof
    for k, (ms, n) in prof.items():
        avg_s = ms / n / 1e3
        nbytes = kernel_bytes("rowpass_stokes" if fused and k == "rowpass" else k, inst, F)
        kernels[k] = {"launches_per_step": n / args.steps, "avg_us": avg_s * 1e6,
                      "alg_bytes": nbytes, "GBps": nbytes / avg_s / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches_per_step"])
    kd = kernels[dom]
    traffic = counter_traffic()
    roofline = {"kernel": dom, "bound": "hbm", "achieved": kd["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kd["GBps"] / HBM_PEAK_GBS, "traffic": traffic.get(dom), "traffic_unit": "bytes per launch",
                "alg_bytes": kd["alg_bytes"]}

    value = samples / dt / 1e9
    nominal_flop = S * F * 5 * N * math.log2(N)      # 5 N log2 N per N-point real frame per stream
    path_bytes = sum(kernel_bytes(k, inst, F)
                     for k in (("colpass", "rowpass_stokes") if fused else ("colpass", "rowpass", "stokes")))
    out = {
        "metric": METRIC, "value": value, "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper-shaped integration: 2 int8 streams at 16 Msps, 2^18-pt rect frames, "
                               "61 frames (0.999424 s), FP32 passes + FP64 accumulation, Stokes; each step a "
                               f"different HBM-resident second of data (ring of {len(ring)}), "
                               + (f"{depth} integrations in flight (integration i on plan i mod {depth}, each "
                                  "plan with its own workspace and HIP stream), "
                                  + ("eager launches" if graph is None else
                                     "each plan's share of the K integrations replayed as one hipGraph")),
                   "n_streams": S, "bits": 8, "fft_len": N, "frames": F, "samples_per_step": samples},
        "x_realtime": (F * N / SAMPLE_RATE) / dt,
        "fft_tflops_nominal_5NlogN": nominal_flop / dt / 1e12,
        "fft_frac_fp32_peak_nominal": nominal_flop / dt / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
        "fft_tflops_real_2.5NlogN": nominal_flop / 2 / dt / 1e12,
        "fft_frac_fp32_peak_real": nominal_flop / 2 / dt / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
        "path_alg_bytes_per_step": path_bytes,
        "path_GBps": path_bytes / dt / 1e9,
        "path_frac_hbm": path_bytes / dt / 1e9 / HBM_PEAK_GBS,
        "ms_per_step_eager": dt_eager * 1e3,
        "ms_per_step_single_stream_graph": None if dt_graph_single is None else dt_graph_single * 1e3,
        "ms_per_step_single_stream_eager": dt_eager_single * 1e3,
        "pipeline": graph,
        "ms_per_step_with_kernel_events": dt_prof * 1e3,
        "kernels": kernels,
        "roofline": roofline,
    }
    if args.main_only:
        print(json.dumps(out), flush=True)
        return
    out["fwd_bwd"] = differentiation_form(pk, torch, dev, max(5, args.steps // 2), 2)
    out["autotune"] = autotune_form(pk, torch, dev, inst, packed, args.steps)
    out["total_power"] = power_form(pk, torch, dev, inst, packed, max(5, args.steps // 4))
    out["overlap_form"] = overlap_form(pk, torch, dev, inst, ring, max(8, args.steps // 2))
    out["table1_modes"] = modes_form(pk, torch, dev, max(8, args.steps // 2), args.ring)
    out["post_reduction"] = post_form(pk, torch, dev, 10)
    out["short_transforms"] = short_form(pk, torch, dev, max(5, args.steps // 4))
    out["long_transforms"] = long_form(pk, torch, dev, max(5, args.steps // 4))
    if not args.no_batching:
        out["batching_form"] = batching_form(pk, torch, dev, max(3, args.steps // 10))
    if not args.no_precision:
        out["precision_form"] = precision_form(pk, torch, dev, max(3, args.steps // 10), 1,
                                               with_oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
