#!/usr/bin/env python3
"""Benchmark: packed approximate FFT overlap-save convolution on one MI355X.

Workload (default): L = 2^22 samples of synthetic audio (AR(1), a = 0.95, unit-variance white
noise, scaled to [-1, 1]), kernel N = 1024 Hann-windowed sinc low-pass (f_c = 0.125), FFT block
W_block = 4096, per-block packing chosen for a model SNR >= 40 dB (calibrated once at
S_q = K_q = 8).  A step is one pass of the whole path over one input signal; the steps rotate
over distinct device buffers (more than the 256 MB last-level cache holds) so every step reads
its input from HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c2|c1|...] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak
FP32_VECTOR_TFLOPS = 157.3   # MI355X FP32 vector peak

WORKLOADS = {
    "c2": dict(L=1 << 22, N=1024, Wb=4096, snr=40.0, core="fft",
               name="FFT overlap-save convolution: L=2^22 AR(1) audio, N=1024 Hann low-pass, "
                    "W_block=4096, per-block packing for SNR>=40 dB"),
    "c3": dict(name="batched cross-correlation matching: 4096 templates (256..4096 taps, excerpts + 20 dB noise) "
                    "against their 64 AR(1) references (2^18..2^20 samples), one persistent launch, autotuned"),
    "c4": dict(name="filter bank: 256 channels x 2^20 pink-noise samples, 32 Hann band-pass FIRs of N=512, "
                    "split-precision FP16 matrix cores (three products, FP32 accumulation)"),
    "c5": dict(name="serving: Poisson arrivals at 2000 req/s for 10 s, L log-uniform in [2^12, 2^22], N log-uniform "
                    "in [16, 4096] (32 sizes, 128 kernels per size), SNR target in {30, 40, 50} dB, admission by a "
                    "32 GiB HBM budget, resident kernels"),
    "c1sweep": dict(name="time-domain sweep: L=2^22 N(0,1) signal, U(-1,1) kernels N in {64,128,256,512,1024}, "
                         "W_block = max(2N, 1024) + N + 1; symmetric and asymmetric M=2 at the largest S_q=K_q, FP32, "
                         "FP64"),
    "sweep": dict(name="paper sweep (Section IV.A, synthetic): L=2^23, U[-128,128] signal and kernel; block sizes "
                       "W in {2,4,8,16,32,64}x2^10 at N=800, and N in {32..8192} at W=32x2^10; FFT core; symmetric and "
                       "asymmetric M=3 at S_q=K_q=16, asymmetric M=2 at 256 (the paper's settings) and at the largest "
                       "in-bound S_q=K_q; FP32 comparator"),
    "delay": dict(name="two-channel delay and correlation (Section IV.C analogue, synthetic): 90 s of AR(1) audio at "
                       "44.1 kHz, channel b = a delayed by 1..200 samples plus 30 dB noise (stereo) or a itself (mono), "
                       "per 1 s segment; blocks of 50/100/200 ms of b correlated with the same block of a in one "
                       "batched launch; S_q=K_q=32"),
    "calib": dict(name="SNR model calibration study (Section IV.D, Fig. 5 analogue, synthetic): cross-correlation of "
                       "2^20-sample sources with a 1025-sample excerpt, W_block=4096; AR(1) audio with a zero-mean "
                       "Laplacian fit and Weibull(0.248, 1.191) features with a Weibull fit; S_q=K_q from 8 to 256 on "
                       "the integer core; model calibrated once at S_q=K_q=8"),
    "c1": dict(L=65536, N=64, Wb=1024, snr=None, core="td", nsig=1024,
               name="time-domain overlap-save convolution, batch of 1024 signals in one launch: L=65536 N(0,1) each, "
                    "N=64 U(-1,1), W_block=1024, asymmetric M=2 at 8 bits (S_q=K_q=127)"),
}


def fft_flops_per_item(Fw: int) -> float:
    """Algorithmic FLOPs of one FFT-core item: forward and inverse complex FFT of Fw/2 points
    (5 M log2 M each) plus the real-split / spectrum product / merge step (~40 per point pair)."""
    M = Fw // 2
    return 2 * 5.0 * M * math.log2(M) + 40.0 * (M // 2 + 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--bufs", type=int, default=16)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the blocks are independent, so the "
                                   "method would shard by block ranges, but no multi-GPU path is implemented"}))
        sys.exit(2)

    import torch

    from paper_1201_3018_amd import apx, synth

    wl = WORKLOADS[args.workload]
    if args.workload == "c3":
        return bench_c3(args, wl)
    if args.workload == "c4":
        return bench_c4(args, wl)
    if args.workload == "c5":
        return bench_c5(args, wl)
    if args.workload == "c1sweep":
        return bench_c1sweep(args, wl)
    if args.workload == "sweep":
        return bench_sweep(args, wl)
    if args.workload == "delay":
        return bench_delay(args, wl)
    if args.workload == "calib":
        return bench_calib(args, wl)
    if args.workload == "c1":
        return bench_c1(args, wl)
    dev = torch.device("cuda:0")
    L, N, Wb = wl["L"], wl["N"], wl["Wb"]
    if args.workload == "c2":
        s = synth.ar1(L, 2001)
        k = synth.hann_lowpass(N)
    else:
        s = synth.gaussian(L, 1001)
        k = synth.uniform(N, 1002)
    nb = max(1, args.bufs if args.workload == "c2" else 1)
    ts = [torch.from_numpy(s).to(dev) for _ in range(nb)]
    tk = torch.from_numpy(k).to(dev)
    outs = [torch.empty(L + N - 1, dtype=torch.float32, device=dev) for _ in range(nb)]
    ctx = apx.Context(0)
    N_odd, W, P = apx.apx_geometry(L, N, Wb)
    core = apx.APX_CORE_FFT if wl["core"] == "fft" else apx.APX_CORE_TIME

    tuned = None
    if args.workload == "c2":
        # calibrate the SNR model once on this signal, then let the autotuner pick the core and
        # FFT implementation of the packed path and of the FP32 comparator at this shape
        k0 = apx.Kernel(ctx, tk, Wb, mode=apx.APX_AUTO_SNR, core=core, snr_min_db=wl["snr"])
        calib = k0.calibrate(ts[0])
        k0.close()
        tuned = {
            "packed": apx.apx_tune(ctx.h, tk, Wb, apx.params(apx.APX_AUTO_SNR, apx.APX_CORE_AUTO,
                                                              snr_min_db=wl["snr"], calib_db=calib), L_hint=L),
            "full_fp32": apx.apx_tune(ctx.h, tk, Wb, apx.params(apx.APX_FULL_FP32, apx.APX_CORE_AUTO), L_hint=L),
        }
        kern = apx.Kernel(ctx, tk, Wb, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_AUTO, snr_min_db=wl["snr"],
                          calib_db=calib)
        full = apx.Kernel(ctx, tk, Wb, mode=apx.APX_FULL_FP32, core=apx.APX_CORE_AUTO)
    else:
        kern = apx.Kernel(ctx, tk, Wb, mode=apx.APX_ASYM2, core=core, Sq=127, Kq=127)
        calib = None
        full = apx.Kernel(ctx, tk, Wb, mode=apx.APX_FULL_FP32, core=core)
    try:
        ref64 = apx.Kernel(ctx, tk, Wb, mode=apx.APX_FULL_FP64, core=apx.APX_CORE_TIME)
    except apx.ApxError as e:  # FP64 reference path needs more LDS than this device offers
        print(f"# FP64 reference unavailable: {e}", file=sys.stderr)
        ref64 = full

    def timed(kh, steps, warmup):
        """K steps captured in one HIP graph (no host launch gaps), bracketed by events on the
        stream the kernels run on."""
        for i in range(warmup):
            kh.run(ts[i % nb], out=outs[i % nb])
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(steps):
                kh.run(ts[i % nb], out=outs[i % nb])
        g.replay()  # untimed replay: first-touch of the graph
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms per step

    ms_packed = timed(kern, args.steps, args.warmup)
    ms_full = timed(full, args.steps, args.warmup)
    # context: the same path at other SNR targets (lower targets admit the symmetric packing)
    snr_sweep = []
    if args.workload == "c2":
        for target in (20.0, 30.0, 50.0):
            kt = apx.Kernel(ctx, tk, Wb, mode=apx.APX_AUTO_SNR, core=apx.APX_CORE_AUTO, snr_min_db=target, calib_db=calib)
            ms_t = timed(kt, max(1, args.steps // 4), 2)
            _, inf_t = kt.run(ts[0], info=True)
            torch.cuda.synchronize()
            m_t = np.bincount(apx.block_info(inf_t)["mode"], minlength=4)
            snr_sweep.append({"snr_min_db": target, "ms_per_step": ms_t, "over_fp32": ms_full / ms_t,
                              "blocks": {"full_fp32": int(m_t[0]), "sym": int(m_t[1]), "asym2": int(m_t[2])}})
            kt.close()

    # the integer matrix-core core (Tier-2 swap: same companding, exact int8 digit products, no
    # FP64 packing) on the same input, at the fixed modes' largest in-bound S_q = K_q; its outputs
    # are compared with the packed FFT core's
    int8_core = []
    if args.workload == "c2":
        for name, mode, q in (("sym", apx.APX_SYM, 0), ("asym2", apx.APX_ASYM2, 0), ("asym2_8bit", apx.APX_ASYM2, 127)):
            ki = apx.Kernel(ctx, tk, Wb, mode=mode, core=apx.APX_CORE_INT8, Sq=q, Kq=q)
            kf_ = apx.Kernel(ctx, tk, Wb, mode=mode, core=apx.APX_CORE_FFT, Sq=q, Kq=q)
            ms_i = timed(ki, max(1, args.steps // 4), 2)
            ms_f = timed(kf_, max(1, args.steps // 4), 2)
            oi, of_ = ki.run(ts[0]), kf_.run(ts[0])
            torch.cuda.synchronize()
            same = bool(torch.equal(oi, of_))
            int8_core.append({"mode": name, "Sq": q or None, "ms_per_step": ms_i, "fft_core_ms_per_step": ms_f,
                              "int8_over_fft": ms_f / ms_i, "outputs_equal_fft_core": same,
                              "kernel": ki.describe()[:80]})
            ki.close()
            kf_.close()

    # per-call latency as a caller sees it (enqueue + completion), packed path
    lat = []
    for i in range(50):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kern.run(ts[i % nb], out=outs[i % nb])
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)

    # accuracy report: per-block SNR against the FP64 time-domain path
    out_p, info = kern.run(ts[0], info=True)
    out_f = full.run(ts[0])
    out_r = ref64.run(ts[0])
    torch.cuda.synchronize()
    info = apx.block_info(info)
    rp, rf, rr = (x.cpu().numpy().astype(np.float64) for x in (out_p, out_f, out_r))

    def block_snr(r):
        v = []
        for w in range(P):
            o, n = (0, W + N_odd - 1) if w == 0 else (N_odd - 1 + W * w, W)
            n = min(n, rr.size - o)
            e = np.sum((r[o:o + n] - rr[o:o + n]) ** 2)
            v.append(np.inf if e == 0 else 10 * np.log10(np.sum(rr[o:o + n] ** 2) / e))
        return np.array(v)

    snr_p, snr_f = block_snr(rp), block_snr(rf)
    outputs = L + N - 1
    value = outputs / (ms_packed * 1e-3)
    modes = np.bincount(info["mode"], minlength=4)

    # roofline of the dominant kernel (the fused FFT / TD block kernel, one launch per step):
    # compulsory bytes, every input sample read once and every output written once; the window
    # bytes (overlapping windows each read whole) are reported beside them
    bytes_alg = L * 4 + outputs * 4
    bytes_win = P * Wb * 4 + outputs * 4
    achieved_gbs = bytes_alg / (ms_packed * 1e-3) / 1e9
    if args.workload == "c2":
        F = 1 << max(9, int(math.ceil(math.log2(Wb))))
        # blocks by mode: asymmetric / FP32 items use F words, symmetric F/2
        items = P + 1
        fl = 0.0
        for m, cnt in enumerate(modes):
            fw = F // 2 if m == apx.APX_SYM else F
            fl += cnt * fft_flops_per_item(fw)
        fl += fft_flops_per_item(F) * (items - P)
    else:
        fl = 2.0 * outputs * N_odd / 2.0      # asymmetric M=2: N FMAs per packed word (2 outputs)
    achieved_tf = fl / (ms_packed * 1e-3) / 1e12
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    alu_frac = achieved_tf / FP64_VECTOR_TFLOPS
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(achieved_tf, 2), "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4)}
    roof["traffic"] = measured_traffic(args.workload)  # scaled FETCH_SIZE + WRITE_SIZE, bytes/launch
    roof["alt"] = {"hbm_GBs": round(achieved_gbs, 1), "hbm_frac": round(hbm_frac, 4),
                   "fp64_TFLOPs": round(achieved_tf, 2), "fp64_frac": round(alu_frac, 4)}
    roof["alt"]["window_bytes_GBs"] = round(bytes_win / (ms_packed * 1e-3) / 1e9, 1)
    roof["kernel"] = kern.describe()
    roof["bytes_per_launch"] = bytes_alg
    roof["window_bytes_per_launch"] = bytes_win
    roof["flops_per_launch"] = fl

    res = {
        "metric": "output samples/s at fixed SNR (>=40 dB per block), packed vs full-precision FP32, 1 GPU",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_packed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "L": L, "N": N, "W_block": Wb, "blocks": P,
                   "snr_min_db": wl["snr"], "calib_db": calib},
        "roofline": roof,
        "full_fp32": {"value": outputs / (ms_full * 1e-3), "ms_per_step": ms_full,
                      "snr_db_min": float(np.min(snr_f))},
        "packed_over_fp32": ms_full / ms_packed,
        "full_fp32_kernel": full.describe(),
        "modes": {"full_fp32": int(modes[0]), "sym": int(modes[1]), "asym2": int(modes[2])},
        "snr_db": {"min": float(np.min(snr_p)), "mean": float(np.mean(snr_p[np.isfinite(snr_p)]))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
    }
    if tuned:
        res["tuned"] = tuned
    if snr_sweep:
        res["snr_sweep"] = snr_sweep
    if int8_core:
        res["int8_core"] = int8_core
    if args.copy_probe:
        res["copy_probe_bytes"] = copy_probe(dev)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(args.workload, s, k, Wb, wl, calib, outputs)
    print(json.dumps(res), flush=True)
    for kh in {id(x): x for x in (kern, full, ref64)}.values():
        kh.close()
    ctx.close()


def c1_batch(n, L, seed=1001):
    """n distinct N(0,1) signals of L samples: 8 generated rows, circularly shifted and sign-flipped."""
    from paper_1201_3018_amd import synth
    base = synth.gaussian(L * 8, seed).reshape(8, L)
    rng = np.random.default_rng(seed + 10)
    host = np.empty((n, L), np.float32)
    for i in range(n):
        host[i] = np.roll(base[i % 8], int(rng.integers(0, L))) * (1.0 if (i // 8) % 2 == 0 else -1.0)
    return host


def bench_c1(args, wl):
    """Time-domain workload as a batch: 1024 signals of 65536 samples through one prepared kernel
    in one launch over every (signal, block) item (apx_many).  A step is one such launch; the
    steps alternate between two input/output sets (1 GB in all, beyond the last-level cache).
    value = output samples/s over the batch, asymmetric M=2 at 8 bits on the default core (the
    integer matrix cores for 65 taps); the packed FP64 time-domain core and the FP32 time-domain
    path are timed the same way beside it."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    n, L, N, Wb = wl["nsig"], wl["L"], wl["N"], wl["Wb"]
    host = c1_batch(n, L)
    k = synth.uniform(N, 1002)
    sets = 2
    ins = [torch.from_numpy(host).to(dev) for _ in range(sets)]
    ctx = apx.Context(0)
    tk = torch.from_numpy(k).to(dev)
    N_odd, W, P = apx.apx_geometry(L, N, Wb)
    outputs = n * (L + N - 1)
    bytes_alg = n * (L * 4 + (L + N - 1) * 4)        # compulsory: every sample read once, every output written once
    bytes_win = n * (P * Wb * 4 + (L + N - 1) * 4)   # every window read whole

    def timed(kh, steps, warmup):
        manys = [apx.Many(kh, [ins[j][i] for i in range(n)]) for j in range(sets)]
        for i in range(warmup):
            manys[i % sets].run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(steps):
                manys[i % sets].run()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        out = torch.stack(manys[0].outs)
        desc = manys[0].describe()
        for m in manys:
            m.close()
        return e0.elapsed_time(e1) / steps, out, desc

    steps = max(1, args.steps // 4)
    packed = apx.Kernel(ctx, tk, Wb, mode=apx.APX_ASYM2, Sq=127, Kq=127)
    ms_packed, out_p, desc = timed(packed, steps, 3)
    td = apx.Kernel(ctx, tk, Wb, mode=apx.APX_ASYM2, Sq=127, Kq=127, core=apx.APX_CORE_TIME)
    ms_td, out_td, _ = timed(td, steps, 3)
    full = apx.Kernel(ctx, tk, Wb, mode=apx.APX_FULL_FP32, core=apx.APX_CORE_TIME)
    ms_full, out_f, _ = timed(full, steps, 3)
    same_td = bool(torch.equal(out_p, out_td))
    # accuracy on sampled signals against FP64 (the FP64 time-domain path, one signal at a time)
    ref64 = apx.Kernel(ctx, tk, Wb, mode=apx.APX_FULL_FP64, core=apx.APX_CORE_TIME)
    snrs, snrs_f = [], []
    for i in (0, 1, 511, 1023):
        rr = ref64.run(ins[0][i]).cpu().numpy().astype(np.float64)
        for arr, dst in ((out_p, snrs), (out_f, snrs_f)):
            e = np.sum((arr[i].cpu().numpy().astype(np.float64) - rr) ** 2)
            dst.append(np.inf if e == 0 else 10 * np.log10(np.sum(rr ** 2) / e))
    value = outputs / (ms_packed * 1e-3)
    gbs = bytes_alg / (ms_packed * 1e-3) / 1e9
    res = {
        "metric": "output samples/s at fixed SNR, packed vs full-precision FP32, 1 GPU",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 3,
        "ms_per_step": ms_packed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": wl["name"], "signals": n, "L": L, "N": N, "W_block": Wb, "blocks_per_signal": P,
                   "items": n * P},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic("c1"),
                     "bytes_per_launch": bytes_alg, "bytes_per_output": round(bytes_alg / outputs, 3),
                     "window_bytes_per_launch": bytes_win,
                     "window_bytes_GBs": round(bytes_win / (ms_packed * 1e-3) / 1e9, 1), "kernel": desc},
        "packed_fp64_time_domain": {"ms_per_step": ms_td, "value": outputs / (ms_td * 1e-3),
                                    "outputs_equal_default_core": same_td},
        "full_fp32": {"ms_per_step": ms_full, "value": outputs / (ms_full * 1e-3),
                      "snr_db_min": float(np.min(snrs_f))},
        "packed_over_fp32": ms_full / ms_packed,
        "full_fp32_kernel": full.describe(),
        "snr_db": {"min": float(np.min(snrs)), "sampled_signals": 4},
    }
    if args.copy_probe:
        res["copy_probe_bytes"] = copy_probe(dev)
    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 10.0:
            x = host[done % n]
            O.conv_blocked(x, k, Wb, O.fixed_params(x, k, Wb, O.ASYM2, 127, 127))
            done += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done * (L + N - 1) / dt, "unit": "samples/s", "cores": O.num_threads(),
                               "kind": "oracle", "sample": f"{done} of the {n} signals, one after the other: "
                                                          f"int64 block convolution, {dt:.1f} s"}
    print(json.dumps(res), flush=True)
    for kh in (packed, td, full, ref64):
        kh.close()
    ctx.close()


def copy_probe(dev):
    """A 256 MiB device copy of known size, three times: the reference that scales the HBM
    counters of a rocprofv3 run (bytes read + written per copy returned)."""
    import torch
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 2 * src.numel() * 4


def bench_c3(args, wl):
    """Batched matching: one step = one run of the whole batch (every pair's correlation at every
    lag and its argmax).  value = correlation lags per second, symmetric packing at the largest
    S_q = K_q; asymmetric M=2 and FP32 timed the same way beside it."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    refs, tmpls, ridx, offs = synth.xcorr_batch()
    tr = [torch.from_numpy(r).to(dev) for r in refs]
    pr = [tr[j] for j in ridx]
    pk = [torch.from_numpy(k).to(dev) for k in tmpls]
    lags_total = int(sum(refs[j].size + k.size - 1 for j, k in zip(ridx, tmpls)))
    ctx = apx.Context(0)
    res_modes = {}
    steps = max(1, min(args.steps, 20))
    warm = max(1, min(args.warmup, 3))
    for name, mode in (("sym", apx.APX_SYM), ("asym2", apx.APX_ASYM2), ("full_fp32", apx.APX_FULL_FP32)):
        print(f"c3: {name}: building and autotuning the batch", file=sys.stderr, flush=True)
        b = apx.Batch(ctx, pr, pk, mode=mode, logW=0)
        print(f"c3: {name}: timing", file=sys.stderr, flush=True)
        lag = torch.empty(len(pk), dtype=torch.int64, device=dev)
        val = torch.empty(len(pk), dtype=torch.float32, device=dev)
        for _ in range(warm):
            b.run(lag, val)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    b.run(lag, val, stream=s)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        wb, lw, nitems = b.blocks()
        lg = lag.cpu().numpy()
        # algorithmic work: every window read once, per item one forward and one inverse FFT
        P = [-(-refs[j].size // (int(w) - (k.size | 1) - 1)) for j, k, w in zip(ridx, tmpls, wb)]
        bytes_alg = sum(4 * p * int(w) for p, w in zip(P, wb))
        fl = nitems * fft_flops_per_item(1 << lw)
        res_modes[name] = {"ms_per_step": ms, "lags_per_s": lags_total / (ms * 1e-3), "logW": lw,
                           "items": nitems, "true_offset_agreement": float(np.mean(lg == offs)),
                           "bytes_per_launch": bytes_alg, "flops_per_launch": fl,
                           "hbm_GBs": bytes_alg / (ms * 1e-3) / 1e9,
                           "alu_TFLOPs": fl / (ms * 1e-3) / 1e12, "kernel": b.describe().split(" tune=")[0]}
        b.close()
    head = res_modes["sym"]
    peak = FP64_VECTOR_TFLOPS
    alu_frac = head["alu_TFLOPs"] / peak
    hbm_frac = head["hbm_GBs"] / HBM_PEAK_GBS
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(head["alu_TFLOPs"], 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(head["hbm_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    roof["traffic"] = measured_traffic("c3")  # scaled FETCH_SIZE + WRITE_SIZE of the symmetric kernel
    roof["kernel"] = head["kernel"]
    res = {
        "metric": "correlation lags/s of batched matching (argmax per template), packed vs FP32, 1 GPU",
        "value": head["lags_per_s"], "unit": "lags/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "pairs": len(pk), "lags": lags_total},
        "roofline": roof, "modes": res_modes,
        "packed_over_fp32": res_modes["full_fp32"]["ms_per_step"] / head["ms_per_step"],
    }
    if args.copy_probe:
        res["copy_probe_bytes"] = copy_probe(dev)
    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        done = 0
        i = 0
        wb_sym = None
        b = apx.Batch(ctx, pr, pk, mode=apx.APX_SYM, logW=head["logW"])
        wb_sym = b.blocks()[0]
        b.close()
        while time.perf_counter() - t0 < 15.0 and i < len(pk):
            c = O.xcorr_blocked(refs[ridx[i]], tmpls[i], int(wb_sym[i]), O.SYM)
            O.argmax_lag_finite(c, tmpls[i].size)
            done += c.size
            i += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done / dt, "unit": "lags/s", "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"first {i} of {len(pk)} pairs ({done} lags), symmetric blocks + argmax, "
                                         f"{dt:.1f} s"}
    print(json.dumps(res), flush=True)
    ctx.close()


MFMA_F16_TFLOPS = 2500.0    # MI355X dense FP16 / BF16 matrix peak


def bench_c4(args, wl):
    """Filter bank: one step = the whole bank (256 x 32 output rows of 2^20 + 511 samples).
    value = output samples/s of the FP16 split path; BF16 split and the FP32 vector path (the
    time-domain FP32 core, one channel timed and scaled by the channel count) beside it, with
    the error against FP64 per channel on sampled outputs."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    C, L, F, N = 256, 1 << 20, 32, 512
    Lout = L + N - 1
    ldy = (Lout + 63) // 64 * 64
    x = synth.pink_noise(C, L, 4001)
    h = synth.bandpass_bank(F, N)
    xd = torch.from_numpy(x).to(dev)
    hd = torch.from_numpy(h).to(dev)
    y = torch.empty(C * F, ldy, dtype=torch.float32, device=dev)
    ctx = apx.Context(0)
    steps = max(1, min(args.steps, 10))
    rng = np.random.default_rng(11)
    chans = rng.choice(C, 8, replace=False)
    ts = rng.integers(0, Lout, 4096)
    xs = {c: np.concatenate([np.zeros(N - 1), x[c].astype(np.float64), np.zeros(N - 1)]) for c in chans}
    ref = {c: xs[c][ts[:, None] + np.arange(N)[None, :]] @ h.astype(np.float64)[:, ::-1].T for c in chans}

    def chan_snr(get):
        out = []
        for c in chans:
            g = get(c)
            e = np.sum((g - ref[c]) ** 2)
            out.append(float("inf") if e == 0 else 10 * math.log10(float(np.sum(ref[c] ** 2)) / e))
        return out

    tsd = torch.from_numpy(ts).to(dev)
    modes = {}
    for name, prec in (("f16x3", apx.APX_FB_F16X3), ("bf16x3", apx.APX_FB_BF16X3)):
        fb = apx.FilterBank(ctx, hd, prec)
        fb.run(xd, y=y, L=L)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fb.run(xd, y=y, L=L)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        yv = y.view(C, F, ldy)
        snr = chan_snr(lambda c: yv[int(c)][:, tsd].cpu().numpy().T.astype(np.float64))
        modes[name] = {"ms_per_step": ms, "samples_per_s": C * F * Lout / (ms * 1e-3),
                       "snr_db_per_channel": [round(v, 1) for v in snr], "kernel": fb.describe()}
        fb.close()
    # FP32 vector path: the FP32 time-domain core, filter by filter, one channel timed
    Wb = 2048
    kerns = [apx.Kernel(ctx, hd[f].contiguous(), Wb, mode=apx.APX_FULL_FP32, core=apx.APX_CORE_TIME) for f in range(F)]
    outs = [torch.empty(Lout, dtype=torch.float32, device=dev) for _ in range(F)]
    for f in range(F):
        kerns[f].run(xd[0], out=outs[f])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for f in range(F):
        kerns[f].run(xd[0], out=outs[f])
    e1.record()
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) * C

    def fp32_get(c):
        g = np.empty((ts.size, F))
        for f in range(F):
            kerns[f].run(xd[int(c)], out=outs[f])
            g[:, f] = outs[f][tsd].cpu().numpy()
        return g
    snr32 = chan_snr(fp32_get)
    modes["fp32_vector"] = {"ms_per_step": ms32, "samples_per_s": C * F * Lout / (ms32 * 1e-3),
                            "snr_db_per_channel": [round(v, 1) for v in snr32],
                            "kernel": kerns[0].describe() + " (one channel timed, x256)"}
    for kk in kerns:
        kk.close()
    head = modes["f16x3"]
    flops = 3 * 2.0 * 512 * 32 * Lout * C                 # executed MFMA work (three products)
    bytes_alg = C * F * Lout * 4 + C * L * 4               # outputs written once + inputs read once
    ach = flops / (head["ms_per_step"] * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(ach, 1), "peak": MFMA_F16_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / MFMA_F16_TFLOPS, 4), "traffic": None,
            "hbm_GBs": round(bytes_alg / (head["ms_per_step"] * 1e-3) / 1e9, 1), "kernel": head["kernel"],
            "flops_per_launch": flops, "bytes_per_launch": bytes_alg}
    res = {
        "metric": "filter-bank output samples/s, split-precision FP16 matrix cores vs FP32 vector path, 1 GPU",
        "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16x3", "data": "synthetic",
        "config": {"workload": wl["name"], "channels": C, "L": L, "filters": F, "N": N},
        "roofline": roof, "modes": modes,
        "speedup_over_fp32_vector": ms32 / head["ms_per_step"],
    }
    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        n = 0
        pairs = 0
        while time.perf_counter() - t0 < 10.0 and pairs < C * F:
            O.conv_direct(x[pairs // F], h[pairs % F])
            n += Lout
            pairs += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / dt, "unit": "samples/s", "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"first {pairs} (channel, filter) rows ({n} outputs), FP64 direct "
                                         f"convolution, {dt:.1f} s"}
    print(json.dumps(res), flush=True)
    ctx.close()


def bench_c5(args, wl, duration: float = 10.0, rate: float = 2000.0):
    """Serving: requests are submitted at their Poisson arrival times to the native server
    (8 streams, 48 requests in flight, 32 GiB budget); latency = completion time - scheduled
    arrival (client lag and waits for a free output buffer included).  Inputs are prefixes of 8
    pinned AR(1) signals; kernels are Hann low-passes, one per (size, pool index)."""
    import torch

    from paper_1201_3018_amd import apx, synth
    reqs = synth.poisson_requests(rate=rate, duration=duration)
    Lmax = max(r["L"] for r in reqs)
    Nmax = max(r["N"] for r in reqs)
    sig = []
    for i in range(8):
        t = torch.empty(Lmax, dtype=torch.float32, pin_memory=True)
        t.copy_(torch.from_numpy(synth.ar1(Lmax, 5100 + i)))
        sig.append(t)
    nbuf = 64
    outs = [torch.empty(Lmax + Nmax - 1, dtype=torch.float32, pin_memory=True) for _ in range(nbuf)]
    free = list(range(nbuf))
    taps = {}

    def kernel_for(r):
        key = (r["N"], r["kernel"])
        if key not in taps:
            taps[key] = synth.hann_lowpass(r["N"], 0.02 + 0.45 * r["kernel"] / 128.0)
        return key[0] * 1000 + key[1], taps[key]

    ctx = apx.Context(0)
    srv = apx.Server(ctx, hbm_budget=32 << 30, n_streams=8, max_inflight=48)
    # warm-up: one request per size so that library code paths are loaded (not timed)
    for N in sorted({r["N"] for r in reqs}):
        key, k = kernel_for({"N": N, "kernel": 0})
        srv.submit(key, k, sig[0], outs[0], 40.0, L=max(4096, N))
        srv.drain()
        srv.poll(max_n=1024)
    srv.close()
    srv = apx.Server(ctx, hbm_budget=32 << 30, n_streams=8, max_inflight=48)
    lat, done_samples, buf_of, arr_of, cores = [], 0, {}, {}, {0: 0, 1: 0, 2: 0}
    t0 = apx.Server.now() + 0.2
    last_done = t0

    def collect(wait_ms=0):
        nonlocal done_samples, last_done
        for c in srv.poll(wait_ms=wait_ms):
            if c["status"] != 0:
                raise RuntimeError(f"request failed: {c}")
            lat.append(c["t_done"] - arr_of.pop(c["ticket"]))
            free.append(buf_of.pop(c["ticket"]))
            done_samples += c["L"] + c["N"] - 1
            cores[c["core"]] += 1
            last_done = max(last_done, c["t_done"])

    for i, r in enumerate(reqs):
        arrival = t0 + r["t"]
        while True:
            collect()
            now = apx.Server.now()
            if now >= arrival and free:
                break
            if not free:
                collect(wait_ms=1)
            elif arrival - now > 0.0004:
                time.sleep(0.0002)
        b = free.pop()
        key, k = kernel_for(r)
        tk = srv.submit(key, k, sig[i % 8], outs[b], r["snr"], L=r["L"])
        buf_of[tk] = b
        arr_of[tk] = arrival
    srv.drain()
    collect()
    st = srv.stats()
    srv.close()
    burst = serve_burst(ctx, sig)
    ctx.close()
    lat = np.array(lat) * 1e3
    span = last_done - t0
    res = {
        "metric": "serving latency p50/p99 and output samples/s under Poisson load, 1 GPU",
        "value": done_samples / span, "unit": "samples/s", "n_gpus": 1, "steps": len(reqs), "warmup": 0,
        "ms_per_step": float(np.mean(lat)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "requests": len(reqs), "rate_req_s": rate, "duration_s": duration},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                       "p99": float(np.percentile(lat, 99)), "max": float(np.max(lat))},
        "served_req_s": len(reqs) / span, "cores": {"time": cores[1], "fft": cores[2]},
        "server": st,
        "burst": burst,
    }
    print(json.dumps(res), flush=True)


def serve_burst(ctx, sig, n=2000, nkern=4, N=256, seed=5002):
    """Saturation: n requests over nkern kernels (N taps, L log-uniform in [2^14, 2^18], SNR
    target 40 dB) submitted at once, so that many are admitted together and run as shared
    launches; against the same requests one at a time (max_inflight = 1, one launch each)."""
    from paper_1201_3018_amd import apx, synth
    rng = np.random.default_rng(seed)
    Ls = np.exp(rng.uniform(np.log(1 << 14), np.log(1 << 18), n)).astype(np.int64)
    taps = [synth.hann_lowpass(N, 0.05 + 0.1 * j) for j in range(nkern)]
    outs = [np.empty(int(L) + N - 1, np.float32) for L in Ls]
    res = {}
    for name, inflight in (("batched", 256), ("one_at_a_time", 1)):
        srv = apx.Server(ctx, hbm_budget=32 << 30, n_streams=8, max_inflight=inflight)
        t0 = apx.Server.now()
        for i in range(n):
            j = i % nkern
            srv.submit(100 + j, taps[j], sig[i % 8], outs[i], 40.0, L=int(Ls[i]))
        srv.drain()
        dt = apx.Server.now() - t0
        srv.poll(max_n=1024)
        st = srv.stats()
        srv.close()
        res[name] = {"s": dt, "samples_per_s": float(np.sum(Ls + N - 1)) / dt, "launches": st["launches"],
                     "requests": st["completed"]}
    res["batching_gain"] = res["batched"]["samples_per_s"] / res["one_at_a_time"]["samples_per_s"]
    res["config"] = f"{n} requests, {nkern} kernels of N={N}, L log-uniform in [2^14, 2^18], SNR 40 dB, host buffers"
    return res


def bench_c1sweep(args, wl):
    """Time-domain core across kernel lengths: per mode, output samples/s, with the measured SNR
    of every mode against the FP64 path on the first 2^18 outputs.  FMAs per output: FP32 and
    FP64 N, asymmetric M=2 N/2, symmetric ceil(N/2)/2 (one packed word carries two outputs).
    Beside them, the integer matrix-core core at the same companding (same outputs)."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    L = 1 << 22
    s = synth.gaussian(L, 1001)
    ts = torch.from_numpy(s).to(dev)
    ctx = apx.Context(0)
    rows = []
    steps = max(1, min(args.steps, 20))
    for N in (64, 128, 256, 512, 1024):
        No = N + 1 - N % 2
        Wb = max(2 * No, 1024) + No + 1
        k = synth.uniform(N, 1002 + N)
        tk = torch.from_numpy(k).to(dev)
        out = torch.empty(L + N - 1, dtype=torch.float32, device=dev)
        ref = None
        first = {}
        row = {"N": N, "W_block": Wb}
        for name, mode, core in (("fp64", apx.APX_FULL_FP64, apx.APX_CORE_TIME),
                                 ("fp32", apx.APX_FULL_FP32, apx.APX_CORE_TIME), ("sym", apx.APX_SYM, apx.APX_CORE_TIME),
                                 ("asym2", apx.APX_ASYM2, apx.APX_CORE_TIME),
                                 ("int8_sym", apx.APX_SYM, apx.APX_CORE_INT8),
                                 ("int8_asym2", apx.APX_ASYM2, apx.APX_CORE_INT8)):
            kern = apx.Kernel(ctx, tk, Wb, mode=mode, core=core)
            kern.run(ts, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                kern.run(ts, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            r = out[: 1 << 18].cpu().numpy().astype(np.float64)
            first[name] = r
            if name == "fp64":
                ref = r
                snr = float("inf")
            else:
                e = float(np.sum((r - ref) ** 2))
                snr = float("inf") if e == 0 else 10 * math.log10(float(np.sum(ref ** 2)) / e)
            row[name] = {"ms": ms, "samples_per_s": (L + N - 1) / (ms * 1e-3), "snr_db": snr}
            kern.close()
        row["int8_equals_packed"] = bool(np.array_equal(first["int8_sym"], first["sym"]) and
                                         np.array_equal(first["int8_asym2"], first["asym2"]))
        row["sym_over_fp64"] = row["fp64"]["ms"] / row["sym"]["ms"]
        row["sym_over_fp32"] = row["fp32"]["ms"] / row["sym"]["ms"]
        row["asym2_over_fp32"] = row["fp32"]["ms"] / row["asym2"]["ms"]
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    big = rows[-1]
    fl = 2.0 * (L + 1023) * ((1025 + 1) // 2) / 2  # symmetric: ceil(N/2) FMAs per packed word of 2 outputs
    ach = fl / (big["sym"]["ms"] * 1e-3) / 1e12
    res = {
        "metric": "time-domain output samples/s, symmetric packing vs FP64 and FP32, 1 GPU",
        "value": big["sym"]["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": big["sym"]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": wl["name"], "L": L},
        "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / FP64_VECTOR_TFLOPS, 4), "traffic": None,
                     "kernel": "k_td symmetric, N=1024", "flops_per_launch": fl},
        "sweep": rows,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def bench_sweep(args, wl):
    """The paper's throughput experiments (Section IV.A) on synthetic data, on the FFT core.

    E1: block size W (outputs per block; W_block = W + N_odd + 1) over {2,...,64} x 2^10 at N = 800.
    E2: kernel length N over {32, ..., 8192} at W = 32 x 2^10, the paper's (the transforms beyond
    2^14 words run on the multi-pass FFT core).
    Modes: the paper's settings (symmetric and asymmetric M=3 at S_q = K_q = 16, asymmetric M=2
    at 256; these exceed the Table 1 bounds at N = 800, so they run with allow_unsafe and their
    SNR includes any unpacking errors), the largest in-bound S_q = K_q of each mode, and the FP32
    comparator.  Each point reports output samples/s and the SNR against the exact convolution
    (FP64 FFT on the host, from the same FP32 inputs).  Points whose transform does not fit the
    FFT core are reported as unsupported."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    L = 1 << 23
    s = synth.uniform(L, 6001) * np.float32(128.0)
    ts = torch.from_numpy(s).to(dev)
    ctx = apx.Context(0)
    steps = max(1, min(args.steps, 10))
    modes = [("fp32", apx.APX_FULL_FP32, 0, False), ("sym16", apx.APX_SYM, 16, True),
             ("asym3_16", apx.APX_ASYM3, 16, True), ("asym2_256", apx.APX_ASYM2, 256, True),
             ("sym_max", apx.APX_SYM, 0, False), ("asym3_max", apx.APX_ASYM3, 0, False),
             ("asym2_max", apx.APX_ASYM2, 0, False)]

    def exact(k):
        n = L + k.size - 1
        nf = 1 << (n - 1).bit_length()
        return np.fft.irfft(np.fft.rfft(s.astype(np.float64), nf) * np.fft.rfft(k.astype(np.float64), nf), nf)[:n]

    def point(N, W, k, tk, ref):
        No = N + 1 - N % 2
        Wb = W + No + 1
        row = {"N": N, "W": W, "W_block": Wb}
        out = torch.empty(L + N - 1, dtype=torch.float32, device=dev)
        for name, mode, q, unsafe in modes:
            try:
                kern = apx.Kernel(ctx, tk, Wb, mode=mode, core=apx.APX_CORE_FFT, Sq=q, Kq=q, allow_unsafe=unsafe)
            except apx.ApxError as e:
                row[name] = {"unsupported": str(e)}
                continue
            kern.run(ts, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                kern.run(ts, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            r = out.cpu().numpy().astype(np.float64)
            err = float(np.sum((r - ref) ** 2))
            snr = float("inf") if err == 0 else 10 * math.log10(float(np.sum(ref ** 2)) / err)
            ent = {"ms": round(ms, 4), "samples_per_s": (L + N - 1) / (ms * 1e-3), "snr_db": round(snr, 2)}
            if q == 0:
                d = kern.describe()
                ent["kernel"] = d[:160]
            row[name] = ent
            kern.close()
        if "ms" in row.get("fp32", {}):
            for name, *_ in modes[1:]:
                if "ms" in row[name]:
                    row[name]["gain_pct_vs_fp32"] = round(100.0 * (row["fp32"]["ms"] / row[name]["ms"] - 1.0), 1)
        print(json.dumps(row), file=sys.stderr, flush=True)
        return row

    e1 = []
    k800 = synth.uniform(800, 6002) * np.float32(128.0)
    ref800 = exact(k800)
    tk800 = torch.from_numpy(k800).to(dev)
    for W in (2, 4, 8, 16, 32, 64):
        e1.append(point(800, W * 1024, k800, tk800, ref800))
    e2 = []
    for N in (32, 64, 128, 256, 512, 1024, 2048, 4096, 8192):
        kN = synth.uniform(N, 6100 + N) * np.float32(128.0)
        W = 32 * 1024 if 2 * (N + 1) <= 32 * 1024 else 2 * (N + 1)
        e2.append(point(N, W, kN, torch.from_numpy(kN).to(dev), exact(kN)))

    # Table 2 analogue: min / max throughput gain over the E1 block sizes, mean SNR, per method
    table2 = {}
    for name, *_ in modes[1:]:
        g = [r[name]["gain_pct_vs_fp32"] for r in e1 if "gain_pct_vs_fp32" in r.get(name, {})]
        sn = [r[name]["snr_db"] for r in e1 if "snr_db" in r.get(name, {})]
        if g:
            table2[name] = {"min_gain_pct": min(g), "max_gain_pct": max(g), "mean_snr_db": round(float(np.mean(sn)), 2),
                            "block_sizes": [r["W"] for r in e1 if "gain_pct_vs_fp32" in r.get(name, {})]}
    head = next(r for r in e1 if r["W"] == 8192)
    hs = head["sym_max"]
    P = -(-L // head["W"])
    bytes_launch = 4.0 * (L + P * (head["W_block"] - head["W"])) + 4.0 * (L + 799)
    ach = bytes_launch / (hs["ms"] * 1e-3) / 1e9
    res = {
        "metric": "output samples/s per packing method vs the FP32 comparator (paper sweep, synthetic), 1 GPU",
        "value": hs["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": hs["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": wl["name"], "L": L},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "FFT core, symmetric packing at the largest in-bound S_q=K_q, N=800, W=8x2^10",
                     "bytes_per_launch": bytes_launch},
        "table2": table2, "e1": e1, "e2": e2,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def bench_delay(args, wl):
    """Inter-channel delay and correlation per block (the paper's multi-channel audio application,
    Section IV.C and Table 4, on synthetic audio).  For each block of the two channels, one batched
    launch correlates block b_i with block a_i at every lag and returns the argmax lag (the delay
    estimate) and its value.  Per method: the share of blocks whose delay differs from the exact
    (FP64) one and the mean relative delay error, the mean relative error of the cross-channel
    correlation coefficient rho = c[lag] / (|a_i| |b_i|), the mono/stereo decision (mono when the
    lag is 0 and rho >= 0.99) against the generator's labels, and channel samples/s.  Methods:
    FP32, the paper's S_q = K_q = 32 for all three packings (symmetric and asymmetric M=3 exceed
    the Table 1 bound at these block lengths and run with allow_unsafe), and the largest in-bound
    S_q = K_q for symmetric and asymmetric M=2."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    fs = 44100
    L = 90 * fs
    a, b, delays, mono = synth.two_channel(L, 7001)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    ctx = apx.Context(0)
    steps = max(1, min(args.steps, 20))
    methods = [("fp32", apx.APX_FULL_FP32, 0, False), ("sym32", apx.APX_SYM, 32, True),
               ("asym2_32", apx.APX_ASYM2, 32, False), ("asym3_32", apx.APX_ASYM3, 32, True),
               ("sym_max", apx.APX_SYM, 0, False), ("asym2_max", apx.APX_ASYM2, 0, False)]
    rows = {}
    for ms_blk in (50, 100, 200):
        n = fs * ms_blk // 1000
        nb = L // n
        A = a[: nb * n].reshape(nb, n).astype(np.float64)
        B = b[: nb * n].reshape(nb, n).astype(np.float64)
        nf = 1 << (2 * n - 1).bit_length()
        C = np.fft.irfft(np.fft.rfft(B, nf, axis=1) * np.conj(np.fft.rfft(A, nf, axis=1)), nf, axis=1)
        full = np.concatenate([C[:, nf - (n - 1):], C[:, :n]], axis=1)  # lags -(n-1) .. n-1
        lag_x = np.argmax(full, axis=1) - (n - 1)
        norm = np.linalg.norm(A, axis=1) * np.linalg.norm(B, axis=1)
        rho_x = np.max(full, axis=1) / norm
        seg = (np.arange(nb) * n) // fs
        truth_mono, truth_d = mono[seg], delays[seg]
        pa = [ta[i * n:(i + 1) * n] for i in range(nb)]
        pb = [tb[i * n:(i + 1) * n] for i in range(nb)]
        row = {"block": n, "blocks": nb, "exact_delay_matches_truth": float(np.mean(lag_x == truth_d))}
        for name, mode, q, unsafe in methods:
            try:
                bt = apx.Batch(ctx, pb, pa, mode=mode, Sq=q, Kq=q, allow_unsafe=unsafe, logW=0)
            except apx.ApxError as e:
                row[name] = {"unsupported": str(e)}
                continue
            lag = torch.empty(nb, dtype=torch.int64, device=dev)
            val = torch.empty(nb, dtype=torch.float32, device=dev)
            bt.run(lag, val)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                bt.run(lag, val)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            lg, vl = lag.cpu().numpy(), val.cpu().numpy().astype(np.float64)
            rho = vl / norm
            det_mono = (lg == 0) & (rho >= 0.99)
            row[name] = {
                "ms": round(ms, 4), "channel_samples_per_s": 2 * nb * n / (ms * 1e-3),
                "delay_mismatch_pct": round(100.0 * float(np.mean(lg != lag_x)), 3),
                "relative_delay_error_pct": round(100.0 * float(np.mean(np.abs(lg - lag_x) /
                                                                        np.maximum(1, np.abs(lag_x)))), 3),
                "correlation_error_pct": round(100.0 * float(np.mean(np.abs(rho - rho_x) / np.abs(rho_x))), 4),
                "mono_stereo_correct_pct": round(100.0 * float(np.mean(det_mono == truth_mono)), 2),
                "kernel": bt.describe().split(" tune=")[0][:120],
            }
            bt.close()
        if "ms" in row.get("fp32", {}):
            for name, *_ in methods[1:]:
                if "ms" in row[name]:
                    row[name]["gain_pct_vs_fp32"] = round(100.0 * (row["fp32"]["ms"] / row[name]["ms"] - 1.0), 1)
        rows[f"{ms_blk}ms"] = row
        print(json.dumps({f"{ms_blk}ms": row}), file=sys.stderr, flush=True)
    head = rows["100ms"]["sym32"]
    n = rows["100ms"]["block"]
    nb = rows["100ms"]["blocks"]
    bytes_launch = 4.0 * 2 * n * nb
    ach = bytes_launch / (head["ms"] * 1e-3) / 1e9
    res = {
        "metric": "channel samples/s of per-block delay and correlation estimation, packed vs FP32, 1 GPU",
        "value": head["channel_samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": wl["name"], "L": L, "fs": fs},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "k_batch, symmetric at S_q=K_q=32, 100 ms blocks", "bytes_per_launch": bytes_launch},
        "blocks": rows,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def bench_calib(args, wl):
    """Fig. 5 analogue: average SNR of the companded correlation against S_q = K_q, measured and
    predicted by eqs. (18)-(19), the prediction calibrated by one measurement at S_q = K_q = 8.
    Two sigma choices in the model: the sources' fitted marginal CDFs (apx_fit_marginal, the
    paper's Section IV.D) and each block's root second moment (the library's default).  The
    integer core gives the exact companded result at every S_q (no packing bound), with the
    per-block model SNR in its block report.  Reference: the FP64 correlation on the host."""
    import torch

    from paper_1201_3018_amd import apx, synth
    dev = torch.device("cuda:0")
    ctx = apx.Context(0)
    L, N, Wb = 1 << 20, 1025, 4096
    W = Wb - N - 1
    P = -(-L // W)
    qs = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256]
    apps = [("audio delay", synth.ar1(L, 9001), apx.APX_MARGINAL_LAPLACE),
            ("feature matching", synth.weibull_features(L, 9002), apx.APX_MARGINAL_WEIBULL)]
    res_apps = {}
    roof = None
    for name, s, model in apps:
        k = s[300000:300000 + N].copy()
        ts, tk = torch.from_numpy(s).to(dev), torch.from_numpy(k).to(dev)
        fs = apx.apx_fit_marginal(ctx.h, ts, model)
        fk = apx.apx_fit_marginal(ctx.h, tk, model)
        nf = 1 << (L + N - 1).bit_length()
        ref = np.fft.irfft(np.fft.rfft(s.astype(np.float64), nf) * np.conj(np.fft.rfft(k.astype(np.float64), nf)), nf)
        ref = np.concatenate([ref[nf - (N - 1):], ref[:L]])  # lags -(N-1) .. L-1
        # kept output range of each block (block 0 from 0)
        spans = [(0, W + N - 1)] + [(N - 1 + W * w, min(N - 1 + W * w + W, L + N - 1)) for w in range(1, P)]
        rows = []
        for q in qs:
            ent = {"Sq": q}
            for tag, ss, sk in (("source_sigma", fs[2], fk[2]), ("block_rms", 0.0, 0.0)):
                kern = apx.Kernel(ctx, tk, Wb, mode=apx.APX_ASYM2, core=apx.APX_CORE_INT8, Sq=q, Kq=q,
                                  op=apx.APX_XCORR, sigma_s=ss, sigma_k=sk)
                out, info = kern.run(ts, info=True)
                torch.cuda.synchronize()
                if tag == "block_rms" and q == 8:
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(10):
                        kern.run(ts, out=out)
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / 10
                    byt = 4.0 * P * Wb + 4.0 * (L + N - 1)
                    ach = byt / (ms * 1e-3) / 1e9
                    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                            "kernel": "k_i8 one digit, S_q=K_q=8, " + name, "bytes_per_launch": byt, "ms": ms}
                r = out.cpu().numpy().astype(np.float64)
                inf = apx.block_info(info)
                kern.close()
                meas = []
                for a0, a1 in spans:
                    e = float(np.sum((r[a0:a1] - ref[a0:a1]) ** 2))
                    p = float(np.sum(ref[a0:a1] ** 2))
                    meas.append(10 * math.log10(p / e) if e > 0 else float("inf"))
                ent[tag] = {"measured_db": float(np.mean(meas)), "model_db": float(np.mean(inf["snr_pred_db"]))}
            rows.append(ent)
        out_app = {"sigma_s_fit": {"scale": fs[0], "shape": fs[1], "sigma": fs[2]},
                   "sigma_k_fit": {"scale": fk[0], "shape": fk[1], "sigma": fk[2]},
                   "signal_rms": float(np.sqrt(np.mean(s.astype(np.float64) ** 2))), "rows": rows}
        for tag in ("source_sigma", "block_rms"):
            off = rows[0][tag]["measured_db"] - rows[0][tag]["model_db"]
            dev_ = [r[tag]["model_db"] + off - r[tag]["measured_db"] for r in rows]
            for r, d in zip(rows, dev_):
                r[tag]["calibrated_model_db"] = r[tag]["model_db"] + off
            out_app[tag] = {"calibration_offset_db": off, "max_abs_deviation_db": float(np.max(np.abs(dev_))),
                            "mean_abs_deviation_db": float(np.mean(np.abs(dev_)))}
        res_apps[name] = out_app
        print(json.dumps({name: out_app}), file=sys.stderr, flush=True)
    worst = max(a["source_sigma"]["max_abs_deviation_db"] for a in res_apps.values())
    res = {
        "metric": "largest deviation of the calibrated SNR model (source sigmas) from the measured average SNR over "
                  "S_q=K_q in 8..256, 1 GPU",
        "value": worst, "unit": "dB", "n_gpus": 1, "steps": 10, "warmup": 1, "ms_per_step": roof["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": wl["name"], "L": L, "N": N, "W_block": Wb},
        "roofline": roof, "applications": res_apps,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


# rocprofv3 counter summary per workload and the kernel sources its figures hold for
TRAFFIC_SUMMARIES = {"c2": ("fft_c2_hbm_counters.md", ("fftw.hip", "fft.h", "internal.h", "items.h")),
                     "c3": ("batch_c3_hbm_counters.md", ("kernels.hip", "fft.h", "internal.h")),
                     "c1": ("int8_c1_hbm_counters.md", ("kernels.hip", "items.h", "internal.h"))}


def measured_traffic(workload: str):
    """HBM bytes per launch of the workload's headline kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since the counters were taken."""
    if workload not in TRAFFIC_SUMMARIES:
        return None
    import hashlib
    fname, srcs = TRAFFIC_SUMMARIES[workload]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, "paper_1201_3018_amd", "csrc", f), "rb").read())
    if rec.get("kernel_sources_sha256_16") != h.hexdigest()[:16]:
        return None
    try:
        return int(rec["traffic_bytes_per_launch"].split()[0])
    except (KeyError, ValueError):
        return None


def cpu_baseline(workload, s, k, Wb, wl, calib, outputs):
    """The oracle, as it stands, on the same workload: the plain per-block integer definition
    (C loops, OpenMP over blocks) with the same block selection, whole signal."""
    import oracle as O
    t0 = time.perf_counter()
    runs = 0
    while True:  # the whole workload, repeated until about 10 s of CPU work
        if workload == "c2":
            ps = O.auto_params(s, k, Wb, wl["snr"], calib)
        else:
            ps = O.fixed_params(s, k, Wb, O.ASYM2, 127, 127)
        O.conv_blocked(s, k, Wb, ps)
        runs += 1
        if time.perf_counter() - t0 >= 10.0:
            break
    dt = time.perf_counter() - t0
    return {"value": runs * outputs / dt, "unit": "samples/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"whole workload ({outputs} outputs) x {runs}: selection + int64 block convolution, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
