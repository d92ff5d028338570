#!/usr/bin/env python3
"""FPTC batch decompression benchmark on one MI355X.

One step = the whole decode path over one batch already resident in HBM:
plan (stream/chunk setup + symlen prefix sums) -> Huffman decode ->
dequantization fused with the inverse DCT, float32 out.  Each step is timed
both ways it can be launched: eager (the library calls, K steps back to back)
and as replays of one captured HIP graph of the same kernels; the step time is
the faster of the two (both are reported, with the mode taken).

Headline workload ("batch"): 4096 synthetic streams, lengths log-uniform in
2^14..2^20 samples, domains EEG / seismic / power-grid / meteorological in
turn, window 64, amplitude quantizer (steps 0.25 / 2.0, threshold 16), one
codebook per domain trained on separate data, L_max 12, fused FP16X2 path.

The same JSON line carries one entry per other workload ("configs"):
  plain      one EEG-like stream of 2^20 samples
  precision  256 x 2^20 samples (EEG / seismic), windows 64 and 256, every
             precision (FP32 SIMT and the MFMA forms)
  grad       256 x 2^18 samples (power / meteorological), window 128, forward
             and backward (scale and coefficient gradients)
  large      64 channels x 2^24 EEG-like samples, window 256, steps 1.0 / 8.0,
             fused FP16X2 against FP32 SIMT
plus the plain per-stream FP32 decoder (one launch sequence per stream), the
batched FP32 SIMT decoder, and the CPU oracle timed on bounded samples, whose
FP64 reconstructions also give each GPU variant's error.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
MFMA_F16_PEAK_TFS = 2500.0  # MI355X dense FP16/BF16 matrix peak
FP32_VEC_PEAK_TFS = 157.3  # MI355X FP32 vector peak
STEP_F, STEP_C, THRESH = 0.25, 2.0, 16.0
PLAN_KERNELS = "k_plan_pass1+k_plan_seg_chunks"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads() -> int:
    """Worker threads for host-side work: the CPUs this process may run on,
    capped at 16, the host's CPU share per GPU."""
    return max(1, min(16, affine_cores()))


def affine_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def quant_for(name: str, w=None):
    from paper_2605_01086_amd import codec as C
    if name == "large":  # window 256, coarse steps 1.0 / 8.0
        return C.quant_params("amp", 256, 256, step_fine=1.0, step_coarse=8.0, threshold=THRESH)
    if name == "paper":  # Table 1's typical values; A0 / A1 from the training data, on the GPU
        return paper_quant(32, 16, w)
    N = {"plain": 64, "batch": 64, "grad": 128}.get(name, 64)
    return C.quant_params("amp", N, N, step_fine=STEP_F, step_coarse=STEP_C, threshold=THRESH)


def paper_quant(N: int, E: int, w, B1: int = 2, B2: int | None = None):
    """The paper quantizer (mu 50, alpha1 0.004) at window N keeping E bins,
    zones [0, B1) mu-law, [B1, B2) deadzone (B2 = E by default, as Table 1's
    N = 32, E = 16, B2 = 16), A0 / A1 the 99.9th percentile of |c| over the
    workload's training signal."""
    from paper_2605_01086_amd import codec as C
    from synth import workloads as W
    B1 = min(B1, E)
    B2 = E if B2 is None else B2
    q = C.quant_params("paper", N, E, B1=B1, B2=B2, mu=50.0, alpha1=0.004)
    q.A0, q.A1 = C.zone_maxima(W.training_signals(w)[0], q, 99.9)
    return q


_SIGNALS = {}


def encode(w, q, threads):
    """Generate a workload's signals and encode them with the library's host
    encoder: (words, symlen, word_off, code-length tables)."""
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    from synth import workloads as W
    x = _SIGNALS.get(w.name)
    if x is None:
        x = W.signals(w, threads)
        if w.name == "sweep":  # every point of the sweep encodes the same signals
            _SIGNALS[w.name] = x
    lens_tab = np.stack([C.train_code_lengths(t, q) for t in W.training_signals(w)])
    sample_off = w.sample_off
    nsym = C.n_windows(w.lengths, q.N) * q.E
    cap_off = np.concatenate([[0], np.cumsum(nsym + 1)]).astype(np.int64)
    words = np.zeros(int(cap_off[-1]), dtype=np.uint64)
    symlen = np.zeros(int(cap_off[-1]), dtype=np.uint8)
    nw = F.fptc_encode_batch_host(x, sample_off, w.book_id, q, lens_tab, cap_off, words, symlen, threads)
    del x
    word_off = np.concatenate([[0], np.cumsum(nw)]).astype(np.int64)
    wc = np.empty(int(word_off[-1]), dtype=np.uint64)
    sc = np.empty(int(word_off[-1]), dtype=np.uint8)
    for i in range(len(nw)):  # compact the per-stream reserved ranges
        wc[word_off[i]:word_off[i + 1]] = words[cap_off[i]:cap_off[i] + nw[i]]
        sc[word_off[i]:word_off[i + 1]] = symlen[cap_off[i]:cap_off[i] + nw[i]]
    return wc, sc, word_off, lens_tab


class Setup:
    """One workload encoded and uploaded."""

    def __init__(self, name: str, threads: int, q=None):
        import torch
        from paper_2605_01086_amd import codec as C
        from synth import workloads as W
        t0 = time.perf_counter()
        self.name = name
        self.w = W.workload(name)
        self.q = q or quant_for(name, self.w)
        self.words, self.symlen, self.word_off, self.lens_tab = encode(self.w, self.q, threads)
        self.sample_off = self.w.sample_off
        self.codec = C.DeviceCodec(self.lens_tab, self.q, 12)
        self.batch = C.DeviceBatch(self.words, self.symlen, self.word_off, self.sample_off, self.q.N, self.q.E,
                                   self.w.book_id if self.codec.n_books > 1 else None)
        torch.cuda.synchronize()
        self.setup_s = time.perf_counter() - t0
        log(f"workload {name}: {self.w.n_streams} streams, {self.batch.n_samples} samples, "
            f"{self.batch.n_words} words, window {self.q.N}, setup {self.setup_s:.1f}s")

    @property
    def n_samples(self):
        return self.batch.n_samples

    @property
    def comp_bytes(self):
        return self.batch.compressed_bytes + self.batch.header_bytes


def kernel_name(stage: str, N: int, precision: str) -> str:
    wide = N == 256
    return {"plan": PLAN_KERNELS, "fused": f"k_w256<{precision}, fused>" if wide else f"k_fused<{precision}>",
            "decode": "k_decode",
            "dequant_idct": "k_dqidct_f32" if precision == "fp32" else
            (f"k_w256<{precision}, split>" if wide else f"k_dqidct_mfma<{precision}>"),
            "backward": ("k_bwd_mfma" if N in (32, 64, 128) else "k_bwd_chunk") + "+k_bwd_streams"}[stage]


def stage_bytes(s: Setup, stage: str) -> int:
    """Algorithmic HBM bytes of one launch of a stage: compressed words 8 B +
    symlen 1 B per word and per-stream headers in, 1 B per decoded symbol
    between the split kernels, 4 B per output sample."""
    b = s.batch
    return {"plan": b.n_words + b.header_bytes, "fused": s.comp_bytes + 4 * b.n_samples,
            "decode": s.comp_bytes + b.n_symbols, "dequant_idct": b.n_symbols + 4 * b.n_samples,
            "backward": 4 * b.n_samples + b.n_symbols + 4 * b.n_symbols}[stage]


def time_stages(dec, stages, steps, warmup, precision):
    """Eager launches with HIP events on the current stream (the stream every
    call is issued on) around each stage; mean ms per stage."""
    import torch
    calls = {"plan": dec.plan, "decode": dec.decode, "fused": lambda: dec.decompress(precision=precision),
             "dequant_idct": lambda: dec.dequant_idct(precision=precision)}
    for _ in range(warmup):
        for st in stages:
            calls[st]()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        for j, st in enumerate(stages):
            calls[st]()
            ev[k][j + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    per = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(len(stages))] for e in ev])
    gpu = np.array([e[0].elapsed_time(e[-1]) for e in ev])
    return wall, per.mean(axis=0), gpu


def time_graph(dec, precision, fused, steps, warmup):
    """ms per replay of the captured step (plan + decode kernels)."""
    import torch
    from paper_2605_01086_amd.graph import CapturedStep
    step = CapturedStep(dec, precision, fused)
    for _ in range(warmup):
        step.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    del step
    return ms


def read_summary(name: str, stage: str, wide: bool = False):
    """key: value lines of profiles/<name>.txt, or None when absent or taken on
    other kernel sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest(stage, wide):
        return None, "kernel changed since the counters were taken"
    return kv, path[len(ROOT) + 1:]


# Sources of each stage's kernels (window 256 has kernels of its own); a
# counter summary in profiles/ applies only while these hash to the digest
# recorded in it.
KERNEL_SOURCES = {
    ("fused", False): ["fused.hip", "decode_common.h", "mfma_common.h", "fptc_internal.h"],
    ("fused", True): ["mfma256.hip", "decode_common.h", "mfma_common.h", "fptc_internal.h"],
    ("decode", False): ["decode.hip", "decode_common.h", "mfma_common.h", "fptc_internal.h"],
    ("dequant_idct", False): ["dqidct_mfma.hip", "dqidct.hip", "mfma_common.h", "fptc_internal.h"],
    ("dequant_idct", True): ["mfma256.hip", "dqidct.hip", "mfma_common.h", "fptc_internal.h"],
    ("plan", False): ["plan.hip", "fptc_internal.h"],
    ("backward", False): ["bwd.hip", "fptc_internal.h"],
}


def source_digest(stage: str, wide: bool = False) -> str:
    import hashlib
    h = hashlib.sha256()
    files = KERNEL_SOURCES.get((stage, wide)) or KERNEL_SOURCES[(stage, False)]
    for f in files:
        with open(os.path.join(ROOT, "paper_2605_01086_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def roofline(s: Setup, stage: str, ms: float, precision: str, tag: str) -> dict:
    alg = stage_bytes(s, stage)
    achieved = alg / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": kernel_name(stage, s.q.N, precision), "achieved": round(achieved, 1),
         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
         "algorithmic_bytes": int(alg), "avg_ms": round(float(ms), 4)}
    wide = s.q.N == 256
    kv, src = read_summary(f"traffic_{tag}", stage, wide)
    r["traffic"] = int(float(kv["traffic_bytes_per_dispatch"])) if kv else None
    r["traffic_source"] = src
    kv, src = read_summary(f"mfma_{tag}", stage, wide)
    if kv and "mfma_util" in kv:
        r["mfma_util"] = float(kv["mfma_util"])
        r["mfma_source"] = src
    if stage in ("fused", "dequant_idct") and precision != "fp32":
        # dense contraction work actually issued: 2 flops per (sample, kept bin) per operand-piece pass
        passes = {"fp16": 1, "bf16": 1, "fp16x2": 2, "bf16x3": 3}[precision]
        tf = 2.0 * s.q.E * passes * s.n_samples / (ms * 1e-3) / 1e12
        r["mfma_tflops"] = round(tf, 1)
        r["mfma_frac_of_peak"] = round(tf / MFMA_F16_PEAK_TFS, 4)
    return r


def batched(s: Setup, launch, precision, fused, steps, warmup):
    """Step time (the faster launch mode), both modes' times and per-stage
    eager HIP-event times."""
    from paper_2605_01086_amd import codec as C
    dec = C.Decoder(s.batch, s.codec, launch)
    stages = ["plan", "fused"] if fused else ["plan", "decode", "dequant_idct"]
    eager_ms, per, gpu = time_stages(dec, stages, steps, warmup, precision)
    graph_ms = time_graph(dec, precision, fused, steps, warmup)
    ms = min(eager_ms, graph_ms)
    modes = {"launch_mode": "graph" if graph_ms < eager_ms else "eager", "eager_ms_per_step": round(eager_ms, 4),
             "graph_ms_per_step": round(graph_ms, 4)}
    st = dec.status.cpu().numpy()
    if np.any(st != 0):
        raise SystemExit(f"decode reported stream errors on {s.name}: {np.flatnonzero(st)[:8]}")
    return dec, ms, modes, dict(zip(stages, per.tolist())), gpu


def time_per_stream(s: Setup, launch, steps, precision):
    """The same decode issued as one plan/decode/dequant+IDCT call sequence per
    stream: 3 calls and 4 kernels (2 plan kernels, decode, dequant+IDCT) each."""
    import ctypes
    import torch
    from paper_2605_01086_amd import fptc as F
    batch, codec = s.batch, s.codec
    dev = batch.word_off.device
    n = batch.n_streams
    wo, so, yo = batch.word_off_h, batch.sample_off_h, batch.sym_off_h
    loc_w = torch.from_numpy(np.stack([np.zeros(n, np.int64), np.diff(wo)], 1).copy()).to(dev)
    loc_s = torch.from_numpy(np.stack([np.zeros(n, np.int64), np.diff(so)], 1).copy()).to(dev)
    lib = F.load()
    lc = launch.c()
    structs = []
    ws_bytes = 0
    for i in range(n):
        b = F.fptc_batch(1, 0, int(wo[i + 1] - wo[i]), int(yo[i + 1] - yo[i]), int(so[i + 1] - so[i]),
                         batch.words.data_ptr() + 8 * int(wo[i]), batch.symlen.data_ptr() + int(wo[i]),
                         loc_w.data_ptr() + 16 * i, loc_s.data_ptr() + 16 * i,
                         None if batch.book_id is None else batch.book_id.data_ptr() + i)
        structs.append(b)
        ws_bytes = max(ws_bytes, F.fptc_workspace_size(b, codec.c, lc))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    sym = torch.empty(max(1, batch.n_symbols), dtype=torch.uint8, device=dev)
    out = torch.empty(max(1, batch.n_samples), dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    by = ctypes.byref
    cp, lp = by(codec.c), by(lc)
    prec = F.PRECISIONS[precision]

    def one_pass():
        for i in range(n):
            bp = by(structs[i])
            sp = status.data_ptr() + 4 * i
            rc = lib.fptc_plan_batch(bp, cp, lp, ws.data_ptr(), ws_bytes, sp, st)
            rc |= lib.fptc_decode_batch(bp, cp, lp, ws.data_ptr(), ws_bytes, sym.data_ptr() + int(yo[i]), sp, st)
            rc |= lib.fptc_dequant_idct(bp, cp, lp, ws.data_ptr(), ws_bytes, sym.data_ptr() + int(yo[i]), None, prec,
                                        out.data_ptr() + 4 * int(so[i]), st)
            if rc:
                raise RuntimeError("per-stream launch failed")

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, out


# ------------------------------------------------------------------ CPU oracle leg


def oracle_params(q):
    from oracle import oracle as O
    if q.kind == 0:
        return O.QuantParams("amp", q.N, q.E, step_f=q.step_fine, step_c=q.step_coarse, T=q.threshold)
    return O.QuantParams("paper", q.N, q.E, B1=q.B1, B2=q.B2, mu=q.mu, alpha1=q.alpha1, A0=q.A0, A1=q.A1)


def oracle_decode(s: Setup, i: int, keep: bool = False):
    """The CPU oracle on stream i: bit-serial decode + FP64 dequant/IDCT."""
    from oracle import oracle as O
    p = oracle_params(s.q)
    L = int(s.sample_off[i + 1] - s.sample_off[i])
    wo = s.word_off
    book = O.Codebook(s.lens_tab[int(s.w.book_id[i]) if s.lens_tab.shape[0] > 1 else 0])
    sym = O.symlen_decode(s.words[wo[i]:wo[i + 1]], s.symlen[wo[i]:wo[i + 1]], book, O.n_windows(L, s.q.N) * s.q.E)
    rec = O.reconstruct(sym, L, p)
    return rec if keep else L


def cpu_oracle(s: Setup, streams, threads, budget_s=None):
    """Time the oracle over `streams` (in order, until the budget is used)."""
    t0 = time.perf_counter()

    def work(i):
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            return 0
        return oracle_decode(s, int(i))

    if threads == 1:
        res = [work(i) for i in streams]
    else:
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(work, streams))
    dt = time.perf_counter() - t0
    samples = int(sum(res))
    return {"value": round(4 * samples / dt / 1e9, 5), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{sum(1 for r in res if r)} of {s.w.n_streams} streams ({samples} samples) in {dt:.1f}s"}


def errors_vs_oracle(s: Setup, outs: dict, streams, threads):
    """max-abs, RMS and max-abs / range of each GPU output against the
    oracle's FP64 reconstruction of the sampled streams."""
    with ThreadPoolExecutor(threads) as ex:
        refs = list(ex.map(lambda i: oracle_decode(s, int(i), keep=True), streams))
    rep = {}
    for k, out in outs.items():
        ma, rms, rel = 0.0, 0.0, 0.0
        for i, ref in zip(streams, refs):
            got = out[s.sample_off[i]:s.sample_off[i + 1]].astype(np.float64)
            d = got - ref
            ma = max(ma, float(np.abs(d).max()))
            rms = max(rms, float(np.sqrt(np.mean(d * d))))
            rel = max(rel, float(np.abs(d).max() / (np.ptp(ref) or 1.0)))
        rep[k] = {"max_abs": float(f"{ma:.3e}"), "rms": float(f"{rms:.3e}"), "max_abs_over_range": float(f"{rel:.3e}")}
    return rep


# ------------------------------------------------------------------ legs


def copy_bandwidth(n_bytes: int = 1 << 30, reps: int = 10) -> dict:
    """Measured HBM bandwidth of a plain device copy (torch copy_ of n_bytes,
    read + write) and of a fill (write only), best of reps by HIP events: the
    practical ceilings beside the 8 TB/s specification."""
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    fbest = float("inf")  # write only: the output side of a decode
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.fill_(1.0)
        e1.record()
        torch.cuda.synchronize()
        fbest = min(fbest, e0.elapsed_time(e1))
    del src, dst
    return {"kernel": "torch copy_ of 1 GiB float32 (read + write)", "GBs": round(2 * n_bytes / (best * 1e-3) / 1e9, 1),
            "best_ms": round(best, 4), "fill_GBs": round(n_bytes / (fbest * 1e-3) / 1e9, 1)}


def release():
    """Return freed device memory to the driver between workloads."""
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def tuned_launch(s: Setup, launch, precision, fused, tune):
    """The launch shape of one leg: the autotuner's pick on this workload when
    tune is set, else `launch`; with a record of which."""
    if not tune:
        return launch, {"picked_by": "default"}
    from paper_2605_01086_amd import autotune
    lt, info = autotune.tune(s.batch, s.codec, precision, fused)
    return lt, {"shape": info["shape"], "picked_by": "autotuner", "tuning_s": round(info["tuning_s"], 2),
                "cached": info["cached"]}


def leg_fused_vs_fp32(s: Setup, launch, steps, warmup, precisions=("fp16x2",), with_fp32=True, tune=False):
    """Decoded GB/s of the fused path per MFMA precision and of the split FP32
    SIMT path, each with its dominant kernel's roofline fraction; outputs kept
    on the host for the error report."""
    res, outs = {}, {}
    for prec in precisions:
        lp, how = tuned_launch(s, launch, prec, True, tune)
        dec, ms, modes, per, _ = batched(s, lp, prec, True, steps, warmup)
        res[f"fused_{prec}"] = {"value": round(4 * s.n_samples / (ms * 1e-3) / 1e9, 2), "ms_per_step": round(ms, 4),
                                **modes, "launch": how,
                                "stage_ms": {k: round(v, 4) for k, v in per.items()},
                                "roofline": roofline(s, "fused", per["fused"], prec, f"fused_{prec}_{s.name}")}
        outs[f"fused_{prec}"] = dec.out[:s.n_samples].cpu().numpy()
        del dec
        release()
    if with_fp32:
        lp, how = tuned_launch(s, launch, "fp32", False, tune)
        dec, ms, modes, per, _ = batched(s, lp, "fp32", False, steps, warmup)
        dom = max(per, key=per.get)
        res["split_fp32"] = {"value": round(4 * s.n_samples / (ms * 1e-3) / 1e9, 2), "ms_per_step": round(ms, 4),
                             **modes, "launch": how,
                             "stage_ms": {k: round(v, 4) for k, v in per.items()},
                             "roofline": roofline(s, dom, per[dom], "fp32", f"{dom}_fp32_{s.name}")}
        if dom == "dequant_idct":  # the FP32 SIMT contraction: E fused multiply-adds per sample
            tf = 2.0 * s.q.E * s.n_samples / (per[dom] * 1e-3) / 1e12
            res["split_fp32"]["fp32_tflops"] = round(tf, 1)
            res["split_fp32"]["fp32_frac_of_vector_peak"] = round(tf / FP32_VEC_PEAK_TFS, 4)
        outs["split_fp32"] = dec.out[:s.n_samples].cpu().numpy()
        del dec
        release()
    return res, outs


def leg_grad(s: Setup, launch, steps, warmup, tune=False):
    """Forward (plan + fused FP16X2, and the split path the backward needs) and
    backward (coefficient + scale gradients) on the grad workload."""
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    res, outs = leg_fused_vs_fp32(s, launch, steps, warmup, ("fp16x2",), True, tune)
    dec = C.Decoder(s.batch, s.codec, launch)
    dec.plan()
    dec.decode()
    torch.cuda.synchronize()
    g = torch.randn(s.n_samples, device="cuda", dtype=torch.float32) * 1e-6
    gc_ = torch.empty(max(1, s.batch.n_symbols), device="cuda", dtype=torch.float32)
    gg = torch.empty((s.batch.n_streams, 3), device="cuda", dtype=torch.float64)

    def bwd():
        F.fptc_dequant_idct_backward(s.batch.c, s.codec.c, dec.lc, dec.ws, dec.symbols, g, gc_, gg)

    for _ in range(warmup):
        bwd()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        bwd()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    alg = stage_bytes(s, "backward")
    res["backward"] = {"ms": round(ms, 4), "value": round(alg / (ms * 1e-3) / 1e9, 1), "unit": "GB/s algorithmic",
                       "outputs": "grad_coeff f32 [all coefficients] + grad_gamma f64 [streams x 3]",
                       "roofline": {"bound": "hbm", "kernel": kernel_name("backward", s.q.N, "fp32"),
                                    "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                    "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                    "algorithmic_bytes": int(alg)}}
    del dec, g, gc_, gg
    release()
    return res, outs


def sweep(threads, steps, warmup, tune=True):
    """Decoded GB/s over window N and kept coefficients E at the paper
    quantizer (zones [0, 2) mu-law, [2, E) deadzone), on 128 EEG-like streams
    of 2^20 samples: the fused FP16X2 path (N >= 32) and the split FP32 SIMT
    path, each point in the autotuner's launch shape for it (tune) and each
    step timed in its faster launch mode."""
    from paper_2605_01086_amd import codec as C
    from synth import workloads as W
    w = W.workload("sweep")
    rows = []
    for N in (16, 32, 64, 128):
        for E in sorted({4, 8, 16, N // 2, N}):
            if E > N:
                continue
            q = paper_quant(N, E, w)
            s = Setup("sweep", threads, q)
            row = {"N": N, "E": E, "bytes_per_sample_in": round(s.comp_bytes / s.n_samples, 4)}
            if N >= 32:
                lf, how = tuned_launch(s, C.Launch(), "fp16x2", True, tune)
                row["fused_launch"] = how.get("shape")
                dec, ms, _, per, _ = batched(s, lf, "fp16x2", True, steps, warmup)
                row["fused_fp16x2_GBs"] = round(4 * s.n_samples / (ms * 1e-3) / 1e9, 1)
                row["fused_ms"] = round(ms, 4)
                row["fused_kernel_frac_hbm"] = roofline(s, "fused", per["fused"], "fp16x2", "sweep")["frac"]
                del dec
            ls, how = tuned_launch(s, C.Launch(), "fp32", False, tune)
            row["split_launch"] = how.get("shape")
            dec, ms, _, per, _ = batched(s, ls, "fp32", False, steps, warmup)
            row["split_fp32_GBs"] = round(4 * s.n_samples / (ms * 1e-3) / 1e9, 1)
            row["split_ms"] = round(ms, 4)
            row["split_stage_ms"] = {k: round(v, 4) for k, v in per.items()}
            del dec, s
            release()
            rows.append(row)
            log(f"sweep N={N} E={E}: {row}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "plain", "precision", "grad", "large", "paper"],
                    help="headline workload")
    ap.add_argument("--precision", default="fp16x2", choices=["fp32", "fp16", "fp16x2", "bf16", "bf16x3"])
    ap.add_argument("--path", default="fused", choices=["fused", "split"],
                    help="fused: one decode+dequant+IDCT kernel; split: decode kernel then dequant+IDCT kernel")
    ap.add_argument("--wpc", type=int, default=0, help="windows per chunk (0 = library default)")
    ap.add_argument("--waves", type=int, default=0, help="waves per block (0 = library default)")
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--group", type=int, default=0, help="chunks per group in the fused schedule (0 = default)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false", default=True,
                    help="use the library's default launch shape instead of the autotuner's")
    ap.add_argument("--configs", default="plain,precision,grad,large,paper",
                    help="other workloads reported in the same line (comma list, or 'none')")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-stream", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the sweep over window N and kept coefficients E at the paper quantizer")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB copy kernel (torch.neg) 3 times: the reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the decode path is measured on one GPU's share of streams "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n_bytes = 1 << 30
        src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"kernel": "torch.neg elementwise", "read_bytes": n_bytes,
                                               "write_bytes": n_bytes, "dispatches": 3}}), flush=True)
        return

    from paper_2605_01086_amd import codec as C
    threads = host_threads()
    if args.sweep:
        rows = sweep(threads, args.steps, args.warmup, args.autotune)
        print(json.dumps({"sweep": rows, "workload": "128 EEG-like streams x 2^20 samples, paper quantizer",
                          "steps": args.steps}), flush=True)
        return
    s = Setup(args.workload, threads)
    fused = args.path == "fused"
    if fused and args.precision == "fp32":
        raise SystemExit("the fused path runs the MFMA precisions (fp16x2, bf16x3, fp16, bf16)")
    launch = C.Launch(args.wpc, args.waves, args.blocks, args.group)
    tuned = None
    if args.autotune and not (args.wpc or args.waves or args.blocks or args.group):
        from paper_2605_01086_amd import autotune
        launch, tuned = autotune.tune(s.batch, s.codec, args.precision, fused)
        log(f"autotune: {launch} in {tuned['tuning_s']:.1f}s ({'cached' if tuned['cached'] else 'measured'})")
    dec, ms_step, modes, per, gpu = batched(s, launch, args.precision, fused, args.steps, args.warmup)
    head_out = dec.out[:s.n_samples]
    value = 4 * s.n_samples / (ms_step * 1e-3) / 1e9
    dom = max(per, key=per.get)
    roof = roofline(s, dom, per[dom], args.precision, f"{dom}_{args.precision}_{s.name}")
    path_alg = s.comp_bytes + 4 * s.n_samples
    path_roof = HBM_PEAK_GBS * 4 * s.n_samples / path_alg
    line = {
        "metric": "decoded GB/s (float32 output) + % HBM roofline, batched vs plain, at 1 MI355X",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} MFMA, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"fptc-{args.workload}", "streams": s.w.n_streams, "samples": s.n_samples,
                   "window": s.q.N, "kept_coeffs": s.q.E,
                   "quantizer": f"amplitude {s.q.step_fine}/{s.q.step_coarse}/T{s.q.threshold:g}", "lmax": 12,
                   "path": args.path, "precision": args.precision,
                   "launch": {"windows_per_chunk": launch.windows_per_chunk, "waves_per_block": launch.waves_per_block,
                              "blocks": launch.blocks, "chunk_group": launch.chunk_group,
                              "picked_by": "autotuner" if tuned else "fixed"},
                   "launch_mode": modes["launch_mode"], "compressed_bytes": int(s.comp_bytes),
                   "bytes_per_sample_in": round(s.comp_bytes / s.n_samples, 4)},
        "roofline": roof,
        "path_roofline": {"algorithmic_bytes": int(path_alg),
                          "achieved_GBs": round(path_alg / (ms_step * 1e-3) / 1e9, 1),
                          "frac": round(path_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "roofline_decoded_GBs": round(path_roof, 1),
                          "decoded_frac_of_roofline": round(value / path_roof, 4)},
        "stage_ms": {k: round(float(v), 4) for k, v in per.items()},
        "eager_ms_per_step": modes["eager_ms_per_step"], "graph_ms_per_step": modes["graph_ms_per_step"],
        "gpu_ms_per_step": {"median": round(float(np.median(gpu)), 4), "min": round(float(gpu.min()), 4),
                            "max": round(float(gpu.max()), 4)},
        "autotune": tuned,
    }
    cb = copy_bandwidth()
    line["copy_bandwidth"] = {**cb, "kernel_frac_of_copy": round(roof["achieved"] / cb["GBs"], 4),
                              "path_frac_of_copy": round(4 * s.n_samples / (ms_step * 1e-3) / 1e9 / cb["GBs"]
                                                         * (4 + s.comp_bytes / s.n_samples) / 4, 4)}
    head_host = head_out.cpu().numpy()
    out32_host = None
    if args.workload == "batch":
        # the batched FP32 SIMT decoder (split path), then the plain decoder:
        # the same FP32 path as one call sequence per stream
        d32, ms32, _, per32, _ = batched(s, launch, "fp32", False, max(5, args.steps // 2), 2)
        out32 = d32.out[:s.n_samples]
        rng32 = float(out32.max() - out32.min())
        rel = float((out32 - head_out).abs().max()) / rng32
        line["batched_fp32_simt"] = {"value": round(4 * s.n_samples / (ms32 * 1e-3) / 1e9, 2),
                                     "ms_per_step": round(ms32, 4),
                                     "stage_ms": {k: round(v, 4) for k, v in per32.items()},
                                     "max_abs_diff_vs_headline_over_range": float(f"{rel:.3e}"),
                                     "headline_speedup": round(ms32 / ms_step, 2)}
        del dec, head_out
        release()
        if not args.no_per_stream:
            ms_ps, out_ps = time_per_stream(s, C.Launch(0, 4, 0), 3, "fp32")
            rel = float((out_ps[:s.n_samples] - out32).abs().max()) / rng32
            line["plain_per_stream_fp32"] = {"value": round(4 * s.n_samples / (ms_ps * 1e-3) / 1e9, 2),
                                             "unit": "GB/s", "ms_per_step": round(ms_ps, 3),
                                             "calls_per_step": 3 * s.batch.n_streams,
                                             "kernels_per_step": 4 * s.batch.n_streams,
                                             "max_abs_diff_vs_batched_fp32_over_range": float(f"{rel:.3e}"),
                                             "batched_speedup": round(ms_ps / ms_step, 2)}
            del out_ps
        out32_host = out32.cpu().numpy()
        del d32, out32
    else:
        del dec, head_out
    release()
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(7)
        order = rng.permutation(s.w.n_streams)
        cb = cpu_oracle(s, order, threads, args.cpu_budget)
        cb["affine_cores"] = affine_cores()
        cb["cpu_model"] = cpu_model()
        cb["note"] = "threads = affine cores capped at 16, the host's CPU share per GPU"
        if args.workload == "batch":
            subset = np.sort(rng.choice(s.w.n_streams, size=64, replace=False))
            cb["single_thread_batch_subset"] = cpu_oracle(s, subset, 1)
            cb["single_thread_batch_subset"]["sample"] += " (a fixed seeded subset of 64 streams)"
        sample = np.sort(rng.choice(s.w.n_streams, size=min(16, s.w.n_streams), replace=False))
        outs = {f"{args.path}_{args.precision}": head_host}
        if out32_host is not None:
            outs["batched_fp32_simt"] = out32_host
        line["oracle_error"] = errors_vs_oracle(s, outs, sample, threads)
        line["oracle_error"]["streams"] = f"{len(sample)} seeded streams"
        line["cpu_baseline"] = cb
    del head_host, out32_host, s
    release()

    configs = [c for c in args.configs.split(",") if c and c != "none" and c != args.workload]
    line["configs"] = {}
    for name in configs:
        t0 = time.perf_counter()
        entry = {}
        try:
            if name == "precision":
                for N in (64, 256):
                    from paper_2605_01086_amd import codec as Cc
                    q = Cc.quant_params("amp", N, N, step_fine=STEP_F, step_coarse=STEP_C, threshold=THRESH)
                    cs = Setup("precision", threads, q)
                    res, outs = leg_fused_vs_fp32(cs, C.Launch(), max(5, args.steps // 2), 2,
                                                  ("fp16x2", "bf16x3", "fp16", "bf16"), True, args.autotune)
                    if not args.no_cpu_baseline:
                        res["oracle_error"] = errors_vs_oracle(cs, outs, [0, 1], threads)
                        res["oracle_error"]["streams"] = "streams 0 (EEG-like) and 1 (seismic-like)"
                    res["samples"] = cs.n_samples
                    res["bytes_per_sample_in"] = round(cs.comp_bytes / cs.n_samples, 4)
                    entry[f"w{N}"] = res
                    del outs, cs
                    release()
            elif name == "grad":
                cs = Setup("grad", threads)
                entry, outs = leg_grad(cs, C.Launch(), max(5, args.steps // 2), 2, args.autotune)
                entry["samples"] = cs.n_samples
                del outs, cs
                release()
            elif name in ("plain", "large", "paper"):
                cs = Setup(name, threads)
                prec = ("fp16x2",)
                entry, outs = leg_fused_vs_fp32(cs, C.Launch(), max(5, args.steps // 2), 2, prec, True, args.autotune)
                if not args.no_cpu_baseline:
                    if name == "plain":
                        entry["cpu_baseline_single_thread"] = cpu_oracle(cs, [0], 1)
                        entry["oracle_error"] = errors_vs_oracle(cs, outs, [0], 1)
                    elif name == "paper":
                        entry["oracle_error"] = errors_vs_oracle(cs, outs, [0, 1], 2)
                        entry["oracle_error"]["streams"] = "streams 0 and 1"
                    else:
                        entry["oracle_error"] = errors_vs_oracle(cs, outs, [5], 1)
                        entry["oracle_error"]["streams"] = "channel 5"
                entry["samples"] = cs.n_samples
                entry["bytes_per_sample_in"] = round(cs.comp_bytes / cs.n_samples, 4)
                if name == "paper":
                    q = cs.q
                    entry["quantizer"] = {"N": q.N, "E": q.E, "B1": q.B1, "B2": q.B2, "mu": q.mu, "alpha1": q.alpha1,
                                          "A0": q.A0, "A1": q.A1, "percentile": 99.9}
                del outs, cs
                release()
            else:
                raise SystemExit(f"unknown config {name}")
        except torch.cuda.OutOfMemoryError as e:
            entry = {"error": f"out of device memory: {e}"}
        entry["leg_s"] = round(time.perf_counter() - t0, 1)
        line["configs"][name] = entry
        log(f"config {name} done in {entry['leg_s']}s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
