#!/usr/bin/env python3
"""FPTC batch decompression benchmark on one MI355X.

One step = the whole decode path over one batch already resident in HBM:
plan (stream/chunk setup + symlen prefix sums) -> Huffman decode with
compaction -> dequantization fused with the inverse DCT, float32 out.

Default workload ("batch"): 4096 synthetic streams, lengths log-uniform in
2^14..2^20 samples, domains EEG / seismic / power-grid / meteorological in
turn, window 64, amplitude quantizer (steps 0.25 / 2.0, threshold 16), one
codebook per domain trained on separate data, L_max 12.  "plain": one EEG-like
stream of 2^20 samples with the same codec.

Prints one JSON line: decoded GB/s (4 bytes per output sample / step time),
the HBM roofline of the dominant kernel measured with HIP events, a
per-stream-launch comparison and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
STEP_F, STEP_C, THRESH = 0.25, 2.0, 16.0


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def make_workload(name: str, threads: int):
    """Signals, stream lengths, per-stream domain and the codebook training data."""
    import synth
    if name == "batch":
        config_id, n = 1, 4096
        rng = np.random.default_rng(np.random.SeedSequence(synth.ROOT_SEED, spawn_key=(2, 1)))
        lens = synth.batch_lengths(n, 14.0, 20.0, rng)
        dom = np.arange(n) % 4
    elif name == "plain":
        config_id, n = 0, 1
        lens = np.array([1 << 20], dtype=np.int64)
        dom = np.zeros(1, dtype=np.int64)
    elif name == "large":
        # 64 channels x 2^24 samples of EEG-like sources mixed by a random 64x64 matrix
        config_id, n_ch, L = 4, 64, 1 << 24
        rng = synth.stream_rng(config_id, 0)
        src = np.empty((n_ch, L), dtype=np.float32)

        def gen_src(i):
            src[i] = synth.eeg_like(L, synth.stream_rng(config_id, 1 + i))

        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(gen_src, range(n_ch)))
        M = (rng.standard_normal((n_ch, n_ch)) / np.sqrt(n_ch)).astype(np.float32)
        x = np.ascontiguousarray((M @ src).reshape(-1))
        del src
        sample_off = np.arange(n_ch + 1, dtype=np.int64) * L
        tr_src = np.stack([synth.eeg_like(1 << 16, synth.training_rng(config_id, i)) for i in range(n_ch)])
        train = [(M.astype(np.float64) @ tr_src).reshape(-1).astype(np.float32)]
        return x, sample_off, np.zeros(n_ch, dtype=np.uint8), train
    else:
        raise SystemExit(f"unknown workload {name}")
    sample_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x = np.empty(int(sample_off[-1]), dtype=np.float32)

    def gen(i):
        x[sample_off[i]:sample_off[i + 1]] = synth.domain_signal(synth.DOMAINS[dom[i]], int(lens[i]),
                                                                 synth.stream_rng(config_id, i))

    order = np.argsort(-lens)  # longest first for balance
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(gen, order))
    n_dom = 4 if name == "batch" else 1
    train = [synth.domain_signal(synth.DOMAINS[d], 1 << 18, synth.training_rng(config_id, d)).astype(np.float32)
             for d in range(n_dom)]
    return x, sample_off, dom.astype(np.uint8), train


def encode(x, sample_off, dom, train, q, threads):
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    lens_tab = np.stack([C.train_code_lengths(t, q) for t in train])
    L = np.diff(sample_off)
    nsym = C.n_windows(L, q.N) * q.E
    cap_off = np.concatenate([[0], np.cumsum(nsym + 1)]).astype(np.int64)
    words = np.zeros(int(cap_off[-1]), dtype=np.uint64)
    symlen = np.zeros(int(cap_off[-1]), dtype=np.uint8)
    nw = F.fptc_encode_batch_host(x, sample_off, dom, q, lens_tab, cap_off, words, symlen, threads)
    word_off = np.concatenate([[0], np.cumsum(nw)]).astype(np.int64)
    # compact the per-stream reserved ranges
    wc = np.empty(int(word_off[-1]), dtype=np.uint64)
    sc = np.empty(int(word_off[-1]), dtype=np.uint8)
    for i in range(len(nw)):
        wc[word_off[i]:word_off[i + 1]] = words[cap_off[i]:cap_off[i] + nw[i]]
        sc[word_off[i]:word_off[i + 1]] = symlen[cap_off[i]:cap_off[i] + nw[i]]
    return wc, sc, word_off, lens_tab


def time_batched(dec, steps, warmup, precision, fused=False):
    """Per step: plan, then the fused kernel or decode + dequant/IDCT.
    Returns host ms/step, mean HIP-event ms of each stage, per-step GPU ms."""
    import torch
    for _ in range(warmup):
        dec.run(precision=precision, fused=fused)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        e = ev[k]
        e[0].record()
        dec.plan()
        e[1].record()
        if fused:
            dec.decompress(precision=precision)
            e[2].record()
        else:
            dec.decode()
            e[2].record()
            dec.dequant_idct(precision=precision)
        e[3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ev])  # ms
    gpu = np.array([e[0].elapsed_time(e[3]) for e in ev])
    return wall / steps * 1e3, per.mean(axis=0), gpu


def time_per_stream(batch, codec, launch, steps, precision):
    """The same decode issued as one plan/decode/dequant+IDCT launch sequence per stream."""
    import ctypes
    import torch
    from paper_2605_01086_amd import fptc as F
    dev = batch.word_off.device
    n = batch.n_streams
    wo, so, yo = batch.word_off_h, batch.sample_off_h, batch.sym_off_h
    loc_w = torch.from_numpy(np.stack([np.zeros(n, np.int64), np.diff(wo)], 1).copy()).to(dev)
    loc_s = torch.from_numpy(np.stack([np.zeros(n, np.int64), np.diff(so)], 1).copy()).to(dev)
    lib = F.load()
    lc = launch.c()
    structs = []
    ws_bytes = 0
    for s in range(n):
        b = F.fptc_batch(1, 0, int(wo[s + 1] - wo[s]), int(yo[s + 1] - yo[s]), int(so[s + 1] - so[s]),
                         batch.words.data_ptr() + 8 * int(wo[s]), batch.symlen.data_ptr() + int(wo[s]),
                         loc_w.data_ptr() + 16 * s, loc_s.data_ptr() + 16 * s,
                         None if batch.book_id is None else batch.book_id.data_ptr() + s)
        structs.append(b)
        ws_bytes = max(ws_bytes, F.fptc_workspace_size(b, codec.c, lc))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    sym = torch.empty(max(1, batch.n_symbols), dtype=torch.uint8, device=dev)
    out = torch.empty(max(1, batch.n_samples), dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    by = ctypes.byref
    cp = by(codec.c)
    lp = by(lc)
    prec = F.PRECISIONS[precision]

    def one_pass():
        for s in range(n):
            bp = by(structs[s])
            sp = status.data_ptr() + 4 * s
            rc = lib.fptc_plan_batch(bp, cp, lp, ws.data_ptr(), ws_bytes, sp, st)
            rc |= lib.fptc_decode_batch(bp, cp, lp, ws.data_ptr(), ws_bytes, sym.data_ptr() + int(yo[s]), sp, st)
            rc |= lib.fptc_dequant_idct(bp, cp, lp, ws.data_ptr(), ws_bytes, sym.data_ptr() + int(yo[s]), None, prec,
                                        out.data_ptr() + 4 * int(so[s]), st)
            if rc:
                raise RuntimeError("per-stream launch failed")

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return ms, out


def cpu_baseline(words, symlen, word_off, sample_off, dom, lens_tab, q, budget_s, threads):
    """The CPU oracle (bit-serial decode + FP64 dequant/IDCT), timed on a bounded
    sample of the same streams: streams in a fixed shuffled order until the
    time budget is used."""
    from oracle import oracle as O
    p = O.QuantParams("amp", q.N, q.E, step_f=q.step_fine, step_c=q.step_coarse, T=q.threshold)
    books = [O.Codebook(lens_tab[b]) for b in range(lens_tab.shape[0])]
    n = len(sample_off) - 1
    order = np.random.default_rng(7).permutation(n)
    done = {"samples": 0, "streams": 0}
    t0 = time.perf_counter()

    def work(s):
        if time.perf_counter() - t0 > budget_s:
            return 0
        L = int(sample_off[s + 1] - sample_off[s])
        nsym = O.n_windows(L, q.N) * q.E
        sym = O.symlen_decode(words[word_off[s]:word_off[s + 1]], symlen[word_off[s]:word_off[s + 1]],
                              books[int(dom[s])], nsym)
        O.reconstruct(sym, L, p)
        return L

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(work, order))
    dt = time.perf_counter() - t0
    done["samples"] = int(sum(res))
    done["streams"] = int(sum(1 for r in res if r))
    return done, dt


# Sources of the kernel each roofline stage names; an HBM-traffic summary in
# profiles/ applies only while these hash to the digest recorded in it.
PLAN_KERNELS = "k_plan_streams+k_plan_seg_sums+k_plan_stream_scan+k_plan_seg_chunks"
KERNEL_SOURCES = {
    "fused": ["fused.hip", "mfma256.hip", "decode_common.h", "mfma_common.h", "fptc_internal.h"],
    "decode": ["decode.hip", "decode_common.h", "mfma_common.h", "fptc_internal.h"],
    "dequant_idct": ["dqidct_mfma.hip", "dqidct.hip", "mfma256.hip", "mfma_common.h", "fptc_internal.h"],
    "plan": ["plan.hip", "fptc_internal.h"],
}


def source_digest(stage: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[stage]:
        with open(os.path.join(ROOT, "paper_2605_01086_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(stage: str, tag: str):
    """HBM bytes per launch from profiles/traffic_<tag>.txt (rocprofv3
    FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the same counters on a
    plain copy kernel of known size), or None when absent or taken on other
    sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest(stage):
        return None, "kernel changed since the counters were taken"
    return int(float(kv["traffic_bytes_per_dispatch"])), path[len(ROOT) + 1:]


def copy_calibration(n_bytes: int = 1 << 30, reps: int = 3):
    """A plain elementwise kernel that reads n_bytes and writes n_bytes once
    each; its HBM counters per dispatch give the counters' scale."""
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "torch.neg elementwise", "read_bytes": n_bytes,
                                           "write_bytes": n_bytes, "dispatches": reps}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "plain", "large"])
    ap.add_argument("--precision", default="fp16x2", choices=["fp32", "fp16", "fp16x2", "bf16", "bf16x3"])
    ap.add_argument("--path", default="fused", choices=["fused", "split"],
                    help="fused: one decode+dequant+IDCT kernel; split: decode kernel then dequant+IDCT kernel")
    ap.add_argument("--wpc", type=int, default=32)
    ap.add_argument("--waves", type=int, default=0, help="waves per block (0 = library default)")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape by timing candidates")
    ap.add_argument("--graph", dest="graph", action="store_true", default=True,
                    help="time the step as replays of one captured HIP graph (plan + decode kernels; default)")
    ap.add_argument("--no-graph", dest="graph", action="store_false", help="time eager launches instead")
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-stream", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB copy kernel (torch.neg) 3 times: the reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the decode path has no multi-GPU split in this build "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    threads = host_threads()
    t_setup = time.perf_counter()
    from paper_2605_01086_amd import codec as C
    if args.workload == "large":  # window 256, coarse steps 1.0 / 8.0
        q = C.quant_params("amp", 256, 256, step_fine=1.0, step_coarse=8.0, threshold=THRESH)
    else:
        q = C.quant_params("amp", 64, 64, step_fine=STEP_F, step_coarse=STEP_C, threshold=THRESH)
    x, sample_off, dom, train = make_workload(args.workload, threads)
    words, symlen, word_off, lens_tab = encode(x, sample_off, dom, train, q, threads)
    n_samples = int(sample_off[-1])
    del x
    t_enc = time.perf_counter() - t_setup
    print(f"[bench] workload {args.workload}: {len(sample_off) - 1} streams, {n_samples} samples, "
          f"{len(words)} words, setup {t_enc:.1f}s", file=sys.stderr, flush=True)

    import torch
    torch.cuda.set_device(0)
    codec = C.DeviceCodec(lens_tab, q, 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, q.N, q.E, dom if args.workload == "batch" else None)
    fused = args.path == "fused"
    if fused and args.precision == "fp32":
        raise SystemExit("the fused path runs the MFMA precisions (fp16x2, bf16x3, fp16, bf16)")
    launch = C.Launch(args.wpc, args.waves, args.blocks)
    tuned = None
    if args.autotune:
        from paper_2605_01086_amd import autotune
        launch, tuned = autotune.tune(batch, codec, args.precision, fused, use_cache=False)
    dec = C.Decoder(batch, codec, launch)
    ms_step, per_kernel, gpu_steps = time_batched(dec, args.steps, args.warmup, args.precision, fused)
    eager_ms = ms_step
    graph_ms = None
    if args.graph:
        from paper_2605_01086_amd.graph import CapturedStep
        step = CapturedStep(dec, args.precision, fused)
        for _ in range(args.warmup):
            step.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
        ms_step = graph_ms
    status = dec.status.cpu().numpy()
    if np.any(status != 0):
        raise SystemExit(f"decode reported stream errors: {np.flatnonzero(status)[:8]}")

    out_bytes = 4 * n_samples
    value = out_bytes / (ms_step * 1e-3) / 1e9
    comp_bytes = batch.compressed_bytes + batch.header_bytes
    # algorithmic bytes of one launch of each stage (measurement):
    # compressed words 8 B + symlen 1 B per word, per-stream headers, 1 B per
    # decoded symbol written or read between the split kernels, 4 B per sample.
    if fused:
        names = ["plan", "fused"]
        stage_ms = per_kernel[:2]
        alg = {"plan": batch.n_words + batch.header_bytes, "fused": comp_bytes + out_bytes}
        kern = {"plan": PLAN_KERNELS, "fused": f"k_fused{'256' if q.N == 256 else ''}<{args.precision}>"}
    else:
        names = ["plan", "decode", "dequant_idct"]
        stage_ms = per_kernel
        alg = {"plan": batch.n_words + batch.header_bytes, "decode": comp_bytes + batch.n_symbols,
               "dequant_idct": batch.n_symbols + out_bytes}
        kern = {"plan": PLAN_KERNELS, "decode": "k_decode",
                "dequant_idct": "k_dqidct_f32" if args.precision == "fp32"
                else f"k_dqidct_mfma{'256' if q.N == 256 else ''}<{args.precision}>"}
    dom_k = int(np.argmax(stage_ms))
    kname = names[dom_k]
    achieved = alg[kname] / (stage_ms[dom_k] * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(kname, f"{kname}_{args.precision}_{args.workload}")
    roof = {"bound": "hbm", "kernel": kern[kname], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": traffic_src, "algorithmic_bytes": int(alg[kname]),
            "avg_ms": round(float(stage_ms[dom_k]), 4)}
    path_alg = comp_bytes + out_bytes
    path_roofline_decoded = HBM_PEAK_GBS * out_bytes / path_alg
    line = {
        "metric": "decoded GB/s (float32 output) + % HBM roofline, batched vs plain, at 1 MI355X",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} MFMA, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"fptc-{args.workload}", "streams": int(len(sample_off) - 1),
                   "samples": n_samples, "window": q.N, "kept_coeffs": q.E, "quantizer": f"amplitude {q.step_fine}/{q.step_coarse}/T{q.threshold:g}",
                   "lmax": 12, "path": args.path, "precision": args.precision,
                   "windows_per_chunk": launch.windows_per_chunk, "waves_per_block": launch.waves_per_block,
                   "blocks": launch.blocks, "hip_graph": bool(args.graph), "compressed_bytes": int(comp_bytes),
                   "bytes_per_sample_in": round(comp_bytes / n_samples, 4)},
        "roofline": roof,
        "path_roofline": {"algorithmic_bytes": int(path_alg), "achieved_GBs": round(path_alg / (ms_step * 1e-3) / 1e9, 1),
                          "frac": round(path_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "roofline_decoded_GBs": round(path_roofline_decoded, 1),
                          "decoded_frac_of_roofline": round(value / path_roofline_decoded, 4)},
        "stage_ms": {k: round(float(v), 4) for k, v in zip(names, stage_ms)},
        "eager_ms_per_step": round(float(eager_ms), 4),
        "autotune_ms": tuned,
        "gpu_ms_per_step": {"median": round(float(np.median(gpu_steps)), 4), "min": round(float(gpu_steps.min()), 4),
                            "max": round(float(gpu_steps.max()), 4)},
    }
    if not args.no_per_stream and args.workload == "batch":
        # the plain decoder: FP32 SIMT dequant+IDCT, one launch sequence per stream
        ms_ps, out_ps = time_per_stream(batch, codec, C.Launch(args.wpc, 4, 0), 3, "fp32")
        a, bref = out_ps[:n_samples], dec.out[:n_samples]
        rel = float((a - bref).abs().max() / (bref.max() - bref.min()))
        line["plain_per_stream_fp32"] = {"value": round(out_bytes / (ms_ps * 1e-3) / 1e9, 2), "unit": "GB/s",
                                         "ms_per_step": round(ms_ps, 3), "launches_per_step": 4 * batch.n_streams,
                                         "max_abs_diff_vs_batched_over_range": rel,
                                         "batched_speedup": round(ms_ps / ms_step, 2)}
    if not args.no_cpu_baseline:
        done, dt = cpu_baseline(words, symlen, word_off, sample_off, dom, lens_tab, q, args.cpu_budget, threads)
        line["cpu_baseline"] = {"value": round(4 * done["samples"] / dt / 1e9, 5), "unit": "GB/s", "cores": threads,
                                "kind": "oracle",
                                "sample": f"{done['streams']} of {len(sample_off) - 1} streams "
                                          f"({done['samples']} samples) in {dt:.1f}s, fixed shuffled order"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
