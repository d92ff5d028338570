"""Full-size workloads on the GPU in the launch configuration the benchmark
times, checked on sampled streams against the FP64 oracle (the oracle
decodes and reconstructs those streams one by one).

* precision workload: 2^28 samples, 128 EEG-like + 128 seismic-like streams of
  2^20, windows 64 and 256, every MFMA variant and FP32, max-abs and RMS error
  against FP64 reported per variant;
* large multichannel workload: 64 channels x 2^24 EEG-like samples mixed by a
  random matrix, window 256, steps 1.0 / 8.0, fused FP16X2 vs FP32;
* batch workload: all 4096 streams (about 1.02e9 samples) compared with the
  oracle stream by stream."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _encode_with_oracle(O, p, signals, books, book_of, threads=16):
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        return O.encode_stream(signals[i], p, books[book_of[i]])

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(signals))))


def _device(p, books, signals, enc, book_of):
    from gpu_helpers import qparams
    from paper_2605_01086_amd import codec as C
    words = np.concatenate([e[0] for e in enc])
    symlen = np.concatenate([e[1] for e in enc])
    word_off = np.concatenate([[0], np.cumsum([len(e[0]) for e in enc])])
    sample_off = np.concatenate([[0], np.cumsum([len(x) for x in signals])])
    codec = C.DeviceCodec(np.stack([b.lengths for b in books]), qparams(p), 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, p.N, p.E, np.asarray(book_of, np.uint8))
    return codec, batch


@pytest.mark.parametrize("N", [64, 256])
def test_precision_workload_sampled(N):
    import torch
    import synth
    from oracle import oracle as O
    from paper_2605_01086_amd import codec as C
    p = O.QuantParams("amp", N, N)
    books = []
    for d, dom in enumerate(["eeg", "seismic"]):
        tr = synth.domain_signal(dom, 1 << 16, synth.training_rng(2, d)).astype(np.float32)
        books.append(O.train_codebook(O.quantize_stream(tr, p)))
    n, L = 256, 1 << 20
    book_of = [i % 2 for i in range(n)]
    signals = [synth.domain_signal(["eeg", "seismic"][book_of[i]], L, synth.stream_rng(2, i)).astype(np.float32)
               for i in range(n)]
    enc = _encode_with_oracle(O, p, signals, books, book_of)
    codec, batch = _device(p, books, signals, enc, book_of)
    sample = np.random.default_rng(N).choice(n, size=6, replace=False)
    refs = {int(i): O.reconstruct(enc[i][2], L, p) for i in sample}
    dec = C.Decoder(batch, codec)
    dec.plan()
    dec.decode()
    torch.cuda.synchronize()
    assert int((dec.status != 0).sum()) == 0
    symbols = dec.symbols.cpu().numpy()
    for i in sample:  # decoded symbols equal the oracle's quantized symbols
        assert np.array_equal(symbols[batch.sym_off_h[i]:batch.sym_off_h[i + 1]], enc[i][2])
    report = {}
    for prec, tol in [("fp32", 1e-5), ("fp16x2", 1e-5), ("bf16x3", 1e-5), ("fp16", 2e-3), ("bf16", 2e-2)]:
        out = dec.dequant_idct(precision=prec).cpu().numpy()
        worst_rel, worst_abs, rms = 0.0, 0.0, 0.0
        for i in sample:
            got = out[batch.sample_off_h[i]:batch.sample_off_h[i + 1]].astype(np.float64)
            ref = refs[int(i)]
            d = got - ref
            worst_abs = max(worst_abs, float(np.abs(d).max()))
            worst_rel = max(worst_rel, float(np.abs(d).max() / np.ptp(ref)))
            rms = max(rms, float(np.sqrt(np.mean(d * d))))
        report[prec] = (worst_abs, rms, worst_rel)
        assert worst_rel <= tol, (prec, worst_rel)
    for prec in ("fp16x2", "bf16x3", "fp16", "bf16"):  # fused path: same samples as the split path
        a = dec.dequant_idct(precision=prec).clone()
        f = dec.decompress(precision=prec)
        assert torch.equal(a, f), prec
    print(f"\nW={N} error vs FP64 over 6 sampled streams (max-abs, RMS, max-abs/range):")
    for k, (a, r, rel) in report.items():
        print(f"  {k:7s} {a:.3e} {r:.3e} {rel:.3e}")


def test_large_multichannel_workload_sampled():
    import torch
    import synth
    from oracle import oracle as O
    from paper_2605_01086_amd import codec as C
    p = O.QuantParams("amp", 256, 256, step_f=1.0, step_c=8.0, T=16.0)
    n_ch, L = 64, 1 << 24
    rng = synth.stream_rng(4, 0)
    M = rng.standard_normal((n_ch, n_ch)) / np.sqrt(n_ch)
    src = np.stack([synth.eeg_like(L, synth.stream_rng(4, 1 + i)) for i in range(n_ch)])
    x = (M @ src).astype(np.float32)
    del src
    tr = (M @ np.stack([synth.eeg_like(1 << 14, synth.training_rng(4, i)) for i in range(n_ch)])).reshape(-1)
    books = [O.train_codebook(O.quantize_stream(tr.astype(np.float32), p))]
    signals = [x[i] for i in range(n_ch)]
    enc = _encode_with_oracle(O, p, signals, books, [0] * n_ch)
    codec, batch = _device(p, books, signals, enc, [0] * n_ch)
    dec = C.Decoder(batch, codec)
    dec.plan()
    fused = dec.decompress(precision="fp16x2").clone()
    dec.decode()
    fp32 = dec.dequant_idct(precision="fp32")
    torch.cuda.synchronize()
    assert int((dec.status != 0).sum()) == 0
    symbols = dec.symbols.cpu().numpy()
    for i in range(n_ch):
        assert np.array_equal(symbols[batch.sym_off_h[i]:batch.sym_off_h[i + 1]], enc[i][2]), i
    out_f, out_32 = fused.cpu().numpy(), fp32.cpu().numpy()
    rng = np.random.default_rng(4)
    nwin = L // 256
    for i in rng.choice(n_ch, size=3, replace=False):
        # decoded symbols of the whole channel equal the oracle's
        s0 = batch.sym_off_h[i]
        for w0 in list(rng.integers(0, nwin - 4096, size=3)) + [nwin - 4096]:
            # the oracle reconstructs 4096 sampled windows of the channel
            ref = O.reconstruct(enc[i][2][w0 * 256:(w0 + 4096) * 256], 4096 * 256, p)
            o0 = batch.sample_off_h[i] + w0 * 256
            for out in (out_f, out_32):
                got = out[o0:o0 + 4096 * 256]
                assert np.abs(got - ref).max() <= 1e-5 * np.ptp(ref)


@pytest.mark.timeout(900)
def test_batch_workload_every_stream():
    """The batch workload at full size (4096 streams of floor(2^U(14, 20))
    samples, four signal domains with a codebook each, window 64): every
    stream encoded by the oracle, decoded on the GPU in the launch shape the
    benchmark times, and compared stream by stream with the oracle -- symbols
    bit-exact (split path), reconstruction within 1e-5 of each stream's range
    for FP32 SIMT (split) and FP16X2 (fused)."""
    import os
    import time
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from synth import workloads as W
    from oracle import oracle as O
    from paper_2605_01086_amd import codec as C
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    w = W.workload("batch")
    p = O.QuantParams("amp", 64, 64, step_f=0.25, step_c=2.0, T=16.0)
    books = [O.train_codebook(O.quantize_stream(t, p)) for t in W.training_signals(w)]
    x = W.signals(w, threads=threads)
    off = w.sample_off

    def enc_one(i):
        return O.encode_stream(x[off[i]:off[i + 1]], p, books[w.book_id[i]])

    with ThreadPoolExecutor(threads) as ex:
        enc = list(ex.map(enc_one, range(w.n_streams)))
    signals_len = [int(L) for L in w.lengths]
    del x
    t_enc = time.perf_counter() - t0
    codec, batch = _device(p, books, [np.empty(L, np.float32) for L in signals_len], enc, w.book_id)
    dec = C.Decoder(batch, codec)
    dec.plan()
    dec.decode()
    split32 = dec.dequant_idct(precision="fp32").cpu().numpy()
    fused = dec.decompress(precision="fp16x2").cpu().numpy()
    status = dec.status.cpu().numpy()
    symbols = dec.symbols.cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(status == 0), np.flatnonzero(status)[:8]
    so, yo = batch.sample_off_h, batch.sym_off_h

    def check(i):
        sym = enc[i][2]
        if not np.array_equal(symbols[yo[i]:yo[i + 1]], sym):
            return (i, "symbols", np.inf, np.inf)
        ref = O.reconstruct(sym, signals_len[i], p)
        rng = float(np.ptp(ref)) or 1.0
        e32 = float(np.abs(split32[so[i]:so[i + 1]] - ref).max()) / rng
        e16 = float(np.abs(fused[so[i]:so[i + 1]] - ref).max()) / rng
        return (i, "ok", e32, e16)

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(check, range(w.n_streams)))
    bad_sym = [r[0] for r in res if r[1] != "ok"]
    assert not bad_sym, f"streams whose symbols differ from the oracle's: {bad_sym[:8]}"
    e32 = np.array([r[2] for r in res])
    e16 = np.array([r[3] for r in res])
    print(f"\nbatch workload: {w.n_streams} streams, {int(off[-1])} samples, oracle encode {t_enc:.1f}s, "
          f"total {time.perf_counter() - t0:.1f}s; worst range-relative error: FP32 split {e32.max():.3e} "
          f"(stream {int(e32.argmax())}), FP16X2 fused {e16.max():.3e} (stream {int(e16.argmax())})")
    assert e32.max() <= 1e-5 and e16.max() <= 1e-5
