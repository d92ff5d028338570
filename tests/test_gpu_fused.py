"""GPU parity of the fused decode + dequant + IDCT entry point: identical
samples to the two-call path with the same precision, within 1e-5 of the FP64
oracle, errors flagged per stream, the symbol array untouched."""
import numpy as np
import pytest

from cases import build_case, paper_params
from gpu_helpers import qparams, check_parity, run_gpu

pytestmark = pytest.mark.gpu


def _amp(N, E=None, **kw):
    from oracle import oracle as O
    return O.QuantParams("amp", N, N if E is None else E, **kw)


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_fused_equals_two_call_path(prec, N):
    rng = np.random.default_rng(N + 7)
    lens = list(np.floor(2.0 ** rng.uniform(5, 13, size=14)).astype(int)) + [1, N - 1, N, N + 1, 40 * N + 3]
    c = build_case(_amp(N), ["eeg", "seismic", "power", "meteo"], lens, config_id=1400 + N)
    a = run_gpu(c, precision=prec)
    f = run_gpu(c, precision=prec, fused=True)
    assert np.array_equal(a["out"], f["out"]), int(np.sum(a["out"] != f["out"]))
    assert np.array_equal(f["status"], a["status"])
    if prec in ("fp16x2", "bf16x3"):
        check_parity(c, f, tol=1e-5, check_symbols=False)


@pytest.mark.parametrize("wpc,waves,blocks", [(32, 8, 0), (32, 1, 1), (64, 4, 3), (96, 2, 0), (7, 4, 0), (1, 8, 5)])
def test_fused_launch_shapes(wpc, waves, blocks):
    from paper_2605_01086_amd import codec as C
    rng = np.random.default_rng(wpc * 10 + waves)
    lens = list(np.floor(2.0 ** rng.uniform(4, 13, size=20)).astype(int))
    c = build_case(_amp(64), ["eeg", "seismic", "power", "meteo"], lens, config_id=1500)
    f = run_gpu(c, precision="fp16x2", fused=True, launch=C.Launch(wpc, waves, blocks))
    check_parity(c, f, tol=1e-5, check_symbols=False)


@pytest.mark.parametrize("N,E", [(32, 16), (64, 20), (64, 64), (128, 100), (256, 180), (256, 256)])
def test_fused_paper_quantizer_with_scales(N, E):
    p = paper_params(N, E, "eeg", 1600 + N)
    c = build_case(p, ["eeg", "seismic"], [N * 150 + 7, 3001, 5, N * 31], config_id=1600 + N, gamma=True)
    for prec in ("fp16x2", "bf16x3"):
        check_parity(c, run_gpu(c, precision=prec, fused=True), tol=1e-5, check_symbols=False)


@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_whole_tile_stores_at_every_alignment(N):
    # streams start at sample offsets 0, 1, 2, 3 (mod 4) and hold whole
    # 32-window tiles, so tile stores meet every 16-byte misalignment; both
    # entry points (split: dequant+IDCT from the symbol array)
    T = 32 * N
    lens = [1, 2 * T + 1, 3 * T + 1, T + 2, 2 * T + 3, 77]
    assert [int(x) % 4 for x in np.cumsum([0] + lens[:-1])] == [0, 1, 2, 3, 1, 0]
    kw = dict(step_f=1.0, step_c=8.0, T=16.0) if N == 256 else {}
    c = build_case(_amp(N, **kw), ["eeg", "seismic", "power", "meteo"], lens, config_id=1900 + N)
    for fused in (False, True):
        check_parity(c, run_gpu(c, precision="fp16x2", fused=fused), tol=1e-5, check_symbols=not fused)


def test_fused_flags_corrupt_streams_and_isolates_the_rest():
    from paper_2605_01086_amd import fptc as F
    lens = [4000, 5000, 6000, 7000, 3000]
    c = build_case(_amp(64), ["eeg", "seismic"], lens, config_id=1700)
    words, symlen, word_off, sample_off = c.concat()
    sl = symlen.copy()
    sl[word_off[1] + 3] -= 1
    sl[word_off[3] + 2] = 200
    res = run_gpu(c, symlen_override=sl, precision="fp16x2", fused=True)
    assert res["status"][1] & F.FPTC_STREAM_BAD_COUNT
    assert res["status"][3] & F.FPTC_STREAM_BAD_SYMLEN
    check_parity(c, res, tol=1e-5, skip={1, 3}, check_symbols=False)


@pytest.mark.parametrize("wpc,waves,blocks", [(32, 8, 0), (40, 0, 3), (7, 8, 1), (1, 0, 0), (33, 8, 5)])
def test_window_256_launch_shapes(wpc, waves, blocks):
    # both entry points at window 256 (8 waves per workgroup, one per parity
    # and column tile), odd chunk sizes and grids
    from paper_2605_01086_amd import codec as C
    c = build_case(_amp(256, step_f=1.0, step_c=8.0, T=16.0), ["eeg"], [256 * 300 + 77, 256 * 33, 100],
                   config_id=1800)
    L = C.Launch(wpc, waves, blocks)
    f = run_gpu(c, precision="fp16x2", fused=True, launch=L)
    check_parity(c, f, tol=1e-5, check_symbols=False)
    s = run_gpu(c, precision="fp16x2", fused=False, launch=L)
    assert np.array_equal(s["out"], f["out"])


def test_window_256_fused_refuses_other_wave_counts():
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    c = build_case(_amp(256), ["eeg"], [256 * 4], config_id=1810, recon=False)
    words, symlen, word_off, sample_off = c.concat()
    codec = C.DeviceCodec(np.stack([b.lengths for b in c.books]), qparams(c.p), 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, 256, 256, c.book_id)
    lc = C.Launch(32, 4, 0).c()
    ws = torch.empty(F.fptc_workspace_size(batch.c, codec.c, lc), dtype=torch.uint8, device="cuda")
    out = torch.empty(batch.n_samples, dtype=torch.float32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(F.FptcError) as e:
        F.fptc_decompress_batch(batch.c, codec.c, lc, ws, None, "fp16x2", out, st)
    assert e.value.code == F.FPTC_ERR_UNSUPPORTED


@pytest.mark.parametrize("N", [64, 256])
def test_precisions_share_one_plan(N):
    # calls of different precisions and both entry points on one plan (no
    # re-planning in between) give exactly what each gives alone: no call
    # writes the workspace except the plan
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    kw = dict(step_f=1.0, step_c=8.0, T=16.0) if N == 256 else {}
    c = build_case(_amp(N, **kw), ["eeg", "seismic"], [N * 70 + 3, N * 41], config_id=1820 + N, recon=False)
    words, symlen, word_off, sample_off = c.concat()
    codec = C.DeviceCodec(np.stack([b.lengths for b in c.books]), qparams(c.p), 12)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, N, N, c.book_id)
    lc = C.Launch().c()
    ws = torch.empty(F.fptc_workspace_size(batch.c, codec.c, lc), dtype=torch.uint8, device="cuda")
    st = torch.zeros(batch.n_streams, dtype=torch.int32, device="cuda")
    sym = torch.empty(batch.n_symbols, dtype=torch.uint8, device="cuda")

    def solo(prec, fused):
        out = torch.empty(batch.n_samples, dtype=torch.float32, device="cuda")
        F.fptc_plan_batch(batch.c, codec.c, lc, ws, st)
        if fused:
            F.fptc_decompress_batch(batch.c, codec.c, lc, ws, None, prec, out, st)
        else:
            F.fptc_decode_batch(batch.c, codec.c, lc, ws, sym, st)
            F.fptc_dequant_idct(batch.c, codec.c, lc, ws, sym, None, prec, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    combos = [(p, f) for p in ("fp16x2", "bf16x3", "fp16") for f in (True, False)]
    alone = {k: solo(*k) for k in combos}
    F.fptc_plan_batch(batch.c, codec.c, lc, ws, st)
    F.fptc_decode_batch(batch.c, codec.c, lc, ws, sym, st)
    outs = {k: torch.empty(batch.n_samples, dtype=torch.float32, device="cuda") for k in combos}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for i, (prec, fused) in enumerate(combos):
        with torch.cuda.stream(side if i % 2 else torch.cuda.current_stream()):
            if fused:
                F.fptc_decompress_batch(batch.c, codec.c, lc, ws, None, prec, outs[(prec, fused)], st)
            else:
                F.fptc_dequant_idct(batch.c, codec.c, lc, ws, sym, None, prec, outs[(prec, fused)])
    torch.cuda.synchronize()
    for k in combos:
        assert np.array_equal(outs[k].cpu().numpy(), alone[k]), k


def test_fused_full_size_plain_stream():
    c = build_case(_amp(64), ["eeg"], [1 << 20], config_id=0)
    check_parity(c, run_gpu(c, precision="fp16x2", fused=True), tol=1e-5, check_symbols=False)
