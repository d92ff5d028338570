"""GPU parity of the fused decode + dequant + IDCT entry point: identical
samples to the two-call path with the same precision, within 1e-5 of the FP64
oracle, errors flagged per stream, the symbol array untouched."""
import numpy as np
import pytest

from cases import build_case, paper_params
from gpu_helpers import check_parity, run_gpu

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


@pytest.mark.parametrize("N,E", [(32, 16), (64, 20), (128, 100), (256, 180)])
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


@pytest.mark.parametrize("wpc,waves", [(32, 8), (64, 4), (7, 2)])
def test_fused_window_256_launch_shapes(wpc, waves):
    from paper_2605_01086_amd import codec as C
    c = build_case(_amp(256, step_f=1.0, step_c=8.0, T=16.0), ["eeg"], [256 * 300 + 77, 256 * 33, 100],
                   config_id=1800)
    f = run_gpu(c, precision="fp16x2", fused=True, launch=C.Launch(wpc, waves, 0))
    check_parity(c, f, tol=1e-5, check_symbols=False)


def test_fused_full_size_plain_stream():
    c = build_case(_amp(64), ["eeg"], [1 << 20], config_id=0)
    check_parity(c, run_gpu(c, precision="fp16x2", fused=True), tol=1e-5, check_symbols=False)
