"""Codes longer than 12 bits (L_max 13..16, Section 3.3's length limit):
the decoders switch to two-level lookup tables built in LDS.  Symbols must
equal the oracle's bit-serial decode exactly, samples the FP64 oracle within
1e-5 of the range, on both entry points, and a corrupt stream is flagged as
the oracle's decode rejects it."""
import numpy as np
import pytest

import synth
from cases import Case
from gpu_helpers import check_parity, run_gpu

pytestmark = pytest.mark.gpu


def _long_case(O, lmax, N=64, config_id=2700, lengths=(5000, 64 * 77, 1, 333, 20000, 64 * 40 + 63)):
    # frequencies that give the symbols common in the data (levels near the
    # zero level) the longest codes, so most lookups take the second level
    r = np.abs(np.arange(256) - 128).astype(np.float64)
    freq = (1 + r ** 3).astype(np.uint64)
    book = O.Codebook(O.package_merge(freq, lmax))
    assert int(book.lengths.max()) == lmax
    kw = dict(step_f=1.0, step_c=8.0, T=16.0) if N == 256 else {}
    p = O.QuantParams("amp", N, N, **kw)
    doms = ["eeg", "seismic", "power", "meteo"]
    sig, W, S, Y, R = [], [], [], [], []
    for i, L in enumerate(lengths):
        x = synth.domain_signal(doms[i % 4], int(L), synth.stream_rng(config_id, i)).astype(np.float32)
        w, sl, sym = O.encode_stream(x, p, book)
        sig.append(x), W.append(w), S.append(sl), Y.append(sym), R.append(O.reconstruct(sym, len(x), p))
    long_frac = np.mean(np.concatenate([book.lengths[y] > 12 for y in Y]))
    assert long_frac > 0.3
    return Case(p, [book], sig, np.zeros(len(sig), np.uint8), W, S, Y, recon=R, lmax=lmax)


@pytest.mark.parametrize("lmax", [13, 14, 16])
@pytest.mark.parametrize("fused", [False, True])
def test_long_codes_match_the_oracle(O, lmax, fused):
    c = _long_case(O, lmax)
    res = run_gpu(c, precision="fp16x2" if fused else "fp32", fused=fused)
    check_parity(c, res, tol=1e-5, check_symbols=not fused)


def test_long_codes_window_256_split_path(O):
    c = _long_case(O, 16, N=256, config_id=2710, lengths=(256 * 50 + 3, 256 * 33))
    res = run_gpu(c, precision="fp16x2", fused=False)
    check_parity(c, res, tol=1e-5)


def test_long_codes_corrupt_stream_flagged(O):
    from paper_2605_01086_amd import fptc as F
    c = _long_case(O, 16, lengths=(4000, 5000, 6000))
    words, symlen, word_off, sample_off = c.concat()
    sl = symlen.copy()
    sl[word_off[1] + 5] += 1  # one symbol too many in a word of stream 1
    res = run_gpu(c, symlen_override=sl, precision="fp32")
    assert res["status"][1] != 0
    assert res["status"][0] == 0 and res["status"][2] == 0
    check_parity(c, res, tol=1e-5, skip={1})
