"""Pins of the oracle's SymLen packing (Section 4.1, Algorithm 1) and its
bit-serial decoder (Section 4.2): hand-worked words, packing invariants,
brute-force decoding of tiny streams, and error detection."""
import itertools

import numpy as np
import pytest

from conftest import read_golden


def tiny_codebook(O):
    lengths = np.zeros(256, dtype=np.uint8)
    lengths[128], lengths[129], lengths[127], lengths[130] = 1, 2, 3, 3
    return O.Codebook(lengths)


def test_worked_words(O):
    cb = tiny_codebook(O)
    for row in read_golden("symlen_worked.txt"):
        case, syms, words, symlen = [p.strip() for p in row.split("|")]
        seq = []
        for tok in syms.split():
            c, s = tok.split("*")
            seq += [int(s)] * int(c)
        w, sl = O.symlen_pack(np.array(seq, dtype=np.uint8), cb)
        assert [format(int(v), "016X") for v in w] == words.split(), case
        assert [int(v) for v in sl] == [int(v) for v in symlen.split()], case
        assert np.array_equal(O.symlen_decode(w, sl, cb, len(seq)), np.array(seq, dtype=np.uint8))


def _bits_of(words, symlen, cb, seq):
    """Check the word-level invariants of Algorithm 1 for one packed sequence."""
    pos = 0
    for wi, (w, n) in enumerate(zip(words, symlen)):
        used = 0
        bitstr = format(int(w), "064b")
        for j in range(int(n)):
            s = seq[pos + j]
            l = int(cb.lengths[s])
            assert bitstr[used:used + l] == format(int(cb.codes[s]), "0%db" % l)
            used += l
        assert set(bitstr[used:]) <= {"0"}, "padding bits are zero"
        pos += int(n)
        if wi + 1 < len(words):
            assert used + int(cb.lengths[seq[pos]]) > 64, "greedy: the next code did not fit"
    assert pos == len(seq)


@pytest.mark.parametrize("domain", ["eeg", "seismic", "power", "meteo"])
def test_pack_invariants_and_identity(O, domain):
    import synth
    p = O.QuantParams("amp", 64, 64)
    tr = synth.domain_signal(domain, 1 << 14, synth.training_rng(9, 0)).astype(np.float32)
    cb = O.train_codebook(O.quantize_stream(tr, p))
    x = synth.domain_signal(domain, 3 * 4096 + 37, synth.stream_rng(9, 1)).astype(np.float32)
    w, sl, sym = O.encode_stream(x, p, cb)
    assert int(sl.astype(np.int64).sum()) == sym.size
    assert sym.size == O.n_windows(x.size, 64) * 64
    _bits_of(w, sl, cb, sym)
    assert np.array_equal(O.symlen_decode(w, sl, cb, sym.size), sym)


def _all_parses(bitstr, n, codes):
    """Every way to read n symbols as a prefix of bitstr (brute force)."""
    if n == 0:
        return [[]]
    out = []
    for s, c in codes.items():
        if bitstr.startswith(c):
            for rest in _all_parses(bitstr[len(c):], n - 1, codes):
                out.append([s] + rest)
    return out


def test_brute_force_tiny_streams(O):
    # every sequence over a 4-symbol alphabet up to length 6, two codebooks
    for lens in ({128: 1, 129: 2, 127: 3, 130: 3}, {10: 2, 11: 2, 12: 2, 13: 2}):
        lengths = np.zeros(256, dtype=np.uint8)
        for s, l in lens.items():
            lengths[s] = l
        cb = O.Codebook(lengths)
        codes = {s: format(int(cb.codes[s]), "0%db" % l) for s, l in lens.items()}
        alphabet = sorted(lens)
        for L in range(1, 7):
            for seq in itertools.product(alphabet, repeat=L):
                seq = np.array(seq, dtype=np.uint8)
                w, sl = O.symlen_pack(seq, cb)
                assert np.array_equal(O.symlen_decode(w, sl, cb, L), seq)
                parses = _all_parses(format(int(w[0]), "064b"), int(sl[0]), codes)
                assert len(parses) == 1 and parses[0] == list(seq[: int(sl[0])])
    # long runs that cross word boundaries
    lengths = np.zeros(256, dtype=np.uint8)
    lengths[[128, 129, 127, 130]] = [1, 2, 3, 3]
    cb = O.Codebook(lengths)
    rng = np.random.default_rng(0)
    for _ in range(50):
        seq = rng.choice([127, 128, 129, 130], size=int(rng.integers(1, 400))).astype(np.uint8)
        w, sl = O.symlen_pack(seq, cb)
        _bits_of(w, sl, cb, seq)
        assert np.array_equal(O.symlen_decode(w, sl, cb, seq.size), seq)


def test_decoder_detects_corruption(O):
    lengths = np.zeros(256, dtype=np.uint8)
    lengths[[128, 129, 127, 130]] = [1, 2, 3, 3]
    cb = O.Codebook(lengths)
    seq = np.array([130] * 22, dtype=np.uint8)
    w, sl = O.symlen_pack(seq, cb)
    # word 0 = 21 codes '111' + one zero pad bit.  Asking for 22 symbols reads the
    # pad bit as the 1-bit code of 128 (padding is harmless, Section 4.2); asking
    # for 23 needs a bit past bit 64, which is an error.
    d = O.symlen_decode(w, np.array([22, 1], dtype=np.uint8), cb, 23)
    assert list(d[:22]) == [130] * 21 + [128]
    with pytest.raises(ValueError):
        O.symlen_decode(w, np.array([23, 1], dtype=np.uint8), cb, 24)
    with pytest.raises(ValueError):  # symbol count does not match the expected total
        O.symlen_decode(w, np.array([20, 1], dtype=np.uint8), cb, 22)
