"""Pins of the oracle's entropy coder (Section 3.3): package-merge optimality
against exhaustive search and a textbook Huffman, Kraft equality, canonical
codes against the RFC 1951 worked example, prefix-freeness."""
import heapq
import itertools

import numpy as np
import pytest

from conftest import read_golden


def cost(freq, lengths):
    return int(np.sum(np.asarray(freq, dtype=np.int64) * np.asarray(lengths, dtype=np.int64)))


def brute_force_optimum(freq, lmax):
    """Smallest sum f*l over all length vectors with l in [1, lmax] and Kraft sum <= 1."""
    n = len(freq)
    best = None
    for ls in itertools.product(range(1, lmax + 1), repeat=n):
        if sum(2.0 ** -l for l in ls) <= 1.0 + 1e-15:
            c = cost(freq, ls)
            if best is None or c < best:
                best = c
    return best


def heap_huffman_lengths(freq):
    """Textbook (unbounded) Huffman by repeatedly merging the two lightest trees."""
    heap = [(f, i, (i,)) for i, f in enumerate(freq)]
    heapq.heapify(heap)
    depth = [0] * len(freq)
    cnt = len(freq)
    while len(heap) > 1:
        f1, _, s1 = heapq.heappop(heap)
        f2, _, s2 = heapq.heappop(heap)
        for s in s1 + s2:
            depth[s] += 1
        heapq.heappush(heap, (f1 + f2, cnt, s1 + s2))
        cnt += 1
    return depth


def kraft_int(lengths, lmax):
    return sum(1 << (lmax - int(l)) for l in lengths if l > 0)


@pytest.mark.parametrize("seed", range(12))
def test_package_merge_is_optimal_small(O, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    lmax = int(rng.integers(int(np.ceil(np.log2(n))), 5))
    freq = rng.integers(1, 60, size=n) ** int(rng.integers(1, 4))
    ls = O.package_merge(freq, lmax)
    assert max(ls) <= lmax and min(ls) >= 1
    assert kraft_int(ls, lmax) == 1 << lmax  # Kraft equality
    assert cost(freq, ls) == brute_force_optimum(freq, lmax)


@pytest.mark.parametrize("seed", range(6))
def test_package_merge_matches_huffman_when_unconstrained(O, seed):
    rng = np.random.default_rng(100 + seed)
    freq = rng.integers(1, 1000, size=256)
    h = heap_huffman_lengths(list(freq))
    ls = O.package_merge(freq, max(h))
    assert cost(freq, ls) == cost(freq, h)
    assert kraft_int(ls, max(h)) == 1 << max(h)


def test_package_merge_length_limit_binds(O):
    freq = np.array([2 ** 40 // (2 ** min(i, 39)) + 1 for i in range(256)], dtype=np.uint64)
    h = heap_huffman_lengths([int(f) for f in freq])
    assert max(h) > 12
    ls = O.package_merge(freq, 12)
    assert max(ls) == 12 and kraft_int(ls, 12) == 4096
    assert cost(freq, ls) >= cost(freq, h)
    with pytest.raises(ValueError):
        O.package_merge(np.ones(256, dtype=np.uint64), 7)  # 256 symbols need >= 8 bits


def test_package_merge_degenerate_alphabets(O):
    f = np.zeros(256, dtype=np.uint64)
    f[7] = 5
    ls = O.package_merge(f, 12)
    assert ls[7] == 1 and ls.sum() == 1
    f[9] = 1
    ls = O.package_merge(f, 12)
    assert ls[7] == 1 and ls[9] == 1 and ls.sum() == 2


def test_canonical_codes_rfc1951_example(O):
    rows = [r.split() for r in read_golden("canonical_rfc1951.txt")]
    lengths = np.zeros(len(rows), dtype=np.uint8)
    for r in rows:
        lengths[int(r[0])] = int(r[1])
    codes = O.canonical_codes(lengths)
    for r in rows:
        s, l, bits = int(r[0]), int(r[1]), r[2]
        assert format(int(codes[s]), "0%db" % l) == bits


def test_trained_codebook_is_prefix_free(O):
    import synth
    p = O.QuantParams("amp", 64, 64)
    x = synth.eeg_like(1 << 14, synth.training_rng(0, 0)).astype(np.float32)
    cb = O.train_codebook(O.quantize_stream(x, p))
    assert kraft_int(cb.lengths, 12) == 4096 and cb.lengths.max() <= 12 and cb.lengths.min() >= 1
    strs = [format(int(cb.codes[s]), "0%db" % cb.lengths[s]) for s in range(256)]
    assert len(set(strs)) == 256
    for a in range(256):
        for b in range(256):
            if a != b:
                assert not strs[b].startswith(strs[a])
    # canonical order: (length, symbol) ascending gives increasing codes when left-aligned
    order = sorted(range(256), key=lambda s: (cb.lengths[s], s))
    left = [int(cb.codes[s]) << (12 - int(cb.lengths[s])) for s in order]
    assert all(left[i] < left[i + 1] for i in range(255))
