"""Seeded test batches built entirely by the CPU oracle (test infrastructure).

A case is a batch of streams: signals from `synth`, one codebook per domain
trained by the oracle on a separate training signal, every stream encoded by
the oracle's sequential encoder, and the oracle's expected symbols and
double-precision reconstruction.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

import synth
from oracle import oracle as O


@dataclass
class Case:
    p: O.QuantParams
    books: list            # oracle Codebook per domain
    signals: list          # float32 arrays
    book_id: np.ndarray    # uint8 per stream
    words: list
    symlen: list
    symbols: list          # oracle quantized symbols per stream
    gamma: np.ndarray = None
    recon: list = field(default_factory=list)
    lmax: int = 12          # longest code of the codebooks

    def concat(self):
        lens = np.array([len(x) for x in self.signals], dtype=np.int64)
        nw = np.array([len(w) for w in self.words], dtype=np.int64)
        words = np.concatenate(self.words) if nw.sum() else np.zeros(0, np.uint64)
        symlen = np.concatenate(self.symlen) if nw.sum() else np.zeros(0, np.uint8)
        return (words.astype(np.uint64), symlen.astype(np.uint8), np.concatenate([[0], np.cumsum(nw)]),
                np.concatenate([[0], np.cumsum(lens)]))


def train_books(p: O.QuantParams, domains, config_id: int, n_train: int = 1 << 15, amplitude: float = 1.0):
    books = []
    for d, dom in enumerate(domains):
        tr = (amplitude * synth.domain_signal(dom, n_train, synth.training_rng(config_id, d))).astype(np.float32)
        books.append(O.train_codebook(O.quantize_stream(tr, p)))
    return books


def paper_params(N: int, E: int, domain: str, config_id: int, B1: int = 2, B2: int | None = None,
                 amplitude: float = 1.0) -> O.QuantParams:
    """Paper quantizer (mu = 50, alpha1 = 0.004) with A0 / A1 the 99.9th
    percentiles of a training signal of the domain scaled by `amplitude`."""
    B2 = E // 2 if B2 is None else B2
    p = O.QuantParams("paper", N, E, B1=B1, B2=B2, mu=50.0, alpha1=0.004)
    tr = (amplitude * synth.domain_signal(domain, 1 << 15, synth.training_rng(config_id, 99))).astype(np.float32)
    p.A0, p.A1 = O.paper_zone_maxima(tr, p, 99.9)
    return p


def build_case(p: O.QuantParams, domains, lengths, config_id: int, gamma=False, recon=True, threads: int = 8,
               stream_domains=None, amplitude: float = 1.0) -> Case:
    books = train_books(p, domains, config_id, amplitude=amplitude)
    n = len(lengths)
    sd = stream_domains if stream_domains is not None else [i % len(domains) for i in range(n)]

    def one(i):
        x = (amplitude * synth.domain_signal(domains[sd[i]], int(lengths[i]),
                                             synth.stream_rng(config_id, i))).astype(np.float32)
        w, sl, sym = O.encode_stream(x, p, books[sd[i]])
        return x, w, sl, sym

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(n)))
    c = Case(p, books, [r[0] for r in res], np.array(sd, dtype=np.uint8), [r[1] for r in res],
             [r[2] for r in res], [r[3] for r in res])
    if gamma:
        rng = np.random.default_rng(config_id + 1000)
        c.gamma = rng.uniform(0.8, 1.25, size=(n, 3))
    if recon:
        def rec(i):
            g = None if c.gamma is None else c.gamma[i]
            return O.reconstruct(c.symbols[i], len(c.signals[i]), p, g)
        with ThreadPoolExecutor(threads) as ex:
            c.recon = list(ex.map(rec, range(n)))
    return c


def range_rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max |got - ref| / (max ref - min ref), the per-stream parity measure."""
    if ref.size == 0:
        return 0.0
    rng = float(ref.max() - ref.min())
    den = rng if rng > 0 else max(1.0, float(np.abs(ref).max()))
    return float(np.max(np.abs(got.astype(np.float64) - ref)) / den)
