"""The five synthetic workloads, as stream shapes and float32 signals.

Nothing here touches the codec: a workload is a list of stream lengths, the
signal domain of each stream, the seeds they are drawn from and the training
signals a codebook is built from.  The benchmark and the full-size tests both
take their inputs from here, so they decode the same streams.

  plain      one EEG-like stream of 2^20 samples
  batch      4096 streams, lengths floor(2^U(14, 20)), domains EEG / seismic /
             power / meteorological in turn (stream i has domain i mod 4)
  precision  256 streams of 2^20 samples, EEG-like and seismic-like 50/50
  grad       256 streams of 2^18 samples, power-grid and meteorological 50/50
  large      64 channels of 2^24 EEG-like samples mixed by a 64 x 64 matrix
             with N(0, 1/64) entries
  paper      256 streams of 2^20 EEG-like samples (the paper's operating
             point is quoted on biomedical recordings)
  sweep      128 streams of 2^20 EEG-like samples, for the sweep over window
             and kept coefficients
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from .signals import DOMAINS, ROOT_SEED, batch_lengths, domain_signal, eeg_like, stream_rng, training_rng

CONFIG_ID = {"plain": 0, "batch": 1, "precision": 2, "grad": 3, "large": 4, "paper": 5, "sweep": 6}


@dataclass
class Workload:
    name: str
    config_id: int
    lengths: np.ndarray      # int64 [n_streams]
    domain: np.ndarray       # index into DOMAINS per stream
    domains_used: tuple      # domains with a codebook, in book order
    book_id: np.ndarray      # uint8 codebook index per stream

    @property
    def n_streams(self) -> int:
        return int(self.lengths.shape[0])

    @property
    def sample_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.lengths)]).astype(np.int64)


def workload(name: str) -> Workload:
    cid = CONFIG_ID[name]
    if name == "plain":
        lens = np.array([1 << 20], dtype=np.int64)
        dom = np.zeros(1, dtype=np.int64)
    elif name == "batch":
        rng = np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=(2, 1)))
        lens = batch_lengths(4096, 14.0, 20.0, rng)
        dom = np.arange(4096) % 4
    elif name == "precision":
        lens = np.full(256, 1 << 20, dtype=np.int64)
        dom = np.where(np.arange(256) % 2 == 0, 0, 1)
    elif name == "grad":
        lens = np.full(256, 1 << 18, dtype=np.int64)
        dom = np.where(np.arange(256) % 2 == 0, 2, 3)
    elif name == "large":
        lens = np.full(64, 1 << 24, dtype=np.int64)
        dom = np.zeros(64, dtype=np.int64)
    elif name == "paper":
        lens = np.full(256, 1 << 20, dtype=np.int64)
        dom = np.zeros(256, dtype=np.int64)
    elif name == "sweep":
        lens = np.full(128, 1 << 20, dtype=np.int64)
        dom = np.zeros(128, dtype=np.int64)
    else:
        raise ValueError(f"unknown workload {name}")
    used = tuple(sorted(set(int(d) for d in dom)))
    book = np.array([used.index(int(d)) for d in dom], dtype=np.uint8)
    return Workload(name, cid, lens, dom, tuple(DOMAINS[d] for d in used), book)


def signals(w: Workload, threads: int = 8, streams=None) -> np.ndarray:
    """float32 samples of every stream (or of `streams` only), concatenated
    in stream order."""
    if w.name == "large":
        return _large(w, threads, streams)
    sel = np.arange(w.n_streams) if streams is None else np.asarray(streams)
    lens = w.lengths[sel]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x = np.empty(int(off[-1]), dtype=np.float32)

    def gen(j):
        i = int(sel[j])
        x[off[j]:off[j + 1]] = domain_signal(DOMAINS[int(w.domain[i])], int(w.lengths[i]),
                                             stream_rng(w.config_id, i))

    order = np.argsort(-lens)  # longest first, for balance
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(gen, order))
    return x


def _mixing(w: Workload) -> np.ndarray:
    n = w.n_streams
    return (stream_rng(w.config_id, 0).standard_normal((n, n)) / np.sqrt(n)).astype(np.float32)


def _large(w: Workload, threads: int, streams) -> np.ndarray:
    n, L = w.n_streams, int(w.lengths[0])
    src = np.empty((n, L), dtype=np.float32)

    def gen_src(i):
        src[i] = eeg_like(L, stream_rng(w.config_id, 1 + i))

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(gen_src, range(n)))
    M = _mixing(w)
    if streams is not None:
        M = M[np.asarray(streams)]
    return np.ascontiguousarray((M @ src).reshape(-1))


def training_signals(w: Workload, n_train: int = 1 << 18) -> list:
    """One float32 training signal per codebook, drawn from seeds disjoint
    from the evaluation streams."""
    if w.name == "large":
        n = w.n_streams
        tr = np.stack([eeg_like(1 << 16, training_rng(w.config_id, i)) for i in range(n)])
        return [(_mixing(w).astype(np.float64) @ tr).reshape(-1).astype(np.float32)]
    return [domain_signal(dom, n_train, training_rng(w.config_id, DOMAINS.index(dom))).astype(np.float32)
            for dom in w.domains_used]
