"""Device-side containers for the FPTC decoder, on top of the ctypes binding.

`DeviceCodec` uploads the per-domain structures (decode lookup tables,
dequantization tables, IDCT basis) built by the library's host builders;
`DeviceBatch` uploads a batch of SymLen streams; `Decoder` owns the workspace
and calls plan -> decode -> dequant+IDCT on the current HIP stream.  torch is
used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import fptc as F


def to_device(a: np.ndarray, dev) -> torch.Tensor:
    """C-contiguous device copy of a host array.  The C ABI takes raw pointers
    to dense row-major buffers, so any other layout is refused here."""
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    if not t.is_contiguous():
        raise ValueError("device buffers passed to libfptc must be contiguous")
    return t


def quant_params(kind: str = "amp", N: int = 64, E: int | None = None, step_fine: float = 0.25,
                 step_coarse: float = 2.0, threshold: float = 16.0, B1: int = 2, B2: int = 16, mu: float = 50.0,
                 alpha1: float = 0.004, A0: float = 1.0, A1: float = 1.0) -> F.fptc_quant_params:
    E = N if E is None else E
    return F.fptc_quant_params(F.FPTC_QUANT_AMPLITUDE if kind == "amp" else F.FPTC_QUANT_PAPER, N, E, B1, B2, 0,
                               step_fine, step_coarse, threshold, mu, alpha1, A0, A1)


class DeviceCodec:
    """Codebooks (one per domain) + dequantization tables + IDCT basis on the GPU."""

    def __init__(self, code_lens, q: F.fptc_quant_params, lmax: int = 12, device="cuda"):
        code_lens = np.atleast_2d(np.asarray(code_lens, dtype=np.uint8))
        self.n_books = code_lens.shape[0]
        self.N, self.E, self.lmax = q.N, q.E, lmax
        luts = np.stack([F.fptc_build_lut(code_lens[b], lmax) for b in range(self.n_books)])
        val, zone, rob = F.fptc_build_dequant(q)
        self.n_rows = val.shape[0]
        # every book shares the quantizer; each has its own table copy so books may differ
        vals = np.tile(val, (self.n_books, 1, 1))
        zones = np.tile(zone, (self.n_books, 1, 1))
        robs = np.tile(rob, (self.n_books, 1))
        basis = F.fptc_build_basis(q.N, q.E)
        dev = torch.device(device)
        self.host = dict(lut=luts, deq_val=vals, deq_zone=zones, row_of_bin=robs, basis=basis, code_lens=code_lens)
        self.lut = to_device(luts.view(np.int16), dev)
        self.deq_val = to_device(vals, dev)
        self.deq_zone = to_device(zones, dev)
        self.row_of_bin = to_device(robs, dev)
        self.basis = to_device(basis, dev)
        self.c = F.fptc_codec(self.N, self.E, lmax, self.n_books, self.n_rows, 0, self.lut.data_ptr(),
                              self.deq_val.data_ptr(), self.deq_zone.data_ptr(), self.row_of_bin.data_ptr(),
                              self.basis.data_ptr())


def n_windows(L, N):
    return (np.asarray(L, dtype=np.int64) + N - 1) // N


class DeviceBatch:
    """A batch of SymLen streams in GPU memory (CSR layout of include/fptc.h)."""

    def __init__(self, words: np.ndarray, symlen: np.ndarray, word_off: np.ndarray, sample_off: np.ndarray,
                 N: int, E: int, book_id=None, device="cuda"):
        dev = torch.device(device)
        self.n_streams = int(sample_off.shape[0] - 1)
        self.word_off_h = np.ascontiguousarray(word_off, dtype=np.int64)
        self.sample_off_h = np.ascontiguousarray(sample_off, dtype=np.int64)
        lens = np.diff(self.sample_off_h)
        self.sym_off_h = np.concatenate([[0], np.cumsum(n_windows(lens, N) * E)]).astype(np.int64)
        self.n_words = int(words.shape[0])
        self.n_symbols = int(self.sym_off_h[-1])
        self.n_samples = int(self.sample_off_h[-1])
        w = np.ascontiguousarray(words, dtype=np.uint64)
        self.words = to_device(w.view(np.int64), dev) if w.size else torch.zeros(1, dtype=torch.int64, device=dev)
        sl = np.ascontiguousarray(symlen, dtype=np.uint8)
        self.symlen = to_device(sl, dev) if sl.size else torch.zeros(1, dtype=torch.uint8, device=dev)
        self.word_off = to_device(self.word_off_h, dev)
        self.sample_off = to_device(self.sample_off_h, dev)
        self.book_id = None
        if book_id is not None:
            self.book_id = to_device(np.ascontiguousarray(book_id, dtype=np.uint8), dev)
        self.c = F.fptc_batch(self.n_streams, 0, self.n_words, self.n_symbols, self.n_samples,
                              self.words.data_ptr(), self.symlen.data_ptr(), self.word_off.data_ptr(),
                              self.sample_off.data_ptr(), None if self.book_id is None else self.book_id.data_ptr())

    @property
    def compressed_bytes(self) -> int:
        """Bytes of the SymLen payload: 8 per word plus 1 symlen byte per word."""
        return 9 * self.n_words

    @property
    def header_bytes(self) -> int:
        """Per-stream metadata read by the decoder (offsets, book ids)."""
        return 16 * (self.n_streams + 1) + (self.n_streams if self.book_id is not None else 0)


@dataclass
class Launch:
    """Launch shape of include/fptc.h's fptc_launch; 0 = library default."""
    windows_per_chunk: int = 0
    waves_per_block: int = 0
    blocks: int = 0
    chunk_group: int = 0

    def c(self) -> F.fptc_launch:
        return F.fptc_launch(self.windows_per_chunk, self.waves_per_block, self.blocks, self.chunk_group)


class Decoder:
    """plan -> decode -> dequant+IDCT for one batch and codec."""

    def __init__(self, batch: DeviceBatch, codec: DeviceCodec, launch: Launch | None = None):
        self.batch, self.codec = batch, codec
        self.launch = launch or Launch()
        self.lc = self.launch.c()
        dev = batch.word_off.device
        nbytes = F.fptc_workspace_size(batch.c, codec.c, self.lc)
        if nbytes == 0:
            raise F.FptcError("fptc_workspace_size", F.FPTC_ERR_INVALID_ARG)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.status = torch.zeros(batch.n_streams, dtype=torch.int32, device=dev)
        self.symbols = torch.empty(max(1, batch.n_symbols), dtype=torch.uint8, device=dev)
        self.out = torch.empty(max(1, batch.n_samples), dtype=torch.float32, device=dev)

    def plan(self):
        F.fptc_plan_batch(self.batch.c, self.codec.c, self.lc, self.ws, self.status)

    def decode(self):
        F.fptc_decode_batch(self.batch.c, self.codec.c, self.lc, self.ws, self.symbols, self.status)
        return self.symbols[: self.batch.n_symbols]

    def dequant_idct(self, gamma=None, precision="fp32", out=None):
        out = self.out if out is None else out
        F.fptc_dequant_idct(self.batch.c, self.codec.c, self.lc, self.ws, self.symbols, gamma, precision, out)
        return out[: self.batch.n_samples]

    def decompress(self, gamma=None, precision="fp16x2", out=None):
        """Fused decode + dequant + IDCT (needs a plan)."""
        out = self.out if out is None else out
        F.fptc_decompress_batch(self.batch.c, self.codec.c, self.lc, self.ws, gamma, precision, out, self.status)
        return out[: self.batch.n_samples]

    def run(self, gamma=None, precision="fp32", fused=False):
        self.plan()
        if fused:
            return self.decompress(gamma, precision)
        self.decode()
        return self.dequant_idct(gamma, precision)


# ---------------------------------------------------------------- host-side encode (product encoder)


def train_code_lengths(train: np.ndarray, q: F.fptc_quant_params, lmax: int = 12) -> np.ndarray:
    """Codebook of a domain from representative data: quantize with the host
    encoder, histogram the bytes with +1 smoothing, package-merge lengths."""
    sym = F.fptc_quantize_host(np.asarray(train, dtype=np.float32), q)
    hist = np.bincount(sym, minlength=256).astype(np.uint64) + np.uint64(1)
    return F.fptc_code_lengths(hist, lmax)


def encode_batch(signals, book_id, q: F.fptc_quant_params, code_lens: np.ndarray, n_threads: int = 0):
    """Host encoder over a list of float32 strips -> (words, symlen, word_off, sample_off)."""
    lens = np.array([len(x) for x in signals], dtype=np.int64)
    sample_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    x = np.concatenate([np.asarray(s, dtype=np.float32) for s in signals]) if len(signals) else np.zeros(0, np.float32)
    nsym = n_windows(lens, q.N) * q.E
    cap_off = np.concatenate([[0], np.cumsum(nsym + 1)]).astype(np.int64)  # >= 1 symbol per word
    words = np.zeros(int(cap_off[-1]), dtype=np.uint64)
    symlen = np.zeros(int(cap_off[-1]), dtype=np.uint8)
    bid = None if book_id is None else np.asarray(book_id, dtype=np.uint8)
    code_lens = np.atleast_2d(np.asarray(code_lens, dtype=np.uint8))
    nw = F.fptc_encode_batch_host(x, sample_off, bid, q, code_lens, cap_off, words, symlen, n_threads)
    word_off = np.concatenate([[0], np.cumsum(nw)]).astype(np.int64)
    idx = np.concatenate([np.arange(cap_off[i], cap_off[i] + nw[i]) for i in range(len(signals))]) \
        if len(signals) else np.zeros(0, np.int64)
    return words[idx], symlen[idx], word_off, sample_off


# ---------------------------------------------------------------- device-side training steps


def zone_maxima(train: np.ndarray, q: F.fptc_quant_params, percentile: float = 99.9, device="cuda"):
    """A0 and A1 of the paper quantizer from a training strip, on the GPU: the
    FP64 forward transform of its windows (fptc_quantize_batch) and the
    percentile of |c| over the bins of zone 0 ([0, B1)) and zone 1 ([B1, B2))
    (fptc_abs_percentile); an empty zone gives 1."""
    train = np.ascontiguousarray(train, dtype=np.float32)
    dev = torch.device(device)
    L = int(train.shape[0])
    nw = int(n_windows(np.array([L]), q.N)[0])
    so = to_device(np.array([0, L], dtype=np.int64), dev)
    yo = to_device(np.array([0, nw * q.E], dtype=np.int64), dev)
    x = to_device(train, dev)
    b = F.fptc_batch(1, 0, 0, nw * q.E, L, None, None, None, so.data_ptr(), None)
    tab = to_device(F.fptc_build_dct_table(q.N, q.E), dev)
    sym = torch.empty(max(1, nw * q.E), dtype=torch.uint8, device=dev)
    coef = torch.empty(max(1, nw * q.E), dtype=torch.float64, device=dev)
    F.fptc_quantize_batch(b, q, tab, yo, x, sym, coef)
    ws = torch.empty(F.fptc_percentile_workspace_size(), dtype=torch.uint8, device=dev)
    out = torch.ones(2, dtype=torch.float64, device=dev)
    if q.B1 > 0:
        F.fptc_abs_percentile(coef, nw, q.E, 0, q.B1, percentile, out[0:1], ws)
    if q.B2 > q.B1:
        F.fptc_abs_percentile(coef, nw, q.E, q.B1, q.B2, percentile, out[1:2], ws)
    a = out.cpu().numpy()
    return float(a[0]), float(a[1])
