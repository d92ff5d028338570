"""Python face of the FPTC CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loads the plain-C double-precision oracle (``fptc_oracle.c``) with ctypes and
adds the few steps that are easier to state with numpy (percentiles, the Adam
loop).  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may use this module; the GPU library never imports it and it never imports
the GPU library.

Sections of the paper followed (each function names its own):
  Section 3.1 (DCT, truncation), Section 3.2 (quantizers), Section 3.3
  (histogram, package-merge, canonical codes), Section 4.1 Algorithm 1 (SymLen
  packing), Section 4.2 (decode, reconstruction), Section 5.1 (CR, PRD).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fptc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LMAX_DEFAULT = 12  # reading: the paper leaves L_max open; 12 keeps a 4096-entry table


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _QP(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("N", ctypes.c_int32), ("E", ctypes.c_int32),
                ("B1", ctypes.c_int32), ("B2", ctypes.c_int32),
                ("step_f", ctypes.c_double), ("step_c", ctypes.c_double), ("T", ctypes.c_double),
                ("mu", ctypes.c_double), ("alpha1", ctypes.c_double), ("A0", ctypes.c_double),
                ("A1", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp, fp, u8p, u64p, u32p = (P(ctypes.c_double), P(ctypes.c_float), P(ctypes.c_uint8),
                                   P(ctypes.c_uint64), P(ctypes.c_uint32))
        i64 = ctypes.c_int64
        L.or_dct_ortho.argtypes = [dp, ctypes.c_int, dp]
        L.or_dct_eq1.argtypes = [dp, ctypes.c_int, dp]
        L.or_idct_ortho.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.or_dct_ortho_tab.argtypes = [dp, ctypes.c_int, dp]
        L.or_idct_ortho_tab.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.or_quant_amp.argtypes = [ctypes.c_double] * 4
        L.or_quant_amp.restype = ctypes.c_int
        L.or_dequant_amp.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3
        L.or_dequant_amp.restype = ctypes.c_double
        L.or_zone_amp.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3
        L.or_zone_amp.restype = ctypes.c_int
        L.or_quant_paper.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4
        L.or_quant_paper.restype = ctypes.c_int
        L.or_dequant_paper.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4
        L.or_dequant_paper.restype = ctypes.c_double
        L.or_package_merge.argtypes = [u64p, ctypes.c_int, ctypes.c_int, u8p]
        L.or_package_merge.restype = ctypes.c_int
        L.or_canonical_codes.argtypes = [u8p, ctypes.c_int, u32p]
        L.or_symlen_pack.argtypes = [u8p, i64, u32p, u8p, u64p, u8p, i64]
        L.or_symlen_pack.restype = i64
        L.or_symlen_decode.argtypes = [u64p, u8p, i64, u8p, ctypes.c_int, u8p, i64]
        L.or_symlen_decode.restype = i64
        L.or_dequantize.argtypes = [ctypes.c_int, ctypes.c_int, P(_QP)]
        L.or_dequantize.restype = ctypes.c_double
        L.or_zone.argtypes = [ctypes.c_int, ctypes.c_int, P(_QP)]
        L.or_zone.restype = ctypes.c_int
        L.or_quantize_stream.argtypes = [fp, i64, P(_QP), u8p]
        L.or_dct_stream.argtypes = [fp, i64, ctypes.c_int, ctypes.c_int, dp]
        L.or_histogram.argtypes = [u8p, i64, u64p]
        L.or_reconstruct.argtypes = [u8p, i64, P(_QP), dp, dp]
        L.or_backward.argtypes = [u8p, i64, P(_QP), dp, dp, dp]
        L.or_prd.argtypes = [fp, dp, i64]
        L.or_prd.restype = ctypes.c_double
        L.or_cr.argtypes = [i64, i64]
        L.or_cr.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# Quantizer parameters (Section 3.2, Table 1)


@dataclass
class QuantParams:
    """kind 'amp': amplitude three-zone quantizer (zero zone |c| < step_f/2,
    fine step step_f up to T, coarse step step_c beyond T).
    kind 'paper': frequency three-zone quantizer of Section 3.2 (mu-law bins
    [0, B1), deadzone bins [B1, B2), zeroed bins [B2, E))."""
    kind: str
    N: int
    E: int
    step_f: float = 0.25
    step_c: float = 2.0
    T: float = 16.0
    B1: int = 2
    B2: int = 16
    mu: float = 50.0
    alpha1: float = 0.004
    A0: float = 1.0
    A1: float = 1.0

    def c(self) -> _QP:
        return _QP(0 if self.kind == "amp" else 1, self.N, self.E, self.B1, self.B2,
                   self.step_f, self.step_c, self.T, self.mu, self.alpha1, self.A0, self.A1)


@dataclass
class Codebook:
    """Code lengths and canonical codes for the 256 byte symbols."""
    lengths: np.ndarray  # uint8[256]
    codes: np.ndarray = field(default=None)  # uint32[256]

    def __post_init__(self):
        self.lengths = np.ascontiguousarray(self.lengths, dtype=np.uint8)
        if self.codes is None:
            self.codes = canonical_codes(self.lengths)


# ---------------------------------------------------------------------------
# Section 3.1


def dct_ortho(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().or_dct_ortho(_ptr(x, ctypes.c_double), x.shape[0], _ptr(out, ctypes.c_double))
    return out


def dct_eq1(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().or_dct_eq1(_ptr(x, ctypes.c_double), x.shape[0], _ptr(out, ctypes.c_double))
    return out


def dct_ortho_tab(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().or_dct_ortho_tab(_ptr(x, ctypes.c_double), x.shape[0], _ptr(out, ctypes.c_double))
    return out


def idct_ortho_tab(X: np.ndarray, N: int, E: int | None = None) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    E = X.shape[0] if E is None else E
    out = np.empty(N, dtype=np.float64)
    lib().or_idct_ortho_tab(_ptr(X, ctypes.c_double), N, E, _ptr(out, ctypes.c_double))
    return out


def idct_ortho(X: np.ndarray, N: int, E: int | None = None) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    E = X.shape[0] if E is None else E
    out = np.empty(N, dtype=np.float64)
    lib().or_idct_ortho(_ptr(X, ctypes.c_double), N, E, _ptr(out, ctypes.c_double))
    return out


def dct_stream(x: np.ndarray, N: int, E: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    nw = n_windows(x.shape[0], N)
    out = np.empty(nw * E, dtype=np.float64)
    lib().or_dct_stream(_ptr(x, ctypes.c_float), x.shape[0], N, E, _ptr(out, ctypes.c_double))
    return out


def n_windows(L: int, N: int) -> int:
    return (int(L) + N - 1) // N


# ---------------------------------------------------------------------------
# Section 3.2


def quant_amp(c: float, step_f: float, step_c: float, T: float) -> int:
    return lib().or_quant_amp(c, step_f, step_c, T)


def dequant_amp(s: int, step_f: float, step_c: float, T: float) -> float:
    return lib().or_dequant_amp(s, step_f, step_c, T)


def zone_amp(s: int, step_f: float, step_c: float, T: float) -> int:
    return lib().or_zone_amp(s, step_f, step_c, T)


def quant_paper(c: float, k: int, p: QuantParams) -> int:
    return lib().or_quant_paper(c, k, p.B1, p.B2, p.mu, p.alpha1, p.A0, p.A1)


def dequant_paper(s: int, k: int, p: QuantParams) -> float:
    return lib().or_dequant_paper(s, k, p.B1, p.B2, p.mu, p.alpha1, p.A0, p.A1)


def dequantize(s: int, k: int, p: QuantParams) -> float:
    qp = p.c()
    return lib().or_dequantize(int(s), int(k), ctypes.byref(qp))


def zone(s: int, k: int, p: QuantParams) -> int:
    qp = p.c()
    return lib().or_zone(int(s), int(k), ctypes.byref(qp))


def quantize_stream(x: np.ndarray, p: QuantParams) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(n_windows(x.shape[0], p.N) * p.E, dtype=np.uint8)
    qp = p.c()
    lib().or_quantize_stream(_ptr(x, ctypes.c_float), x.shape[0], ctypes.byref(qp), _ptr(out, ctypes.c_uint8))
    return out


def paper_zone_maxima(train: np.ndarray, p: QuantParams, percentile: float = 99.9) -> tuple[float, float]:
    """A0 and A1: the clipped percentile of |c| over every window's bins of
    zone 0 and zone 1 (Section 3.2; Table 1 percentile 99.9)."""
    coef = dct_stream(train, p.N, p.E).reshape(-1, p.E)
    z0 = np.abs(coef[:, :p.B1]).ravel()
    z1 = np.abs(coef[:, p.B1:p.B2]).ravel()
    A0 = float(np.percentile(z0, percentile, method="linear")) if z0.size else 1.0
    A1 = float(np.percentile(z1, percentile, method="linear")) if z1.size else 1.0
    return A0, A1


# ---------------------------------------------------------------------------
# Section 3.3


def histogram(sym: np.ndarray) -> np.ndarray:
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    h = np.zeros(256, dtype=np.uint64)
    lib().or_histogram(_ptr(sym, ctypes.c_uint8), sym.shape[0], _ptr(h, ctypes.c_uint64))
    return h


def package_merge(freq: np.ndarray, lmax: int) -> np.ndarray:
    freq = np.ascontiguousarray(freq, dtype=np.uint64)
    out = np.zeros(freq.shape[0], dtype=np.uint8)
    rc = lib().or_package_merge(_ptr(freq, ctypes.c_uint64), freq.shape[0], lmax, _ptr(out, ctypes.c_uint8))
    if rc != 0:
        raise ValueError("package-merge: L_max too small for the alphabet")
    return out


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = np.zeros(lengths.shape[0], dtype=np.uint32)
    lib().or_canonical_codes(_ptr(lengths, ctypes.c_uint8), lengths.shape[0], _ptr(out, ctypes.c_uint32))
    return out


def train_codebook(train_symbols: np.ndarray, lmax: int = LMAX_DEFAULT) -> Codebook:
    """Histogram of representative symbols with +1 smoothing (so every byte
    has a code, reading), then length-limited lengths and canonical codes."""
    h = histogram(train_symbols) + np.uint64(1)
    return Codebook(package_merge(h, lmax))


# ---------------------------------------------------------------------------
# Section 4.1, Algorithm 1 and Section 4.2


def symlen_pack(sym: np.ndarray, cb: Codebook) -> tuple[np.ndarray, np.ndarray]:
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    cap = max(1, sym.shape[0])  # at least one symbol per word
    words = np.zeros(cap, dtype=np.uint64)
    symlen = np.zeros(cap, dtype=np.uint8)
    n = lib().or_symlen_pack(_ptr(sym, ctypes.c_uint8), sym.shape[0], _ptr(cb.codes, ctypes.c_uint32),
                             _ptr(cb.lengths, ctypes.c_uint8), _ptr(words, ctypes.c_uint64),
                             _ptr(symlen, ctypes.c_uint8), cap)
    if n < 0:
        raise ValueError("SymLen packing failed (symbol without code)")
    return words[:n].copy(), symlen[:n].copy()


def symlen_decode(words: np.ndarray, symlen: np.ndarray, cb: Codebook, n_expected: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint64)
    symlen = np.ascontiguousarray(symlen, dtype=np.uint8)
    out = np.zeros(max(1, n_expected), dtype=np.uint8)
    n = lib().or_symlen_decode(_ptr(words, ctypes.c_uint64), _ptr(symlen, ctypes.c_uint8), words.shape[0],
                               _ptr(cb.lengths, ctypes.c_uint8), 256, _ptr(out, ctypes.c_uint8), n_expected)
    if n < 0:
        raise ValueError(f"SymLen decode error {n}")
    return out[:n_expected]


def encode_stream(x: np.ndarray, p: QuantParams, cb: Codebook):
    """Sequential encoder: windows -> DCT -> quantize -> SymLen words."""
    sym = quantize_stream(x, p)
    words, symlen = symlen_pack(sym, cb)
    return words, symlen, sym


def reconstruct(symbols: np.ndarray, L: int, p: QuantParams, gamma=None) -> np.ndarray:
    symbols = np.ascontiguousarray(symbols, dtype=np.uint8)
    out = np.zeros(int(L), dtype=np.float64)
    qp = p.c()
    g = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
    lib().or_reconstruct(_ptr(symbols, ctypes.c_uint8), int(L), ctypes.byref(qp),
                         None if g is None else _ptr(g, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def backward(symbols: np.ndarray, L: int, p: QuantParams, gx: np.ndarray, want_coef: bool = True):
    """(dLoss/dchat [n_win*E] or None, dLoss/dgamma [3]) for output gradient gx."""
    symbols = np.ascontiguousarray(symbols, dtype=np.uint8)
    gx = np.ascontiguousarray(gx, dtype=np.float64)
    gc = np.zeros(n_windows(L, p.N) * p.E, dtype=np.float64) if want_coef else None
    gg = np.zeros(3, dtype=np.float64)
    qp = p.c()
    lib().or_backward(_ptr(symbols, ctypes.c_uint8), int(L), ctypes.byref(qp), _ptr(gx, ctypes.c_double),
                      None if gc is None else _ptr(gc, ctypes.c_double), _ptr(gg, ctypes.c_double))
    return gc, gg


def dequant_table(p: QuantParams):
    """v[k, s] and zone[k, s] for every kept bin k and symbol s (oracle side)."""
    v = np.zeros((p.E, 256))
    z = np.zeros((p.E, 256), dtype=np.int64)
    for k in range(p.E):
        for s in range(256):
            v[k, s] = dequantize(s, k, p)
            z[k, s] = zone(s, k, p)
    return v, z


def prd(x: np.ndarray, xhat: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    xhat = np.ascontiguousarray(xhat, dtype=np.float64)
    return lib().or_prd(_ptr(x, ctypes.c_float), _ptr(xhat, ctypes.c_double), x.shape[0])


def cr(orig_bytes: int, comp_bytes: int) -> float:
    return lib().or_cr(int(orig_bytes), int(comp_bytes))


def compressed_bytes(n_words: int) -> int:
    """8 bytes per word plus one symlen byte per word."""
    return 9 * int(n_words)


def mse_loss_and_grad(xhat: np.ndarray, x: np.ndarray, M: int):
    d = xhat - x.astype(np.float64)
    return float(np.sum(d * d) / M), 2.0 * d / M


def adam_refit(streams, p: QuantParams, steps: int = 20, lr: float = 1e-2,
               betas=(0.9, 0.999), eps: float = 1e-8):
    """Refit per-stream, per-zone reconstruction scales gamma by Adam on the
    batch MSE (global mean over all samples).  streams: list of
    (symbols, original float32 signal).  Returns (gamma [n,3], losses)."""
    n = len(streams)
    M = sum(int(x.shape[0]) for _, x in streams)
    gamma = np.ones((n, 3))
    m1 = np.zeros_like(gamma)
    m2 = np.zeros_like(gamma)
    losses = []
    for t in range(1, steps + 1):
        grad = np.zeros_like(gamma)
        loss = 0.0
        for i, (sym, x) in enumerate(streams):
            xh = reconstruct(sym, x.shape[0], p, gamma[i])
            d = xh - x.astype(np.float64)
            loss += float(np.sum(d * d))
            _, gg = backward(sym, x.shape[0], p, 2.0 * d / M, want_coef=False)
            grad[i] = gg
        losses.append(loss / M)
        m1 = betas[0] * m1 + (1 - betas[0]) * grad
        m2 = betas[1] * m2 + (1 - betas[1]) * grad * grad
        mh = m1 / (1 - betas[0] ** t)
        vh = m2 / (1 - betas[1] ** t)
        gamma = gamma - lr * mh / (np.sqrt(vh) + eps)
    # loss at the final gamma
    loss = 0.0
    for i, (sym, x) in enumerate(streams):
        xh = reconstruct(sym, x.shape[0], p, gamma[i])
        loss += float(np.sum((xh - x.astype(np.float64)) ** 2))
    losses.append(loss / M)
    return gamma, losses
