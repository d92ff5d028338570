"""ctypes binding of libfptc.so (include/fptc.h), same names as the C ABI.

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the decode path runs in the library's HIP
kernels.  The library is loaded from this package directory (built in-tree by
``build.py``); a missing library is an error, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfptc.so")

FPTC_OK, FPTC_ERR_INVALID_ARG, FPTC_ERR_UNSUPPORTED, FPTC_ERR_WORKSPACE, FPTC_ERR_HIP = range(5)
FPTC_STREAM_BAD_COUNT, FPTC_STREAM_OVERRUN, FPTC_STREAM_BAD_SYMLEN, FPTC_STREAM_BAD_HEADER = 1, 2, 4, 8
FPTC_FP32_SIMT, FPTC_FP16, FPTC_FP16X2, FPTC_BF16, FPTC_BF16X3 = range(5)
FPTC_NOALLOC_WS_BYTES = 16 << 20  # static workspace of fptc_decompress_batch_noalloc, per device
PRECISIONS = {"fp32": FPTC_FP32_SIMT, "fp16": FPTC_FP16, "fp16x2": FPTC_FP16X2, "bf16": FPTC_BF16,
              "bf16x3": FPTC_BF16X3}
FPTC_QUANT_AMPLITUDE, FPTC_QUANT_PAPER = 0, 1

_vp = ctypes.c_void_p


class fptc_batch(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("n_words", ctypes.c_int64),
                ("n_symbols", ctypes.c_int64), ("n_samples", ctypes.c_int64), ("words", _vp), ("symlen", _vp),
                ("word_off", _vp), ("sample_off", _vp), ("book_id", _vp)]


class fptc_codec(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("E", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("n_books", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("lut", _vp), ("deq_val", _vp), ("deq_zone", _vp), ("row_of_bin", _vp), ("basis", _vp)]


class fptc_launch(ctypes.Structure):
    _fields_ = [("windows_per_chunk", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("chunk_group", ctypes.c_int32)]


class fptc_quant_params(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("N", ctypes.c_int32), ("E", ctypes.c_int32), ("B1", ctypes.c_int32),
                ("B2", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("step_fine", ctypes.c_double),
                ("step_coarse", ctypes.c_double), ("threshold", ctypes.c_double), ("mu", ctypes.c_double),
                ("alpha1", ctypes.c_double), ("A0", ctypes.c_double), ("A1", ctypes.c_double)]


# Every function the header declares: name -> (restype, argtypes).
_P = ctypes.POINTER
_SIGS = {
    "fptc_abi_version": (ctypes.c_int32, []),
    "fptc_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "fptc_init": (ctypes.c_int32, []),
    "fptc_workspace_size": (ctypes.c_size_t, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch)]),
    "fptc_plan_batch": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp, ctypes.c_size_t,
                                         _vp, _vp]),
    "fptc_decode_batch": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp, ctypes.c_size_t,
                                           _vp, _vp, _vp]),
    "fptc_dequant_idct": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp, ctypes.c_size_t,
                                           _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "fptc_decompress_batch": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp,
                                               ctypes.c_size_t, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "fptc_dequant_idct_backward": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp,
                                                    ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]),
    "fptc_decompress_batch_noalloc": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_codec), _P(fptc_launch), _vp,
                                                       ctypes.c_int32, _vp, _vp, _vp]),
    "fptc_quantize_batch": (ctypes.c_int32, [_P(fptc_batch), _P(fptc_quant_params), _vp, _vp, _vp, _vp, _vp, _vp]),
    "fptc_histogram_batch": (ctypes.c_int32, [_P(fptc_batch), _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "fptc_percentile_workspace_size": (ctypes.c_size_t, []),
    "fptc_abs_percentile": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, _vp, _vp, ctypes.c_size_t, _vp]),
    "fptc_build_dct_table": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _vp]),
    "fptc_build_lut": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp]),
    "fptc_canonical_codes": (ctypes.c_int32, [_vp, _vp]),
    "fptc_code_lengths": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp]),
    "fptc_build_basis": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _vp]),
    "fptc_build_dequant": (ctypes.c_int32, [_P(fptc_quant_params), _vp, _vp, _vp, _P(ctypes.c_int32)]),
    "fptc_quantize_host": (ctypes.c_int32, [_vp, ctypes.c_int64, _P(fptc_quant_params), _vp]),
    "fptc_symlen_pack_host": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_int64,
                                               _P(ctypes.c_int64)]),
    "fptc_encode_batch_host": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _P(fptc_quant_params), _vp, _vp,
                                                _vp, _vp, _vp, ctypes.c_int32]),
}

_lib = None


class FptcError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({status_string(code)})")
        self.code = code


def load():
    """Load libfptc.so.  torch is imported first so that the library binds to
    the HIP runtime torch already loaded (same soname)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (or paper_2605_01086_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return list(_SIGS)


def status_string(code: int) -> str:
    return load().fptc_status_string(int(code)).decode()


def _check(fn, rc):
    if rc != FPTC_OK:
        raise FptcError(fn, rc)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError("host arrays passed to libfptc must be C-contiguous")
        return t.ctypes.data
    if not t.is_contiguous():
        raise ValueError("tensors passed to libfptc must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def fptc_abi_version() -> int:
    return load().fptc_abi_version()


def fptc_status_string(code: int) -> str:
    return status_string(code)


def fptc_init() -> None:
    _check("fptc_init", load().fptc_init())


def fptc_workspace_size(batch: fptc_batch, codec: fptc_codec, launch: fptc_launch) -> int:
    return int(load().fptc_workspace_size(ctypes.byref(batch), ctypes.byref(codec), ctypes.byref(launch)))


def fptc_plan_batch(batch, codec, launch, ws, status, stream=None):
    _check("fptc_plan_batch", load().fptc_plan_batch(ctypes.byref(batch), ctypes.byref(codec), ctypes.byref(launch),
                                                     _ptr(ws), ws.numel() * ws.element_size(), _ptr(status),
                                                     _stream(stream)))


def fptc_decode_batch(batch, codec, launch, ws, symbols_out, status, stream=None):
    _check("fptc_decode_batch", load().fptc_decode_batch(ctypes.byref(batch), ctypes.byref(codec),
                                                         ctypes.byref(launch), _ptr(ws),
                                                         ws.numel() * ws.element_size(), _ptr(symbols_out),
                                                         _ptr(status), _stream(stream)))


def fptc_dequant_idct(batch, codec, launch, ws, symbols, gamma, precision, out, stream=None):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    _check("fptc_dequant_idct", load().fptc_dequant_idct(ctypes.byref(batch), ctypes.byref(codec),
                                                         ctypes.byref(launch), _ptr(ws),
                                                         ws.numel() * ws.element_size(), _ptr(symbols), _ptr(gamma),
                                                         int(precision), _ptr(out), _stream(stream)))


def fptc_dequant_idct_backward(batch, codec, launch, ws, symbols, grad_out, grad_coeff, grad_gamma, stream=None):
    _check("fptc_dequant_idct_backward", load().fptc_dequant_idct_backward(
        ctypes.byref(batch), ctypes.byref(codec), ctypes.byref(launch), _ptr(ws), ws.numel() * ws.element_size(),
        _ptr(symbols), _ptr(grad_out), _ptr(grad_coeff), _ptr(grad_gamma), _stream(stream)))


def fptc_decompress_batch(batch, codec, launch, ws, gamma, precision, out, status, stream=None):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    _check("fptc_decompress_batch", load().fptc_decompress_batch(ctypes.byref(batch), ctypes.byref(codec),
                                                                 ctypes.byref(launch), _ptr(ws),
                                                                 ws.numel() * ws.element_size(), _ptr(gamma),
                                                                 int(precision), _ptr(out), _ptr(status),
                                                                 _stream(stream)))


def fptc_decompress_batch_noalloc(batch, codec, launch, gamma, precision, out, status, stream=None):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    _check("fptc_decompress_batch_noalloc", load().fptc_decompress_batch_noalloc(
        ctypes.byref(batch), ctypes.byref(codec), ctypes.byref(launch), _ptr(gamma), int(precision), _ptr(out),
        _ptr(status), _stream(stream)))


def fptc_quantize_batch(batch, q, dct_table, sym_off, x, symbols_out, coef_out=None, stream=None):
    _check("fptc_quantize_batch", load().fptc_quantize_batch(ctypes.byref(batch), ctypes.byref(q), _ptr(dct_table),
                                                             _ptr(sym_off), _ptr(x), _ptr(symbols_out),
                                                             _ptr(coef_out), _stream(stream)))


def fptc_histogram_batch(batch, sym_off, symbols, n_books, counts, stream=None):
    _check("fptc_histogram_batch", load().fptc_histogram_batch(ctypes.byref(batch), _ptr(sym_off), _ptr(symbols),
                                                               int(n_books), _ptr(counts), _stream(stream)))


def fptc_percentile_workspace_size() -> int:
    return int(load().fptc_percentile_workspace_size())


def fptc_abs_percentile(coef, n_windows, E, k0, k1, p, out, ws, stream=None):
    _check("fptc_abs_percentile", load().fptc_abs_percentile(_ptr(coef), int(n_windows), int(E), int(k0), int(k1),
                                                             float(p), _ptr(out), _ptr(ws),
                                                             ws.numel() * ws.element_size(), _stream(stream)))


# ------------------------------------------------------------ host calls


def fptc_build_dct_table(N: int, E: int) -> np.ndarray:
    t = np.zeros((E, N + 1), dtype=np.float64)
    _check("fptc_build_dct_table", load().fptc_build_dct_table(int(N), int(E), _ptr(t)))
    return t



def fptc_build_lut(code_len: np.ndarray, lmax: int) -> np.ndarray:
    code_len = np.ascontiguousarray(code_len, dtype=np.uint8)
    lut = np.zeros(1 << lmax, dtype=np.uint16)
    _check("fptc_build_lut", load().fptc_build_lut(_ptr(code_len), int(lmax), _ptr(lut)))
    return lut


def fptc_canonical_codes(code_len: np.ndarray) -> np.ndarray:
    code_len = np.ascontiguousarray(code_len, dtype=np.uint8)
    out = np.zeros(256, dtype=np.uint32)
    _check("fptc_canonical_codes", load().fptc_canonical_codes(_ptr(code_len), _ptr(out)))
    return out


def fptc_code_lengths(freq: np.ndarray, lmax: int) -> np.ndarray:
    freq = np.ascontiguousarray(freq, dtype=np.uint64)
    out = np.zeros(256, dtype=np.uint8)
    _check("fptc_code_lengths", load().fptc_code_lengths(_ptr(freq), int(lmax), _ptr(out)))
    return out


def fptc_build_basis(N: int, E: int) -> np.ndarray:
    out = np.zeros((E, N), dtype=np.float32)
    _check("fptc_build_basis", load().fptc_build_basis(int(N), int(E), _ptr(out)))
    return out


def fptc_build_dequant(q: fptc_quant_params):
    val = np.zeros((4, 256), dtype=np.float32)
    zone = np.zeros((4, 256), dtype=np.uint8)
    rob = np.zeros(q.E, dtype=np.uint8)
    nr = ctypes.c_int32(0)
    _check("fptc_build_dequant", load().fptc_build_dequant(ctypes.byref(q), _ptr(val), _ptr(zone), _ptr(rob),
                                                           ctypes.byref(nr)))
    return val[:nr.value].copy(), zone[:nr.value].copy(), rob


def fptc_quantize_host(x: np.ndarray, q: fptc_quant_params) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    nw = (x.shape[0] + q.N - 1) // q.N
    out = np.zeros(nw * q.E, dtype=np.uint8)
    _check("fptc_quantize_host", load().fptc_quantize_host(_ptr(x), x.shape[0], ctypes.byref(q), _ptr(out)))
    return out


def fptc_symlen_pack_host(symbols: np.ndarray, code_len: np.ndarray):
    symbols = np.ascontiguousarray(symbols, dtype=np.uint8)
    code_len = np.ascontiguousarray(code_len, dtype=np.uint8)
    cap = max(1, symbols.shape[0])
    words = np.zeros(cap, dtype=np.uint64)
    symlen = np.zeros(cap, dtype=np.uint8)
    n = ctypes.c_int64(0)
    _check("fptc_symlen_pack_host", load().fptc_symlen_pack_host(_ptr(symbols), symbols.shape[0], _ptr(code_len),
                                                                 _ptr(words), _ptr(symlen), cap, ctypes.byref(n)))
    return words[:n.value].copy(), symlen[:n.value].copy()


def fptc_encode_batch_host(x: np.ndarray, sample_off: np.ndarray, book_id, q: fptc_quant_params,
                           code_len: np.ndarray, word_cap_off: np.ndarray, words: np.ndarray, symlen: np.ndarray,
                           n_threads: int = 0) -> np.ndarray:
    n = sample_off.shape[0] - 1
    n_words = np.zeros(n, dtype=np.int64)
    bid = None if book_id is None else np.ascontiguousarray(book_id, dtype=np.uint8)
    code_len = np.ascontiguousarray(code_len, dtype=np.uint8)
    _check("fptc_encode_batch_host", load().fptc_encode_batch_host(
        _ptr(x), _ptr(sample_off), n, _ptr(bid), ctypes.byref(q), _ptr(code_len), _ptr(word_cap_off),
        _ptr(words), _ptr(symlen), _ptr(n_words), int(n_threads)))
    return n_words
