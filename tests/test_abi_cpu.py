"""CPU checks of the C ABI library: it loads without a GPU, exports every
symbol its header declares, its host table builders and host encoder agree
with the oracle, and argument errors return before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from conftest import ROOT

F = pytest.importorskip("paper_2605_01086_amd.fptc")


def header_functions():
    src = open(os.path.join(ROOT, "include", "fptc.h")).read()
    return sorted(set(re.findall(r"FPTC_API[^;(]*?\b(fptc_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = F.load()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(F.exported_names()) == names
    assert F.fptc_abi_version() == 1


def _trained_lengths(O, domain, N=64):
    p = O.QuantParams("amp", N, N)
    x = synth.domain_signal(domain, 1 << 15, synth.training_rng(3, 0)).astype(np.float32)
    return O.train_codebook(O.quantize_stream(x, p)).lengths


@pytest.mark.parametrize("domain", ["eeg", "seismic", "power", "meteo", "long16"])
def test_lut_matches_oracle_canonical_codes(O, domain):
    if domain == "long16":  # codes up to 16 bits
        r = np.abs(np.arange(256) - 128).astype(np.float64)
        lens, lmax = O.package_merge((1 + r ** 3).astype(np.uint64), 16), 16
        assert lens.max() == 16
    else:
        lens, lmax = _trained_lengths(O, domain), 12
    codes = O.canonical_codes(lens)
    assert np.array_equal(F.fptc_canonical_codes(lens), codes)
    lut = F.fptc_build_lut(lens, lmax)
    expect = np.zeros(1 << lmax, dtype=np.uint16)
    for s in range(256):
        l = int(lens[s])
        for tail in range(1 << (lmax - l)):
            expect[(int(codes[s]) << (lmax - l)) | tail] = (l << 8) | s
    assert np.array_equal(lut, expect)


@pytest.mark.parametrize("lmax", [13, 14, 16])
def test_code_lengths_at_long_limits_cost_the_oracle_optimum(O, lmax):
    # length-limited optimum (package-merge) above 12 bits: same cost as the
    # oracle's, Kraft equality, the limit reached
    rng = np.random.default_rng(lmax)
    freq = np.floor(2.0 ** rng.uniform(0, 30, 256)).astype(np.uint64)
    ours = F.fptc_code_lengths(freq, lmax)
    ref = O.package_merge(freq, lmax)
    assert int(ours.max()) <= lmax and int(ref.max()) == lmax
    assert sum(int(f) * int(l) for f, l in zip(freq, ours)) == sum(int(f) * int(l) for f, l in zip(freq, ref))
    assert sum(1 << (lmax - int(l)) for l in ours if l) == 1 << lmax


def test_lut_rejects_bad_lengths():
    lens = np.zeros(256, dtype=np.uint8)
    lens[:3] = 1  # Kraft sum 3/2
    with pytest.raises(F.FptcError):
        F.fptc_build_lut(lens, 12)
    lens[:] = 0
    lens[0] = 13
    with pytest.raises(F.FptcError):
        F.fptc_build_lut(lens, 12)


@pytest.mark.parametrize("seed", range(5))
def test_code_lengths_are_optimal_like_oracle(O, seed):
    rng = np.random.default_rng(seed)
    freq = (rng.pareto(1.0, size=256) * 100 + 1).astype(np.uint64)
    a = F.fptc_code_lengths(freq, 12)
    b = O.package_merge(freq, 12)
    cost = lambda l: int(np.sum(freq.astype(np.int64) * l.astype(np.int64)))
    assert cost(a) == cost(b)
    assert a.max() <= 12 and sum(1 << (12 - int(l)) for l in a) == 4096


@pytest.mark.parametrize("N,E", [(4, 4), (64, 64), (128, 96), (256, 256)])
def test_basis_matches_oracle_dct(O, N, E):
    B = F.fptc_build_basis(N, E)
    ref = np.stack([O.dct_ortho(np.eye(N)[n]) for n in range(N)], axis=1)[:E]
    assert np.max(np.abs(B - ref)) <= 2.0 ** -24


@pytest.mark.parametrize("kind", ["amp", "paper"])
def test_dequant_tables_match_oracle(O, kind):
    from paper_2605_01086_amd import codec as C
    if kind == "amp":
        p = O.QuantParams("amp", 64, 64, step_f=1.0, step_c=8.0, T=16.0)
        q = C.quant_params("amp", 64, 64, step_fine=1.0, step_coarse=8.0, threshold=16.0)
    else:
        p = O.QuantParams("paper", 32, 16, B1=2, B2=10, mu=50.0, alpha1=0.004, A0=41.5, A1=7.25)
        q = C.quant_params("paper", 32, 16, B1=2, B2=10, mu=50.0, alpha1=0.004, A0=41.5, A1=7.25)
    val, zone, rob = F.fptc_build_dequant(q)
    for k in range(p.E):
        for s in range(256):
            v = O.dequantize(s, k, p)
            assert val[rob[k], s] == np.float32(v)
            assert zone[rob[k], s] == O.zone(s, k, p)


@pytest.mark.parametrize("kind,domain", [("amp", "eeg"), ("amp", "seismic"), ("paper", "meteo")])
def test_host_encoder_matches_oracle(O, kind, domain):
    from paper_2605_01086_amd import codec as C
    if kind == "amp":
        p = O.QuantParams("amp", 64, 64)
        q = C.quant_params("amp", 64, 64)
    else:
        p = O.QuantParams("paper", 32, 16, B1=2, B2=10, mu=50.0, alpha1=0.004, A0=60.0, A1=3.0)
        q = C.quant_params("paper", 32, 16, B1=2, B2=10, mu=50.0, alpha1=0.004, A0=60.0, A1=3.0)
    x = synth.domain_signal(domain, 64 * 300 + 19, synth.stream_rng(4, 0)).astype(np.float32)
    cb = O.train_codebook(O.quantize_stream(x, p))
    sym = F.fptc_quantize_host(x, q)
    assert np.array_equal(sym, O.quantize_stream(x, p))
    w, sl = F.fptc_symlen_pack_host(sym, cb.lengths)
    wo, slo = O.symlen_pack(sym, cb)
    assert np.array_equal(w, wo) and np.array_equal(sl, slo)
    # batch encoder, several streams and two books
    xs = [x, x[:1000], x[:1], x[5:64 * 7]]
    words, symlen, word_off, sample_off = C.encode_batch(xs, [0, 1, 0, 1], q, np.stack([cb.lengths, cb.lengths]))
    for i, xi in enumerate(xs):
        wi, si, _ = O.encode_stream(xi, p, cb)
        assert np.array_equal(words[word_off[i]:word_off[i + 1]], wi)
        assert np.array_equal(symlen[word_off[i]:word_off[i + 1]], si)


def _fake_structs():
    b = F.fptc_batch(2, 0, 10, 128, 100, 16, 16, 16, 16, None)
    c = F.fptc_codec(64, 64, 12, 1, 1, 0, 16, 16, 16, 16, 16)
    l = F.fptc_launch(0, 0, 0, 0)
    return b, c, l


def test_argument_errors_return_before_any_launch():
    lib = F.load()
    b, c, l = _fake_structs()
    ok = F.fptc_workspace_size(b, c, l)
    assert ok > 0
    by = ctypes.byref
    # too-small workspace
    assert lib.fptc_plan_batch(by(b), by(c), by(l), 16, ok - 1, 16, None) == F.FPTC_ERR_WORKSPACE
    assert lib.fptc_decode_batch(by(b), by(c), by(l), 16, ok - 1, 16, 16, None) == F.FPTC_ERR_WORKSPACE
    assert lib.fptc_dequant_idct(by(b), by(c), by(l), 16, ok - 1, 16, None, 0, 16, None) == F.FPTC_ERR_WORKSPACE
    # precision out of range
    assert lib.fptc_dequant_idct(by(b), by(c), by(l), 16, ok, 16, None, 9, 16, None) == F.FPTC_ERR_INVALID_ARG
    # NULL workspace / outputs
    assert lib.fptc_plan_batch(by(b), by(c), by(l), None, ok, 16, None) == F.FPTC_ERR_INVALID_ARG
    assert lib.fptc_decode_batch(by(b), by(c), by(l), 16, ok, None, 16, None) == F.FPTC_ERR_INVALID_ARG
    # invalid batch and codec fields
    for field, bad in [("n_streams", 0), ("n_words", -1), ("word_off", None), ("sample_off", None)]:
        bb, cc, ll = _fake_structs()
        setattr(bb, field, bad)
        assert F.fptc_workspace_size(bb, cc, ll) == 0
        assert lib.fptc_plan_batch(by(bb), by(cc), by(ll), 16, 1 << 30, 16, None) == F.FPTC_ERR_INVALID_ARG
    for field, bad in [("N", 3), ("N", 512), ("E", 0), ("E", 65), ("lmax", 17), ("lmax", 0), ("n_books", 9), ("n_rows", 0),
                       ("lut", None), ("basis", None)]:
        bb, cc, ll = _fake_structs()
        setattr(cc, field, bad)
        assert F.fptc_workspace_size(bb, cc, ll) == 0
        assert lib.fptc_decode_batch(by(bb), by(cc), by(ll), 16, 1 << 30, 16, 16, None) == F.FPTC_ERR_INVALID_ARG
    for field, bad in [("windows_per_chunk", -1), ("waves_per_block", 17), ("blocks", -2)]:
        bb, cc, ll = _fake_structs()
        setattr(ll, field, bad)
        assert F.fptc_workspace_size(bb, cc, ll) == 0
    # a decode chunk whose symbol buffers cannot fit in LDS is refused before launch
    bb, cc, ll = _fake_structs()
    bb.n_symbols = 1 << 20
    cc.N, cc.E, ll.windows_per_chunk, ll.waves_per_block = 256, 256, 1024, 16
    size = F.fptc_workspace_size(bb, cc, ll)
    assert size > 0
    assert lib.fptc_decode_batch(by(bb), by(cc), by(ll), 16, size, 16, 16, None) == F.FPTC_ERR_UNSUPPORTED
    # the fused path: unsupported precision / window size / LDS budget
    bb, cc, ll = _fake_structs()
    size = F.fptc_workspace_size(bb, cc, ll)
    assert lib.fptc_decompress_batch(by(bb), by(cc), by(ll), 16, size, None, 0, 16, 16, None) == F.FPTC_ERR_UNSUPPORTED
    cc.N, cc.E = 16, 16
    size = F.fptc_workspace_size(bb, cc, ll)
    assert lib.fptc_decompress_batch(by(bb), by(cc), by(ll), 16, size, None, 2, 16, 16, None) == F.FPTC_ERR_UNSUPPORTED
    cc.N, cc.E, cc.n_books = 128, 128, 8
    ll.windows_per_chunk, ll.waves_per_block = 1024, 16
    size = F.fptc_workspace_size(bb, cc, ll)
    assert lib.fptc_decompress_batch(by(bb), by(cc), by(ll), 16, size, None, 4, 16, 16, None) == F.FPTC_ERR_UNSUPPORTED


def test_codec_tables_are_dense_row_major_per_book(O):
    # regression: per-book table copies must reach the C ABI as dense
    # [n_books][n_rows][256] buffers whatever numpy layout they were built in
    from paper_2605_01086_amd import codec as C
    lens = np.stack([_trained_lengths(O, d) for d in ("eeg", "seismic", "power")])
    q = C.quant_params("paper", 32, 16, B1=2, B2=10, mu=50.0, alpha1=0.004, A0=41.5, A1=7.25)
    cd = C.DeviceCodec(lens, q, 12, device="cpu")
    val, zone, rob = F.fptc_build_dequant(q)
    for t in (cd.lut, cd.deq_val, cd.deq_zone, cd.row_of_bin, cd.basis):
        assert t.is_contiguous()
    flat = cd.deq_val.numpy().ravel()
    for b in range(3):
        assert np.array_equal(flat[b * 3 * 256:(b + 1) * 3 * 256], val.ravel())
        assert np.array_equal(cd.lut.numpy().view(np.uint16)[b], F.fptc_build_lut(lens[b], 12))
    with pytest.raises(ValueError):
        F._ptr(np.zeros((4, 4))[:, ::2])


@pytest.mark.parametrize("N", [4, 16, 64, 256])
def test_dct_table_gives_the_oracle_transform_bit_for_bit(O, N):
    # the table's cosines and scales, summed in n order with separately
    # rounded products and sums (the GPU encoder's arithmetic), reproduce the
    # oracle's FP64 DCT-II exactly; and the transform is the orthonormal one
    import scipy.fft
    tab = F.fptc_build_dct_table(N, N)
    assert tab.shape == (N, N + 1)
    rng = np.random.default_rng(N)
    for _ in range(3):
        x = rng.normal(0, 30, N).astype(np.float32).astype(np.float64)
        got = np.empty(N)
        for k in range(N):
            s = 0.0
            for n in range(N):
                s = s + float(x[n]) * float(tab[k, n])
            got[k] = float(tab[k, N]) * s
        assert np.array_equal(got, O.dct_stream(x.astype(np.float32), N, N))
        np.testing.assert_allclose(got, scipy.fft.dct(x, type=2, norm="ortho"), rtol=0, atol=1e-12 * np.abs(x).sum())


def test_dct_table_rejects_bad_sizes():
    with pytest.raises(F.FptcError):
        F.fptc_build_dct_table(12, 4)
    with pytest.raises(F.FptcError):
        F.fptc_build_dct_table(64, 65)


def test_window_sample_index_matches_a_loop():
    # the output position of every window sample (the coefficient input of
    # the autograd Function scatters through it)
    from paper_2605_01086_amd.refit import window_sample_index
    for N, lens in [(4, [0, 1, 4, 5, 9]), (64, [64 * 3 + 7, 0, 1, 128]), (256, [300, 256, 2])]:
        so = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        want = []
        for s, L in enumerate(lens):
            for w in range((L + N - 1) // N):
                for n in range(N):
                    pos = w * N + n
                    want.append(so[s] + pos if pos < L else -1)
        assert np.array_equal(window_sample_index(so, N), np.array(want, dtype=np.int64))
