"""GPU parity of the encode-side steps against the CPU oracle: the FP64
forward transform and quantizer (symbols bit-exact, coefficients bit-exact),
the per-codebook symbol histogram (exact counts) and the clipped zone maxima
A0 / A1 (the oracle's numpy percentile, bit-exact)."""
import numpy as np
import pytest

import synth
from cases import paper_params

pytestmark = pytest.mark.gpu


def _strips(domains, lengths, config_id):
    xs = [synth.domain_signal(domains[i % len(domains)], int(L), synth.stream_rng(config_id, i)).astype(np.float32)
          for i, L in enumerate(lengths)]
    return xs


def _gpu_quantize(q, xs, book_id=None, want_coef=True):
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    lens = np.array([len(x) for x in xs], dtype=np.int64)
    sample_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    sym_off = np.concatenate([[0], np.cumsum(C.n_windows(lens, q.N) * q.E)]).astype(np.int64)
    dev = torch.device("cuda")
    so = torch.from_numpy(sample_off).to(dev)
    yo = torch.from_numpy(sym_off).to(dev)
    bid = None if book_id is None else torch.from_numpy(np.asarray(book_id, np.uint8)).to(dev)
    x = torch.from_numpy(np.concatenate(xs) if xs else np.zeros(0, np.float32)).to(dev)
    n_sym = int(sym_off[-1])
    b = F.fptc_batch(len(xs), 0, 0, n_sym, int(sample_off[-1]), None, None, None, so.data_ptr(),
                     None if bid is None else bid.data_ptr())
    tab = torch.from_numpy(F.fptc_build_dct_table(q.N, q.E)).to(dev)
    sym = torch.full((n_sym + 64,), 0xA5, dtype=torch.uint8, device=dev)
    coef = torch.full((n_sym + 8,), -1.0, dtype=torch.float64, device=dev) if want_coef else None
    F.fptc_quantize_batch(b, q, tab, yo, x, sym, coef)
    torch.cuda.synchronize()
    s = sym.cpu().numpy()
    assert np.all(s[n_sym:] == 0xA5), "quantize wrote past the symbol array"
    c = None
    if want_coef:
        c = coef.cpu().numpy()
        assert np.all(c[n_sym:] == -1.0)
        c = c[:n_sym]
    return dict(sym=s[:n_sym], coef=c, sym_off=sym_off, batch=b, yo=yo, symt=sym, coeft=coef, keep=(so, bid, x))


def _qp(p):
    from paper_2605_01086_amd import codec as C
    if p.kind == "amp":
        return C.quant_params("amp", p.N, p.E, step_fine=p.step_f, step_coarse=p.step_c, threshold=p.T)
    return C.quant_params("paper", p.N, p.E, B1=p.B1, B2=p.B2, mu=p.mu, alpha1=p.alpha1, A0=p.A0, A1=p.A1)


CASES = [("amp", 64, 64, {}), ("amp", 16, 8, {}), ("amp", 256, 256, dict(step_f=1.0, step_c=8.0)),
         ("amp", 128, 100, {}), ("paper", 32, 16, {}), ("paper", 128, 100, {}), ("paper", 4, 4, {})]


@pytest.mark.parametrize("kind,N,E,kw", CASES)
def test_quantize_matches_oracle_bit_exact(O, kind, N, E, kw):
    if kind == "amp":
        p = O.QuantParams("amp", N, E, **kw)
    else:
        p = paper_params(N, E, "eeg", 2400 + N, B1=min(2, E), B2=min(E, max(2, E // 2)))
    rng = np.random.default_rng(2400 + N + E)
    lens = list(np.floor(2.0 ** rng.uniform(4, 15, size=10)).astype(int)) + [1, N - 1 if N > 1 else 1, N, 3 * N + 1]
    xs = _strips(["eeg", "seismic", "power", "meteo"], lens, 2400 + N)
    g = _gpu_quantize(_qp(p), xs)
    for i, x in enumerate(xs):
        a, b = g["sym_off"][i], g["sym_off"][i + 1]
        want = O.quantize_stream(x, p)
        got = g["sym"][a:b]
        assert np.array_equal(got, want), f"stream {i}: symbols differ at {np.flatnonzero(got != want)[:8]}"
        cw = O.dct_stream(x, N, E)
        assert np.array_equal(g["coef"][a:b], cw), f"stream {i}: coefficients differ"


def test_histogram_per_book_matches_oracle(O):
    import torch
    from paper_2605_01086_amd import fptc as F
    p = O.QuantParams("amp", 64, 64)
    rng = np.random.default_rng(2500)
    lens = list(np.floor(2.0 ** rng.uniform(6, 16, size=24)).astype(int)) + [1, 64]
    book = (np.arange(len(lens)) % 3).astype(np.uint8)
    xs = _strips(["eeg", "seismic", "power"], lens, 2500)
    g = _gpu_quantize(_qp(p), xs, book_id=book, want_coef=False)
    counts = torch.zeros((4, 256), dtype=torch.int64, device="cuda")
    F.fptc_histogram_batch(g["batch"], g["yo"], g["symt"], 4, counts)
    F.fptc_histogram_batch(g["batch"], g["yo"], g["symt"], 4, counts)  # adds: twice the counts
    torch.cuda.synchronize()
    got = counts.cpu().numpy().astype(np.uint64)
    want = np.zeros((4, 256), dtype=np.uint64)
    for i, x in enumerate(xs):
        want[book[i]] += O.histogram(O.quantize_stream(x, p))
    assert np.array_equal(got, 2 * want)
    assert got[3].sum() == 0


@pytest.mark.parametrize("N,E,B1,B2", [(32, 16, 2, 16), (64, 64, 4, 32), (128, 100, 1, 50)])
def test_zone_maxima_match_oracle_bit_exact(O, N, E, B1, B2):
    import torch
    from paper_2605_01086_amd import fptc as F
    p = O.QuantParams("paper", N, E, B1=B1, B2=B2)
    train = (3.0 * synth.domain_signal("eeg", (1 << 16) + 13, synth.training_rng(2600 + N, 0))).astype(np.float32)
    g = _gpu_quantize(_qp(p), [train])
    coef_dev = g["coeft"]
    nw = O.n_windows(len(train), N)
    ws = torch.empty(F.fptc_percentile_workspace_size(), dtype=torch.uint8, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    want0, want1 = O.paper_zone_maxima(train, p, 99.9)
    F.fptc_abs_percentile(coef_dev, nw, E, 0, B1, 99.9, out[0:1], ws)
    F.fptc_abs_percentile(coef_dev, nw, E, B1, B2, 99.9, out[1:2], ws)
    # other percentiles and ranges against numpy on the oracle's coefficients
    ref = np.abs(O.dct_stream(train, N, E).reshape(-1, E))
    extra = [(0, E, 50.0), (0, E, 0.0), (0, E, 100.0), (B1, E, 37.3)]
    for j, (k0, k1, pc) in enumerate(extra):
        F.fptc_abs_percentile(coef_dev, nw, E, k0, k1, pc, out[2 + j:3 + j], ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[0] == want0 and got[1] == want1, (got[:2], want0, want1)
    for j, (k0, k1, pc) in enumerate(extra):
        assert got[2 + j] == np.percentile(ref[:, k0:k1].ravel(), pc, method="linear"), (k0, k1, pc)
