"""Helpers for the GPU parity tests: run the HIP path through the C ABI on an
oracle-built case, with sentinel guard bands around every output buffer."""
from __future__ import annotations

import numpy as np

from cases import Case, range_rel_err

PAD = 256  # guard elements after every output buffer
SENT_U8 = 0xA5
SENT_F32 = np.float32(-12345.678)


def qparams(p):
    from paper_2605_01086_amd import codec as C
    if p.kind == "amp":
        return C.quant_params("amp", p.N, p.E, step_fine=p.step_f, step_coarse=p.step_c, threshold=p.T)
    return C.quant_params("paper", p.N, p.E, B1=p.B1, B2=p.B2, mu=p.mu, alpha1=p.alpha1, A0=p.A0, A1=p.A1)


def run_gpu(case: Case, launch=None, precision="fp32", use_gamma=True, words_override=None, symlen_override=None,
            repeat=1, fused=False):
    import torch
    from paper_2605_01086_amd import codec as C
    from paper_2605_01086_amd import fptc as F
    p = case.p
    words, symlen, word_off, sample_off = case.concat()
    if words_override is not None:
        words = words_override
    if symlen_override is not None:
        symlen = symlen_override
    codec = C.DeviceCodec(np.stack([b.lengths for b in case.books]), qparams(p), case.lmax)
    batch = C.DeviceBatch(words, symlen, word_off, sample_off, p.N, p.E, case.book_id)
    L = launch or C.Launch()
    lc = L.c()
    dev = batch.word_off.device
    ws = torch.empty(F.fptc_workspace_size(batch.c, codec.c, lc), dtype=torch.uint8, device=dev)
    status = torch.full((batch.n_streams,), -1, dtype=torch.int32, device=dev)
    sym = torch.full((batch.n_symbols + PAD,), SENT_U8, dtype=torch.uint8, device=dev)
    out = torch.full((batch.n_samples + PAD,), float(SENT_F32), dtype=torch.float32, device=dev)
    gamma = None
    if use_gamma and case.gamma is not None:
        gamma = torch.from_numpy(case.gamma.astype(np.float32)).to(dev)
    results = []
    for _ in range(repeat):
        F.fptc_plan_batch(batch.c, codec.c, lc, ws, status)
        if fused:
            F.fptc_decompress_batch(batch.c, codec.c, lc, ws, gamma, precision, out, status)
        else:
            F.fptc_decode_batch(batch.c, codec.c, lc, ws, sym, status)
            F.fptc_dequant_idct(batch.c, codec.c, lc, ws, sym, gamma, precision, out)
        torch.cuda.synchronize()
        results.append((sym.cpu().numpy().copy(), out.cpu().numpy().copy(), status.cpu().numpy().copy()))
    s_h, o_h, st_h = results[-1]
    if fused:
        assert np.all(s_h == SENT_U8), "the fused path must not touch the symbol array"
    assert np.all(s_h[batch.n_symbols:] == SENT_U8), "decode wrote past the symbol array"
    assert np.all(o_h[batch.n_samples:] == SENT_F32), "dequant+IDCT wrote past the output array"
    return dict(sym=s_h[:batch.n_symbols], out=o_h[:batch.n_samples], status=st_h, batch=batch, runs=results)


def _diagnose(case: Case, res) -> str:
    """Describe which windows of which streams disagree."""
    batch = res["batch"]
    N = case.p.N
    lines = []
    nbad_streams = 0
    for i in range(len(case.signals)):
        o0, o1 = batch.sample_off_h[i], batch.sample_off_h[i + 1]
        d = np.abs(res["out"][o0:o1].astype(np.float64) - case.recon[i])
        rng = float(np.ptp(case.recon[i])) if case.recon[i].size else 1.0
        bad = np.flatnonzero(d > 1e-5 * max(rng, 1e-30))
        if bad.size:
            nbad_streams += 1
            wins = np.unique(bad // N)
            if len(lines) < 6:
                lines.append(f"stream {i}: L={o1 - o0} bad samples {bad.size} in {wins.size} windows "
                             f"(first {wins[:6].tolist()}), got {res['out'][o0 + bad[0]]:.4f} "
                             f"want {case.recon[i][bad[0]]:.4f}")
    lines.insert(0, f"{nbad_streams} of {len(case.signals)} streams disagree")
    return "\n".join(lines)


def check_parity(case: Case, res, tol=1e-5, skip=(), check_symbols=True):
    batch = res["batch"]
    worst = 0.0
    for i in range(len(case.signals)):
        if i in skip:
            continue
        assert res["status"][i] == 0, (i, res["status"][i])
        s0, s1 = batch.sym_off_h[i], batch.sym_off_h[i + 1]
        got = res["sym"][s0:s1]
        if check_symbols:
            assert np.array_equal(got, case.symbols[i]), \
                f"stream {i}: symbols differ at {np.flatnonzero(got != case.symbols[i])[:8]}"
        o0, o1 = batch.sample_off_h[i], batch.sample_off_h[i + 1]
        err = range_rel_err(res["out"][o0:o1], case.recon[i])
        worst = max(worst, err)
        if err > tol:
            raise AssertionError(f"stream {i}: range-relative error {err:.3e} > {tol}\n" + _diagnose(case, res))
    return worst
